"""Batches: many scenes stepped by one graph launch give, scene by scene,
bitwise the results of the scene stepped alone, and the oracle's results
element by element."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
requires_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU")

FIELDS = ("ptype", "i", "j", "code", "flags", "d", "E", "G", "Hpsd", "g", "row_ptr", "col", "val")


def _scenes():
    return [synth.woven_patch(seed=11, n_warp=2, n_weft=3, verts_per_rod=64),
            synth.folded_cloth(seed=12, n=40, gaps=()),
            synth.woven_patch(seed=13, n_warp=4, n_weft=4, verts_per_rod=96),
            synth.folded_cloth(seed=14, n=72, gaps=(950.0,), l_mid=4000.0, l_conv=2000.0),
            synth.helix_loop_rod(),
            synth.folded_cloth(seed=15, n=24, gaps=())]


def _fill_outputs(cs):
    for t in (cs.l_E, cs.l_G, cs.l_H, cs.E, cs.g, cs.val):
        t.fill_(float("nan"))
    for t in (cs.a_i, cs.a_j, cs.col, cs.row_ptr):
        t.fill_(-7)


@requires_gpu
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("lanes", [1, 2, 0])
def test_batch_equals_alone(prec, lanes):
    import paper_2510_10256_amd as bfc
    p = bfc.BF_FP64 if prec == "fp64" else bfc.BF_MIXED
    scenes = _scenes()
    print(f"[batch] prec={prec} lanes={lanes} scenes={len(scenes)}", flush=True)
    dev = torch.device("cuda:0")
    css, xs, alone = [], [], []
    for sc in scenes:
        cs = bfc.ContactScene(sc, prec=p, device=dev)
        x = torch.tensor(sc.x, dtype=torch.float64, device=dev)
        cs.run(x)
        alone.append(cs.results())
        oc = oracle.counts(oracle.evaluate(sc, mode=1, derivs=False))
        for k in ("n_c", "n_filt", "n_act", "n_infeasible"):
            assert alone[-1]["counts"][k] == oc[k], (sc.name, k)
        _fill_outputs(cs)
        css.append(cs)
        xs.append(x)
    batch = bfc.Batch(css, xs, lanes=lanes)
    print(f"[batch] lanes in use {batch.lanes}", flush=True)
    for rep in range(3):  # replays keep giving the same results
        for cs in css:
            _fill_outputs(cs)
        batch.step()
        torch.cuda.synchronize()
        for k, cs in enumerate(css):
            got = cs.results()
            assert got["counts"] == alone[k]["counts"], (k, rep)
            for f in FIELDS:
                assert np.array_equal(got[f], alone[k][f], equal_nan=True), (k, rep, f)
            assert got["E_total"] == alone[k]["E_total"]
    batch.close()
    for cs in css:
        cs.close()


@requires_gpu
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_scenes_match_the_oracle(prec):
    # every scene of a batch step (four lanes), element by element against the
    # oracle: active set, counts, per-pair values and the assembly
    import paper_2510_10256_amd as bfc
    from tests.parity import compare
    p = bfc.BF_FP64 if prec == "fp64" else bfc.BF_MIXED
    scenes = _scenes()
    print(f"[batch vs oracle] prec={prec} scenes={len(scenes)}", flush=True)
    dev = torch.device("cuda:0")
    css, xs = [], []
    for sc in scenes:
        cs = bfc.ContactScene(sc, prec=p, device=dev)
        x = torch.tensor(sc.x, dtype=torch.float64, device=dev)
        cs.run(x)
        _fill_outputs(cs)
        css.append(cs)
        xs.append(x)
    batch = bfc.Batch(css, xs, lanes=0)
    batch.step()
    torch.cuda.synchronize()
    for sc, cs in zip(scenes, css):
        g = cs.results()
        g["x"] = sc.x
        rep = compare(g, oracle.evaluate(sc, mode=1), sc.n_verts, kappa=sc.kappa,
                      tau=1e-10 if prec == "fp64" else 1e-5)
        print(sc.name, g["counts"], rep, flush=True)
    batch.close()
    for cs in css:
        cs.close()


@requires_gpu
def test_steps_repeat_bitwise():
    # the same inputs give bitwise the same outputs from step to step (no
    # result depends on the order in which atomics complete)
    import paper_2510_10256_amd as bfc
    sc = synth.folded_cloth(seed=16, n=96, gaps=(950.0,), l_mid=4000.0, l_conv=2000.0)
    print(f"[repeat] V={sc.n_verts}", flush=True)
    cs = bfc.ContactScene(sc, device="cuda:0")
    x = torch.tensor(sc.x, dtype=torch.float64, device="cuda:0")
    cs.run(x)
    first = cs.results()
    for _ in range(3):
        _fill_outputs(cs)
        cs.step(x)
        got = cs.results()
        assert np.array_equal(got["cand"], first["cand"])
        for f in FIELDS:
            assert np.array_equal(got[f], first[f], equal_nan=True), f
    cs.close()
