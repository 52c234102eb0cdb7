"""GPU edge cases of the step against the oracle: nothing in contact, a
single pair, a pair inside the offset (infeasible), a shell without contact,
and a scene whose only candidates are filtered stencil neighbours.

Every case runs the four calls of a step and must equal the oracle (active
set, counts, energies, gradients, assembled blocks); the empty cases must
give zero counts, a zero energy and gradient and an empty block matrix.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.parity import compare

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
requires_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU")

H, ETA = 300.0, 270.0


def _rods(segments, h=H, eta=ETA, name="rods"):
    """Polylines given as lists of points; arc length per vertex."""
    xs, es, ref, base = [], [], [], 0
    for pts in segments:
        p = np.asarray(pts, float)
        xs.append(p)
        n = len(p)
        es.append(np.stack([np.arange(n - 1), np.arange(1, n)], 1) + base)
        ref.append(np.concatenate([[0.0], np.cumsum(np.linalg.norm(np.diff(p, axis=0), axis=1))]))
        base += n
    return synth.scenes.Scene(name, "rod", np.concatenate(xs), np.concatenate(es).astype(np.int32),
                              np.zeros((0, 3), np.int32), np.concatenate(ref), h=h, eta=eta, seed=0)


def _sheet(n, ell, z=0.0):
    g = np.arange(n) * ell
    X, Y = np.meshgrid(g, g, indexing="ij")
    x = np.stack([X.ravel(), Y.ravel(), np.full(n * n, z)], 1)
    idx = np.arange(n * n).reshape(n, n)
    tris = []
    for i in range(n - 1):
        for j in range(n - 1):
            a, b, c, d = idx[i, j], idx[i + 1, j], idx[i, j + 1], idx[i + 1, j + 1]
            tris += [(a, b, d), (a, d, c)]
    tris = np.array(tris, np.int32)
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
    e = np.unique(np.sort(e, axis=1), axis=0).astype(np.int32)
    return synth.scenes.Scene("sheet", "shell", x, e, tris, x[:, :2].copy(), h=1000.0, eta=900.0, seed=0)


CASES = {
    # two straight rods 5 mm apart: no candidate at all
    "far_rods": lambda: _rods([[(0, 0, 0), (400, 0, 0), (800, 0, 0)], [(0, 5000, 0), (400, 5000, 0), (800, 5000, 0)]]),
    # two single-edge rods crossing 280 apart: one active edge-edge pair
    "one_pair": lambda: _rods([[(-200, 0, 0), (200, 0, 0)], [(0, -200, 280), (0, 200, 280)]]),
    # the same 250 apart: inside the offset, infeasible
    "infeasible": lambda: _rods([[(-200, 0, 0), (200, 0, 0)], [(0, -200, 250), (0, 200, 250)]]),
    # one straight rod with segments shorter than h: only filtered stencil neighbours
    "filtered_only": lambda: _rods([[(k * 100.0, 0, 0) for k in range(12)]]),
    # a flat sheet at rest: candidates, all filtered
    "sheet_rest": lambda: _sheet(6, 400.0),
}


@requires_gpu
@pytest.mark.parametrize("name", list(CASES))
def test_edge_case_matches_the_oracle(name):
    import paper_2510_10256_amd as bfc
    sc = CASES[name]()
    print(f"[edge] {name} V={sc.n_verts} E={sc.n_edges} F={sc.n_tris}", flush=True)
    cs = bfc.ContactScene(sc, device=torch.device("cuda:0"))
    st = cs.run(sc.x)
    g = cs.results()
    cs.close()
    o = oracle.evaluate(sc, mode=1)
    compare(g, o, sc.n_verts, kappa=sc.kappa, tau=1e-10)
    c = g["counts"]
    print(name, c, g["E_total"], flush=True)
    if name == "far_rods":
        assert c["n_bp"] == 0
    if name in ("far_rods", "filtered_only", "sheet_rest"):
        assert c["n_act"] == 0 and g["E_total"] == 0.0 and not np.any(g["g"])
        assert c["nnzb"] == 0 and not np.any(g["row_ptr"])
    if name == "filtered_only":
        assert c["n_c"] > 0 and c["n_filt"] == c["n_c"]
    if name == "one_pair":
        assert c["n_act"] == 1 and c["n_infeasible"] == 0 and g["E_total"] > 0.0 and c["nnzb"] == 16
    if name == "infeasible":
        assert c["n_infeasible"] == 1 and st & bfc.BF_S_INFEASIBLE and g["E_total"] == float("inf")


@requires_gpu
def test_capacity_overflow_reports_sizes_and_retry_matches_the_oracle():
    # every device store of the step is guarded by its buffer's capacity: a
    # list that does not fit sets its status bit and its counter still holds
    # the size required; growing the buffers to those sizes and stepping again
    # gives the oracle's results
    import ctypes as C
    import paper_2510_10256_amd as bfc
    from paper_2510_10256_amd import binding as B
    sc = synth.woven_patch(n_warp=4, n_weft=4, verts_per_rod=80)
    print(f"[overflow] {sc.name} V={sc.n_verts}", flush=True)
    o = oracle.evaluate(sc, mode=1)
    oc = oracle.counts(o)
    cs = bfc.ContactScene(sc, cand_cap=256, act_cap=64, bsr_cap=64, device="cuda:0")
    x = cs._as_x(sc.x)

    def grow(cand=None, act=None, bsr=None):
        cs.cand_cap = cand or cs.cand_cap
        cs.act_cap = act or cs.act_cap
        cs.bsr_cap = bsr or cs.bsr_cap
        B._check(B.lib().bf_scene_reserve(cs.handle, cs.cand_cap, cs.act_cap), "bf_scene_reserve")
        cs._alloc()

    cs.step(x)
    st = cs.status(clear=True)
    assert st & B.BF_S_CAND_OVERFLOW
    need_cand = int(cs.c_n.item())
    assert need_cand > 256
    grow(cand=need_cand)
    cs.step(x)
    st = cs.status(clear=True)
    assert not (st & B.BF_S_CAND_OVERFLOW) and int(cs.c_n.item()) == need_cand
    assert st & B.BF_S_ACT_OVERFLOW
    need_act = int(cs.a_n.item())
    assert need_act == oc["n_act"] and int(cs.counters[2].item()) == oc["n_act"] and need_act > 64
    grow(act=need_act)
    cs.step(x)
    st = cs.status(clear=True)
    assert not (st & (B.BF_S_CAND_OVERFLOW | B.BF_S_ACT_OVERFLOW))
    assert st & B.BF_S_BSR_OVERFLOW
    need_bsr = int(cs.nnzb.item())
    assert need_bsr > 64
    grow(bsr=need_bsr)
    cs.step(x)
    st = cs.status(clear=True)
    assert not (st & (B.BF_S_CAND_OVERFLOW | B.BF_S_ACT_OVERFLOW | B.BF_S_BSR_OVERFLOW)), st
    g = cs.results()
    g["x"] = sc.x
    assert g["counts"]["nnzb"] == need_bsr
    rep = compare(g, o, sc.n_verts, kappa=sc.kappa, tau=1e-10)
    print(g["counts"], rep, flush=True)
    cs.close()
