"""GPU parity: the HIP path against the CPU oracle on the same seeded inputs."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gpu_available():
    return torch.cuda.is_available()


requires_gpu = pytest.mark.skipif(not _gpu_available(), reason="no GPU")


def run_gpu(scene, **kw):
    import paper_2510_10256_amd as bfc
    cs = bfc.ContactScene(scene, **kw)
    cs.run(scene.x)
    out = cs.results()
    out["info"] = cs.info()
    cs.close()
    return out


SMALL = {
    "rod": lambda: synth.helix_loop_rod(),
    "yarn": lambda: synth.woven_patch(n_warp=4, n_weft=4, verts_per_rod=80),
    "cloth": lambda: synth.folded_cloth(n=72, gaps=(950.0,), l_mid=4000.0, l_conv=2000.0),
}


@requires_gpu
@pytest.mark.parametrize("name", list(SMALL))
def test_precompute_matches(name):
    from tests.parity import compare  # noqa: F401
    sc = SMALL[name]()
    print(f"[precompute] {name} V={sc.n_verts}", flush=True)
    g = run_gpu(sc)
    comp, d2, d = oracle.precompute(sc)
    gcomp, gd2, gd = g["info"]
    assert np.array_equal(gcomp, comp)
    assert np.array_equal(gd2, d2) and np.array_equal(gd, d)


@requires_gpu
@pytest.mark.parametrize("name", list(SMALL))
def test_small_parity_fp64(name):
    from tests.parity import compare
    sc = SMALL[name]()
    print(f"[parity fp64] {name} V={sc.n_verts}", flush=True)
    g = run_gpu(sc)
    o = oracle.evaluate(sc, mode=1)
    rep = compare(g, o, sc.n_verts, kappa=sc.kappa, tau=1e-10)
    print(name, g["counts"], rep, flush=True)


@requires_gpu
@pytest.mark.parametrize("name", list(SMALL))
def test_small_parity_no_offset(name):
    # eta = 0: the filter of Eq. 4 reduces to that of Eq. 1 (the rest distance
    # as activation, no offset) and the other pairs take the plain barrier
    # with activation h
    from tests.parity import compare
    sc = SMALL[name]()
    print(f"[parity eta=0] {name} V={sc.n_verts}", flush=True)
    g = run_gpu(sc, eta=0.0)
    o = oracle.evaluate(sc, mode=1, eta=0.0)
    assert np.all(o["eta"] == 0.0)
    rep = compare(g, o, sc.n_verts, kappa=sc.kappa, tau=1e-10)
    print(name, g["counts"], rep, flush=True)


@requires_gpu
@pytest.mark.parametrize("name", list(SMALL))
def test_small_parity_unfiltered(name):
    # no filter (plain offset barrier on every pair, the comparison setting):
    # stencil neighbours closer than h at rest are active too, most of them
    # infeasible
    import paper_2510_10256_amd as bfc
    from tests.parity import compare
    sc = SMALL[name]()
    print(f"[parity unfiltered] {name} V={sc.n_verts}", flush=True)
    g = run_gpu(sc, filter_mode=bfc.BF_FILTER_NONE)
    o = oracle.evaluate(sc, mode=1, filter_mode=1)
    assert g["counts"]["n_filt"] == 0 and g["counts"]["n_infeasible"] > 0
    rep = compare(g, o, sc.n_verts, kappa=sc.kappa, tau=1e-10)
    print(name, g["counts"], rep, flush=True)


@requires_gpu
@pytest.mark.parametrize("name", list(SMALL))
def test_small_parity_mixed(name):
    # FP32 screen in the narrow phase, FP32 derivative terms: the active set
    # stays exact, values within tau = 1e-5
    import paper_2510_10256_amd as bfc
    from tests.parity import compare
    sc = SMALL[name]()
    print(f"[parity mixed] {name} V={sc.n_verts}", flush=True)
    g = run_gpu(sc, prec=bfc.BF_MIXED)
    o = oracle.evaluate(sc, mode=1)
    rep = compare(g, o, sc.n_verts, kappa=sc.kappa, tau=1e-5)
    print(name, g["counts"], rep, flush=True)


@requires_gpu
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("seed", [11, 12, 13])
def test_seeded_moved_parity(seed, prec):
    # other seeds of the generators, at positions moved along a seeded
    # displacement: pairs close in, and on the cloth some cross the offset
    # (infeasible, E = +inf)
    import paper_2510_10256_amd as bfc
    from tests.parity import compare
    for name, sc in (("yarn", synth.woven_patch(seed=seed, n_warp=4, n_weft=4, verts_per_rod=80)),
                     ("cloth", synth.folded_cloth(seed=seed, n=48, gaps=(950.0,), l_mid=4000.0, l_conv=2000.0))):
        x = sc.x + 0.05 * synth.search_direction(sc, seed=seed + 100)
        print(f"[parity seed] {name} seed={seed} {prec} V={sc.n_verts}", flush=True)
        cs = bfc.ContactScene(sc, prec=bfc.BF_FP64 if prec == "fp64" else bfc.BF_MIXED)
        cs.run(x)
        g = cs.results()
        cs.close()
        o = oracle.evaluate(sc, x, mode=1)
        rep = compare(g, o, sc.n_verts, kappa=sc.kappa, tau=1e-10 if prec == "fp64" else 1e-5)
        print(name, seed, prec, g["counts"], rep, flush=True)
        if name == "cloth":
            assert g["counts"]["n_infeasible"] > 0


@requires_gpu
def test_full_yarn_patch_parity_mixed():
    import paper_2510_10256_amd as bfc
    from tests.parity import compare
    sc = synth.woven_patch()
    print(f"[parity mixed] woven_patch V={sc.n_verts}", flush=True)
    g = run_gpu(sc, prec=bfc.BF_MIXED)
    o = oracle.evaluate(sc, mode=1)
    rep = compare(g, o, sc.n_verts, kappa=sc.kappa, tau=1e-5)
    print(g["counts"], rep, flush=True)


@requires_gpu
def test_full_yarn_patch_parity_fp64():
    # the 32 x 32 woven patch (32,704 edges): full comparison
    from tests.parity import compare
    sc = synth.woven_patch()
    print(f"[parity fp64] woven_patch V={sc.n_verts}", flush=True)
    g = run_gpu(sc)
    o = oracle.evaluate(sc, mode=1)
    rep = compare(g, o, sc.n_verts, kappa=sc.kappa, tau=1e-10)
    print(g["counts"], rep, flush=True)


@requires_gpu
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_full_cloth_parity(prec):
    # the 256 x 256 folded cloth: active set and counts exactly; per-pair
    # values on a sample re-evaluated pair by pair; assembly by its
    # size-independent properties and the oracle's energy sum
    import math
    import paper_2510_10256_amd as bfc
    from tests.parity import active_view
    sc = synth.folded_cloth()
    print(f"[parity {prec}] folded_cloth V={sc.n_verts}", flush=True)
    g = run_gpu(sc, prec=bfc.BF_FP64 if prec == "fp64" else bfc.BF_MIXED)
    o = oracle.evaluate(sc, mode=1, derivs=False)
    oc = oracle.counts(o)
    for k in ("n_c", "n_filt", "n_act", "n_infeasible"):
        assert g["counts"][k] == oc[k], (k, g["counts"][k], oc[k])
    gi, oi = active_view(g), active_view(o)
    for k in ("ptype", "i", "j"):
        assert np.array_equal(g[k][gi], o[k][oi])
    assert np.array_equal(g["flags"][gi] & 5, o["flags"][oi] & 5)
    rng = np.random.default_rng(7)
    sample = rng.choice(len(gi), size=min(4000, len(gi)), replace=False)
    tau = 1e-10 if prec == "fp64" else 1e-5
    worst = 0.0
    for s in sample:
        k, q = gi[s], oi[s]
        verts = o["verts"][q]
        X = sc.x[verts].reshape(12)
        r = oracle.pair_barrier(int(o["ptype"][q]), X, o["a"][q], o["eta"][q], sc.kappa)
        w = o["a"][q] - o["eta"][q]
        bref = sc.kappa * (w / 2) ** 2 * math.log(2)
        assert abs(g["E"][k] - r["E"]) <= tau * (abs(r["E"]) + bref)
        assert np.linalg.norm(g["G"][k] - r["G"]) <= tau * (np.linalg.norm(r["G"]) + bref / w)
        dH = np.linalg.norm(g["Hpsd"][k] - r["Hpsd"])
        tolH = tau * (np.linalg.norm(r["Hpsd"]) + bref / w ** 2)
        worst = max(worst, dH / tolH)
        assert dH <= tolH
    # assembly: total energy, translation invariance of g and of every BSR row
    Eo = float(np.sum(o["E"][(o["flags"] & oracle.F_ACTIVE) != 0]))
    bsum = np.sum(sc.kappa * ((o["a"][oi] - o["eta"][oi]) / 2) ** 2 * math.log(2) + np.abs(o["E"][oi]))
    assert abs(g["E_total"] - Eo) <= tau * bsum
    gscale = np.abs(g["G"]).max()
    assert np.abs(g["g"].sum(0)).max() <= 1e-9 * gscale * math.sqrt(len(gi))
    rows = np.repeat(np.arange(sc.n_verts), np.diff(g["row_ptr"]))
    rowsum = np.zeros((sc.n_verts, 3, 3))
    np.add.at(rowsum, rows, g["val"])
    assert np.abs(rowsum).max() <= 1e-9 * np.abs(g["val"]).max()
    # symmetry of the assembled matrix: block (r, c) = block (c, r)^T
    key = {(int(r), int(c)): b for r, c, b in zip(rows, g["col"], g["val"])}
    for (r, c), b in list(key.items())[:20000]:
        assert np.allclose(key[(c, r)].T, b, rtol=0, atol=1e-9 * np.abs(b).max() + 1e-300)
    print(g["counts"], "H worst ratio", worst, flush=True)


@requires_gpu
def test_unaligned_hessian_buffer_is_refused():
    # eval_barrier writes H two doubles at a time: a buffer off 16-byte
    # alignment is refused on the host (no kernel runs)
    import ctypes as C
    import paper_2510_10256_amd as bfc
    from paper_2510_10256_amd import binding as B
    sc = SMALL["yarn"]()
    cs = bfc.ContactScene(sc, device=torch.device("cuda:0"))
    x = torch.tensor(sc.x, dtype=torch.float64, device="cuda:0")
    cs.run(x)
    Hx = torch.zeros(cs.act_cap * 144 + 1, dtype=torch.float64, device="cuda:0")
    loc = B.Local(cs.l_E.data_ptr(), cs.l_G.data_ptr(), Hx.data_ptr() + 8, cs.act_cap)
    rc = B.lib().eval_barrier(cs.handle, B._ptr(x), C.byref(cs._act), C.byref(loc), C.c_void_p(cs._stream()))
    assert rc == 1  # BF_E_ARG
    torch.cuda.synchronize()
    cs.close()
