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
    out["x"] = np.asarray(scene.x)
    cs.close()
    return out


SMALL = {
    "rod": lambda: synth.helix_loop_rod(),
    "yarn": lambda: synth.woven_patch(n_warp=4, n_weft=4, verts_per_rod=80),
    "cloth": lambda: synth.folded_cloth(n=72, gaps=(950.0,), l_mid=4000.0, l_conv=2000.0),
    # no in-plane shear: the fold's stacked layers line up vertex over vertex,
    # and lattice pairs sit exactly at h apart
    "cloth_noshear": lambda: synth.folded_cloth(n=72, gaps=(950.0,), l_mid=4000.0, l_conv=2000.0, shear=0.0),
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
    # the mixed mode (the projection's iteration stops at a looser tolerance):
    # the active set stays exact, values within tau = 1e-5
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
    # the 256 x 256 folded cloth (6.7 M pairs within h, 1.5 M active), element
    # by element: active set and counts exactly, every active pair's energy,
    # gradient and projected Hessian, the assembled energy, gradient and
    # block matrix (pattern exactly, values within the summed bounds)
    import paper_2510_10256_amd as bfc
    from tests.parity import compare
    sc = synth.folded_cloth()
    print(f"[parity {prec}] folded_cloth V={sc.n_verts}", flush=True)
    g = run_gpu(sc, prec=bfc.BF_FP64 if prec == "fp64" else bfc.BF_MIXED)
    del g["cand"]
    o = oracle.evaluate(sc, mode=1)
    rep = compare(g, o, sc.n_verts, kappa=sc.kappa, tau=1e-10 if prec == "fp64" else 1e-5)
    print(g["counts"], rep, flush=True)


@requires_gpu
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_packed_hessian_layout(prec):
    # H_d holds the upper triangle by 3 x 3 blocks (the layout of bf_local in
    # include/bfc.h): block-row s at 0, 33, 57, 72; block (s, s) as xx, xy, xz,
    # yy, yz, zz, then blocks (s, t > s) row-major; doubles, or floats in the
    # mixed mode.  The raw records of the small yarn equal the oracle's
    # projected Hessians entry by entry.
    from tests.parity import active_view
    import paper_2510_10256_amd as bfc
    p = bfc.BF_FP64 if prec == "fp64" else bfc.BF_MIXED
    sc = SMALL["yarn"]()
    cs_out = run_gpu(sc, prec=p)
    cs = bfc.ContactScene(sc, prec=p, device=torch.device("cuda:0"))
    cs.run(sc.x)
    torch.cuda.synchronize()
    n = cs.counts()["n_act"]
    assert cs.l_H.dtype == (torch.float64 if prec == "fp64" else torch.float32)
    raw = cs.l_H[:n].cpu().numpy().astype(np.float64)
    cs.close()
    o = oracle.evaluate(sc, mode=1)
    gi, oi = active_view(cs_out), active_view(o)
    starts = [0, 33, 57, 72]
    worst = 0.0
    for s_ in range(4):
        q = starts[s_]
        for (i, j) in [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]:
            ref = o["Hpsd"][oi][:, 3 * s_ + i, 3 * s_ + j]
            worst = max(worst, np.max(np.abs(raw[gi, q] - ref) / (np.abs(o["Hpsd"][oi]).max((1, 2)) + 1e-300)))
            q += 1
        for t in range(s_ + 1, 4):
            for i in range(3):
                for j in range(3):
                    ref = o["Hpsd"][oi][:, 3 * s_ + i, 3 * t + j]
                    worst = max(worst, np.max(np.abs(raw[gi, q] - ref) / (np.abs(o["Hpsd"][oi]).max((1, 2)) + 1e-300)))
                    q += 1
        assert q == (starts[s_ + 1] if s_ < 3 else 78)
    assert worst < (1e-9 if prec == "fp64" else 1e-5), worst


@requires_gpu
def test_exact_tie_scenes():
    # lattice geometry exactly at h and at d_min (two vertex-aligned sheets
    # h apart, parallel rods h apart, a sheet at rest) and one ulp either
    # side: the decisions equal the oracle's, which equal exact rational
    # decisions (tests/test_oracle_assembly.py)
    from tests.parity import compare
    from tests.test_oracle_assembly import _tie_scenes
    for sc in _tie_scenes():
        print(f"[ties] {sc.name} V={sc.n_verts} gap={sc.x[:, 2].max() - sc.x[:, 2].min()!r}", flush=True)
        g = run_gpu(sc)
        o = oracle.evaluate(sc, mode=0)
        rep = compare(g, o, sc.n_verts, kappa=sc.kappa, tau=1e-10)
        print(sc.name, g["counts"], rep, flush=True)
