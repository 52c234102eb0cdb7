"""GPU parity under the Euclidean reading of the reference distance
(BF_REFDIST_EUCLID_REST: dbar between the primitives at a rest pose)
against the oracle: components and d_min bit for bit, then the whole path
element by element, at rest and at moved positions."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
requires_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU")


def _flat_rest(sc):
    return np.c_[sc.ref, np.zeros(sc.n_verts)]


CASES = {
    # rest pose = the input pose: the loop's successive turns are filtered
    "rod": lambda: synth.helix_loop_rod().with_euclid_rest(),
    "yarn": lambda: synth.woven_patch(n_warp=4, n_weft=4, verts_per_rod=80).with_euclid_rest(),
    # rest pose = the flat sheet (u, v, 0): the same filter as the parametric reading
    "cloth_flat_rest": lambda: (lambda sc: sc.with_euclid_rest(_flat_rest(sc)))(
        synth.folded_cloth(n=72, gaps=(950.0,), l_mid=4000.0, l_conv=2000.0)),
    # the same on the lattice without shear: rest distances exactly at h
    "cloth_noshear_flat_rest": lambda: (lambda sc: sc.with_euclid_rest(_flat_rest(sc)))(
        synth.folded_cloth(n=72, gaps=(950.0,), l_mid=4000.0, l_conv=2000.0, shear=0.0)),
    # rest pose = the folded pose: the stacked layers are filtered
    "cloth_folded_rest": lambda: synth.folded_cloth(n=72, gaps=(950.0,), l_mid=4000.0, l_conv=2000.0)
    .with_euclid_rest(),
}


@requires_gpu
@pytest.mark.parametrize("name", list(CASES))
def test_euclidean_reading_matches_the_oracle(name):
    import paper_2510_10256_amd as bfc
    from tests.parity import compare
    sc = CASES[name]()
    print(f"[refdist euclid] {name} V={sc.n_verts}", flush=True)
    cs = bfc.ContactScene(sc, device="cuda:0")
    try:
        comp, d2, dm = oracle.precompute(sc)
        gcomp, gd2, gd = cs.info()
        assert np.array_equal(gcomp, comp)
        assert np.array_equal(gd2, d2) and np.array_equal(gd, dm)
        for k, x in enumerate((sc.x, sc.x + 0.05 * synth.search_direction(sc, seed=21))):
            cs.run(x)
            g = cs.results()
            g["x"] = np.asarray(x)
            o = oracle.evaluate(sc, x, mode=1)
            rep = compare(g, o, sc.n_verts, kappa=sc.kappa, tau=1e-10)
            print(name, k, g["counts"], rep, flush=True)
            if k == 0:
                assert g["counts"]["n_filt"] > 0
    finally:
        cs.close()


@requires_gpu
def test_touching_rest_pose_is_refused():
    # one polyline whose fourth edge passes through its first at rest
    import paper_2510_10256_amd as bfc
    pts = np.array([[0, 0, 0], [200, 0, 0], [200, 200, 0], [100, 200, 0], [100, -100, 0]], np.float64)
    s = np.concatenate([[0.0], np.cumsum(np.linalg.norm(np.diff(pts, axis=0), axis=1))])
    sc = synth.Scene("self_touching", "rod", pts, np.array([[0, 1], [1, 2], [2, 3], [3, 4]], np.int32),
                     np.zeros((0, 3), np.int32), s, 50.0, 45.0).with_euclid_rest()
    print(f"[refdist euclid] {sc.name}", flush=True)
    with pytest.raises(RuntimeError, match="touch"):
        bfc.ContactScene(sc, device="cuda:0")
    # the parametric reading has no such condition
    bfc.ContactScene(synth.Scene("self_touching", "rod", pts, sc.edges, sc.tris, s, 50.0, 45.0),
                     device="cuda:0").close()
