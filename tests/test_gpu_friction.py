"""GPU parity of the lagged friction against the oracle.

The active pairs at the lagged positions (the scene's step there), their
lagged data (normal force, closest-point weights, normal), then the
friction at positions moved by a seeded displacement whose slips straddle
the smoothing width eh (both branches of f0).  Bar: closest-point weights
and normals to 1e-12, lambda to tau = 1e-10 of the barrier's force scale;
per-pair energy, gradient and Hessian within tau of the pair's scale
(mu lambda' eh, mu lambda', mu lambda' / eh with lambda' = lambda plus the
force scale of the barrier's band); the assembled energy, gradient
and blocks within the summed bounds.  Accumulation onto the contact terms
equals contact plus friction bit for bit; after a step at the new positions
(a new contact list) the friction still runs over the lagged list.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
requires_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU")

MU, EH, TAU = 0.3, 1.0, 1e-10

SCENES = {
    "yarn": lambda: synth.woven_patch(n_warp=4, n_weft=4, verts_per_rod=80),
    "cloth": lambda: synth.folded_cloth(n=72, gaps=(950.0,), l_mid=4000.0, l_conv=2000.0),
    "yarn_full": lambda: synth.workload("woven_patch"),
}


def _keyed(ptype, i, j):
    return {(int(a), int(b), int(c)): k for k, (a, b, c) in enumerate(zip(ptype, i, j))}


@requires_gpu
@pytest.mark.parametrize("name", list(SCENES))
def test_lagged_friction_matches_the_oracle(name):
    sc = SCENES[name]()
    print(f"[friction] {name} V={sc.n_verts}", flush=True)
    _check_friction(sc, synth.search_direction(sc), name)


@requires_gpu
@pytest.mark.parametrize("seed", [11, 12])
def test_friction_other_seeds(seed):
    # other seeds of the yarn and cloth generators and of the slip direction
    for name, sc in (("yarn", synth.woven_patch(seed=seed, n_warp=4, n_weft=4, verts_per_rod=80)),
                     ("cloth", synth.folded_cloth(seed=seed, n=48, gaps=(950.0,), l_mid=4000.0, l_conv=2000.0))):
        print(f"[friction] {name} seed={seed} V={sc.n_verts}", flush=True)
        _check_friction(sc, synth.search_direction(sc, seed=seed + 100), name)


def _check_friction(sc, p, name):
    import paper_2510_10256_amd as bfc
    xl = sc.x
    x = xl + 0.02 * p   # slips of about one eh
    dev = torch.device("cuda:0")
    cs = bfc.ContactScene(sc, device=dev)
    XL = torch.tensor(xl, dtype=torch.float64, device=dev)
    X = torch.tensor(x, dtype=torch.float64, device=dev)
    cs.run(XL)                       # active list at the lagged positions
    cs.friction_lag(XL)
    # accumulate onto the contact terms of the lagged list at x: contact + friction
    cs.eval_barrier(X)
    E_c = cs.l_E.clone()
    G_c = cs.l_G.clone()
    cs.friction_eval(X, MU, EH)
    f_E, f_G = cs.fl_E.clone(), cs.fl_G.clone()
    cs.friction_eval(X, MU, EH, accumulate=True)
    torch.cuda.synchronize()
    na = int(cs.f_cnt.item())
    fin = np.isfinite(E_c[:na].cpu().numpy())
    assert np.array_equal(cs.l_E[:na].cpu().numpy()[fin], (E_c[:na] + f_E[:na]).cpu().numpy()[fin])
    assert np.array_equal(cs.l_G[:na].cpu().numpy()[fin], (G_c[:na] + f_G[:na]).cpu().numpy()[fin])
    # a step at x replaces the contact list; the friction keeps the lagged one
    cs.run(X)
    with pytest.raises(RuntimeError):
        cs.friction_eval(X, MU, EH, accumulate=True)
    cs.friction_eval(X, MU, EH)
    cs.friction_assemble()
    g = cs.friction_results()
    # the assembly structure belongs to the lagged list: another list is refused
    import ctypes as C
    from paper_2510_10256_amd import binding as B
    rc = B.lib().friction_assemble(cs.handle, C.byref(cs._act), C.byref(cs._floc), B._ptr(cs.f_E), B._ptr(cs.f_g),
                                   C.byref(cs._fbsr), C.c_void_p(cs._stream()))
    assert rc == 5   # BF_E_STATE
    assert cs.status(clear=True) & bfc.BF_S_BSR_OVERFLOW == 0
    lag = oracle.friction_lag(sc, xl)
    o = oracle.friction_eval(lag, x, xl, MU, EH)
    gk = _keyed(g["ptype"], g["i"], g["j"])
    ok = _keyed(lag["ptype"], lag["i"], lag["j"])
    assert len(gk) == na and set(gk) == set(ok)
    gi = np.array([gk[k] for k in ok])
    oi = np.array([ok[k] for k in ok])
    lo = lag["lam"][oi]
    # lambda = kappa |b'(d)| on the scale of the barrier's force in the band
    # (kappa b_ref / (a - eta), b_ref = (a - eta)^2 ln 2 / 4), as the contact
    # gradients are compared
    res0 = oracle.evaluate(sc, xl, mode=1, derivs=False)
    act0 = (res0["flags"] & oracle.F_ACTIVE) != 0
    k0 = _keyed(res0["ptype"][act0], res0["i"][act0], res0["j"][act0])
    band0 = res0["a"][act0] - res0["eta"][act0]
    wband = band0[np.array([k0[k] for k in ok], dtype=np.int64)]
    fref = sc.kappa * wband * np.log(2) / 4
    dl = np.abs(g["lam"][gi] - lo) / (lo + fref)
    dw = np.abs(g["w"][gi] - lag["w"][oi]).max(axis=1)
    dn = np.abs(g["n"][gi] - lag["n"][oi]).max(axis=1)
    # the friction is linear in lambda, so its terms take lambda's scale:
    # near d = a the force vanishes quadratically and its value relative to
    # itself is rounding noise (both sides round d differently)
    s = MU * (lo + fref)
    rE = np.abs(g["E"][gi] - o["E"][oi]) / (np.abs(o["E"][oi]) + s * EH + 1e-300)
    rG = np.linalg.norm(g["G"][gi] - o["G"][oi], axis=1) / (np.linalg.norm(o["G"][oi], axis=1) + s + 1e-300)
    rH = np.linalg.norm((g["Hpsd"][gi] - o["Hpsd"][oi]).reshape(len(oi), -1), axis=1) / \
        (np.linalg.norm(o["Hpsd"][oi].reshape(len(oi), -1), axis=1) + s / EH + 1e-300)
    print(name, "worst: lam", dl.max(), "w", dw.max(), "n", dn.max(), "E", rE.max(), "G", rG.max(), "H", rH.max(),
          flush=True)
    assert dl.max() <= TAU and dw.max() <= 1e-12 and dn.max() <= 1e-12
    assert rE.max() <= TAU and rG.max() <= TAU and rH.max() <= TAU
    y_small = int(np.sum(o["E"][oi] < MU * lo * EH * 0.999))   # pairs in the smoothing branch
    print(name, "pairs", len(oi), "below eh", y_small, "E", g["E_total"], float(np.sum(o["E"])), flush=True)
    assert 0 < y_small < len(oi)
    # the friction assembled over the lagged list
    res = dict(flags=np.full(len(oi), oracle.F_ACTIVE), verts=lag["verts"], E=o["E"], G=o["G"], Hpsd=o["Hpsd"])
    asm = oracle.assemble(res, sc.n_verts)
    sl = np.empty(len(oi))
    sl[oi] = s                                          # the pairs' scales in the oracle's order
    assert abs(g["E_total"] - asm["E"]) <= TAU * float(np.sum(np.abs(o["E"]) + sl * EH)) + 1e-300
    gb = np.zeros(sc.n_verts)
    for q in range(4):
        np.add.at(gb, lag["verts"][:, q], TAU * (np.linalg.norm(o["G"], axis=1) + sl))
    assert np.all(np.linalg.norm(g["g"] - asm["g"], axis=1) <= gb + 1e-300)
    assert np.array_equal(g["row_ptr"], asm["row_ptr"]) and np.array_equal(g["col"], asm["col"])
    # each pair's bound on the 16 blocks (a, b) of its stencil, found by the
    # key a * V + b among the CSR's (row-major, columns sorted) keys
    nv = sc.n_verts
    keys = np.repeat(np.arange(nv, dtype=np.int64), np.diff(asm["row_ptr"])) * nv + asm["col"]
    V4 = lag["verts"].astype(np.int64)
    idx = np.searchsorted(keys, np.repeat(V4, 4, axis=1) * nv + np.tile(V4, (1, 4)))
    assert np.array_equal(keys[idx], np.repeat(V4, 4, axis=1) * nv + np.tile(V4, (1, 4)))
    sck = TAU * (np.linalg.norm(o["Hpsd"].reshape(len(oi), -1), axis=1) + sl / EH)
    hb = np.zeros(len(g["col"]))
    np.add.at(hb, idx.ravel(), np.repeat(sck, 16))
    assert np.all(np.abs(g["val"] - asm["val"]).reshape(len(hb), -1).max(axis=1) <= hb + 1e-300)
    cs.close()
