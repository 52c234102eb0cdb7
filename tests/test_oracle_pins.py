"""Pins of the CPU oracle against what the paper and the mathematics fix.

The paper prints no worked numerical example for this path, so every pin is a
closed form (Eq. 2, Eq. 3, Eq. 4 and the geometry of the distance types), an
independent computation (mpmath at 50 digits, a convex minimiser for
distances, LAPACK for eigenvalues, exact rationals for threshold decisions),
finite differences, or an invariant (translation/rotation, rest states).
"""
import math
from fractions import Fraction

import mpmath
import numpy as np
import pytest
from scipy.optimize import minimize

import oracle
import synth

mpmath.mp.dps = 50
RNG = np.random.default_rng(1234)


# ---------------------------------------------------------------------------
# Barrier: Eq. 2 (IPC log barrier) and Eq. 3 (offset b(d, a, eta) = b(d - eta, a - eta))
# ---------------------------------------------------------------------------

def mp_b(d, a, eta):
    """Eq. 2 and Eq. 3 exactly as printed, in 50-digit arithmetic."""
    d, a, eta = mpmath.mpf(d), mpmath.mpf(a), mpmath.mpf(eta)
    dd, aa = d - eta, a - eta
    if dd >= aa:
        return mpmath.mpf(0)
    return -(dd - aa) ** 2 * mpmath.log(dd / aa)


@pytest.mark.parametrize("d,a,eta", [(0.5, 1, 0), (195, 200, 190), (285, 300, 270), (950, 1000, 900),
                                     (40, 50, 0), (191.3, 200, 190), (12.5, 50, 0), (999.9, 1000, 900),
                                     (46.0, 200, 45)])
def test_barrier_matches_mpmath(d, a, eta):
    b, b1, b2 = oracle.barrier_scalar(d, a, eta)
    f = lambda t: mp_b(t, a, eta)
    rb, rb1, rb2 = f(d), mpmath.diff(f, d), mpmath.diff(f, d, 2)
    assert abs(b - float(rb)) <= 1e-14 * abs(float(rb)) + 1e-300
    assert abs(b1 - float(rb1)) <= 1e-13 * abs(float(rb1))
    assert abs(b2 - float(rb2)) <= 1e-13 * abs(float(rb2))


@pytest.mark.parametrize("a,eta", [(1, 0), (200, 190), (300, 270), (1000, 900), (50, 0), (200, 45)])
def test_barrier_midband_closed_form(a, eta):
    # at the middle of the band, (d - eta)/(a - eta) = 1/2:
    # b = ((a - eta)/2)^2 ln 2 and b'' = 5 + 2 ln 2 for every band width
    d = 0.5 * (a + eta)
    b, b1, b2 = oracle.barrier_scalar(d, a, eta)
    w = a - eta
    assert b == pytest.approx((w / 2) ** 2 * math.log(2), rel=1e-14)
    assert b1 == pytest.approx(-w * math.log(2) - w / 2, rel=1e-14)   # -2uL - u^2/w
    assert b2 == pytest.approx(5 + 2 * math.log(2), rel=1e-14)


@pytest.mark.parametrize("a,eta", [(1, 0), (200, 190), (1000, 900), (50, 0)])
def test_barrier_vanishes_c2_at_activation(a, eta):
    assert oracle.barrier_scalar(a, a, eta) == (0.0, 0.0, 0.0)
    b, b1, b2 = oracle.barrier_scalar(a * (1 - 1e-9), a, eta)
    assert b > 0 and b1 < 0 and b2 > 0


def test_barrier_scale_covariance():
    for _ in range(20):
        a = RNG.uniform(1, 1000)
        eta = RNG.uniform(0, 0.95) * a
        d = eta + RNG.uniform(0.01, 0.99) * (a - eta)
        lam = RNG.uniform(0.1, 10)
        b, b1, b2 = oracle.barrier_scalar(d, a, eta)
        c, c1, c2 = oracle.barrier_scalar(lam * d, lam * a, lam * eta)
        assert c == pytest.approx(lam ** 2 * b, rel=1e-12)
        assert c1 == pytest.approx(lam * b1, rel=1e-12)
        assert c2 == pytest.approx(b2, rel=1e-12)


# ---------------------------------------------------------------------------
# Distances (Sec. 3: unsigned distance between the deformed primitives)
# ---------------------------------------------------------------------------

def X12(*pts):
    return np.array(pts, dtype=np.float64).reshape(12)


def test_distance_hand_placed_point_triangle():
    tri = [(0, 0, 0), (4, 0, 0), (0, 4, 0)]
    D, code = oracle.pair_distance(0, X12((1, 1, 3), *tri))        # above interior
    assert (D, code) == (9.0, 6)
    D, code = oracle.pair_distance(0, X12((2, -3, 4), *tri))       # beyond edge t0-t1
    assert (D, code) == (25.0, 3)
    D, code = oracle.pair_distance(0, X12((-3, -4, 0), *tri))      # beyond vertex t0
    assert (D, code) == (25.0, 0)
    D, code = oracle.pair_distance(0, X12((3, 3, 1), *tri))        # beyond edge t1-t2
    assert D == pytest.approx(2.0 + 1.0, rel=1e-15) and code == 4
    D, code = oracle.pair_distance(0, X12((7, -4, 0), *tri))       # beyond vertex t1
    assert (D, code) == (25.0, 1)


def test_distance_hand_placed_edge_edge():
    # perpendicular skew segments crossing at gap g
    g = 2.5
    D, code = oracle.pair_distance(1, X12((-1, 0, 0), (1, 0, 0), (0, -1, g), (0, 1, g)))
    assert (D, code) == (g * g, 15)
    # parallel overlapping segments at offset g: point-segment fallback
    D, code = oracle.pair_distance(1, X12((0, 0, 0), (4, 0, 0), (1, g, 0), (6, g, 0)))
    assert D == g * g and code in (11, 12, 13, 14)
    # collinear rod edges: distance is the gap between the facing endpoints
    D, code = oracle.pair_distance(1, X12((0, 0, 0), (50, 0, 0), (150, 0, 0), (200, 0, 0)))
    assert (D, code) == (100.0 ** 2, 9)
    # skew, closest points at an endpoint of one edge and inside the other
    D, code = oracle.pair_distance(1, X12((0, 0, 0), (4, 0, 0), (2, 3, 1), (2, 9, 1)))
    assert (D, code) == (10.0, 13)


def _min_dist_pt(X):
    p, a, b, c = X.reshape(4, 3)

    def f(z):
        q = a + z[0] * (b - a) + z[1] * (c - a)
        return float(np.dot(p - q, p - q))
    cons = [{"type": "ineq", "fun": lambda z: 1 - z[0] - z[1]}]
    best = min((minimize(f, z0, method="SLSQP", bounds=[(0, 1), (0, 1)], constraints=cons,
                         options=dict(ftol=1e-16, maxiter=500)) for z0 in ([0.3, 0.3], [0.8, 0.1], [0.1, 0.8])),
               key=lambda r: r.fun)
    return best.fun


def _min_dist_ee(X):
    a0, a1, b0, b1 = X.reshape(4, 3)

    def f(z):
        q = a0 + z[0] * (a1 - a0) - b0 - z[1] * (b1 - b0)
        return float(np.dot(q, q))
    best = min((minimize(f, z0, method="L-BFGS-B", bounds=[(0, 1), (0, 1)],
                         options=dict(ftol=1e-16, gtol=1e-14, maxiter=1000)) for z0 in ([0.5, 0.5], [0.1, 0.9], [0.9, 0.1])),
               key=lambda r: r.fun)
    return best.fun


def test_distance_against_convex_minimiser():
    # the distance is the minimum of a convex quadratic over the primitives'
    # parameter domains; a general-purpose minimiser is an independent check
    for k in range(150):
        X = RNG.normal(0, 1, 12)
        ptype = k % 2
        D, code = oracle.pair_distance(ptype, X)
        ref = _min_dist_pt(X) if ptype == 0 else _min_dist_ee(X)
        assert D == pytest.approx(ref, rel=1e-7, abs=1e-12), (k, code)


def _mp_case(code, X):
    P = [mpmath.matrix([mpmath.mpf(float(v)) for v in X[3 * i:3 * i + 3]]) for i in range(4)]
    kind = oracle.CASE_KIND[code]
    slots = {0: [(0, 1), (0, 2), (0, 3)], 7: [(0, 2), (0, 3), (1, 2), (1, 3)]}
    cross = lambda u, v: mpmath.matrix([u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]])
    dot = lambda u, v: u[0] * v[0] + u[1] * v[1] + u[2] * v[2]
    table = {0: (0, 1), 1: (0, 2), 2: (0, 3), 7: (0, 2), 8: (0, 3), 9: (1, 2), 10: (1, 3)}
    pe = {3: (0, 1, 2), 4: (0, 2, 3), 5: (0, 3, 1), 11: (0, 2, 3), 12: (1, 2, 3), 13: (2, 0, 1), 14: (3, 0, 1)}
    if kind == 0:
        i, j = table[code]
        r = P[i] - P[j]
        return dot(r, r)
    if kind == 1:
        i, j, k = pe[code]
        r, e = P[i] - P[j], P[k] - P[j]
        c = cross(r, e)
        return dot(c, c) / dot(e, e)
    if kind == 2:
        n = cross(P[2] - P[1], P[3] - P[1])
        s = dot(P[0] - P[1], n)
        return s * s / dot(n, n)
    n = cross(P[1] - P[0], P[3] - P[2])
    s = dot(P[0] - P[2], n)
    return s * s / dot(n, n)


def test_distance_formulas_against_mpmath():
    # every sub-case formula, in double and in binary128, against 50 digits
    for k in range(400):
        X = RNG.normal(0, 100, 12)
        code = k % 16
        Dd, hi, lo = oracle.case_distance(code, X)
        ref = _mp_case(code, X)
        assert abs(Dd - float(ref)) <= 1e-12 * float(ref)
        assert abs(mpmath.mpf(hi) + mpmath.mpf(lo) - ref) <= mpmath.mpf(1e-30) * ref


def test_threshold_decision_is_exact():
    # knife-edge PP pairs: D within a few ulps of a^2; compare with exact rationals
    lib = oracle.lib()
    import ctypes as C
    lib.orc_decide.argtypes = [C.c_int32, C.c_void_p, C.c_double, C.c_int32, C.c_void_p]
    lib.orc_decide.restype = C.c_int32
    n_ext = 0
    for k in range(300):
        base = RNG.normal(0, 1000, 3)
        dirn = RNG.normal(0, 1, 3)
        dirn /= np.linalg.norm(dirn)
        a = float(RNG.choice([50.0, 200.0, 353.5533905932738, 1000.0]))
        q = base + a * dirn * (1 + RNG.integers(-8, 9) * 2.0 ** -52)
        X = np.concatenate([base, q, RNG.normal(0, 1, 3), RNG.normal(0, 1, 3)])
        ext = np.zeros(1, np.int32)
        got = lib.orc_decide(0, X.ctypes.data_as(C.c_void_p), a, 1, ext.ctypes.data_as(C.c_void_p))
        n_ext += int(ext[0])
        exact = sum((Fraction(float(base[i])) - Fraction(float(q[i]))) ** 2 for i in range(3))
        assert bool(got) == (exact < Fraction(a) ** 2)
        got_le = lib.orc_decide(0, X.ctypes.data_as(C.c_void_p), a, 0, ext.ctypes.data_as(C.c_void_p))
        assert bool(got_le) == (exact <= Fraction(a) ** 2)
    assert n_ext > 250


# ---------------------------------------------------------------------------
# Derivatives: finite differences of the oracle's own energy and gradient
# ---------------------------------------------------------------------------

def _random_active_pair(ptype, want_kind, a, eta):
    for _ in range(10000):
        X = RNG.normal(0, 1, 12) * 60.0
        if ptype == 0:
            X[:3] = X[3:6] / 3 + X[6:9] / 3 + X[9:12] / 3 + RNG.normal(0, 30, 3)
        D, code = oracle.pair_distance(ptype, X)
        d = math.sqrt(D)
        if oracle.CASE_KIND[code] == want_kind and eta + 0.05 * (a - eta) < d < a - 0.05 * (a - eta):
            return X
    raise RuntimeError("no sample")


@pytest.mark.parametrize("ptype,kind", [(0, 0), (0, 1), (0, 2), (1, 0), (1, 1), (1, 3)])
def test_gradient_hessian_finite_differences(ptype, kind):
    a, eta = 60.0, 20.0
    for _ in range(3):
        X = _random_active_pair(ptype, kind, a, eta)
        r = oracle.pair_barrier(ptype, X, a, eta)
        step = 1e-5 * 60.0
        G_fd = np.zeros(12)
        H_fd = np.zeros((12, 12))
        for k in range(12):
            Xp, Xm = X.copy(), X.copy()
            Xp[k] += step
            Xm[k] -= step
            rp, rm = oracle.pair_barrier(ptype, Xp, a, eta), oracle.pair_barrier(ptype, Xm, a, eta)
            assert rp["code"] == r["code"] == rm["code"]
            G_fd[k] = (rp["E"] - rm["E"]) / (2 * step)
            H_fd[:, k] = (rp["G"] - rm["G"]) / (2 * step)
        assert np.linalg.norm(G_fd - r["G"]) <= 1e-6 * np.linalg.norm(r["G"])
        assert np.linalg.norm(H_fd - r["Hraw"]) <= 1e-5 * np.linalg.norm(r["Hraw"])


# ---------------------------------------------------------------------------
# PSD projection (the projected Newton solver of App. A; eigenvalue clamp)
# ---------------------------------------------------------------------------

def test_psd_projection_against_lapack():
    for n in (3, 6, 9, 12):
        for _ in range(10):
            M = RNG.normal(0, 1, (n, n))
            A = M + M.T
            Ap, ev = oracle.psd_project(A)
            w, V = np.linalg.eigh(A)
            ref = (V * np.maximum(w, 0)) @ V.T
            assert np.allclose(Ap, ref, rtol=0, atol=1e-12 * np.abs(A).max())
            assert np.allclose(np.sort(ev), w, atol=1e-12 * np.abs(A).max())
            assert np.array_equal(Ap, Ap.T)
            assert np.linalg.norm(A - Ap) ** 2 == pytest.approx(np.sum(np.minimum(w, 0) ** 2), rel=1e-10)
            Ap2, _ = oracle.psd_project(Ap)
            assert np.allclose(Ap2, Ap, atol=1e-12 * np.abs(A).max())


def test_pair_hessian_psd_and_null_space():
    a, eta = 60.0, 20.0
    for ptype, kind in [(0, 2), (1, 3), (1, 1), (0, 0)]:
        X = _random_active_pair(ptype, kind, a, eta)
        r = oracle.pair_barrier(ptype, X, a, eta)
        H, Hp = r["Hraw"], r["Hpsd"]
        w = np.linalg.eigvalsh(Hp)
        assert w.min() >= -1e-12 * np.abs(H).max()
        # translation null space: sum of gradient blocks and H+ (1 (x) t) vanish
        assert np.abs(r["G"].reshape(4, 3).sum(0)).max() <= 1e-12 * np.abs(r["G"]).max()
        T = np.tile(np.eye(3), (4, 1))
        assert np.abs(Hp @ T).max() <= 1e-10 * np.abs(H).max()
        # rotation: sum_k x_k x g_k = 0 (the distance is rotation invariant)
        torque = np.cross(X.reshape(4, 3), r["G"].reshape(4, 3)).sum(0)
        assert np.abs(torque).max() <= 1e-9 * np.abs(r["G"]).max() * np.abs(X).max()


def test_point_point_projection_closed_form():
    # PP type: d = |p - q|, H = [[M, -M], [-M, M]] with M = b'' g g^T + (b'/d)(I - g g^T);
    # b' < 0 inside the band, so the projection keeps M+ = b'' g g^T
    a, eta = 60.0, 20.0
    X = _random_active_pair(1, 0, a, eta)
    r = oracle.pair_barrier(1, X, a, eta)
    code = r["code"]
    i, j = {7: (0, 2), 8: (0, 3), 9: (1, 2), 10: (1, 3)}[code]
    P = X.reshape(4, 3)
    diff = P[i] - P[j]
    d = np.linalg.norm(diff)
    ghat = diff / d
    b, b1, b2 = oracle.barrier_scalar(d, a, eta)
    Mp = b2 * np.outer(ghat, ghat)
    ref = np.zeros((12, 12))
    for (s, t, sg) in [(i, i, 1), (j, j, 1), (i, j, -1), (j, i, -1)]:
        ref[3 * s:3 * s + 3, 3 * t:3 * t + 3] = sg * Mp
    assert np.allclose(r["Hpsd"], ref, atol=1e-10 * np.abs(ref).max())
    assert r["E"] == pytest.approx(b, rel=1e-13)


# ---------------------------------------------------------------------------
# Mesh-side precompute (Sec. 3.2): components, parametric d_min
# ---------------------------------------------------------------------------

def _grid(n, lx, ly, flip=False):
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    u = np.stack([lx * i.ravel(), ly * j.ravel()], 1).astype(np.float64)
    v00 = (i[:-1, :-1] * n + j[:-1, :-1]).ravel()
    v10, v01, v11 = v00 + n, v00 + 1, v00 + n + 1
    if not flip:
        tris = np.concatenate([np.stack([v00, v10, v11], 1), np.stack([v00, v11, v01], 1)])
    else:
        tris = np.concatenate([np.stack([v00, v10, v01], 1), np.stack([v10, v11, v01], 1)])
    e = set()
    for t in tris:
        for a_, b_ in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0])):
            e.add((min(a_, b_), max(a_, b_)))
    edges = np.array(sorted(e), np.int32)
    x = np.concatenate([u, np.zeros((len(u), 1))], 1)
    return synth.Scene("grid", "shell", x, edges, tris.astype(np.int32), u, h=1000.0, eta=900.0)


@pytest.mark.parametrize("flip", [False, True])
def test_dmin_regular_grid(flip):
    # right-triangle grid: the closest non-incident stencil is a vertex and the
    # opposite diagonal, at the triangle's altitude l/sqrt(2)
    comp, d2, d = oracle.precompute(_grid(12, 500.0, 500.0, flip))
    assert comp.max() == 0 and d2[0] == 125000.0 and d[0] == math.sqrt(125000.0)
    comp, d2, d = oracle.precompute(_grid(10, 300.0, 400.0, flip))
    assert d2[0] == 57600.0 and d[0] == 240.0   # altitude 300*400/500


def test_dmin_rods_and_components():
    r = synth.helix_loop_rod()
    comp, d2, d = oracle.precompute(r)
    assert comp.max() == 0 and d[0] == 50.0
    w = synth.woven_patch(n_warp=3, n_weft=4, verts_per_rod=40)
    comp, d2, d = oracle.precompute(w)
    assert comp.max() + 1 == 7
    assert np.all(d == 20.0)   # min interior edge of the graded rods
    assert np.array_equal(comp, np.repeat(np.arange(7), 40))


# ---------------------------------------------------------------------------
# The paper's central claims as exact invariants (Sec. 1, Sec. 3.2, App. A)
# ---------------------------------------------------------------------------

def _straight_rod(n=200, ell=50.0, h=200.0, eta=190.0):
    s = ell * np.arange(n, dtype=np.float64)
    x = np.stack([s, np.zeros(n), np.zeros(n)], 1)
    edges = np.stack([np.arange(n - 1), np.arange(1, n)], 1).astype(np.int32)
    return synth.Scene("straight", "rod", x, edges, np.zeros((0, 3), np.int32), s, h=h, eta=eta)


def test_filtered_rod_has_no_rest_forces():
    r = _straight_rod()
    res = oracle.evaluate(r, mode=0)
    c = oracle.counts(res)
    assert c["n_filt"] == 197 + 196 + 195 and c["n_act"] == 0 and c["n_infeasible"] == 0
    assert c["n_c"] == 197 + 196 + 195       # d = gap exactly; gap 200 = h is not < h


def test_filtered_flat_sheet_has_no_rest_forces():
    g = _grid(10, 500.0, 500.0)
    res = oracle.evaluate(g, mode=0)
    c = oracle.counts(res)
    assert c["n_act"] == 0 and c["n_c"] == c["n_filt"] > 0


def test_unfiltered_rod_energy_closed_form():
    # plain offset barrier (no filter), eta = 0.9 min(h, dmin) = 45 as in the
    # paper's comparison setting: every gap-50/100/150 pair is active
    r = _straight_rod(eta=45.0)
    res = oracle.evaluate(r, mode=0, filter_mode=1)
    E = float(oracle.assemble(res, r.n_verts)["E"])
    ref = 197 * mp_b(50, 200, 45) + 196 * mp_b(100, 200, 45) + 195 * mp_b(150, 200, 45)
    assert E == pytest.approx(float(ref), rel=1e-13)
    assert E == pytest.approx(17441752.5437827, rel=1e-13)


def test_unfiltered_rod_with_large_offset_is_infeasible():
    # App. A: without the filter a large eta fails at the start (d = 50 <= eta)
    res = oracle.evaluate(_straight_rod(eta=190.0), mode=0, filter_mode=1)
    c = oracle.counts(res)
    assert c["n_infeasible"] == c["n_act"] == 197 + 196 + 195
    assert np.all(np.isinf(res["E"][(res["flags"] & oracle.F_INFEASIBLE) != 0]))
    # with the filter the same rod is feasible and force-free
    c2 = oracle.counts(oracle.evaluate(_straight_rod(eta=190.0), mode=0))
    assert c2["n_infeasible"] == 0 and c2["n_act"] == 0


# ---------------------------------------------------------------------------
# Whole-scene consistency
# ---------------------------------------------------------------------------

def _small_scenes():
    return [synth.helix_loop_rod(), synth.woven_patch(n_warp=4, n_weft=4, verts_per_rod=80),
            synth.folded_cloth(n=72, gaps=(950.0,), l_mid=4000.0, l_conv=2000.0)]


def test_brute_force_equals_sweep():
    for sc in _small_scenes():
        a = oracle.evaluate(sc, mode=0, derivs=False)
        b = oracle.evaluate(sc, mode=1, derivs=False)
        for k in ("ptype", "i", "j", "code", "flags", "d", "a", "eta", "E"):
            assert np.array_equal(a[k], b[k]), (sc.name, k)


def test_signed_axis_permutation_keeps_active_set():
    sc = synth.woven_patch(n_warp=4, n_weft=4, verts_per_rod=80)
    base = oracle.evaluate(sc, mode=1)
    for perm, sgn in [((1, 2, 0), (1, -1, 1)), ((2, 0, 1), (-1, -1, 1)), ((0, 2, 1), (1, 1, -1))]:
        x = sc.x[:, perm] * np.array(sgn)
        r = oracle.evaluate(sc, x=x, mode=1)
        for k in ("ptype", "i", "j", "flags"):
            assert np.array_equal(base[k], r[k])
        assert np.allclose(base["E"], r["E"], rtol=1e-12, atol=0)


def test_rotation_translation_keeps_energy():
    sc = synth.woven_patch(n_warp=4, n_weft=4, verts_per_rod=80)
    base = oracle.evaluate(sc, mode=1)
    q, _ = np.linalg.qr(RNG.normal(0, 1, (3, 3)))
    x = sc.x @ q.T + 1e4
    r = oracle.evaluate(sc, x=x, mode=1)
    assert np.array_equal(base["flags"] & oracle.F_ACTIVE, r["flags"] & oracle.F_ACTIVE)
    act = (base["flags"] & oracle.F_ACTIVE) != 0
    bref = ((base["a"] - base["eta"]) / 2) ** 2 * math.log(2)
    assert np.all(np.abs(base["E"][act] - r["E"][act]) <= 1e-9 * (np.abs(base["E"][act]) + bref[act]))


def test_generators_reproducible_and_feasible():
    for make in (synth.helix_loop_rod, lambda: synth.woven_patch(n_warp=8, n_weft=8, verts_per_rod=128)):
        a, b = make(), make()
        assert np.array_equal(a.x, b.x) and np.array_equal(a.ref, b.ref)
        c = oracle.counts(oracle.evaluate(a, mode=1, derivs=False))
        assert c["n_infeasible"] == 0 and c["n_act"] > 0 and c["n_filt"] > 0
    r = synth.helix_loop_rod()
    chords = np.linalg.norm(np.diff(r.x, axis=0), axis=1)
    assert np.all(np.abs(chords - 50.0) < 1e-9)


@pytest.mark.slow
def test_full_size_workloads_feasible():
    for name in ("woven_patch", "folded_cloth"):
        sc = synth.workload(name)
        c = oracle.counts(oracle.evaluate(sc, mode=1, derivs=False))
        assert c["n_infeasible"] == 0 and c["n_act"] > 0 and c["n_filt"] > 0, name
