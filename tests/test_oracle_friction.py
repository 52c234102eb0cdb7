"""Pins of the oracle's lagged friction (CPU only).

The friction of an active pair (IPC's lagged model, which the paper uses
with its contact energy, App. A) is the work of a Coulomb force mu lambda
over the tangential slip of the pair's closest points, smoothed below the
slip eh.  Pinned against what the mechanics fixes:

* lambda is the barrier's normal force kappa |b'(d)| at the lagged distance
  (checked against a central difference of the closed-form barrier);
* a point sliding a distance s >= eh over a triangle face (or an edge along
  a crossing edge, or a point past a point) costs exactly mu lambda s, with
  the force mu lambda along the slip on the moving side, distributed by the
  barycentric weights of the contact point on the other;
* below eh the energy is the smoothing cubic; motion along the normal and a
  common translation of the stencil cost nothing beyond f0(0) = eh / 3;
* the gradient equals central differences of the energy, and the Hessian of
  the exact energy is positive semidefinite (no projection needed).
"""
import math

import numpy as np
import pytest

import oracle

H, ETA, KAPPA = 300.0, 270.0, 1.0
MU, EH = 0.3, 10.0


def _barrier(d, a=H, eta=ETA):
    return -(d - a) ** 2 * math.log((d - eta) / (a - eta))


def _lam(d):
    step = 1e-4
    return KAPPA * abs((_barrier(d + step) - _barrier(d - step)) / (2 * step))


def _lag_pt(d):
    # point above the interior of a triangle in z = 0, at height d
    X = np.array([3.0, 2.0, d, -20, -20, 0, 40, -20, 0, -20, 40, 0], float)
    D, code = oracle.pair_distance(0, X)
    lo, w, n = np.zeros(1), np.zeros(4), np.zeros(3)
    oracle.lib().orc_friction_lag(code, oracle._p(X), math.sqrt(D), H, ETA, KAPPA, oracle._p(lo), oracle._p(w),
                                  oracle._p(n))
    return X, dict(lam=lo, w=w[None], n=n[None], verts=np.arange(4)[None]), code


def _energy(lag, X, Xl):
    return float(oracle.friction_eval(lag, X.reshape(4, 3), Xl.reshape(4, 3), MU, EH, derivs=False)["E"][0])


@pytest.mark.parametrize("d", [272.0, 285.0, 299.0])
def test_normal_force_and_point_face_slip(d):
    Xl, lag, code = _lag_pt(d)
    assert code == 6
    lam = float(lag["lam"][0])
    assert abs(lam - _lam(d)) <= 1e-6 * lam
    # barycentric weights of the contact point (3, 2) in the triangle
    b1, b2 = (3 + 20) / 60.0, (2 + 20) / 60.0
    assert np.allclose(lag["w"][0], [1, -(1 - b1 - b2), -b1, -b2], atol=1e-14)
    for s in (50.0, 12.0):   # above the smoothing width
        slip = np.array([0.6, 0.8, 0.0]) * s
        X = Xl.copy()
        X[:3] += slip
        E = _energy(lag, X, Xl)
        assert abs(E - MU * lam * s) <= 1e-12 * MU * lam * s
        r = oracle.friction_eval(lag, X.reshape(4, 3), Xl.reshape(4, 3), MU, EH)
        G = r["G"][0].reshape(4, 3)
        f = MU * lam * slip / s
        assert np.allclose(G[0], f, rtol=1e-10, atol=1e-12 * MU * lam)
        for k, b in enumerate([1 - b1 - b2, b1, b2]):
            assert np.allclose(G[k + 1], -b * f, rtol=1e-10, atol=1e-12 * MU * lam)


def test_small_slip_normal_motion_and_translation():
    Xl, lag, _ = _lag_pt(285.0)
    lam = float(lag["lam"][0])
    y = 4.0
    X = Xl.copy()
    X[:3] += [y, 0.0, 7.0]                     # slip 4 < eh plus 7 along the normal
    expect = MU * lam * (-y ** 3 / (3 * EH ** 2) + y ** 2 / EH + EH / 3)
    assert abs(_energy(lag, X, Xl) - expect) <= 1e-12 * expect
    X = Xl + np.tile([13.0, -5.0, 2.0], 4)     # common translation: no slip
    assert abs(_energy(lag, X, Xl) - MU * lam * EH / 3) <= 1e-12 * MU * lam * EH


def _lag_pair(ptype, Xl):
    D, code = oracle.pair_distance(ptype, Xl)
    lo, w, n = np.zeros(1), np.zeros(4), np.zeros(3)
    oracle.lib().orc_friction_lag(code, oracle._p(Xl), math.sqrt(D), H, ETA, KAPPA, oracle._p(lo), oracle._p(w),
                                  oracle._p(n))
    return dict(lam=lo, w=w[None], n=n[None], verts=np.arange(4)[None]), code


def test_edge_edge_and_point_point_slip():
    # crossing edges 280 apart: contact at both midpoints
    Xl = np.array([-50, 0, 0, 50, 0, 0, 0, -50, 280, 0, 50, 280], float)
    lag, code = _lag_pair(1, Xl)
    assert code == 15 and np.allclose(lag["w"][0], [0.5, 0.5, -0.5, -0.5])
    X = Xl.copy()
    X[0:6] += np.tile([30.0, 0, 0], 2)           # edge a slides 30 along itself
    lam = float(lag["lam"][0])
    assert abs(_energy(lag, X, Xl) - MU * lam * 30.0) <= 1e-12 * MU * lam * 30
    # collinear edges with facing ends 290 apart: point-point contact
    Xl = np.array([0, 0, 0, 100, 0, 0, 390, 0, 0, 490, 0, 0], float)
    lag, code = _lag_pair(1, Xl)
    assert code == 9 and np.allclose(lag["w"][0], [0, 1, -1, 0])
    X = Xl.copy()
    X[6:] += np.tile([0.0, 25.0, 0.0], 2)        # the second edge moves sideways by 25
    lam = float(lag["lam"][0])
    assert abs(_energy(lag, X, Xl) - MU * lam * 25.0) <= 1e-12 * MU * lam * 25


def test_gradient_against_differences_and_psd_hessian():
    rng = np.random.default_rng(11)
    for trial in range(40):
        ptype = trial % 2
        while True:
            Xl = rng.normal(scale=150.0, size=12)
            D, code = oracle.pair_distance(ptype, Xl)
            if ETA + 2 < math.sqrt(D) < H - 2:
                break
        lag, _ = _lag_pair(ptype, Xl)
        X = Xl + rng.normal(scale=(3.0, 30.0)[trial % 4 // 2], size=12)
        r = oracle.friction_eval(lag, X.reshape(4, 3), Xl.reshape(4, 3), MU, EH)
        G, Hm = r["G"][0], r["H"][0]
        step = 1e-4
        for k in range(12):
            e = np.zeros(12)
            e[k] = step
            fd = (_energy(lag, X + e, Xl) - _energy(lag, X - e, Xl)) / (2 * step)
            assert abs(fd - G[k]) <= 1e-5 * (abs(G[k]) + MU * lag["lam"][0]), (trial, k, fd, G[k])
        ev = np.linalg.eigvalsh(Hm)
        assert ev.min() >= -1e-9 * max(1.0, np.abs(ev).max()), (trial, ev.min())
        assert np.allclose(r["Hpsd"][0], Hm, atol=1e-9 * max(1.0, np.abs(ev).max()))


@pytest.mark.parametrize("theta", [1e-3, 3e-5, 1.2e-5])
def test_nearly_parallel_edges_weights_exact(theta):
    # edge b at height 280 over edge a, turned by theta in the plane: the
    # closest points are the lines' crossing in projection.  The weights
    # solve a 2 x 2 system whose determinant is |ea|^2 |eb|^2 sin^2 theta;
    # compare with the exact rational solution for the stored coordinates.
    # (Edges with sin^2 theta below 1e-10 are classified as parallel and
    # take a point-edge sub-case instead.)
    from fractions import Fraction as Fr
    c, s = math.cos(theta), math.sin(theta)
    Xl = np.array([-100, 0, 0, 100, 0, 0, 37 - 100 * c, -100 * s, 280, 37 + 100 * c, 100 * s, 280], float)
    lag, code = _lag_pair(1, Xl)
    assert code == 15
    Q = [Fr(float(v)) for v in Xl]
    sub = lambda a, b: [Q[a + k] - Q[b + k] for k in range(3)]
    dot = lambda u, v: sum(p * q for p, q in zip(u, v))
    ea, eb, r = sub(3, 0), sub(9, 6), sub(0, 6)
    A, B, C, D, E = dot(ea, ea), dot(ea, eb), dot(eb, eb), dot(ea, r), dot(eb, r)
    den = A * C - B * B
    al, be = (B * E - C * D) / den, (A * E - B * D) / den
    exact = [float(1 - al), float(al), float(-(1 - be)), float(-be)]
    assert abs(float(al) - 0.685) < 1e-6 and abs(float(be) - 0.5) < 1e-6
    assert np.allclose(lag["w"][0], exact, rtol=0, atol=4e-16), (lag["w"][0], exact)
