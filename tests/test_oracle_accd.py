"""Pins of the oracle's line-search functions (CPU only).

ACCD (additive CCD of Li et al. 2021, applied with the filtered offsets as
Sec. 3.3's last paragraph asks) is pinned by closed forms and invariants that
a slip in its steps would break:

* head-on approach at relative speed v from distance d0 to offset xi: the
  first step closes (1 - s) of the gap and the second falls below s of it,
  so t = (1 - s)(d0 - xi) / v exactly (edge-edge endpoints and point-face);
* a displacement common to the four vertices changes no distance, so it must
  not change t (the mean displacement is removed before bounding the motion);
* no relative motion, or motion that never closes the gap: the full step 1;
* a start at or inside the offset: t = 0;
* safety on random pairs: dense sampling of the distance along x + tau p for
  tau in [0, t] never reaches the offset, and a step below 1 means the pair
  does come within s of its initial gap before ACCD's next step.

The pair set of max_step (swept boxes within h) is pinned by an independent
numpy enumeration; the offsets by the filter (Eq. 4: 0 for filtered
stencils, eta otherwise); the energy by the closed form of the barrier.
"""
import math

import numpy as np
import pytest

import oracle
import synth

S = 0.1


def _edge_pair_x(d0):
    # two collinear edges along x with facing endpoints d0 apart
    return np.array([0, 0, 0, 10, 0, 0, 10 + d0, 0, 0, 20 + d0, 0, 0], float)


@pytest.mark.parametrize("s", [S, 0.3])
@pytest.mark.parametrize("d0,xi,v", [(100.0, 20.0, 120.0), (50.0, 0.0, 400.0), (300.0, 270.0, 45.0),
                                     (1e-3, 0.0, 1e-2), (1e4, 9e3, 2e4)])
def test_head_on_edges_closed_form(d0, xi, v, s):
    X = _edge_pair_x(d0)
    P = np.array([v / 2, 0, 0, v / 2, 0, 0, -v / 2, 0, 0, -v / 2, 0, 0], float)
    t, it = oracle.accd_pair(1, X, P, xi, s)
    expect = (1 - s) * (d0 - xi) / v
    assert expect < 1
    assert abs(t - expect) <= 1e-12 * expect, (t, expect, it)
    assert it == 2
    # a common translation of the stencil does not change the step
    shift = np.tile([3.0 * v, -7.0 * v, 11.0 * v], 4)
    t2, _ = oracle.accd_pair(1, X, P + shift, xi, s)
    assert abs(t2 - t) <= 1e-12 * t


@pytest.mark.parametrize("u,w", [(10.0, 30.0), (0.0, 80.0), (55.0, 0.0)])
def test_head_on_point_face_closed_form(u, w):
    d0, xi = 120.0, 90.0
    # point above the interior of a triangle in z = 0, approaching its face
    X = np.array([1.0, 1.0, d0, -20, -20, 0, 40, -20, 0, -20, 40, 0], float)
    P = np.array([0, 0, -u, 0, 0, w, 0, 0, w, 0, 0, w], float)
    t, _ = oracle.accd_pair(0, X, P, xi, S)
    expect = min(1.0, (1 - S) * (d0 - xi) / (u + w))
    assert abs(t - expect) <= 1e-12 * expect, (t, expect)


def test_full_step_cases():
    X = _edge_pair_x(100.0)
    assert oracle.accd_pair(1, X, np.tile([5.0, -2.0, 1.0], 4), 20.0, S)[0] == 1.0   # no relative motion
    P = np.array([-30, 0, 0, -30, 0, 0, 30, 0, 0, 30, 0, 0], float)                  # separating
    assert oracle.accd_pair(1, X, P, 20.0, S)[0] == 1.0
    # sliding at constant distance over a large triangle: many steps, then 1
    Xt = np.array([0, 0, 50, -1e4, -1e4, 0, 3e4, -1e4, 0, -1e4, 3e4, 0], float)
    Pt = np.array([400, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0], float)
    t, it = oracle.accd_pair(0, Xt, Pt, 0.0, S)
    assert t == 1.0 and it > 3


def test_inside_the_offset_gives_zero():
    X = _edge_pair_x(10.0)
    P = np.array([1, 0, 0, 1, 0, 0, -1, 0, 0, -1, 0, 0], float)
    assert oracle.accd_pair(1, X, P, 10.0, S)[0] == 0.0
    assert oracle.accd_pair(1, X, P, 12.0, S)[0] == 0.0


def _sampled_gap(ptype, X, P, xi, taus):
    out = []
    for tau in taus:
        D, _ = oracle.pair_distance(ptype, X + tau * P)
        out.append(math.sqrt(D) - xi)
    return np.array(out)


def test_random_pairs_are_safe_and_stop_only_near_contact():
    rng = np.random.default_rng(20251010)
    checked_short = 0
    for trial in range(120):
        ptype = int(trial % 2)
        X = rng.normal(scale=60.0, size=12)
        P = rng.normal(scale=150.0, size=12)
        xi = float(rng.uniform(0.0, 20.0))
        sf = (S, 0.2, 0.5)[trial % 3]
        D0, _ = oracle.pair_distance(ptype, X)
        gap0 = math.sqrt(D0) - xi
        if gap0 <= 1.0:
            continue
        t, it = oracle.accd_pair(ptype, X, P, xi, sf)
        assert 0.0 < t <= 1.0
        taus = np.linspace(0.0, t, 801)
        assert _sampled_gap(ptype, X, P, xi, taus).min() > 0.0, trial
        if t < 1.0 and it < 65536:
            checked_short += 1
            # the pair comes within s of its initial gap before the next step
            # ACCD would take (0.9 of the gap at t over the relative-motion
            # bound lp), up to the sampling step times lp
            Pm = (P.reshape(4, 3) - P.reshape(4, 3).mean(axis=0))
            nrm = np.linalg.norm(Pm, axis=1)
            lp = nrm[0] + nrm[1:].max() if ptype == 0 else nrm[:2].max() + nrm[2:].max()
            gap_t = _sampled_gap(ptype, X, P, xi, [t])[0]
            taus = np.linspace(0.0, t + 0.9 * gap_t / lp, 4001)
            assert _sampled_gap(ptype, X, P, xi, taus).min() < sf * gap0 + lp * (taus[1] + 1e-12), trial
    assert checked_short > 10


def _tiny_rod():
    # two crossing rods plus a tight zigzag in the first (filtered stencils)
    return synth.workload("helix_loop_rod")


def _swept_pairs_numpy(sc, x, p):
    e = np.asarray(sc.edges)
    xe = x + p
    lo = np.minimum(np.minimum(x[e[:, 0]], x[e[:, 1]]), np.minimum(xe[e[:, 0]], xe[e[:, 1]]))
    hi = np.maximum(np.maximum(x[e[:, 0]], x[e[:, 1]]), np.maximum(xe[e[:, 0]], xe[e[:, 1]]))
    out = set()
    for a in range(len(e)):
        gap = np.maximum(lo[a + 1:] - hi[a], lo[a] - hi[a + 1:]).max(axis=1)
        for b in np.nonzero(gap < sc.h)[0] + a + 1:
            if len({e[a, 0], e[a, 1], e[b, 0], e[b, 1]}) == 4:
                out.add((a, int(b)))
    return out


def test_max_step_pair_set_offsets_and_minimum():
    sc = _tiny_rod()
    rng = np.random.default_rng(7)
    p = rng.normal(scale=40.0, size=sc.x.shape)
    r = oracle.max_step(sc, sc.x, p, s=S)
    got = set(zip(r["i"].tolist(), r["j"].tolist()))
    assert got == _swept_pairs_numpy(sc, sc.x, p)
    assert np.all(r["ptype"] == 1)
    # Eq. 4: filtered stencils have no offset, every other pair has eta
    assert np.all(r["xi"][r["filtered"] == 1] == 0.0)
    assert np.all(r["xi"][r["filtered"] == 0] == sc.eta)
    assert r["filtered"].sum() > 0 and (r["filtered"] == 0).sum() > 0
    assert r["t"] == r["tpair"].min()
    # the pruned enumeration finds the same pairs and steps
    r0 = oracle.max_step(sc, sc.x, p, s=S, mode=0)
    assert np.array_equal(r0["i"], r["i"]) and np.array_equal(r0["j"], r["j"])
    assert np.array_equal(r0["tpair"], r["tpair"])


def test_energy_closed_form_two_edges():
    # two parallel rods 250 apart in z, h = 300, eta = 270: every active pair
    # has d = 250 < eta, so the configuration is infeasible (+inf) ...
    class Sc:
        kind = "rod"
        n_verts, n_edges, n_tris = 4, 2, 0
        edges = np.array([[0, 1], [2, 3]], np.int32)
        tris = np.zeros((0, 3), np.int32)
        ref = np.array([0.0, 100.0, 0.0, 100.0])
        h, eta, kappa = 300.0, 270.0, 1.0
    x = np.array([[0, 0, 0], [100, 0, 0], [0, 0, 250], [100, 0, 250]], float)
    E, _ = oracle.energy(Sc, x)
    assert math.isinf(E)
    # ... while at 285 (inside the band) the energy is the barrier's closed form
    x[2:, 2] = 285.0
    E, res = oracle.energy(Sc, x)
    d, a, eta = 285.0, 300.0, 270.0
    expect = -(d - a) ** 2 * math.log((d - eta) / (a - eta))
    assert abs(E - expect) <= 1e-12 * abs(expect)
    assert len(res["E"]) == 1
