"""Pins of the temporary zero offset (Sec. 3.4) in the oracle (CPU only).

Two straight rods cross at right angles with centrelines `z` apart (h = 300,
eta = 270, 100 um segments whose midpoints sit over the crossing).  The
edge-edge distances near the crossing are sqrt(z^2 + dx^2 + dy^2) with dx, dy
in {0, 50, 150, ...} (the nearest points of the two segments), so which pairs
are inside the core, their energies and which ones a move releases are known
in closed form:

* z = 250: the 3 x 3 pairs with dx, dy <= 50 are at d <= 259.8 < 270, all
  other pairs at d >= 291.5; core_mark returns exactly those nine;
* with the core set, each of them has the single-phase energy of Eq. 1 with
  activation h, -(d - h)^2 ln(d / h), and is feasible; without it they are
  infeasible (+inf);
* at z = 262 the four pairs with dx = dy = 50 are at 271.4 > 270 and are
  released, the other five (<= 266.7) stay; at z = 280 all nine are released
  and then take the biphasic energy -(d - h)^2 ln((d - eta)/(h - eta)).
"""
import math

import numpy as np

import oracle
import synth

H, ETA = 300.0, 270.0


def _Cross(z):
    return synth.crossing_rods(z, n=14, ell=100.0, h=H, eta=ETA)


def _mid_edges(sc):
    # edges of rod A and rod B whose midpoints are at -100..100 (dx or dy in {0, 50})
    n = sc.n_verts // 2
    mids = (sc.x[sc.edges[:, 0]] + sc.x[sc.edges[:, 1]]) / 2
    ea = [k for k in range(n - 1) if abs(mids[k, 0]) <= 100]
    eb = [k for k in range(n - 1, 2 * (n - 1)) if abs(mids[k, 1]) <= 100]
    return ea, eb


def _d(sc, ea, eb):
    mids = (sc.x[sc.edges[:, 0]] + sc.x[sc.edges[:, 1]]) / 2
    # nearest points: the segment end closest to the crossing (or the crossing)
    dx = max(0.0, abs(mids[ea, 0]) - 50.0)
    dy = max(0.0, abs(mids[eb, 1]) - 50.0)
    z = sc.x[-1, 2]
    return math.sqrt(z * z + dx * dx + dy * dy)


def test_core_mark_is_the_nine_crossing_pairs():
    sc = _Cross(250.0)
    ea, eb = _mid_edges(sc)
    assert len(ea) == 3 and len(eb) == 3
    cp, ci, cj = oracle.core_mark(sc, sc.x)
    assert np.all(cp == 1)
    assert set(zip(ci.tolist(), cj.tolist())) == {(a, b) for a in ea for b in eb}


def test_core_pairs_take_the_single_phase_energy():
    sc = _Cross(250.0)
    core = oracle.core_mark(sc, sc.x)
    plain = oracle.evaluate(sc, sc.x, derivs=False)
    key = {(int(i), int(j)): k for k, (i, j) in enumerate(zip(plain["i"], plain["j"]))}
    for i, j in zip(core[1], core[2]):
        assert math.isinf(plain["E"][key[(int(i), int(j))]])
    res = oracle.evaluate(sc, sc.x, derivs=False, core=core)
    key = {(int(i), int(j)): k for k, (i, j) in enumerate(zip(res["i"], res["j"]))}
    for i, j in zip(core[1], core[2]):
        k = key[(int(i), int(j))]
        d = _d(sc, int(i), int(j))
        assert res["flags"][k] & oracle.F_CORE and not res["flags"][k] & oracle.F_INFEASIBLE
        assert res["eta"][k] == 0.0 and res["a"][k] == H
        expect = -(d - H) ** 2 * math.log(d / H)
        assert abs(res["E"][k] - expect) <= 1e-12 * abs(expect)
    assert not np.any(res["flags"] & oracle.F_INFEASIBLE)
    # non-stencil pairs outside the set keep their offset
    other = (res["flags"] & (oracle.F_CORE | oracle.F_FILTERED)) == 0
    assert other.any() and np.all(res["eta"][other] == ETA)


def test_release_when_the_pair_leaves_the_core():
    sc = _Cross(250.0)
    core = oracle.core_mark(sc, sc.x)
    up = _Cross(262.0)
    rel = oracle.core_release(up, up.x, core)
    mids = (up.x[up.edges[:, 0]] + up.x[up.edges[:, 1]]) / 2
    corner = np.array([abs(mids[i, 0]) > 1 and abs(mids[j, 1]) > 1 for i, j in zip(core[1], core[2])])
    assert np.array_equal(rel, corner) and rel.sum() == 4
    far = _Cross(280.0)
    assert oracle.core_release(far, far.x, core).all()
    # released pairs take the biphasic energy of Eq. 3 again
    res = oracle.evaluate(far, far.x, derivs=False, core=None)
    key = {(int(i), int(j)): k for k, (i, j) in enumerate(zip(res["i"], res["j"]))}
    for i, j in zip(core[1], core[2]):
        k = key[(int(i), int(j))]
        d = _d(far, int(i), int(j))
        expect = -(d - H) ** 2 * math.log((d - ETA) / (H - ETA))
        assert abs(res["E"][k] - expect) <= 1e-12 * abs(expect)


def test_filtered_stencils_are_never_core():
    # the helix rod squeezed along its axis: successive turns come closer
    # than eta (core pairs), while the rod's own neighbours, much closer
    # still, are filtered stencils and must stay out of the core set
    sc = synth.helix_loop_rod()
    x = sc.x * np.array([1.0, 1.0, 0.9])
    res = oracle.evaluate(sc, x, derivs=False)
    cp, ci, cj = oracle.core_mark(sc, x)
    got = set(zip(ci.tolist(), cj.tolist()))
    filt = {(int(i), int(j)) for i, j, f in zip(res["i"], res["j"], res["flags"]) if f & oracle.F_FILTERED}
    near = {(int(i), int(j)) for i, j, d in zip(res["i"], res["j"], res["d"]) if d <= sc.eta}
    assert got and not (got & filt)
    assert got == near - filt
