"""Pins of the oracle under the Euclidean reading of the reference distance
(dbar measured between the primitives at the rest pose, Eq. 1 and Sec. 3.2
read literally) against the parametric reading (arc length for rods, 2D rest
coordinates for shells; Sec. 1 and Sec. 3.4).

* On a straight rod and a flat sheet at rest the two readings are the same
  distance, so every result is the same, bit for bit.
* On the helix-and-loop rod the Euclidean reading also filters the pairs of
  successive turns, which are close in space but far apart along the rod:
  its filtered set, its d_min and which pairs stay active are checked
  against rest distances from an independent numpy computation (a ternary
  search over one segment of the point-to-segment distance, convex along it).
* The filter follows the rest pose, not the deformed one.
"""
import numpy as np

import oracle
import synth


def _point_seg(p, b0, b1):
    e = b1 - b0
    t = np.clip(np.einsum("...k,...k", p - b0, e) / np.einsum("...k,...k", e, e), 0.0, 1.0)
    q = b0 + t[..., None] * e
    return np.linalg.norm(p - q, axis=-1)


def _seg_seg(a0, a1, b0, b1, iters=200):
    """Distance between segments (arrays [n,3]) by ternary search on the
    convex function s -> dist(a0 + s (a1 - a0), [b0, b1])."""
    lo = np.zeros(len(a0))
    hi = np.ones(len(a0))
    f = lambda s: _point_seg(a0 + s[:, None] * (a1 - a0), b0, b1)
    for _ in range(iters):
        m1 = lo + (hi - lo) / 3.0
        m2 = hi - (hi - lo) / 3.0
        left = f(m1) <= f(m2)
        hi = np.where(left, m2, hi)
        lo = np.where(left, lo, m1)
    ends = np.stack([f(lo), f(hi), f(np.zeros_like(lo)), f(np.ones_like(lo))], 1)
    return ends.min(1)


def _rest_dist_ee(sc, i, j):
    X = sc.xrest
    e = sc.edges
    return _seg_seg(X[e[i, 0]], X[e[i, 1]], X[e[j, 0]], X[e[j, 1]])


def _same(a, b, keys=("ptype", "i", "j", "code", "flags", "d", "a", "eta", "E", "G", "Hpsd")):
    for k in keys:
        assert np.array_equal(a[k], b[k]), k


def test_readings_agree_where_rest_distance_is_the_parametric_one():
    # straight rod along x with s_k = x_k, flat sheet with x = (u, v, 0)
    for sc in (synth.straight_rod(100.0, length=5000.0), synth.flat_sheet(250.0, side=5000.0)):
        x = sc.x.copy()
        x[:, 2] += 0.3 * sc.h * np.sin(x[:, 0] / 700.0)  # a deformed pose: pairs come closer than d_min
        se = sc.with_euclid_rest(sc.x)
        cp, dp, dmp = oracle.precompute(sc)
        ce, de, dme = oracle.precompute(se)
        assert np.array_equal(cp, ce) and np.array_equal(dp, de) and np.array_equal(dmp, dme)
        op, oe = oracle.evaluate(sc, x, mode=1), oracle.evaluate(se, x, mode=1)
        assert oracle.counts(op)["n_filt"] > 0 and oracle.counts(op) == oracle.counts(oe)
        _same(op, oe)


def test_helix_loop_turn_pairs_are_filtered_only_under_the_euclidean_reading():
    sc = synth.helix_loop_rod()
    se = sc.with_euclid_rest()  # rest pose = the input pose
    op, oe = oracle.evaluate(sc, mode=1), oracle.evaluate(se, mode=1)
    assert np.array_equal(op["i"], oe["i"]) and np.array_equal(op["j"], oe["j"])  # d < h does not depend on it
    i, j = op["i"], op["j"]
    e = sc.edges
    s = sc.ref
    gap = np.maximum(np.minimum(s[e[j, 0]], s[e[j, 1]]) - np.maximum(s[e[i, 0]], s[e[i, 1]]),
                     np.minimum(s[e[i, 0]], s[e[i, 1]]) - np.maximum(s[e[j, 0]], s[e[j, 1]]))
    dist = _rest_dist_ee(se, i, j)
    fp, fe = (op["flags"] & 1) != 0, (oe["flags"] & 1) != 0
    h = sc.h
    # parametric: filtered iff 0 < gap < h; Euclidean: iff dbar < h (pairs far from h)
    assert np.array_equal(fp, (gap > 0) & (gap < h))
    clear = np.abs(dist - h) > 1e-6 * h
    assert clear.sum() > 0.99 * len(dist)
    assert np.array_equal(fe[clear], dist[clear] < h)
    # the difference is exactly the pairs of successive turns (far along the
    # rod, close in space), and there are many of them
    turn = (gap >= h) & (dist < h)
    assert turn.sum() >= 100
    assert np.array_equal(fe & ~fp, turn)
    assert not np.any(fp & ~fe)  # a chord is never longer than the arc
    # d_min: the smallest rest distance of a filtered pair
    _, d2p, _ = oracle.precompute(sc)
    _, d2e, dme = oracle.precompute(se)
    assert d2p[0] == 2500.0  # one edge of 50 between edges two apart
    ref_min = np.min(dist[fe])
    assert abs(dme[0] - ref_min) <= 1e-9 * ref_min and d2e[0] <= d2p[0]
    # the parametric reading keeps the turns in contact (offset barrier, h);
    # the Euclidean one gives them activation d_min and no offset: inactive
    act_p, act_e = (op["flags"] & 2) != 0, (oe["flags"] & 2) != 0
    assert np.all(act_p[turn]) and not np.any(act_e[turn])
    assert np.all(op["a"][turn] == h) and np.all(oe["a"][turn] == dme[0]) and np.all(oe["eta"][turn] == 0.0)


def test_euclidean_filter_follows_the_rest_pose():
    sc = synth.helix_loop_rod()
    se = sc.with_euclid_rest()
    x = sc.x + 0.05 * synth.search_direction(sc, seed=7)
    o0, o1 = oracle.evaluate(se, mode=1), oracle.evaluate(se, x, mode=1)
    k0 = {(a, b): f & 1 for a, b, f in zip(o0["i"], o0["j"], o0["flags"])}
    common = [(a, b, f & 1) for a, b, f in zip(o1["i"], o1["j"], o1["flags"]) if (a, b) in k0]
    assert len(common) > 500
    assert all(k0[(a, b)] == f for a, b, f in common)
    # and the rest pose decides: the same moved positions with the moved pose
    # as rest filter a different set
    o2 = oracle.evaluate(sc.with_euclid_rest(x), x, mode=1)
    assert not np.array_equal(o2["flags"] & 1, o1["flags"] & 1)


def test_euclidean_reading_per_component_on_yarns():
    # crossing yarns are separate components: their pairs are contacts under
    # either reading, never stencils, and d_min is per component
    sc = synth.woven_patch(n_warp=3, n_weft=3, verts_per_rod=64)
    se = sc.with_euclid_rest()
    oe = oracle.evaluate(se, mode=1)
    comp, d2, dm = oracle.precompute(se)
    i, j = oe["i"], oe["j"]
    e = sc.edges
    ci, cj = comp[e[i, 0]], comp[e[j, 0]]
    fe = (oe["flags"] & 1) != 0
    dist = _rest_dist_ee(se, i, j)
    assert np.sum(ci != cj) > 0 and not np.any(fe[ci != cj])
    assert np.any(dist[ci != cj] < sc.h)  # crossings closer than h that are not filtered
    same = ci == cj
    clear = np.abs(dist - sc.h) > 1e-6 * sc.h
    assert np.array_equal(fe[same & clear], dist[same & clear] < sc.h)
    for c in np.unique(ci[fe]):
        m = fe & (ci == c)
        assert abs(dm[c] - dist[m].min()) <= 1e-9 * dist[m].min()
