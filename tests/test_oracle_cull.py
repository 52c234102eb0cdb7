"""Pins of the comparison modes and the contact-locking experiment (CPU only).

A straight rod at rest with uniform segments ell (the paper's locking toy,
Fig. self_pushing_toy_example and App. A: eta = 0.9 min(h, dbar_min)): edges k
apart are collinear with a gap of (k - 1) ell, so the pairs in contact at
rest are known in closed form,

* no filter (plain offset barrier): every pair with k >= 2 and
  (k - 1) ell < h is active, E - k pairs for each such k (E edges);
* culling with radius r (Kaldor): the same with k > r;
* the paper's filter: none (every such pair is a stencil pair whose
  activation d_min = ell is not above its rest distance),

and the energy of each active pair is the barrier of Eq. 2-3 at d = (k - 1)
ell.  Culling follows positions along the polyline: a closed loop culls
across its seam, and renumbering the edges changes nothing.
"""
import math

import numpy as np
import pytest

import oracle
import synth

H = 300.0


def _closed_form(E, ell, lo):
    K = 1
    while (K * ell) < H:      # (k - 1) ell < h for k = K + 1
        K += 1
    return sum(E - k for k in range(lo, K + 1) if k <= E - 1)


@pytest.mark.parametrize("ell", [600.0, 300.0, 200.0, 100.0, 50.0, 25.0])
def test_rest_state_counts_and_energies(ell):
    sc = synth.straight_rod(ell, length=10000.0, h=H)
    E = sc.n_edges
    for mode, r, lo in [(1, 11, 2), (2, 11, 12), (2, 5, 6), (0, 11, None)]:
        res = oracle.evaluate(sc, mode=1, derivs=False, filter_mode=mode, cull_radius=r)
        n_act = oracle.counts(res)["n_act"]
        expect = 0 if lo is None else _closed_form(E, ell, lo)
        assert n_act == expect, (ell, mode, r, n_act, expect)
        act = (res["flags"] & oracle.F_ACTIVE) != 0
        for i, j, e in zip(res["i"][act], res["j"][act], res["E"][act]):
            d = (abs(int(j) - int(i)) - 1) * ell
            a, eta = H, sc.eta
            ref = -(d - a) ** 2 * math.log((d - eta) / (a - eta))
            assert abs(e - ref) <= 1e-12 * abs(ref)


def _ring(n, radius=1000.0):
    th = 2 * np.pi * np.arange(n) / n
    x = np.stack([radius * np.cos(th), radius * np.sin(th), np.zeros(n)], 1)
    e = np.stack([np.arange(n), (np.arange(n) + 1) % n], 1).astype(np.int32)
    ell = 2 * radius * math.sin(math.pi / n)
    s = np.arange(n) * ell
    return synth.scenes.Scene("ring", "rod", x, e, np.zeros((0, 3), np.int32), s, h=H,
                              eta=0.9 * min(H, ell), seed=0)


def test_culling_wraps_around_a_closed_loop_and_ignores_numbering():
    sc = _ring(200)      # 200 edges of about 31.4 um: edges within 9 steps are within h
    base = oracle.evaluate(sc, mode=1, derivs=False, filter_mode=2, cull_radius=5)
    # every active pair is more than 5 steps apart the short way round
    for i, j in zip(base["i"], base["j"]):
        k = abs(int(j) - int(i))
        assert min(k, 200 - k) > 5
    # pairs across the seam (edge 0 with edges 190..194) are there too
    assert any(int(i) == 0 and int(j) >= 190 for i, j in zip(base["i"], base["j"]))
    # renumber the edges: the same vertex pairs are in contact
    perm = np.random.default_rng(3).permutation(200)
    sc2 = synth.scenes.Scene("ring2", "rod", sc.x, sc.edges[perm], sc.tris, sc.ref, h=sc.h, eta=sc.eta, seed=0)
    res2 = oracle.evaluate(sc2, mode=1, derivs=False, filter_mode=2, cull_radius=5)
    key = lambda s_, res: {tuple(sorted((tuple(s_.edges[int(i)]), tuple(s_.edges[int(j)])))) for i, j in
                           zip(res["i"], res["j"])}
    assert key(sc, base) == key(sc2, res2)
