"""More pins of the CPU oracle, for the parts that the per-pair pins leave open.

* Assembly (the Newton system of App. A): the assembled gradient against
  central differences of the assembled energy E(x), and the assembled block
  matrix (summed from the pairs' Hessians before projection) against central
  differences of the assembled gradient, on small rod, yarn and cloth scenes.
  A transposed off-diagonal block and a wrong stencil map, planted in the
  oracle, each fail these pins.
* The binary128 derivative branch (interior edge-edge pairs of nearly
  parallel edges, sin^2 below 1e-4) against 50-digit arithmetic of Eq. 2-3
  composed with the line-line distance.
* Exact ties (Eq. 1, Eq. 2: "0 for d >= a"; Eq. 4: filtered iff dbar < h):
  lattice geometry placed exactly at h and at d_min, and one ulp either
  side, decided by the oracle as exact rational arithmetic decides.
"""
import math
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import oracle
import synth

mpmath.mp.dps = 50


# ---------------------------------------------------------------------------
# Assembly against finite differences
# ---------------------------------------------------------------------------

def _scenes():
    cloth = synth.folded_cloth(n=36, gaps=(950.0,), l_mid=2500.0, l_conv=1500.0)
    # jitter: exactly parallel lattice edges make the distance a minimum of
    # several smooth pieces (a kink that finite differences straddle)
    cloth.x = cloth.x + np.random.default_rng(7).normal(0.0, 3.0, cloth.x.shape)
    return [synth.helix_loop_rod(), synth.woven_patch(n_warp=4, n_weft=4, verts_per_rod=96), cloth]


def _assembled(sc, x, hess="Hpsd"):
    r = oracle.evaluate(sc, x, mode=1, derivs=True)
    return r, oracle.assemble(r, sc.n_verts, hess=hess)


def _bsr_matvec(A, v):
    rows = np.repeat(np.arange(len(A["row_ptr"]) - 1), np.diff(A["row_ptr"]))
    out = np.zeros_like(v)
    np.add.at(out, rows, np.einsum("bij,bj->bi", A["val"], v[A["col"]]))
    return out


EPS = 1e-6  # um: small beside the edges' sin(angle) * length of the most nearly parallel pairs


def _grad_pin(sc, seed=0, ndir=2):
    """max relative error of g.v against (E(x + eps v) - E(x - eps v)) / (2 eps)"""
    rng = np.random.default_rng(seed)
    r, A = _assembled(sc, sc.x)
    assert ((r["flags"] & oracle.F_ACTIVE) != 0).sum() > 100
    worst = 0.0
    for _ in range(ndir):
        v = rng.normal(size=sc.x.shape)
        Ep, _ = oracle.energy(sc, sc.x + EPS * v)
        Em, _ = oracle.energy(sc, sc.x - EPS * v)
        fd = (Ep - Em) / (2 * EPS)
        an = float(np.sum(A["g"] * v))
        worst = max(worst, abs(an - fd) / abs(fd))
    return worst


def _hess_pin(sc, seed=1, ndir=1):
    """max relative error of H v against (g(x + eps v) - g(x - eps v)) / (2 eps)"""
    rng = np.random.default_rng(seed)
    _, A = _assembled(sc, sc.x, hess="Hraw")
    worst = 0.0
    for _ in range(ndir):
        v = rng.normal(size=sc.x.shape)
        gp = _assembled(sc, sc.x + EPS * v)[1]["g"]
        gm = _assembled(sc, sc.x - EPS * v)[1]["g"]
        fd = (gp - gm) / (2 * EPS)
        worst = max(worst, np.linalg.norm(_bsr_matvec(A, v) - fd) / np.linalg.norm(fd))
    return worst


@pytest.mark.parametrize("k", [0, 1, 2])
def test_assembled_gradient_and_hessian_match_differences(k):
    sc = _scenes()[k]
    assert _grad_pin(sc) < 2e-6, sc.name
    assert _hess_pin(sc) < 2e-6, sc.name


def test_assembled_pattern_and_symmetry():
    # every feasible active pair's 16 blocks are present (zero blocks too), and
    # the assembled matrix is symmetric block for block
    sc = _scenes()[1]
    r, A = _assembled(sc, sc.x)
    feas = ((r["flags"] & oracle.F_ACTIVE) != 0) & ((r["flags"] & oracle.F_INFEASIBLE) == 0)
    want = {(int(a), int(b)) for vs in r["verts"][feas] for a in vs for b in vs}
    rows = np.repeat(np.arange(sc.n_verts), np.diff(A["row_ptr"]))
    got = set(zip(rows.tolist(), A["col"].tolist()))
    assert got == want
    pos = {key: q for q, key in enumerate(zip(rows.tolist(), A["col"].tolist()))}
    for (a, b), q in pos.items():
        assert np.array_equal(A["val"][q], A["val"][pos[(b, a)]].T)


def test_planted_transposed_block_fails(monkeypatch):
    # a mistake that transposes every off-diagonal block goes unseen by the
    # symmetric diagonal but fails the Hessian pin
    sc = _scenes()[1]
    monkeypatch.setattr(oracle, "_block",
                        lambda H, r, c: (H[..., 3 * r:3 * r + 3, 3 * c:3 * c + 3].swapaxes(-1, -2) if r != c
                                         else H[..., 3 * r:3 * r + 3, 3 * c:3 * c + 3]))
    assert _hess_pin(sc) > 1e-3


def test_planted_wrong_stencil_map_fails(monkeypatch):
    # a mistake that swaps two stencil slots sends gradient and blocks to the
    # wrong vertices: both pins fail
    sc = _scenes()[1]
    monkeypatch.setattr(oracle, "_stencil", lambda res, k: res["verts"][k][..., [0, 2, 1, 3]])
    assert _grad_pin(sc) > 1e-3
    assert _hess_pin(sc) > 1e-3


# ---------------------------------------------------------------------------
# Binary128 derivative branch: nearly parallel edges
# ---------------------------------------------------------------------------

def _mp_energy_ee_interior(X, a, eta):
    """kappa = 1; Eq. 2 and Eq. 3 at d = distance of the two lines (the
    interior edge-edge sub-case), in 50-digit arithmetic."""
    P = [[mpmath.mpf(float(X[3 * s + c])) for c in range(3)] for s in range(4)]

    def f(*t):
        Q = [[P[s][c] + sum(t[q] * DIRS[q][3 * s + c] for q in range(len(t))) for c in range(3)] for s in range(4)]
        ea = [Q[1][c] - Q[0][c] for c in range(3)]
        eb = [Q[3][c] - Q[2][c] for c in range(3)]
        n = [ea[1] * eb[2] - ea[2] * eb[1], ea[2] * eb[0] - ea[0] * eb[2], ea[0] * eb[1] - ea[1] * eb[0]]
        w = [Q[0][c] - Q[2][c] for c in range(3)]
        s_ = w[0] * n[0] + w[1] * n[1] + w[2] * n[2]
        d = mpmath.sqrt(s_ * s_ / (n[0] ** 2 + n[1] ** 2 + n[2] ** 2))
        return -(d - a) ** 2 * mpmath.log((d - eta) / (a - eta))
    return f


DIRS = []


def _near_parallel_pair(rng, sin2, gap, L=400.0):
    """Two edges whose lines cross (in projection) at their midpoints, angle
    theta with sin^2 theta = sin2, offset `gap` along the common normal; then
    a random rotation and translation."""
    th = math.asin(math.sqrt(sin2))
    a0, a1 = np.array([-L / 2, 0, 0]), np.array([L / 2, 0, 0])
    u = np.array([math.cos(th), math.sin(th), 0.0])
    b0, b1 = -0.45 * L * u + [0, 0, gap], 0.55 * L * u + [0, 0, gap]
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    t = rng.normal(0, 1000, 3)
    return np.concatenate([Q @ p + t for p in (a0, a1, b0, b1)])


def test_binary128_derivative_branch_against_mpmath():
    rng = np.random.default_rng(42)
    a, eta = 1000.0, 900.0
    for sin2 in (2e-10, 1e-8, 1e-6, 3e-5):
        X = _near_parallel_pair(rng, sin2, gap=950.0 + rng.uniform(-30, 30))
        r = oracle.pair_barrier(1, X, a, eta, quad=True)
        assert r["code"] == 15
        v, w = rng.normal(size=12), rng.normal(size=12)
        DIRS[:] = [v, w]
        f = _mp_energy_ee_interior(X, a, eta)
        E = f(0, 0)
        gv = mpmath.diff(lambda t: f(t, 0), 0)
        vHw = mpmath.diff(f, (0, 0), (1, 1))
        assert abs(r["E"] - float(E)) <= 1e-13 * abs(float(E)), sin2
        assert abs(r["G"] @ v - float(gv)) <= 1e-13 * (np.linalg.norm(r["G"]) * np.linalg.norm(v)), sin2
        scale = np.linalg.norm(r["Hraw"]) * np.linalg.norm(v) * np.linalg.norm(w)
        assert abs(v @ r["Hraw"] @ w - float(vHw)) <= 1e-13 * scale, sin2


def test_evaluate_routes_near_parallel_edges_to_binary128():
    # two rods (separate components) whose middle edges are nearly parallel
    # at an active distance: the whole-scene evaluation gives the binary128
    # derivatives of that pair
    rng = np.random.default_rng(3)
    X = _near_parallel_pair(rng, 1e-6, gap=960.0)
    P = X.reshape(4, 3)
    ea, eb = P[1] - P[0], P[3] - P[2]
    x = np.stack([P[0] - ea, P[0], P[1], P[1] + ea, P[2] - eb, P[2], P[3], P[3] + eb])
    edges = np.array([[0, 1], [1, 2], [2, 3], [4, 5], [5, 6], [6, 7]], np.int32)
    s = np.array([0, 400, 800, 1200, 0, 400, 800, 1200], np.float64)
    sc = synth.Scene("parallel", "rod", x, edges, np.zeros((0, 3), np.int32), s, h=1000.0, eta=900.0)
    res = oracle.evaluate(sc, mode=0)
    k = [q for q in range(len(res["i"])) if (res["i"][q], res["j"][q]) == (1, 4)]
    assert len(k) == 1 and res["code"][k[0]] == 15 and res["flags"][k[0]] & oracle.F_ACTIVE
    q = oracle.pair_barrier(1, X, 1000.0, 900.0, quad=True)
    assert np.array_equal(res["G"][k[0]], q["G"]) and np.array_equal(res["Hraw"][k[0]], q["Hraw"])


# ---------------------------------------------------------------------------
# Exact ties against rational arithmetic
# ---------------------------------------------------------------------------

def _frac_case(code, X):
    """The squared-distance formula of sub-case `code`, exactly, in rationals
    of the double inputs."""
    P = [[Fraction(float(v)) for v in X[3 * i:3 * i + 3]] for i in range(4)]
    sub = lambda u, v: [u[0] - v[0], u[1] - v[1], u[2] - v[2]]
    dot = lambda u, v: u[0] * v[0] + u[1] * v[1] + u[2] * v[2]
    cross = lambda u, v: [u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]]
    kind = oracle.CASE_KIND[code]
    pp = {0: (0, 1), 1: (0, 2), 2: (0, 3), 7: (0, 2), 8: (0, 3), 9: (1, 2), 10: (1, 3)}
    pe = {3: (0, 1, 2), 4: (0, 2, 3), 5: (0, 3, 1), 11: (0, 2, 3), 12: (1, 2, 3), 13: (2, 0, 1), 14: (3, 0, 1)}
    if kind == 0:
        r = sub(*[P[k] for k in pp[code]])
        return dot(r, r)
    if kind == 1:
        i, j, k = pe[code]
        c = cross(sub(P[i], P[j]), sub(P[k], P[j]))
        e = sub(P[k], P[j])
        return dot(c, c) / dot(e, e)
    if kind == 2:
        n = cross(sub(P[2], P[1]), sub(P[3], P[1]))
        s = dot(sub(P[0], P[1]), n)
        return s * s / dot(n, n)
    n = cross(sub(P[1], P[0]), sub(P[3], P[2]))
    s = dot(sub(P[0], P[2]), n)
    return s * s / dot(n, n)


def _universe(sc):
    """(ptype, i, j, X) of every non-incident pair (rods: edge-edge only)."""
    out = []
    x, E, T = sc.x, sc.edges, sc.tris
    if sc.kind == "shell":
        for v in range(sc.n_verts):
            for t in range(len(T)):
                if v not in T[t]:
                    out.append((0, v, t, np.concatenate([x[v], x[T[t]].ravel()])))
    for a in range(len(E)):
        for b in range(a + 1, len(E)):
            if len(set(E[a]) | set(E[b])) == 4:
                out.append((1, a, b, np.concatenate([x[E[a]].ravel(), x[E[b]].ravel()])))
    return out


def _two_sheets(n, ell, gap, shift=(0.0, 0.0), h=1000.0, eta=900.0):
    """Two vertex-aligned lattice sheets (two components) `gap` apart in z;
    the upper one moved in plane by `shift`."""
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    u = np.stack([ell * i.ravel(), ell * j.ravel()], 1).astype(np.float64)
    v00 = (i[:-1, :-1] * n + j[:-1, :-1]).ravel()
    tris = np.concatenate([np.stack([v00, v00 + n, v00 + n + 1], 1), np.stack([v00, v00 + n + 1, v00 + 1], 1)])
    e = sorted({(min(a, b), max(a, b)) for t in tris for a, b in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0]))})
    nv = n * n
    x0 = np.concatenate([u, np.zeros((nv, 1))], 1)
    x1 = np.concatenate([u + np.array(shift), np.full((nv, 1), gap)], 1)
    return synth.Scene("two_sheets", "shell", np.concatenate([x0, x1]),
                       np.concatenate([np.array(e), np.array(e) + nv]).astype(np.int32),
                       np.concatenate([tris, tris + nv]).astype(np.int32),
                       np.concatenate([u, u]), h=h, eta=eta)


def _parallel_rods(gap, h=1000.0, eta=900.0, ell=500.0, n=5, rot=False):
    s = ell * np.arange(n, dtype=np.float64)
    a = np.stack([s, np.zeros(n), np.zeros(n)], 1)
    b = np.stack([s + 0.5 * ell, np.full(n, gap), np.zeros(n)], 1)
    x = np.concatenate([a, b])
    if rot:  # scaled by 5 and turned by the rotation (3/5, 4/5) about z: integers stay integers
        x = np.stack([3 * x[:, 0] - 4 * x[:, 1], 4 * x[:, 0] + 3 * x[:, 1], 5 * x[:, 2]], 1)
        h, eta = 5 * h, 5 * eta
    edges = np.concatenate([np.stack([np.arange(n - 1), np.arange(1, n)], 1)] * 2)
    edges[n - 1:] += n
    return synth.Scene("parallel_rods", "rod", x, edges.astype(np.int32), np.zeros((0, 3), np.int32),
                       np.concatenate([s, s]) * (5 if rot else 1), h=h, eta=eta)


def _tie_scenes():
    ulp = np.spacing(1000.0)
    out = []
    for gap in (1000.0, 1000.0 - ulp, 1000.0 + ulp):
        out.append(_two_sheets(4, 500.0, gap))
        out.append(_two_sheets(4, 500.0, gap, shift=(250.0, 125.0)))
        out.append(_parallel_rods(gap))
        out.append(_parallel_rods(gap, rot=True))
    out.append(_grid_at_rest())
    return out


def _grid_at_rest(n=5, ell=500.0):
    s = _two_sheets(n, ell, 0.0)
    nv = n * n
    keep = s.edges.max(1) < nv
    return synth.Scene("sheet_at_rest", "shell", s.x[:nv], s.edges[keep], s.tris[: len(s.tris) // 2], s.ref[:nv],
                       h=1000.0, eta=900.0)


def test_exact_ties_against_rationals():
    """Every pair of the universe whose double distance lies within 1e-6 of a
    threshold: membership of N_c (d < h), activity (d < a) and feasibility
    (d > eta) as the rational value of its formula decides."""
    n_tie = n_near = 0
    for sc in _tie_scenes():
        comp, dmin2, dmin = oracle.precompute(sc)
        res = oracle.evaluate(sc, mode=0, derivs=False)
        got = {(int(p), int(i), int(j)): (int(f), float(a)) for p, i, j, f, a in
               zip(res["ptype"], res["i"], res["j"], res["flags"], res["a"])}
        h2 = Fraction(sc.h) ** 2
        for (p, i, j, X) in _universe(sc):
            D, code = oracle.pair_distance(p, X)
            thr = [float(h2)]
            filt = None
            if (p, i, j) in got:
                filt = bool(got[(p, i, j)][0] & oracle.F_FILTERED)
                thr.append(got[(p, i, j)][1] ** 2)
            if not any(abs(D - t) <= 1e-6 * t for t in thr):
                continue
            Dx = _frac_case(code, X)
            n_tie += Dx == h2
            n_near += Dx != h2
            assert ((p, i, j) in got) == (Dx < h2), (sc.name, p, i, j, float(Dx - h2))
            if (p, i, j) not in got:
                continue
            c = comp[i] if p == 0 else comp[sc.edges[i][0]]
            a2 = (Fraction(dmin2[c]) if sc.kind == "shell" else Fraction(dmin[c]) ** 2) if filt else h2
            assert bool(got[(p, i, j)][0] & oracle.F_ACTIVE) == (Dx < a2), (sc.name, p, i, j)
            if not filt and Dx < a2:
                assert bool(got[(p, i, j)][0] & oracle.F_INFEASIBLE) == (Dx <= Fraction(sc.eta) ** 2)
    assert n_tie > 100 and n_near > 100, (n_tie, n_near)


def test_lattice_aligned_cloth_decisions_are_exact():
    """The folded cloth without in-plane shear: stacked fold layers line up
    vertex over vertex and lattice pairs sit at h or d_min up to the
    generator's rounding.  Every pair whose double distance lies within 1e-9
    of h, or of its activation a, is decided as exact rational arithmetic
    decides: membership of N_c (d < h, checked against a second listing at a
    slightly larger h), activity (d < a) and feasibility (d > eta).  Some of
    these pairs are exact ties and some lie 1e-25 from a threshold: a fixed
    tie band of binary128 values, or binary128 alone, gets one kind wrong."""
    import dataclasses
    sc = synth.folded_cloth(n=72, gaps=(950.0,), l_mid=4000.0, l_conv=2000.0, shear=0.0)
    comp, dmin2, dmin = oracle.precompute(sc)
    r = oracle.evaluate(sc, mode=1, derivs=False)
    wide = oracle.evaluate(dataclasses.replace(sc, h=sc.h * (1 + 1e-6)), mode=1, derivs=False)
    inside = set(zip(r["ptype"].tolist(), r["i"].tolist(), r["j"].tolist()))
    h2 = Fraction(sc.h) ** 2
    n_tie_h = n_close = n_checked = 0
    for k in range(len(wide["i"])):
        D = wide["d"][k] ** 2
        if abs(D - float(h2)) > 1e-9 * float(h2):
            continue
        X = sc.x[wide["verts"][k]].ravel()
        Dx = _frac_case(int(wide["code"][k]), X)
        key = (int(wide["ptype"][k]), int(wide["i"][k]), int(wide["j"][k]))
        assert (key in inside) == (Dx < h2), key
        n_tie_h += Dx == h2
        n_checked += 1
    ext = np.nonzero((r["flags"] & oracle.F_EXTENDED) != 0)[0]
    for k in ext:
        X = sc.x[r["verts"][k]].ravel()
        Dx = _frac_case(int(r["code"][k]), X)
        filt = bool(r["flags"][k] & oracle.F_FILTERED)
        a2 = Fraction(dmin2[0]) if filt else h2
        assert bool(r["flags"][k] & oracle.F_ACTIVE) == (Dx < a2), (int(r["i"][k]), int(r["j"][k]))
        if Dx < a2 and not filt:
            assert bool(r["flags"][k] & oracle.F_INFEASIBLE) == (Dx <= Fraction(sc.eta) ** 2)
        n_close += Dx != a2 and abs(float((Dx - a2) / a2)) < 1e-20
        n_checked += 1
    assert n_tie_h > 0 and n_close > 0 and n_checked > 1000, (n_tie_h, n_close, n_checked)
