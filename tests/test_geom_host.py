"""CPU check of the library's exact threshold decisions (bfc_geom.h), built
for the host: on pairs whose distance lies within the FP64 guard band of a
threshold (d = h, d = d_min, d = eta) -- lattice ties of the shear-free
folded cloth and of hand-placed lattice scenes, and the near-ties of
generator rounding -- the exact FP64 evaluation (when it applies), the
point-edge fixed-point sum (when it applies) and the expansion arithmetic
give the sign of D - T that exact rationals give."""
import os
import subprocess
import tempfile
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from tests.test_oracle_assembly import _frac_case, _tie_scenes

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2510_10256_amd", "csrc")


@pytest.fixture(scope="module")
def exe():
    d = tempfile.mkdtemp(prefix="geom_host_")
    out = os.path.join(d, "geom_host")
    cmd = ["/opt/rocm/bin/hipcc", "-O2", "-std=c++17", "-I", CSRC, os.path.join(HERE, "host", "geom_host.cpp"),
           "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("hipcc host build failed: " + r.stderr[-500:])
    return out


def _dd(v):
    hi = float(v)
    return hi, float(v - Fraction(hi))


def _records(sc, res, comp, dmin2, dmin):
    """(code, X, T) for every pair of res in the FP64 band of one of its thresholds."""
    recs = []
    h2 = Fraction(sc.h) ** 2
    for k in range(len(res["i"])):
        X = sc.x[res["verts"][k]].ravel()
        code = int(res["code"][k])
        D = float(res["d"][k]) ** 2
        c = comp[res["i"][k]] if res["ptype"][k] == 0 else comp[sc.edges[res["i"][k]][0]]
        thr = [h2, Fraction(sc.eta) ** 2]
        if res["flags"][k] & oracle.F_FILTERED:
            thr.append(Fraction(dmin2[c]) if sc.kind == "shell" else Fraction(dmin[c]) ** 2)
        for T in thr:
            if T > 0 and abs(D - float(T)) <= 1e-9 * float(T):
                recs.append((code, X, T))
    return recs


def _run(exe, recs):
    d = tempfile.mkdtemp(prefix="geom_io_")
    fi, fo = os.path.join(d, "in.bin"), os.path.join(d, "out.bin")
    with open(fi, "wb") as f:
        np.array([len(recs)], np.int64).tofile(f)
        for code, X, T in recs:
            np.array([code, *X, *_dd(T)], np.float64).tofile(f)
    r = subprocess.run([exe, fi, fo], capture_output=True)
    assert r.returncode == 0, r
    return np.fromfile(fo, np.float64).reshape(-1, 4)


def test_exact_decisions_match_rationals(exe):
    recs = []
    for sc in _tie_scenes() + [synth.folded_cloth(n=72, gaps=(950.0,), l_mid=4000.0, l_conv=2000.0, shear=0.0),
                               synth.folded_cloth(n=72, gaps=(950.0,), l_mid=4000.0, l_conv=2000.0)]:
        comp, dmin2, dmin = oracle.precompute(sc)
        res = oracle.evaluate(sc, mode=0 if sc.n_verts < 200 else 1, derivs=False)
        recs += _records(sc, res, comp, dmin2, dmin)
    out = _run(exe, recs)
    n_ties = n_fp64 = n_fix = 0
    for (code, X, T), (fp64, xp, ddv, fix) in zip(recs, out):
        Dx = _frac_case(code, X)
        want = (Dx > T) - (Dx < T)
        n_ties += want == 0
        assert xp == want, (code, float(Dx - T))
        if fp64 != 2:
            n_fp64 += 1
            assert fp64 == want, (code, float(Dx - T))
        if fix != 2:
            n_fix += 1
            assert fix == want, (code, float(Dx - T))
        if abs(float((Dx - T) / T)) > 1e-20:
            assert ddv == want  # outside 1e-20 double-double decides
    assert n_ties > 1000 and n_fp64 > 1000 and n_fix > 1000, (n_ties, n_fp64, n_fix, len(recs))
    print(f"{len(recs)} decisions in the band, {n_ties} exact ties, {n_fp64} settled in exact FP64, "
          f"{n_fix} by the point-edge fixed-point sum")


def test_point_edge_fixed_point_near_ties(exe):
    # a point straight across an edge at distance h (the edge tilted by the
    # rounding of a non-integer base, or rotated, or the point jittered by
    # 1e-9), exact lattice ties with a threshold as a double-double, and
    # random pairs at thresholds near D: the fixed-point sum's sign is the
    # rational one wherever it applies
    rng = np.random.default_rng(7)
    recs = []
    for k in range(1500):
        base = rng.uniform(-1e5, 1e5, 3)
        L, h = rng.choice([250.0, 500.0, 1000.0]), rng.choice([500.0, 1000.0, 707.1067811865476])
        e0, e1 = base, base + np.array([L, 0.0, 0.0]) * (1 if k % 2 else -1)
        p = base + np.array([rng.uniform(-L, 2 * L), h, 0.0]) + (rng.normal(0, 1e-9, 3) if k % 3 == 0 else 0.0)
        R = np.linalg.qr(rng.normal(size=(3, 3)))[0] if k % 5 == 0 else np.eye(3)
        X = np.concatenate([R @ (p - base) + base, R @ (e0 - base) + base, R @ (e1 - base) + base, base + 3.0])
        recs.append((3, X, Fraction(h) ** 2))
    for k in range(800):
        b = rng.integers(-5000, 5000, 3).astype(float)
        e0, e1, p = b, b + rng.integers(-50, 50, 3), b + rng.integers(-50, 50, 3)
        X = np.concatenate([p, rng.normal(size=3), e0, e1])
        if not (e1 - e0).any():
            continue
        hi, lo = _dd(_frac_case(4, X))
        recs.append((4, X, Fraction(hi) + Fraction(lo)))  # a tie wherever D is a double-double
    for k in range(1200):
        X = rng.normal(size=12) * 10.0 ** rng.uniform(-3, 5)
        code = int(rng.choice([3, 4, 5, 11, 12, 13, 14]))
        T = _frac_case(code, X) * (1 + Fraction(rng.normal()) * Fraction(10) ** int(rng.integers(-16, -2)))
        hi, lo = _dd(T)
        recs.append((code, X, Fraction(hi) + Fraction(lo)))  # the threshold as the double-double it is passed as
    out = _run(exe, recs)
    n_fix = n_ties = 0
    for (code, X, T), row in zip(recs, out):
        Dx = _frac_case(code, X)
        want = (Dx > T) - (Dx < T)
        assert row[1] == want
        if row[3] != 2:
            n_fix += 1
            n_ties += want == 0
            assert row[3] == want, (code, float((Dx - T) / T))
    assert n_fix > 1500 and n_ties > 300, (n_fix, n_ties)
