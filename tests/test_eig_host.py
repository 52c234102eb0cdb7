"""CPU check of the library's PSD projection (tridiagonal QR, bfc_eig.h),
built for the host: against LAPACK (numpy eigh) on random, structured and
degenerate symmetric matrices, and on reduced pair Hessians of the workloads
(from the oracle)."""
import os
import subprocess
import tempfile

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2510_10256_amd", "csrc")


@pytest.fixture(scope="module")
def exe():
    d = tempfile.mkdtemp(prefix="eig_host_")
    out = os.path.join(d, "eig_host")
    cmd = ["/opt/rocm/bin/hipcc", "-O2", "-std=c++17", "-I", CSRC, os.path.join(HERE, "host", "eig_host.cpp"),
           "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("hipcc host build failed: " + r.stderr[-500:])
    return out


def _upper(A):
    n = A.shape[-1]
    iu = np.triu_indices(n)
    return A[..., iu[0], iu[1]]


def _full(U, n):
    A = np.zeros(U.shape[:-1] + (n, n))
    iu = np.triu_indices(n)
    A[..., iu[0], iu[1]] = U
    A[..., iu[1], iu[0]] = U
    return A


def _project(exe, mats, tol=2.2e-16):
    n = mats.shape[-1]
    d = tempfile.mkdtemp(prefix="eig_io_")
    fi, fo = os.path.join(d, "in.bin"), os.path.join(d, "out.bin")
    with open(fi, "wb") as f:
        np.array([len(mats), n], np.int64).tofile(f)
        np.ascontiguousarray(_upper(mats), np.float64).tofile(f)
    r = subprocess.run([exe, fi, fo, repr(tol)], capture_output=True)
    assert r.returncode == 0, r
    return _full(np.fromfile(fo, np.float64).reshape(len(mats), -1), n)


def _reference(mats):
    w, V = np.linalg.eigh(mats)
    return np.einsum("nij,nj,nkj->nik", V, np.maximum(w, 0.0), V)


def _cases(n, rng):
    out = []
    for _ in range(200):  # random, random scale
        B = rng.normal(size=(n, n)) * 10.0 ** rng.uniform(-6, 6)
        out.append(B + B.T)
    for _ in range(50):   # low rank (repeated zero eigenvalues), mixed signs
        U = rng.normal(size=(n, 3))
        out.append(U @ np.diag(rng.normal(size=3)) @ U.T)
    for _ in range(50):   # repeated eigenvalues of both signs
        Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
        lam = rng.choice([-2.0, -1e-9, 0.0, 1.0, 3.0], size=n)
        out.append(Q @ np.diag(lam) @ Q.T)
    out.append(np.zeros((n, n)))
    out.append(np.diag(rng.normal(size=n)))
    T = np.diag(rng.normal(size=n)) + np.diag(rng.normal(size=n - 1), 1)
    out.append(T + np.triu(T, 1).T)
    out.append(np.eye(n) * -1.0)
    return np.array(out)


def _split_cases(n, rng):
    """Matrices whose tridiagonal form splits inside (an exact zero off the
    diagonal above the last entry): a null row and column, block-diagonal
    matrices, split tridiagonals, and a dense block beside a null block."""
    out = []
    for k in range(n):  # symmetric with row/column k zero
        B = rng.normal(size=(n, n))
        A = B + B.T
        A[k, :] = 0.0
        A[:, k] = 0.0
        out.append(A)
    for p in range(1, n):  # two dense diagonal blocks, sizes p and n - p
        A = np.zeros((n, n))
        B1 = rng.normal(size=(p, p))
        B2 = rng.normal(size=(n - p, n - p))
        A[:p, :p] = B1 + B1.T
        A[p:, p:] = B2 + B2.T
        out.append(A)
    for p in range(1, n - 1):  # tridiagonal with e[p-1] = 0 (a split above the bottom pair)
        d = rng.normal(size=n)
        e = rng.normal(size=n - 1)
        e[p - 1] = 0.0
        out.append(np.diag(d) + np.diag(e, 1) + np.diag(e, -1))
    for _ in range(20):  # block-diagonal with random orthogonal blocks and mixed signs, permuted
        p = int(rng.integers(1, n))
        Q1, _ = np.linalg.qr(rng.normal(size=(p, p)))
        Q2, _ = np.linalg.qr(rng.normal(size=(n - p, n - p)))
        A = np.zeros((n, n))
        A[:p, :p] = Q1 @ np.diag(rng.normal(size=p)) @ Q1.T
        A[p:, p:] = Q2 @ np.diag(rng.normal(size=n - p)) @ Q2.T
        P = np.eye(n)[rng.permutation(n)]
        out.append(P @ A @ P.T)
    return np.array(out)


@pytest.mark.parametrize("n", [6, 9])
def test_projection_split_tridiagonal(exe, n):
    # a zero inside the tridiagonal decouples the blocks: each block needs its
    # own QR steps (a chase started at the top stops at the zero)
    rng = np.random.default_rng(11 + n)
    mats = _split_cases(n, rng)
    got = _project(exe, mats)
    ref = _reference(mats)
    scale = np.linalg.norm(mats, axis=(1, 2)) + 1e-300
    err = np.linalg.norm(got - ref, axis=(1, 2)) / scale
    assert err.max() < 1e-13, (err.max(), int(err.argmax()))


@pytest.mark.parametrize("n", [6, 9])
def test_projection_matches_lapack(exe, n):
    rng = np.random.default_rng(5 + n)
    mats = _cases(n, rng)
    got = _project(exe, mats)
    ref = _reference(mats)
    scale = np.linalg.norm(mats, axis=(1, 2)) + 1e-300
    err = np.linalg.norm(got - ref, axis=(1, 2)) / scale
    assert err.max() < 1e-13, (err.max(), int(err.argmax()))
    # the projection is PSD and idempotent
    w = np.linalg.eigvalsh(got)
    assert (w >= -1e-13 * scale[:, None]).all()


def test_pair_hessians_of_the_workloads(exe):
    # reduced (translation-free) Hessians of active pairs of the yarn and cloth
    # workloads, from the oracle: 9x9 for edge-edge / point-triangle, 6x6 for
    # point-edge
    import oracle
    import synth
    W4 = 0.5 * np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], float)
    for sc in (synth.woven_patch(n_warp=8, n_weft=8, verts_per_rod=128),
               synth.folded_cloth(n=72, gaps=(950.0,), l_mid=4000.0, l_conv=2000.0)):
        r = oracle.evaluate(sc, mode=1, derivs=True)
        act = ((r["flags"] & 2) != 0) & ((r["flags"] & 4) == 0)
        H, codes = r["Hraw"][act], r["code"][act]
        tri = (codes == 6) | (codes == 15)
        if tri.any():
            Wf = np.kron(W4, np.eye(3))
            mats = np.einsum("ia,nij,jb->nab", Wf, H[tri], Wf)
            got = _project(exe, mats)
            ref = _reference(mats)
            err = np.linalg.norm(got - ref, axis=(1, 2)) / (np.linalg.norm(mats, axis=(1, 2)) + 1e-300)
            assert err.max() < 1e-13, (sc.name, err.max())


@pytest.mark.parametrize("n", [6, 9])
def test_single_precision_projection_of_the_mixed_mode(exe, n):
    # the mixed mode's projection (scaled to the largest entry, FP32, QR steps
    # stopping at 1e-6 of |A|) against LAPACK: within a few 1e-6 of |A| on the
    # random, degenerate and split cases, and exactly zero on the zero matrix
    rng = np.random.default_rng(17 + n)
    mats = np.concatenate([_cases(n, rng), _split_cases(n, rng)])
    got = _project(exe, mats, tol=-1.0)
    ref = _reference(mats)
    scale = np.linalg.norm(mats, axis=(1, 2)) + 1e-300
    err = np.linalg.norm(got - ref, axis=(1, 2)) / scale
    assert err.max() < 5e-6, (err.max(), int(err.argmax()))
    assert err.max() > 1e-9  # it is the single-precision path
    zero = np.all(mats == 0.0, axis=(1, 2))
    assert zero.any() and np.all(got[zero] == 0.0)


def test_single_precision_projection_with_tiny_entries(exe):
    # entries spanning far more decades than FP32 holds (pairs whose Hessian
    # has a stiff direction and tiny couplings): no NaN, and within the bound
    rng = np.random.default_rng(23)
    mats = []
    for _ in range(200):
        B = rng.normal(size=(9, 9))
        A = B + B.T
        A[0, :] *= 1e-25
        A[:, 0] *= 1e-25
        A[4, 5] = A[5, 4] = 1e-30
        A *= 10.0 ** rng.uniform(-20, 20)
        mats.append(A)
    mats = np.array(mats)
    got = _project(exe, mats, tol=-1.0)
    ref = _reference(mats)
    assert np.all(np.isfinite(got))
    err = np.linalg.norm(got - ref, axis=(1, 2)) / np.linalg.norm(mats, axis=(1, 2))
    assert err.max() < 5e-6, err.max()


def test_single_precision_projection_on_pair_hessians(exe):
    # the reduced Hessians of the small cloth's active pairs (entries span
    # some thirty decades), with denormals kept and with them flushed as on
    # the device: all finite and within the bound
    import oracle
    import synth
    W4 = 0.5 * np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], float)
    sc = synth.folded_cloth(n=72, gaps=(950.0,), l_mid=4000.0, l_conv=2000.0)
    r = oracle.evaluate(sc, mode=1, derivs=True)
    act = ((r["flags"] & 2) != 0) & ((r["flags"] & 4) == 0)
    H, codes = r["Hraw"][act], r["code"][act]
    tri = (codes == 6) | (codes == 15)
    Wf = np.kron(W4, np.eye(3))
    mats = np.einsum("ia,nij,jb->nab", Wf, H[tri], Wf)
    ref = _reference(mats)
    for flush in (-1.0, -2.0):
        got = _project(exe, mats, tol=flush)
        assert np.all(np.isfinite(got)), flush
        err = np.linalg.norm(got - ref, axis=(1, 2)) / (np.linalg.norm(mats, axis=(1, 2)) + 1e-300)
        assert err.max() < 5e-6, (flush, err.max())
