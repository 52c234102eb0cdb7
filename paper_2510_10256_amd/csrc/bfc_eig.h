// Projection of a small symmetric matrix onto the PSD cone (App. A: the
// projected Newton solver clamps each pair Hessian's eigenvalues at zero):
//   A+ = Z max(L, 0) Z^T,  A = Z L Z^T.
//
// The eigensystem comes from a Householder reduction to tridiagonal form
// followed by implicit symmetric QR steps with Wilkinson shifts on the
// unreduced block that ends at the bottom, deflating from the bottom and
// splitting wherever an off-diagonal entry is negligible (Golub and Van Loan,
// Matrix Computations, Alg. 8.3.1, 8.3.2 and 8.3.3; the orthogonal factor
// formed from the reflectors by backward accumulation, Sec. 5.1.6).  For n = 9 this costs about a quarter of the FP64 operations of
// cyclic Jacobi (which needs about seven sweeps of 36 rotations here).  All
// array indices are compile-time constants (registers, no scratch); the only
// data-dependent control is the number of QR steps per deflation stage, a loop
// that the lanes of a wave leave together once every lane has converged, and
// the start of the unreduced block, which selects identity rotations.
//
// Written for host and device so that it can be checked on the CPU.
#pragma once
#include <hip/hip_runtime.h>

#include <math.h>

namespace bfc {

#define BFC_HD __host__ __device__ __forceinline__

// upper-triangle index of an N x N symmetric matrix (i <= j)
template <int N> BFC_HD constexpr int eig_uix(int i, int j) {
  return i <= j ? i * N - (i * (i - 1)) / 2 + (j - i) : j * N - (j * (j - 1)) / 2 + (i - j);
}

// true when the predicate holds on every active lane of the wave (device), or
// on this thread (host)
BFC_HD bool eig_all(bool p) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __all(p ? 1 : 0) != 0;
#else
  return p;
#endif
}

// Plane rotation that maps (x, z) to (r, 0): c = x / r, s = z / r,
// r = |(x, z)|, from one reciprocal square root (a square root and a
// division per rotation lengthen the dependent chain of a QR step).
template <class T> BFC_HD void eig_givens(T x, T z, T& c, T& s, T& r) {
  const T q = x * x + z * z;
  if (q > T(0)) {
#if defined(__HIP_DEVICE_COMPILE__)
    T ir;
    if constexpr (sizeof(T) == 4) ir = rsqrtf(q);
    else ir = rsqrt(q);
#else
    const T ir = T(1) / sqrt(q);
#endif
    c = x * ir;
    s = z * ir;
    r = q * ir;
  } else {
    c = T(1);
    s = T(0);
    r = T(0);
  }
}

// One implicit symmetric QR step with Wilkinson shift on the unreduced block
// p..L of the tridiagonal (d, e), p known at run time only (e[p-1] = 0, or
// p = 0): the loop runs over 0..L with compile-time indices and the
// rotations below p are the identity (c = 1, s = 0 leave every entry exactly
// as it was), so a block split inside the matrix gets its own QR steps
// (Golub and Van Loan, Alg. 8.3.3).  The rotations are then applied to the
// columns of Z (N x N, row-major) one row at a time (each element sees the
// same operations in the same order as rotation by rotation; a row in flight
// at a time keeps the live set small).
template <int N, int L, class T> BFC_HD void eig_qr_step(T* d, T* e, T (*Z)[N], int p) {
  const T dl = T(0.5) * (d[L - 1] - d[L]);
  const T b2 = e[L - 1] * e[L - 1];
  const T rt = sqrt(dl * dl + b2);
  const T den = dl >= T(0) ? dl + rt : dl - rt;
  const T mu = den != T(0) ? d[L] - b2 / den : d[L];
  T x = T(0), z = T(0);
  T cr[L], sr[L];
#pragma unroll
  for (int k = 0; k < L; ++k) {
    if (k == p) {
      x = d[k] - mu;
      z = e[k];
    }
    T c, s, r;
    eig_givens(x, z, c, s, r);
    if (k < p) {
      c = T(1);
      s = T(0);
    }
    cr[k] = c;
    sr[k] = s;
    if (k > p) e[k - 1] = r;
    const T a = d[k], b = e[k], cc = d[k + 1];
    const T c2 = c * c, s2 = s * s, cs = c * s;
    d[k] = c2 * a + T(2) * cs * b + s2 * cc;
    d[k + 1] = s2 * a - T(2) * cs * b + c2 * cc;
    e[k] = cs * (cc - a) + (c2 - s2) * b;
    if (k + 1 < L) {
      z = s * e[k + 1];
      e[k + 1] = c * e[k + 1];
      x = e[k];
    }
  }
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T zk = Z[i][0];
#pragma unroll
    for (int k = 0; k < L; ++k) {
      const T zk1 = Z[i][k + 1];
      Z[i][k] = cr[k] * zk + sr[k] * zk1;
      zk = cr[k] * zk1 - sr[k] * zk;
    }
    Z[i][L] = zk;
  }
}

// Deflation stages L = N-1 down to 1: QR steps on the unreduced block that
// ends at L until |e[L-1]| <= lim on every lane (at most 48 steps a stage).
// Before each step, off-diagonal entries at or below lim inside the block are
// set to zero and the block starts after the last of them.  Returns false on
// a lane whose stage hit the step limit (its projection is then not exact).
template <int N, int L, class T> BFC_HD bool eig_stages(T* d, T* e, T (*Z)[N], T lim) {
  if constexpr (L >= 1) {
    bool ok = true;
    int it = 0;
    for (; it < 48; ++it) {
      const bool conv = !(fabs(e[L - 1]) > lim);
      if (eig_all(conv)) break;
      if (!conv) {
        int p = 0;
#pragma unroll
        for (int k = 0; k + 1 < L; ++k)
          if (!(fabs(e[k]) > lim)) {
            e[k] = T(0);
            p = k + 1;
          }
        eig_qr_step<N, L, T>(d, e, Z, p);
      }
    }
    if (it == 48 && fabs(e[L - 1]) > lim) ok = false;
    e[L - 1] = T(0);
    return eig_stages<N, L - 1, T>(d, e, Z, lim) && ok;
  }
  return true;
}

// A: upper triangle of the symmetric N x N input (destroyed); P: upper
// triangle of A+.  tol: relative size (to |A|) below which an off-diagonal
// element of the tridiagonal counts as zero.  Returns false when a deflation
// stage did not converge within its step limit.  T = float expects A scaled
// to a largest entry of 1.
//
// Live data is kept small so that the whole projection stays in registers:
// the reduction stores its reflectors in the entries of A it zeroes (Z is not
// carried through it), Z is formed from them afterwards, and A+ is built row
// by row while the rows of Z that are no longer needed die.
template <int N, class T = double> BFC_HD bool psd_project(T* A, T* P, T tol) {
  // Householder reduction: step k zeroes entries k+2.. of row k and keeps
  // v[k+2..] there, v[k+1] in vh[k] and 2 / (v^T v) in bh[k] (0: identity)
  T vh[N > 2 ? N - 2 : 1], bh[N > 2 ? N - 2 : 1];
#pragma unroll
  for (int k = 0; k < N - 2; ++k) {
    T v[N];
    T sig = T(0);
#pragma unroll
    for (int j = k + 2; j < N; ++j) sig += A[eig_uix<N>(k, j)] * A[eig_uix<N>(k, j)];
    const T x0 = A[eig_uix<N>(k, k + 1)];
    vh[k] = T(0);
    bh[k] = T(0);
    // already tridiagonal in this row (the same on every lane of typical
    // input).  In single precision (inputs scaled to a largest entry of 1) a
    // row whose remaining entries are below 1e-15 counts as reduced too: a
    // reflector for it would need 1 / |v|^2 beyond the float range.
    if (!(sig > (sizeof(T) == 4 ? T(1e-30) : T(0)))) continue;
    const T nrm = sqrt(x0 * x0 + sig);
    const T alpha = x0 >= T(0) ? -nrm : nrm;
    const T beta = T(1) / (alpha * (alpha - x0));  // 2 / (v^T v)
#pragma unroll
    for (int j = 0; j < N; ++j) v[j] = T(0);
    v[k + 1] = x0 - alpha;
#pragma unroll
    for (int j = k + 2; j < N; ++j) v[j] = A[eig_uix<N>(k, j)];
    // p = beta A_sub v, w = p - (beta/2)(v^T p) v on indices k+1..N-1
    T p[N];
    T vp = T(0);
#pragma unroll
    for (int i = k + 1; i < N; ++i) {
      T acc = T(0);
#pragma unroll
      for (int j = k + 1; j < N; ++j) acc += A[eig_uix<N>(i, j)] * v[j];
      p[i] = beta * acc;
      vp += v[i] * p[i];
    }
    const T kk = T(0.5) * beta * vp;
#pragma unroll
    for (int i = k + 1; i < N; ++i) p[i] -= kk * v[i];
#pragma unroll
    for (int i = k + 1; i < N; ++i)
#pragma unroll
      for (int j = i; j < N; ++j) A[eig_uix<N>(i, j)] -= v[i] * p[j] + p[i] * v[j];
    A[eig_uix<N>(k, k + 1)] = alpha;
    vh[k] = v[k + 1];
    bh[k] = beta;  // v[k+2..] stay in row k of A
  }
  T d[N], e[N];
  T anorm = T(0);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    d[i] = A[eig_uix<N>(i, i)];
    e[i] = i + 1 < N ? A[eig_uix<N>(i, i + 1)] : T(0);
  }
#pragma unroll
  for (int i = 0; i < N; ++i) anorm = fmax(anorm, fabs(d[i]) + fabs(e[i]) + (i > 0 ? fabs(e[i - 1]) : T(0)));
  // Z = H_0 H_1 ... H_{N-3}, accumulated from the last reflector (H_k acts on
  // indices k+1..N-1, where the product so far is still the identity outside)
  T Z[N][N];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) Z[i][j] = i == j ? T(1) : T(0);
#pragma unroll
  for (int k = N - 3; k >= 0; --k) {
    T v[N];
    v[k + 1] = vh[k];
#pragma unroll
    for (int j = k + 2; j < N; ++j) v[j] = A[eig_uix<N>(k, j)];
#pragma unroll
    for (int j = k + 1; j < N; ++j) {
      T w = T(0);
#pragma unroll
      for (int i = k + 1; i < N; ++i) w += v[i] * Z[i][j];
      w *= bh[k];
#pragma unroll
      for (int i = k + 1; i < N; ++i) Z[i][j] -= w * v[i];
    }
  }
  const bool ok = eig_stages<N, N - 1, T>(d, e, Z, tol * anorm);
  T lam[N];
#pragma unroll
  for (int k = 0; k < N; ++k) lam[k] = fmax(d[k], T(0));
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T zl[N];
#pragma unroll
    for (int k = 0; k < N; ++k) zl[k] = Z[i][k] * lam[k];
#pragma unroll
    for (int j = i; j < N; ++j) {
      T acc = T(0);
#pragma unroll
      for (int k = 0; k < N; ++k) acc += zl[k] * Z[j][k];
      P[eig_uix<N>(i, j)] = acc;
    }
  }
  return ok;
}

}  // namespace bfc
