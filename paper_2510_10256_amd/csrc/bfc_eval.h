// Per-pair barrier energy, gradient and PSD-projected Hessian (device code).
//
// Every distance formula depends on positions only through translation-free
// difference vectors y (Sec. 3 distances are invariant under rigid
// translation):
//   PP: y = (r)          r = x_i - x_j                      D = r.r
//   PE: y = (r, e)       r = x_p - x_e0, e = x_e1 - x_e0    D = |r x e|^2 / e.e
//   PT: y = (r, u, v)    r = p - t0, u = t1 - t0, v = t2 - t0
//   EE: y = (r, u, v)    r = a0 - b0, u = a1 - a0, v = b1 - b0
//                        D = (r.n)^2 / n.n, n = u x v
// The gradient and Hessian of D are written out in y, the barrier's chain rule
// (d = sqrt(D)) is applied in y, and the Hessian is expressed in an
// orthonormal basis of the translation complement of the participating
// vertices (W), where its eigenvalues are clamped at zero (App. A, projected
// Newton).  Mapping back through W gives the projected 12x12 Hessian, whose
// translation null space is exact by construction.
#pragma once
#include "bfc_eig.h"
#include "bfc_geom.h"

namespace bfc {

template <class T> struct M3 {
  T a[3][3];
};

// [a]x : the matrix with [a]x b = a x b
template <class T> __device__ __forceinline__ void skew(V3<T> a, T m[3][3], T sgn) {
  m[0][0] = 0; m[0][1] = -sgn * a.z; m[0][2] = sgn * a.y;
  m[1][0] = sgn * a.z; m[1][1] = 0; m[1][2] = -sgn * a.x;
  m[2][0] = -sgn * a.y; m[2][1] = sgn * a.x; m[2][2] = 0;
}
template <class T> __device__ __forceinline__ T comp(V3<T> a, int i) { return i == 0 ? a.x : (i == 1 ? a.y : a.z); }

// Upper-triangle index of an N x N symmetric matrix.
template <int N> __device__ __forceinline__ constexpr int uix(int i, int j) {
  return i <= j ? i * N - (i * (i - 1)) / 2 + (j - i) : j * N - (j * (j - 1)) / 2 + (i - j);
}

// Select one of four vertices without indexing a register array at run time
// (which would place it in scratch memory).
__device__ __forceinline__ d3 pick4(const d3* P, int s) { return pick<double>(P, s); }

// Scale factors of the barrier chain rule on D:
//   g_y = cg * dD,  H_y = c1 * dD dD^T + c2 * d2D
// with d = sqrt(D): grad d = dD/(2d), hess d = d2D/(2d) - dD dD^T/(4 d^3).
struct Chain {
  double E, cg, c1, c2;
  bool zero;
};
__device__ __forceinline__ Chain chain_coeffs(double D, double a, double eta, double kappa) {
  Chain ch;
  double d = sqrt(D);
  if (!(d < a)) {  // Eq. 2: zero at and beyond the activation distance
    ch.zero = true;
    ch.E = ch.cg = ch.c1 = ch.c2 = 0.0;
    return ch;
  }
  double b, b1, b2;
  barrier3<double>(d, a, eta, b, b1, b2);
  ch.zero = false;
  ch.E = kappa * b;
  ch.cg = kappa * b1 / (2.0 * d);
  ch.c1 = kappa * (b2 / (4.0 * D) - b1 / (4.0 * D * d));
  ch.c2 = kappa * b1 / (2.0 * d);
  return ch;
}

// A pair's results: the energy, and the projected Hessian in the reduced
// form it is computed in, from which hess_row() produces the rows of the
// 12 x 12 matrix one at a time (the caller streams them out).  The gradient
// is stored directly (G, 12 doubles).
enum { H_ZERO = 0, H_PP = 1, H_PE = 2, H_TRI = 3 };
struct PairOut {
  double E;
  int kind;      // H_*
  int eig_ok;    // 0: the projection's QR iteration hit its step limit
  int sl[3];     // PP: slots (s0, s1); PE: slots (point, e0, e1)
  double A[45];  // TRI: projected 9 x 9 (upper); PE: projected 6 x 6 (upper, 21);
                 // PP: r (3), eigenvalue along r, across r, 1 / D
};
__device__ __forceinline__ void zero_grad(double* G) {
#pragma unroll
  for (int q = 0; q < 12; ++q) G[q] = 0.0;
}

// ---- PP: closed-form projection ------------------------------------------
// H_y = c1 (2r)(2r)^T + 2 c2 I has eigenvalue kappa b'' along r and kappa b'/d
// across it; the projection keeps the positive parts.
__device__ __forceinline__ void eval_pp(const d3* P, int s0, int s1, double a, double eta, double kappa,
                                        double* G, PairOut& h) {
  d3 r = pick4(P, s0) - pick4(P, s1);
  double D = dot(r, r);
  Chain ch = chain_coeffs(D, a, eta, kappa);
  h.E = ch.E;
  zero_grad(G);
  if (ch.zero) return;
  double rr[3] = {r.x, r.y, r.z};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double g = 2.0 * ch.cg * rr[i];
    G[3 * s0 + i] = g;
    G[3 * s1 + i] = -g;
  }
  h.kind = H_PP;
  h.sl[0] = s0;
  h.sl[1] = s1;
  h.A[0] = r.x; h.A[1] = r.y; h.A[2] = r.z;
  h.A[3] = fmax(4.0 * ch.c1 * D + 2.0 * ch.c2, 0.0);  // eigenvalue along r
  h.A[4] = fmax(2.0 * ch.c2, 0.0);                    // eigenvalue across r
  h.A[5] = 1.0 / D;
}

// Projection of the reduced system A (upper triangle, N x N) into P.  FP64:
// psd_project in double.  FP32 (the mixed mode): A is scaled by its largest
// entry (the projection commutes with a positive scale, and the scale keeps
// FP32 away from overflow and underflow), projected in float with QR
// iterations that stop at 1e-6 of |A|, and scaled back; the FP32 arithmetic
// and the stopping rule each leave errors of order 1e-6 |A|.
template <int N, bool FP32>
__device__ __forceinline__ bool project_reduced(double* A, double* P, double tol) {
  constexpr int M = N * (N + 1) / 2;
  if constexpr (FP32) {
    double amax = 0.0;
#pragma unroll
    for (int k = 0; k < M; ++k) amax = fmax(amax, fabs(A[k]));
    if (!(amax > 0.0) || !(amax <= 1.7e308)) {  // zero, or not finite: the FP64 path decides
      return psd_project<N>(A, P, tol);
    }
    const double sc = 1.0 / amax;
    float Af[M], Pf[M];
    // entries below 1e-18 of the largest go to zero: their squares would be
    // FP32 denormals, which the device flushes (a Householder norm of zero
    // with a nonzero pivot), and they are far below the tolerance
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const double y = A[k] * sc;
      Af[k] = fabs(y) < 1e-18 ? 0.0f : (float)y;
    }
    const bool ok = psd_project<N, float>(Af, Pf, 1e-6f);
#pragma unroll
    for (int k = 0; k < M; ++k) P[k] = (double)Pf[k] * amax;
    return ok;
  } else {
    return psd_project<N>(A, P, tol);
  }
}

// ---- PE: 6 x 6 reduced system ----------------------------------------------
// Orthonormal basis of the translation complement of slots (p, e0, e1):
// w1 = (1, -1, 0)/sqrt2, w2 = (1, 1, -2)/sqrt6.  With y = (r, e) = Y x the
// coupling b = Y W is [[sqrt2, 0], [1/sqrt2, -3/sqrt6]].
template <bool FP32>
__device__ __forceinline__ void eval_pe(const d3* P, int sp, int se0, int se1, double a, double eta,
                                        double kappa, double tol, double* G, PairOut& h) {
  const double S2 = 1.4142135623730951, IS2 = 0.70710678118654752, IS6 = 0.40824829046386302;
  d3 xp = pick4(P, sp), x0 = pick4(P, se0), x1 = pick4(P, se1);
  d3 r = xp - x0, e = x1 - x0;
  double s = dot(r, e), m = dot(e, e), im = 1.0 / m;
  d3 c = cross(r, e);
  double D = dot(c, c) * im;
  Chain ch = chain_coeffs(D, a, eta, kappa);
  h.E = ch.E;
  if (ch.zero) {
    zero_grad(G);
    return;
  }
  double rv[3] = {r.x, r.y, r.z}, ev[3] = {e.x, e.y, e.z};
  double gr[3], ge[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    gr[i] = 2.0 * rv[i] - 2.0 * s * im * ev[i];
    ge[i] = -2.0 * s * im * rv[i] + 2.0 * s * s * im * im * ev[i];
  }
  double Yrr[3][3], Yre[3][3], Yee[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double dl = i == j ? 1.0 : 0.0;
      double hrr = 2.0 * dl - 2.0 * im * ev[i] * ev[j];
      double hre = -2.0 * im * ev[i] * rv[j] - 2.0 * s * im * dl + 4.0 * s * im * im * ev[i] * ev[j];
      double hee = -2.0 * im * rv[i] * rv[j] + 4.0 * s * im * im * (rv[i] * ev[j] + ev[i] * rv[j]) +
                   2.0 * s * s * im * im * dl - 8.0 * s * s * im * im * im * ev[i] * ev[j];
      Yrr[i][j] = ch.c1 * gr[i] * gr[j] + ch.c2 * hrr;
      Yre[i][j] = ch.c1 * gr[i] * ge[j] + ch.c2 * hre;
      Yee[i][j] = ch.c1 * ge[i] * ge[j] + ch.c2 * hee;
    }
  const double br[2] = {S2, 0.0}, be[2] = {IS2, -3.0 * IS6};
  double A[21];
#pragma unroll
  for (int al = 0; al < 2; ++al)
#pragma unroll
    for (int bt = al; bt < 2; ++bt)
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          int I = 3 * al + i, J = 3 * bt + j;
          if (I > J) continue;
          A[uix<6>(I, J)] = br[al] * br[bt] * Yrr[i][j] + br[al] * be[bt] * Yre[i][j] +
                            be[al] * br[bt] * Yre[j][i] + be[al] * be[bt] * Yee[i][j];
        }
  // the gradient goes out first: nothing but A stays live through the projection
  // (slot of the pair missing from the stencil gets a zero gradient)
  zero_grad(G);
#pragma unroll
  for (int i = 0; i < 3; ++i) {  // Y rows: r = (1, -1, 0), e = (0, -1, 1) on (p, e0, e1)
    double grx = ch.cg * gr[i], gex = ch.cg * ge[i];
    G[3 * sp + i] = grx;
    G[3 * se0 + i] = -grx - gex;
    G[3 * se1 + i] = gex;
  }
  h.eig_ok = project_reduced<6, FP32>(A, h.A, tol);
  h.kind = H_PE;
  h.sl[0] = sp;
  h.sl[1] = se0;
  h.sl[2] = se1;
}

// ---- PT and EE: 9 x 9 reduced system --------------------------------------
// Hadamard basis of the translation complement of four slots:
// w1 = (1,1,-1,-1)/2, w2 = (1,-1,1,-1)/2, w3 = (1,-1,-1,1)/2.
// Couplings b = Y W (rows r, u, v):
//   PT (r = p-t0, u = t1-t0, v = t2-t0):  r (0,1,1)  u (-1,1,0)  v (-1,0,1)
//   EE (r = a0-b0, u = a1-a0, v = b1-b0): r (1,0,1)  u (0,-1,-1) v (0,-1,1)
template <bool FP32>
__device__ __forceinline__ void eval_tri(const d3* P, bool is_pt, double a, double eta, double kappa, double tol,
                                         double* G, PairOut& h) {
  d3 r, u, v;
  if (is_pt) {
    r = P[0] - P[1]; u = P[2] - P[1]; v = P[3] - P[1];
  } else {
    r = P[0] - P[2]; u = P[1] - P[0]; v = P[3] - P[2];
  }
  d3 n = cross(u, v);
  double s = dot(r, n), m = dot(n, n), im = 1.0 / m;
  double D = s * s * im;
  Chain ch = chain_coeffs(D, a, eta, kappa);
  h.E = ch.E;
  if (ch.zero) {
    zero_grad(G);
    return;
  }
  double uu = dot(u, u), vv = dot(v, v), uv = dot(u, v);
  d3 gs[3] = {n, cross(v, r), cross(r, u)};
  d3 gm[3] = {{0.0, 0.0, 0.0}, 2.0 * (vv * u - uv * v), 2.0 * (uu * v - uv * u)};
  const double ks = 2.0 * s * im, km = -s * s * im * im;
  double g[9];
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int i = 0; i < 3; ++i) g[3 * b + i] = ks * comp(gs[b], i) + km * comp(gm[b], i);
  const double k_ss = 2.0 * im, k_hs = 2.0 * s * im, k_sm = -2.0 * s * im * im, k_hm = -s * s * im * im,
               k_mm = 2.0 * s * s * im * im * im;
  double Sru[3][3], Srv[3][3], Suv[3][3];
  skew(v, Sru, -1.0);
  skew(u, Srv, 1.0);
  skew(r, Suv, -1.0);
  double Y[3][3][3][3];
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int c = b; c < 3; ++c)
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          double gsi = comp(gs[b], i), gsj = comp(gs[c], j), gmi = comp(gm[b], i), gmj = comp(gm[c], j);
          double hs = 0.0, hm = 0.0;
          double dl = i == j ? 1.0 : 0.0;
          if (b == 0 && c == 1) hs = Sru[i][j];
          if (b == 0 && c == 2) hs = Srv[i][j];
          if (b == 1 && c == 2) hs = Suv[i][j];
          if (b == 1 && c == 1) hm = 2.0 * vv * dl - 2.0 * comp(v, i) * comp(v, j);
          if (b == 2 && c == 2) hm = 2.0 * uu * dl - 2.0 * comp(u, i) * comp(u, j);
          if (b == 1 && c == 2) hm = 4.0 * comp(u, i) * comp(v, j) - 2.0 * comp(v, i) * comp(u, j) - 2.0 * uv * dl;
          double d2 = k_ss * gsi * gsj + k_hs * hs + k_sm * (gsi * gmj + gmi * gsj) + k_hm * hm + k_mm * gmi * gmj;
          Y[b][c][i][j] = ch.c1 * g[3 * b + i] * g[3 * c + j] + ch.c2 * d2;
        }
  const float BPT[3][3] = {{0, 1, 1}, {-1, 1, 0}, {-1, 0, 1}};
  const float BEE[3][3] = {{1, 0, 1}, {0, -1, -1}, {0, -1, 1}};
  double A[45];
#pragma unroll
  for (int al = 0; al < 3; ++al)
#pragma unroll
    for (int bt = al; bt < 3; ++bt)
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          int I = 3 * al + i, J = 3 * bt + j;
          if (I > J) continue;
          double acc = 0.0;
#pragma unroll
          for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              double w = (double)(is_pt ? BPT[b][al] * BPT[c][bt] : BEE[b][al] * BEE[c][bt]);
              double y = b <= c ? Y[b][c][i][j] : Y[c][b][j][i];
              acc += w * y;
            }
          A[uix<9>(I, J)] = acc;
        }
  // the gradient goes out first: nothing but A stays live through the projection
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double gr = ch.cg * g[i], gu = ch.cg * g[3 + i], gv = ch.cg * g[6 + i];
    if (is_pt) {  // r = p - t0, u = t1 - t0, v = t2 - t0
      G[i] = gr;
      G[3 + i] = -gr - gu - gv;
      G[6 + i] = gu;
      G[9 + i] = gv;
    } else {      // r = a0 - b0, u = a1 - a0, v = b1 - b0
      G[i] = gr - gu;
      G[3 + i] = gu;
      G[6 + i] = -gr - gv;
      G[9 + i] = gv;
    }
  }
  h.eig_ok = project_reduced<9, FP32>(A, h.A, tol);
  h.kind = H_TRI;
}

// Row I (compile-time) of a pair's projected 12 x 12 Hessian, from its
// reduced form: H = W A W^T with W the orthonormal basis of the translation
// complement (Hadamard rows for four vertices, (1,-1,0)/sqrt2 and
// (1,1,-2)/sqrt6 for point-edge), and the point-point closed form.
template <int I> __device__ __forceinline__ void hess_row(const PairOut& h, double* out) {
  constexpr int s = I / 3, i = I % 3;
#pragma unroll
  for (int q = 0; q < 12; ++q) out[q] = 0.0;
  if (h.kind == H_TRI) {
    constexpr float W[4][3] = {{0.5f, 0.5f, 0.5f}, {0.5f, -0.5f, -0.5f}, {-0.5f, 0.5f, -0.5f}, {-0.5f, -0.5f, 0.5f}};
    double C[3][3];  // C[bt][j] = sum_al W[s][al] A[3al+i][3bt+j]
#pragma unroll
    for (int bt = 0; bt < 3; ++bt)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        double c = 0.0;
#pragma unroll
        for (int al = 0; al < 3; ++al) c += (double)W[s][al] * h.A[uix<9>(3 * al + i, 3 * bt + j)];
        C[bt][j] = c;
      }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        out[3 * t + j] = (double)W[t][0] * C[0][j] + (double)W[t][1] * C[1][j] + (double)W[t][2] * C[2][j];
  } else if (h.kind == H_PE) {
    const double IS2 = 0.70710678118654752, IS6 = 0.40824829046386302;
    // local index (0, 1, 2) of a slot in the stencil (point, e0, e1); basis rows
    // (1,-1,0)/sqrt2 and (1,1,-2)/sqrt6 over the local indices
    auto w0 = [&](int slot) { return slot == h.sl[0] ? IS2 : slot == h.sl[1] ? -IS2 : 0.0; };
    auto w1 = [&](int slot) { return slot == h.sl[0] || slot == h.sl[1] ? IS6 : slot == h.sl[2] ? -2.0 * IS6 : 0.0; };
    const double ws0 = w0(s), ws1 = w1(s);
    double C[2][3];
#pragma unroll
    for (int bt = 0; bt < 2; ++bt)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        C[bt][j] = ws0 * h.A[uix<6>(i, 3 * bt + j)] + ws1 * h.A[uix<6>(3 + i, 3 * bt + j)];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const double wt0 = w0(t), wt1 = w1(t);
#pragma unroll
      for (int j = 0; j < 3; ++j) out[3 * t + j] = wt0 * C[0][j] + wt1 * C[1][j];
    }
  } else if (h.kind == H_PP) {
    // blocks (s0,s0) = (s1,s1) = M, (s0,s1) = (s1,s0) = -M,
    // M = (l_r - l_t) r r^T / D + l_t I
    const double sr = s == h.sl[0] ? 1.0 : s == h.sl[1] ? -1.0 : 0.0;
    const double ri = h.A[i], lr = h.A[3], lt = h.A[4], iD = h.A[5];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const double st = t == h.sl[0] ? sr : t == h.sl[1] ? -sr : 0.0;
#pragma unroll
      for (int j = 0; j < 3; ++j) out[3 * t + j] = st * ((lr - lt) * ri * h.A[j] * iD + (i == j ? lt : 0.0));
    }
  }
}

// Evaluate one active pair with the sub-case `code` fixed by the narrow
// phase.  MIXED: the PSD projection of the reduced system runs in FP32
// (project_reduced); distances, energy, gradient and the Hessian before the
// projection stay FP64 on both paths (FP32 derivative terms lose up to 1e-2
// relative accuracy for nearly parallel edges, successive turns of a coiled
// rod).
template <bool MIXED>
__device__ __forceinline__ void eval_pair(const d3* P, int code, double a, double eta, double kappa, double* G,
                                          PairOut& h) {
  const double tol = 2.2e-16;
  int kind = case_kind(code);
  if (kind == K_PT || kind == K_EE) {
    eval_tri<MIXED>(P, kind == K_PT, a, eta, kappa, tol, G, h);
    return;
  }
  int s0, s1, s2;
  case_slots(code, s0, s1, s2);
  if (kind == K_PP) eval_pp(P, s0, s1, a, eta, kappa, G, h);
  else eval_pe<MIXED>(P, s0, s1, s2, a, eta, kappa, tol, G, h);
}

}  // namespace bfc
