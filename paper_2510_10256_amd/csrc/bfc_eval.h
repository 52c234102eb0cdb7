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

// Cyclic Jacobi eigen-decomposition of the symmetric N x N matrix A (upper
// triangle, destroyed) followed by A+ = V max(L, 0) V^T written to P (upper).
// Converges when the off-diagonal mass is below 1e-32 of the Frobenius mass.
template <int N> __device__ __forceinline__ void psd_jacobi(double* A, double* P) {
  constexpr int NU = N * (N + 1) / 2;
  double V[N][N];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) V[i][j] = i == j ? 1.0 : 0.0;
  double fro = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = i; j < N; ++j) fro += (i == j ? 1.0 : 2.0) * A[uix<N>(i, j)] * A[uix<N>(i, j)];
  for (int sweep = 0; sweep < 15; ++sweep) {
    double off = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = i + 1; j < N; ++j) off += A[uix<N>(i, j)] * A[uix<N>(i, j)];
    if (!(off > 1e-32 * fro)) break;
#pragma unroll
    for (int p = 0; p < N - 1; ++p) {
#pragma unroll
      for (int q = p + 1; q < N; ++q) {
        double apq = A[uix<N>(p, q)];
        if (apq != 0.0) {
          double tau = (A[uix<N>(q, q)] - A[uix<N>(p, p)]) / (2.0 * apq);
          double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          double c = 1.0 / sqrt(1.0 + t * t);
          double s = t * c;
          A[uix<N>(p, p)] -= t * apq;
          A[uix<N>(q, q)] += t * apq;
          A[uix<N>(p, q)] = 0.0;
#pragma unroll
          for (int k = 0; k < N; ++k) {
            if (k == p || k == q) continue;
            double akp = A[uix<N>(k, p)], akq = A[uix<N>(k, q)];
            A[uix<N>(k, p)] = c * akp - s * akq;
            A[uix<N>(k, q)] = s * akp + c * akq;
          }
#pragma unroll
          for (int k = 0; k < N; ++k) {
            double vkp = V[k][p], vkq = V[k][q];
            V[k][p] = c * vkp - s * vkq;
            V[k][q] = s * vkp + c * vkq;
          }
        }
      }
    }
  }
  double lam[N];
#pragma unroll
  for (int k = 0; k < N; ++k) lam[k] = fmax(A[uix<N>(k, k)], 0.0);
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = i; j < N; ++j) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) acc += V[i][k] * lam[k] * V[j][k];
      P[uix<N>(i, j)] = acc;
    }
  (void)NU;
}

// Output helpers: packed upper triangle of the 12 x 12 Hessian.
__device__ __forceinline__ int hix(int I, int J) { return I * 12 - (I * (I - 1)) / 2 + (J - I); }

struct PairOut {
  double E;
  double G[12];
  double H[78];
};

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

// ---- PP: closed-form projection ------------------------------------------
// H_y = c1 (2r)(2r)^T + 2 c2 I has eigenvalue kappa b'' along r and kappa b'/d
// across it; the projection keeps the positive parts.
__device__ __forceinline__ void eval_pp(const d3* P, int s0, int s1, double a, double eta, double kappa,
                                        PairOut& o) {
  d3 r = P[s0] - P[s1];
  double D = dot(r, r);
  Chain ch = chain_coeffs(D, a, eta, kappa);
  o.E = ch.E;
  if (ch.zero) return;
  double g[3] = {2.0 * ch.cg * r.x, 2.0 * ch.cg * r.y, 2.0 * ch.cg * r.z};
  double lr = 4.0 * ch.c1 * D + 2.0 * ch.c2;  // eigenvalue along r
  double lt = 2.0 * ch.c2;                    // eigenvalue across r
  lr = fmax(lr, 0.0);
  lt = fmax(lt, 0.0);
  double rr[3] = {r.x, r.y, r.z};
  double M[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) M[i][j] = (lr - lt) * rr[i] * rr[j] / D + (i == j ? lt : 0.0);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    o.G[3 * s0 + i] = g[i];
    o.G[3 * s1 + i] = -g[i];
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      int I0 = 3 * s0 + i, I1 = 3 * s1 + i, J0 = 3 * s0 + j, J1 = 3 * s1 + j;
      if (I0 <= J0) o.H[hix(I0, J0)] = M[i][j];
      if (I1 <= J1) o.H[hix(I1, J1)] = M[i][j];
      if (I0 <= J1) o.H[hix(I0, J1)] = -M[i][j];
      if (I1 <= J0) o.H[hix(I1, J0)] = -M[i][j];
    }
}

// ---- PE: 6 x 6 reduced system ----------------------------------------------
// Orthonormal basis of the translation complement of slots (p, e0, e1):
// w1 = (1, -1, 0)/sqrt2, w2 = (1, 1, -2)/sqrt6.  With y = (r, e) = Y x the
// coupling b = Y W is [[sqrt2, 0], [1/sqrt2, -3/sqrt6]].
__device__ __forceinline__ void eval_pe(const d3* P, int sp, int se0, int se1, double a, double eta,
                                        double kappa, PairOut& o) {
  const double S2 = 1.4142135623730951, IS2 = 0.70710678118654752, IS6 = 0.40824829046386302;
  d3 r = P[sp] - P[se0], e = P[se1] - P[se0];
  double s = dot(r, e), m = dot(e, e), im = 1.0 / m;
  d3 c = cross(r, e);
  double D = dot(c, c) * im;
  Chain ch = chain_coeffs(D, a, eta, kappa);
  o.E = ch.E;
  if (ch.zero) return;
  double rv[3] = {r.x, r.y, r.z}, ev[3] = {e.x, e.y, e.z};
  // gradient of D in y
  double gr[3], ge[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    gr[i] = 2.0 * rv[i] - 2.0 * s * im * ev[i];
    ge[i] = -2.0 * s * im * rv[i] + 2.0 * s * s * im * im * ev[i];
  }
  // Hessian blocks of D in y
  double Hrr[3][3], Hre[3][3], Hee[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double dl = i == j ? 1.0 : 0.0;
      Hrr[i][j] = 2.0 * dl - 2.0 * im * ev[i] * ev[j];
      Hre[i][j] = -2.0 * im * ev[i] * rv[j] - 2.0 * s * im * dl + 4.0 * s * im * im * ev[i] * ev[j];
      Hee[i][j] = -2.0 * im * rv[i] * rv[j] + 4.0 * s * im * im * (rv[i] * ev[j] + ev[i] * rv[j]) +
                  2.0 * s * s * im * im * dl - 8.0 * s * s * im * im * im * ev[i] * ev[j];
    }
  // energy Hessian in y: Hy = c1 g g^T + c2 H
  double Yrr[3][3], Yre[3][3], Yee[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      Yrr[i][j] = ch.c1 * gr[i] * gr[j] + ch.c2 * Hrr[i][j];
      Yre[i][j] = ch.c1 * gr[i] * ge[j] + ch.c2 * Hre[i][j];
      Yee[i][j] = ch.c1 * ge[i] * ge[j] + ch.c2 * Hee[i][j];
    }
  // reduced A = (b x I)^T Hy (b x I), blocks alpha,beta in {1,2}:
  // b[r] = (S2, 0), b[e] = (IS2, -3 IS6)
  const double br1 = S2, br2 = 0.0, be1 = IS2, be2 = -3.0 * IS6;
  double A[21];
#pragma unroll
  for (int al = 0; al < 2; ++al)
#pragma unroll
    for (int be = al; be < 2; ++be) {
      double ra = al == 0 ? br1 : br2, ea = al == 0 ? be1 : be2;
      double rb = be == 0 ? br1 : br2, eb = be == 0 ? be1 : be2;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          int I = 3 * al + i, J = 3 * be + j;
          if (I > J) continue;
          A[uix<6>(I, J)] = ra * rb * Yrr[i][j] + ra * eb * Yre[i][j] + ea * rb * Yre[j][i] + ea * eb * Yee[i][j];
        }
    }
  double Ap[21];
  psd_jacobi<6>(A, Ap);
  // gradient: x-gradient of slot k = sum over y-vectors of Y[y][k] * g_y
  // Y rows: r = (1, -1, 0), e = (0, -1, 1) on (p, e0, e1)
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double grx = ch.cg * gr[i], gex = ch.cg * ge[i];
    o.G[3 * sp + i] = grx;
    o.G[3 * se0 + i] = -grx - gex;
    o.G[3 * se1 + i] = gex;
  }
  // back to slots: H+[s][t] = sum W[s][al] W[t][be] A+[al][be]
  const int sl[3] = {sp, se0, se1};
  const double W[3][2] = {{IS2, IS6}, {-IS2, IS6}, {0.0, -2.0 * IS6}};
#pragma unroll
  for (int u = 0; u < 3; ++u)
#pragma unroll
    for (int w = 0; w < 3; ++w)
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          int I = 3 * sl[u] + i, J = 3 * sl[w] + j;
          if (I > J) continue;
          double acc = 0.0;
#pragma unroll
          for (int al = 0; al < 2; ++al)
#pragma unroll
            for (int be = 0; be < 2; ++be) acc += W[u][al] * W[w][be] * Ap[uix<6>(3 * al + i, 3 * be + j)];
          o.H[hix(I, J)] = acc;
        }
}

// ---- PT and EE: 9 x 9 reduced system --------------------------------------
// Hadamard basis of the translation complement of four slots:
// w1 = (1,1,-1,-1)/2, w2 = (1,-1,1,-1)/2, w3 = (1,-1,-1,1)/2.
// Couplings b = Y W (rows r, u, v):
//   PT (r = p-t0, u = t1-t0, v = t2-t0):  r (0,1,1)  u (-1,1,0)  v (-1,0,1)
//   EE (r = a0-b0, u = a1-a0, v = b1-b0): r (1,0,1)  u (0,-1,-1) v (0,-1,1)
__device__ __forceinline__ void eval_tri(const d3* P, bool is_pt, double a, double eta, double kappa,
                                         PairOut& o) {
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
  o.E = ch.E;
  if (ch.zero) return;
  double uu = dot(u, u), vv = dot(v, v), uv = dot(u, v);
  // gradients of s and m in y = (r, u, v)
  d3 gs[3] = {n, cross(v, r), cross(r, u)};
  d3 gm[3] = {{0.0, 0.0, 0.0}, 2.0 * (vv * u - uv * v), 2.0 * (uu * v - uv * u)};
  // dD = (2 s / m) gs - (s^2/m^2) gm
  const double ks = 2.0 * s * im, km = -s * s * im * im;
  double g[9];
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int i = 0; i < 3; ++i) g[3 * b + i] = ks * comp(gs[b], i) + km * comp(gm[b], i);
  // d2D = (2/m) gs gs^T + (2s/m) Hs - (2s/m^2)(gs gm^T + gm gs^T) - (s^2/m^2) Hm + (2 s^2/m^3) gm gm^T
  const double k_ss = 2.0 * im, k_hs = 2.0 * s * im, k_sm = -2.0 * s * im * im, k_hm = -s * s * im * im,
               k_mm = 2.0 * s * s * im * im * im;
  // Hs blocks: [r,u] = -[v]x, [r,v] = [u]x, [u,v] = -[r]x (and transposes)
  double Sru[3][3], Srv[3][3], Suv[3][3];
  skew(v, Sru, -1.0);
  skew(u, Srv, 1.0);
  skew(r, Suv, -1.0);
  // energy Hessian in y, blocks Y[b][c] (b <= c): Hy = c1 g g^T + c2 d2D
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
  // couplings
  const float BPT[3][3] = {{0, 1, 1}, {-1, 1, 0}, {-1, 0, 1}};
  const float BEE[3][3] = {{1, 0, 1}, {0, -1, -1}, {0, -1, 1}};
  double A[45];
#pragma unroll
  for (int al = 0; al < 3; ++al)
#pragma unroll
    for (int be = al; be < 3; ++be)
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          int I = 3 * al + i, J = 3 * be + j;
          if (I > J) continue;
          double acc = 0.0;
#pragma unroll
          for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              double w = (double)(is_pt ? BPT[b][al] * BPT[c][be] : BEE[b][al] * BEE[c][be]);
              // Y[b][c][i][j] for b <= c, Y[c][b][j][i] otherwise
              double y = b <= c ? Y[b][c][i][j] : Y[c][b][j][i];
              acc += w * y;
            }
          A[uix<9>(I, J)] = acc;
        }
  double Ap[45];
  psd_jacobi<9>(A, Ap);
  // gradient in slots: Y rows per pair type
  double gr[3], gu[3], gv[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    gr[i] = ch.cg * g[i];
    gu[i] = ch.cg * g[3 + i];
    gv[i] = ch.cg * g[6 + i];
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    if (is_pt) {  // r = p - t0, u = t1 - t0, v = t2 - t0
      o.G[i] = gr[i];
      o.G[3 + i] = -gr[i] - gu[i] - gv[i];
      o.G[6 + i] = gu[i];
      o.G[9 + i] = gv[i];
    } else {      // r = a0 - b0, u = a1 - a0, v = b1 - b0
      o.G[i] = gr[i] - gu[i];
      o.G[3 + i] = gu[i];
      o.G[6 + i] = -gr[i] - gv[i];
      o.G[9 + i] = gv[i];
    }
  }
  // back to slots through the Hadamard basis
  const float W[4][3] = {{0.5f, 0.5f, 0.5f}, {0.5f, -0.5f, -0.5f}, {-0.5f, 0.5f, -0.5f}, {-0.5f, -0.5f, 0.5f}};
#pragma unroll
  for (int st = 0; st < 4; ++st)
#pragma unroll
    for (int tt = st; tt < 4; ++tt)
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          int I = 3 * st + i, J = 3 * tt + j;
          if (I > J) continue;
          double acc = 0.0;
#pragma unroll
          for (int al = 0; al < 3; ++al)
#pragma unroll
            for (int be = 0; be < 3; ++be)
              acc += (double)(W[st][al] * W[tt][be]) * Ap[uix<9>(3 * al + i, 3 * be + j)];
          o.H[hix(I, J)] = acc;
        }
}

// Evaluate one active pair with the sub-case `code` fixed by the narrow phase.
__device__ __forceinline__ void eval_pair(const d3* P, int code, double a, double eta, double kappa,
                                          PairOut& o) {
  o.E = 0.0;
#pragma unroll
  for (int k = 0; k < 12; ++k) o.G[k] = 0.0;
#pragma unroll
  for (int k = 0; k < 78; ++k) o.H[k] = 0.0;
  int kind = case_kind(code);
  if (kind == K_PT || kind == K_EE) {
    eval_tri(P, kind == K_PT, a, eta, kappa, o);
    return;
  }
  int s0, s1, s2;
  case_slots(code, s0, s1, s2);
  if (kind == K_PP) eval_pp(P, s0, s1, a, eta, kappa, o);
  else eval_pe(P, s0, s1, s2, a, eta, kappa, o);
}

}  // namespace bfc
