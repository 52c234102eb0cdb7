// Device geometry for barrier-filtered contact evaluation on gfx950.
//
// Distances between contact primitives (point-triangle and edge-edge pairs,
// Sec. 3), the exact threshold decisions of the filter and the barrier, the
// offset IPC barrier (Eq. 2 with the shift of Eq. 3), its derivatives and the
// projection of each pair Hessian onto the PSD cone (App. A: projected Newton).
//
// Local layout of a pair: four stencil vertices (slots), point-triangle pairs
// (p, t0, t1, t2), edge-edge pairs (a0, a1, b0, b1).  Distance sub-case codes:
//   point-triangle: 0 PP(0,1) 1 PP(0,2) 2 PP(0,3) 3 PE(0;1,2) 4 PE(0;2,3) 5 PE(0;3,1) 6 PT
//   edge-edge:      7 PP(0,2) 8 PP(0,3) 9 PP(1,2) 10 PP(1,3)
//                   11 PE(0;2,3) 12 PE(1;2,3) 13 PE(2;0,1) 14 PE(3;0,1) 15 EE
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

namespace bfc {

// Host and device: the geometry and its exact decisions are also built for
// the CPU tests.
#define BFC_GD __host__ __device__ __forceinline__

// ---------------------------------------------------------------------------
// double-double arithmetic (about 106 significant bits), used to re-decide
// threshold comparisons that fall inside the FP64 guard band.  Its
// error-free transformations need every product and sum rounded on its own:
// each function turns FP contraction off, or the compiler would fuse a
// product into the following two-sum as an FMA and lose the error term.
// ---------------------------------------------------------------------------
struct dd {
  double hi, lo;
};
BFC_GD dd dd_two_sum(double a, double b) {
#pragma clang fp contract(off)
  double s = a + b;
  double bb = s - a;
  double e = (a - (s - bb)) + (b - bb);
  return {s, e};
}
BFC_GD dd dd_fast(double a, double b) {
#pragma clang fp contract(off)
  double s = a + b;
  return {s, b - (s - a)};
}
BFC_GD dd operator+(dd a, dd b) {
#pragma clang fp contract(off)
  dd s = dd_two_sum(a.hi, b.hi);
  dd t = dd_two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = dd_fast(s.hi, s.lo);
  s.lo += t.lo;
  return dd_fast(s.hi, s.lo);
}
BFC_GD dd operator-(dd a) { return {-a.hi, -a.lo}; }
BFC_GD dd operator-(dd a, dd b) { return a + (-b); }
BFC_GD dd operator*(dd a, dd b) {
#pragma clang fp contract(off)
  double p = a.hi * b.hi;
  double e = fma(a.hi, b.hi, -p);
  e += a.hi * b.lo + a.lo * b.hi;
  return dd_fast(p, e);
}
BFC_GD dd operator/(dd a, dd b) {
#pragma clang fp contract(off)
  double q1 = a.hi / b.hi;
  dd r = a - dd{q1, 0.0} * b;
  double q2 = r.hi / b.hi;
  r = r - dd{q2, 0.0} * b;
  double q3 = r.hi / b.hi;
  dd q = dd_fast(q1, q2);
  return q + dd{q3, 0.0};
}
BFC_GD bool dd_lt(dd a, dd b) { return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo); }
BFC_GD bool dd_le(dd a, dd b) { return a.hi < b.hi || (a.hi == b.hi && a.lo <= b.lo); }
BFC_GD dd dd_of(double v) { return {v, 0.0}; }
// exact square of a double
BFC_GD dd dd_sq(double v) {
#pragma clang fp contract(off)
  double p = v * v;
  return {p, fma(v, v, -p)};
}

// ---------------------------------------------------------------------------
// 3-vectors over a scalar type (double, float or dd)
// ---------------------------------------------------------------------------
template <class T> struct V3 {
  T x, y, z;
};
template <class T> BFC_GD V3<T> operator-(V3<T> a, V3<T> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class T> BFC_GD V3<T> operator+(V3<T> a, V3<T> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class T> BFC_GD V3<T> operator*(T s, V3<T> a) { return {s * a.x, s * a.y, s * a.z}; }
template <class T> BFC_GD T dot(V3<T> a, V3<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class T> BFC_GD V3<T> cross(V3<T> a, V3<T> b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
typedef V3<double> d3;
typedef V3<dd> q3;

BFC_GD q3 q3_of(d3 a) { return {dd_of(a.x), dd_of(a.y), dd_of(a.z)}; }

// ---------------------------------------------------------------------------
// Sub-case table
// ---------------------------------------------------------------------------
enum { K_PP = 0, K_PE = 1, K_PT = 2, K_EE = 3 };
BFC_GD int case_kind(int code) {
  // 0-2 PP, 3-5 PE, 6 PT, 7-10 PP, 11-14 PE, 15 EE
  return code <= 2 ? K_PP : code <= 5 ? K_PE : code == 6 ? K_PT : code <= 10 ? K_PP : code <= 14 ? K_PE : K_EE;
}
// participating slots; PP: (s0, s1); PE: point s0, edge (s1, s2); PT/EE: all four
BFC_GD void case_slots(int code, int& s0, int& s1, int& s2) {
  switch (code) {
    case 0: s0 = 0; s1 = 1; s2 = -1; break;
    case 1: s0 = 0; s1 = 2; s2 = -1; break;
    case 2: s0 = 0; s1 = 3; s2 = -1; break;
    case 3: s0 = 0; s1 = 1; s2 = 2; break;
    case 4: s0 = 0; s1 = 2; s2 = 3; break;
    case 5: s0 = 0; s1 = 3; s2 = 1; break;
    case 7: s0 = 0; s1 = 2; s2 = -1; break;
    case 8: s0 = 0; s1 = 3; s2 = -1; break;
    case 9: s0 = 1; s1 = 2; s2 = -1; break;
    case 10: s0 = 1; s1 = 3; s2 = -1; break;
    case 11: s0 = 0; s1 = 2; s2 = 3; break;
    case 12: s0 = 1; s1 = 2; s2 = 3; break;
    case 13: s0 = 2; s1 = 0; s2 = 1; break;
    case 14: s0 = 3; s1 = 0; s2 = 1; break;
    default: s0 = 0; s1 = 1; s2 = 2; break;
  }
}

// ---------------------------------------------------------------------------
// Squared-distance formulas per kind (any scalar type)
// ---------------------------------------------------------------------------
template <class T> BFC_GD T sqd_pp(V3<T> p, V3<T> q) {
  V3<T> r = p - q;
  return dot(r, r);
}
template <class T> BFC_GD T sqd_pe(V3<T> p, V3<T> e0, V3<T> e1) {
  V3<T> e = e1 - e0;
  V3<T> c = cross(p - e0, e);
  return dot(c, c) / dot(e, e);
}
// plane / line-line form shared by PT and EE: (r . (u x v))^2 / |u x v|^2
template <class T> BFC_GD T sqd_tri(V3<T> r, V3<T> u, V3<T> v) {
  V3<T> n = cross(u, v);
  T s = dot(r, n);
  return s * s / dot(n, n);
}
// one of four vertices, chosen by value selects (indexing the array with a
// run-time slot, or selecting between element addresses, would keep the
// array in scratch memory)
template <class T> BFC_GD T sel4(int s, T a, T b, T c, T d) {
  T lo = s == 0 ? a : b;
  T hi = s == 2 ? c : d;
  return s < 2 ? lo : hi;
}
template <class T> BFC_GD V3<T> pick(const V3<T>* P, int s) {
  const V3<T> p0 = P[0], p1 = P[1], p2 = P[2], p3 = P[3];
  return {sel4(s, p0.x, p1.x, p2.x, p3.x), sel4(s, p0.y, p1.y, p2.y, p3.y), sel4(s, p0.z, p1.z, p2.z, p3.z)};
}
template <class T> BFC_GD T sqd_case(int code, const V3<T>* P) {
  int k = case_kind(code);
  if (k == K_PT) return sqd_tri(P[0] - P[1], P[2] - P[1], P[3] - P[1]);
  if (k == K_EE) return sqd_tri(P[0] - P[2], P[1] - P[0], P[3] - P[2]);
  int s0, s1, s2;
  case_slots(code, s0, s1, s2);
  if (k == K_PP) return sqd_pp(pick(P, s0), pick(P, s1));
  return sqd_pe(pick(P, s0), pick(P, s1), pick(P, s2));
}

// ---------------------------------------------------------------------------
// Classification in FP64: nearest features of the two primitives
// ---------------------------------------------------------------------------
struct Near {
  double D;
  int code;
};
// point p against segment (e0, e1): vertex e0, vertex e1, or interior
BFC_GD Near near_pseg(d3 p, d3 e0, d3 e1, int c0, int c1, int ce) {
  d3 e = e1 - e0, r = p - e0;
  double re = dot(r, e), ee = dot(e, e);
  if (re <= 0.0) return {dot(r, r), c0};
  if (re >= ee) {
    d3 q = p - e1;
    return {dot(q, q), c1};
  }
  d3 c = cross(r, e);
  return {dot(c, c) / ee, ce};
}
// Keep the first-listed candidate among ties: a later one must be closer by
// more than a relative 1e-12 (exactly parallel edges make several
// point-segment sub-cases equidistant; the listing order picks one).
BFC_GD void take_min(Near& best, Near c) {
  if (c.D < best.D * (1.0 - 1e-12)) best = c;
}
BFC_GD Near classify_pt(const d3* P) {
  d3 u = P[2] - P[1], v = P[3] - P[1], r = P[0] - P[1];
  double uu = dot(u, u), uv = dot(u, v), vv = dot(v, v), ru = dot(r, u), rv = dot(r, v);
  double det = uu * vv - uv * uv;
  double bn = vv * ru - uv * rv;  // barycentric weight of t1 times det
  double gn = uu * rv - uv * ru;  // barycentric weight of t2 times det
  if (bn > 0.0 && gn > 0.0 && bn + gn < det) return {sqd_tri(r, u, v), 6};
  Near best = near_pseg(P[0], P[1], P[2], 0, 1, 3);
  take_min(best, near_pseg(P[0], P[2], P[3], 1, 2, 4));
  take_min(best, near_pseg(P[0], P[3], P[1], 2, 0, 5));
  return best;
}
// |ea x eb|^2 below this fraction of |ea|^2 |eb|^2: treat the edges as parallel
// and take the nearest of the four point-segment sub-cases
#define BFC_PARALLEL_TOL 1e-10
BFC_GD Near classify_ee(const d3* P) {
  d3 ea = P[1] - P[0], eb = P[3] - P[2], r = P[0] - P[2];
  double A = dot(ea, ea), B = dot(ea, eb), C = dot(eb, eb);
  d3 n = cross(ea, eb);
  double nn = dot(n, n);
  if (!(nn < BFC_PARALLEL_TOL * A * C)) {
    double Dd = dot(ea, r), Ee = dot(eb, r);
    double den = A * C - B * B;
    double sn = B * Ee - C * Dd;  // line parameter on edge a, times den
    double tn = A * Ee - B * Dd;  // line parameter on edge b, times den
    if (sn > 0.0 && sn < den && tn > 0.0 && tn < den) return {sqd_tri(r, ea, eb), 15};
  }
  Near best = near_pseg(P[0], P[2], P[3], 7, 8, 11);
  take_min(best, near_pseg(P[1], P[2], P[3], 9, 10, 12));
  take_min(best, near_pseg(P[2], P[0], P[1], 7, 9, 13));
  take_min(best, near_pseg(P[3], P[0], P[1], 8, 10, 14));
  return best;
}

// ---------------------------------------------------------------------------
// Exact arithmetic on expansions (Shewchuk, "Adaptive Precision
// Floating-Point Arithmetic and Fast Robust Geometric Predicates", 1997): a
// value is kept as an unevaluated sum of non-overlapping doubles of
// increasing magnitude; the two-sum and the FMA two-product are error free,
// so every sum and product below is exact.  Used for the rare threshold
// decisions whose double-double value lies within 1e-20 of the threshold
// (exact ties of lattice geometry, and values closer to it than
// double-double resolves), in a kernel of their own (k_exact): each thread
// works on a slab of XP_WS doubles of its own.
// ---------------------------------------------------------------------------
constexpr int XP_CAP = 32;                // doubles per expansion
constexpr int XP_SLOTS = 12;              // expansions per slab
constexpr int XP_WS = XP_CAP * XP_SLOTS;  // doubles of LDS per wave

// h = e + b (e: n components); the length, or -1 past XP_CAP
BFC_GD int xp_grow(const double* e, int n, double b, double* h) {
#pragma clang fp contract(off)
  double q = b;
  int m = 0;
  for (int i = 0; i < n; ++i) {
    const dd s = dd_two_sum(q, e[i]);
    if (s.lo != 0.0) {
      if (m >= XP_CAP) return -1;
      h[m++] = s.lo;
    }
    q = s.hi;
  }
  if (q != 0.0 || m == 0) {
    if (m >= XP_CAP) return -1;
    h[m++] = q;
  }
  return m;
}
// in place: the fewest components (largest last)
BFC_GD int xp_compress(double* e, int n) {
#pragma clang fp contract(off)
  if (n <= 1) return n;
  int bottom = n - 1;
  double Q = e[n - 1];
  for (int i = n - 2; i >= 0; --i) {
    const dd s = dd_fast(Q, e[i]);
    if (s.lo != 0.0) {
      e[bottom--] = s.hi;
      Q = s.lo;
    } else {
      Q = s.hi;
    }
  }
  e[bottom] = Q;
  int top = 0;
  for (int i = bottom + 1; i < n; ++i) {
    const dd s = dd_fast(e[i], Q);
    if (s.lo != 0.0) e[top++] = s.lo;
    Q = s.hi;
  }
  e[top++] = Q;
  return top;
}
// h = e + f (h may not alias e or f; t: scratch of XP_CAP); -1 past XP_CAP
BFC_GD int xp_add(const double* e, int ne, const double* f, int nf, double* h, double* t) {
  if (ne < 0 || nf < 0) return -1;
  double* cur = h;
  double* oth = t;
  for (int i = 0; i < ne; ++i) cur[i] = e[i];
  int n = ne;
  for (int j = 0; j < nf && n >= 0; ++j) {
    n = xp_grow(cur, n, f[j], oth);
    double* x = cur;
    cur = oth;
    oth = x;
  }
  if (n < 0) return -1;
  n = xp_compress(cur, n);
  if (cur != h)
    for (int i = 0; i < n; ++i) h[i] = cur[i];
  return n;
}
// h = -e
BFC_GD int xp_neg(const double* e, int n, double* h) {
  for (int i = 0; i < n; ++i) h[i] = -e[i];
  return n;
}
// h = e * b; -1 past XP_CAP
BFC_GD int xp_scale(const double* e, int n, double b, double* h) {
#pragma clang fp contract(off)
  if (n < 0 || 2 * n > XP_CAP) return -1;
  if (n == 0 || b == 0.0) {
    h[0] = 0.0;
    return 1;
  }
  int m = 0;
  double p = e[0] * b;
  double lo = fma(e[0], b, -p);
  if (lo != 0.0) h[m++] = lo;
  double Q = p;
  for (int i = 1; i < n; ++i) {
    const double T = e[i] * b, t = fma(e[i], b, -T);
    dd s = dd_two_sum(Q, t);
    if (s.lo != 0.0) h[m++] = s.lo;
    s = dd_fast(T, s.hi);
    if (s.lo != 0.0) h[m++] = s.lo;
    Q = s.hi;
  }
  if (Q != 0.0 || m == 0) h[m++] = Q;
  return m;
}
// h = e * f (t1, t2, t3: scratch of XP_CAP); -1 past XP_CAP
BFC_GD int xp_mul(const double* e, int ne, const double* f, int nf, double* h, double* t1,
                                      double* t2, double* t3) {
  if (ne < 0 || nf < 0) return -1;
  int n = 0;
  for (int j = 0; j < nf; ++j) {
    const int ns = xp_scale(e, ne, f[j], t1);
    if (ns < 0) return -1;
    n = xp_add(h, n, t1, ns, t2, t3);
    if (n < 0) return -1;
    for (int i = 0; i < n; ++i) h[i] = t2[i];
  }
  return n;
}
BFC_GD int xp_sign(const double* e, int n) {
  const double top = n > 0 ? e[n - 1] : 0.0;
  return top > 0.0 ? 1 : (top < 0.0 ? -1 : 0);
}
// h = a - b exactly (two components)
BFC_GD int xp_diff(double a, double b, double* h) {
  const dd s = dd_two_sum(a, -b);
  if (s.lo != 0.0) {
    h[0] = s.lo;
    h[1] = s.hi;
    return 2;
  }
  h[0] = s.hi;
  return 1;
}

// Exact sign of (squared distance of sub-case `code` at the FP64 vertices
// p0..p3) - T, T = T.hi + T.lo exactly: -1, 0 or 1.  D = num / den with
// den > 0 (a zero den, a degenerate primitive, counts as above T); ws: the
// thread's slab.  Returns 2 when an expansion outgrew XP_CAP (the caller
// then keeps the double-double decision).
__host__ __device__ __noinline__ int xp_sign_sq_minus(int code, d3 p0, d3 p1, d3 p2, d3 p3, dd T, double* ws) {
  const d3 P[4] = {p0, p1, p2, p3};
  double *A = ws, *B = ws + XP_CAP, *C = ws + 2 * XP_CAP, *N0 = ws + 3 * XP_CAP, *N1 = ws + 4 * XP_CAP,
         *N2 = ws + 5 * XP_CAP, *NUM = ws + 6 * XP_CAP, *DEN = ws + 7 * XP_CAP, *T1 = ws + 8 * XP_CAP,
         *T2 = ws + 9 * XP_CAP, *T3 = ws + 10 * XP_CAP, *DF = ws + 11 * XP_CAP;
  // DF holds nine two-component differences: u (0..5), v (6..11), r (12..17)
  int nd[9];
  auto diff3 = [&](int slot, d3 a, d3 b) {
    nd[3 * slot] = xp_diff(a.x, b.x, DF + 6 * slot);
    nd[3 * slot + 1] = xp_diff(a.y, b.y, DF + 6 * slot + 2);
    nd[3 * slot + 2] = xp_diff(a.z, b.z, DF + 6 * slot + 4);
  };
  auto comp = [&](int slot, int c) { return DF + 6 * slot + 2 * c; };
  auto ncomp = [&](int slot, int c) { return nd[3 * slot + c]; };
  // dot of two difference vectors (slots a, b) into H
  auto dot_d = [&](int a, int b, double* H) {
    int n = 0;
    for (int c = 0; c < 3 && n >= 0; ++c) {
      const int m = xp_mul(comp(a, c), ncomp(a, c), comp(b, c), ncomp(b, c), T1, T2, T3, C);
      if (m < 0) return -1;
      n = xp_add(H, n, T1, m, B, T2);
      if (n < 0) return -1;
      for (int i = 0; i < n; ++i) H[i] = B[i];
    }
    return n;
  };
  // n = (slot a) x (slot b) into N0, N1, N2
  int nn[3];
  auto cross_d = [&](int a, int b) {
    double* Nc[3] = {N0, N1, N2};
    for (int c = 0; c < 3; ++c) {
      const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
      const int m1 = xp_mul(comp(a, c1), ncomp(a, c1), comp(b, c2), ncomp(b, c2), A, T1, T2, T3);
      const int m2 = xp_mul(comp(a, c2), ncomp(a, c2), comp(b, c1), ncomp(b, c1), B, T1, T2, T3);
      if (m1 < 0 || m2 < 0) return false;
      xp_neg(B, m2, T1);
      nn[c] = xp_add(A, m1, T1, m2, Nc[c], T2);
      if (nn[c] < 0) return false;
    }
    return true;
  };
  auto dot_n = [&](double* H, const double* const* X, const int* nx, const double* const* Y, const int* ny) {
    int n = 0;
    for (int c = 0; c < 3; ++c) {
      const int m = xp_mul(X[c], nx[c], Y[c], ny[c], T1, T2, T3, C);
      if (m < 0) return -1;
      n = xp_add(H, n, T1, m, A, T2);
      if (n < 0) return -1;
      for (int i = 0; i < n; ++i) H[i] = A[i];
    }
    return n;
  };
  const int kind = case_kind(code);
  int s0, s1, s2;
  case_slots(code, s0, s1, s2);
  int nnum = -1, nden = -1;
  if (kind == K_PP) {
    diff3(0, pick(P, s0), pick(P, s1));
    nnum = dot_d(0, 0, NUM);
    DEN[0] = 1.0;
    nden = 1;
  } else if (kind == K_PE) {
    const d3 p = pick(P, s0), e0 = pick(P, s1), e1 = pick(P, s2);
    diff3(0, p, e0);   // r
    diff3(1, e1, e0);  // e
    if (cross_d(0, 1)) {
      const double* Nc[3] = {N0, N1, N2};
      nnum = dot_n(NUM, Nc, nn, Nc, nn);
    }
    nden = dot_d(1, 1, DEN);
  } else {
    if (kind == K_PT) {
      diff3(0, P[2], P[1]);  // u = t1 - t0
      diff3(1, P[3], P[1]);  // v = t2 - t0
      diff3(2, P[0], P[1]);  // r = p - t0
    } else {
      diff3(0, P[1], P[0]);  // u = a1 - a0
      diff3(1, P[3], P[2]);  // v = b1 - b0
      diff3(2, P[0], P[2]);  // r = a0 - b0
    }
    if (cross_d(0, 1)) {
      const double* Nc[3] = {N0, N1, N2};
      const double* R[3] = {comp(2, 0), comp(2, 1), comp(2, 2)};
      const int nr[3] = {ncomp(2, 0), ncomp(2, 1), ncomp(2, 2)};
      const int ns = dot_n(DEN, R, nr, Nc, nn);  // s = r . n (DEN as a temporary)
      if (ns >= 0) nnum = xp_mul(DEN, ns, DEN, ns, NUM, T1, T2, T3);
      nden = dot_n(DEN, Nc, nn, Nc, nn);
    }
  }
  if (nnum < 0 || nden < 0) return 2;
  if (xp_sign(DEN, nden) <= 0) return 1;
  // num - T den
  double tt[2] = {T.lo, T.hi};
  const int nt = T.lo != 0.0 ? 2 : 1;
  const int m = xp_mul(DEN, nden, nt == 2 ? tt : tt + 1, nt, A, T1, T2, T3);
  if (m < 0) return 2;
  xp_neg(A, m, B);
  const int r = xp_add(NUM, nnum, B, m, C, T1);
  if (r < 0) return 2;
  return xp_sign(C, r);
}

// Exact: is the 2D squared distance from p to the segment (a, b) below H2
// (exactly T.hi + T.lo)?  1 yes, 0 no, 2 past XP_CAP.  The branch tests
// (closest point at a, at b, or inside) are exact too.
__host__ __device__ __noinline__ int xp_seg2_below(double px, double py, double ax, double ay, double bx, double by, dd H2,
                                          double* ws) {
  double *EX = ws, *EY = ws + 2, *RX = ws + 4, *RY = ws + 6, *A = ws + XP_CAP, *B = ws + 2 * XP_CAP,
         *C = ws + 3 * XP_CAP, *V = ws + 4 * XP_CAP, *W = ws + 5 * XP_CAP, *T1 = ws + 6 * XP_CAP,
         *T2 = ws + 7 * XP_CAP, *T3 = ws + 8 * XP_CAP, *T4 = ws + 9 * XP_CAP;
  const int nex = xp_diff(bx, ax, EX), ney = xp_diff(by, ay, EY);
  const int nrx = xp_diff(px, ax, RX), nry = xp_diff(py, ay, RY);
  // V = x1 y1 + x2 y2 (the inputs two-component differences)
  auto dot2 = [&](const double* x1, int n1, const double* y1, int m1, const double* x2, int n2, const double* y2,
                  int m2, double* out, int sign2) {
    const int a = xp_mul(x1, n1, y1, m1, A, T1, T2, T3);
    int b = xp_mul(x2, n2, y2, m2, B, T1, T2, T3);
    if (a < 0 || b < 0) return -1;
    if (sign2 < 0) b = xp_neg(B, b, C);
    return xp_add(A, a, sign2 < 0 ? C : B, b, out, T4);
  };
  double tt[2] = {H2.lo, H2.hi};
  const double* Th = H2.lo != 0.0 ? tt : tt + 1;
  const int nt = H2.lo != 0.0 ? 2 : 1;
  const int nre = dot2(RX, nrx, EX, nex, RY, nry, EY, ney, V, 1);   // r . e
  const int nee = dot2(EX, nex, EX, nex, EY, ney, EY, ney, W, 1);   // e . e
  if (nre < 0 || nee < 0) return 2;
  int nval;
  if (xp_sign(V, nre) <= 0) {         // closest point a: |r|^2 - H2
    nval = dot2(RX, nrx, RX, nrx, RY, nry, RY, nry, V, 1);
  } else {
    xp_neg(W, nee, T4);
    const int nd = xp_add(V, nre, T4, nee, C, T1);  // r . e - e . e
    if (nd < 0) return 2;
    if (xp_sign(C, nd) >= 0) {        // closest point b: |p - b|^2
      const int nqx = xp_diff(px, bx, RX), nqy = xp_diff(py, by, RY);
      nval = dot2(RX, nqx, RX, nqx, RY, nqy, RY, nqy, V, 1);
    } else {                          // inside: c^2 / ee with c = r x e (2D)
      const int nc = dot2(RX, nrx, EY, ney, RY, nry, EX, nex, V, -1);
      if (nc < 0) return 2;
      for (int i = 0; i < nc; ++i) C[i] = V[i];
      nval = xp_mul(C, nc, C, nc, V, T1, T2, T3);  // c^2
      if (nval < 0) return 2;
      for (int i = 0; i < nee; ++i) C[i] = W[i];
      const int nh = xp_mul(C, nee, Th, nt, W, T1, T2, T3);  // H2 ee
      if (nh < 0) return 2;
      xp_neg(W, nh, T4);
      const int nr = xp_add(V, nval, T4, nh, C, T1);
      return nr < 0 ? 2 : (xp_sign(C, nr) < 0 ? 1 : 0);
    }
  }
  if (nval < 0) return 2;
  for (int i = 0; i < nt; ++i) W[i] = -Th[i];
  const int nr = xp_add(V, nval, W, nt, C, T1);
  return nr < 0 ? 2 : (xp_sign(C, nr) < 0 ? 1 : 0);
}

// ---------------------------------------------------------------------------
// Exactness in FP64: the sub-case formulas as num / den evaluated in double,
// checking that no operation rounded (every sum's two-sum error and every
// product's FMA residual is zero).  Then num and den are the exact values and
// num - T den is decided exactly from five doubles.  Lattice geometry (exact
// ties at d_min or h) passes this check: it settles those ties without
// expansion arithmetic.
// ---------------------------------------------------------------------------
struct ExactD {
  bool ok;
  BFC_GD double add(double a, double b) {
#pragma clang fp contract(off)
    const dd s = dd_two_sum(a, b);
    ok = ok && s.lo == 0.0;
    return s.hi;
  }
  BFC_GD double sub(double a, double b) { return add(a, -b); }
  BFC_GD double mul(double a, double b) {
#pragma clang fp contract(off)
    const double p = a * b;
    ok = ok && fma(a, b, -p) == 0.0;
    return p;
  }
  BFC_GD d3 sub3(d3 a, d3 b) { return {sub(a.x, b.x), sub(a.y, b.y), sub(a.z, b.z)}; }
  BFC_GD double dot3(d3 a, d3 b) { return add(add(mul(a.x, b.x), mul(a.y, b.y)), mul(a.z, b.z)); }
  BFC_GD d3 cross3(d3 a, d3 b) {
    return {sub(mul(a.y, b.z), mul(a.z, b.y)), sub(mul(a.z, b.x), mul(a.x, b.z)), sub(mul(a.x, b.y), mul(a.y, b.x))};
  }
};
// sign of num - T den (num, den, T.hi, T.lo exact doubles, den > 0), exactly:
// the five terms summed as an expansion (Shewchuk's grow with zero elimination)
BFC_GD int sign_num_minus_tden(double num, double den, dd T) {
#pragma clang fp contract(off)
  const double p1 = T.hi * den, e1 = fma(T.hi, den, -p1);
  const double p2 = T.lo * den, e2 = fma(T.lo, den, -p2);
  const double t[5] = {num, -p1, -e1, -p2, -e2};
  double h[5];
  int m = 0;
#pragma unroll
  for (int k = 0; k < 5; ++k) {  // h <- h + t[k]; h stays non-overlapping, increasing
    double q = t[k];
    int m2 = 0;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      if (i >= m) break;
      const dd s = dd_two_sum(q, h[i]);
      if (s.lo != 0.0) h[m2++] = s.lo;
      q = s.hi;
    }
    h[m2++] = q;
    m = m2;
  }
  const double top = h[m - 1];  // the largest component: the sign of the sum (zero only if all are zero)
  return top > 0.0 ? 1 : (top < 0.0 ? -1 : 0);
}
// -1 / 0 / 1: sign of D - T, exact, when sub-case `code` evaluates without
// rounding in FP64; 2 otherwise
BFC_GD int exact_in_double(int code, const d3* P, dd T) {
  ExactD E{true};
  double num, den;
  const int k = case_kind(code);
  if (k == K_PT || k == K_EE) {
    const d3 r = k == K_PT ? E.sub3(P[0], P[1]) : E.sub3(P[0], P[2]);
    const d3 u = k == K_PT ? E.sub3(P[2], P[1]) : E.sub3(P[1], P[0]);
    const d3 v = k == K_PT ? E.sub3(P[3], P[1]) : E.sub3(P[3], P[2]);
    const d3 n = E.cross3(u, v);
    const double sc = E.dot3(r, n);
    num = E.mul(sc, sc);
    den = E.dot3(n, n);
  } else {
    int s0, s1, s2;
    case_slots(code, s0, s1, s2);
    if (k == K_PP) {
      const d3 r = E.sub3(pick(P, s0), pick(P, s1));
      num = E.dot3(r, r);
      den = 1.0;
    } else {
      const d3 r = E.sub3(pick(P, s0), pick(P, s1)), e = E.sub3(pick(P, s2), pick(P, s1));
      const d3 c = E.cross3(r, e);
      num = E.dot3(c, c);
      den = E.dot3(e, e);
    }
  }
  if (!E.ok || !(den > 0.0) || !(fabs(num) <= 1.7976931348623157e308) || !(den <= 1.7976931348623157e308)) return 2;
  return sign_num_minus_tden(num, den, T);
}

// Exact sign of D - T for a point-edge sub-case, D = |r x e|^2 / |e|^2, as
// the sign of |r x e|^2 - T |e|^2 summed in 256-bit fixed point (no memory:
// the near ties of lattice-like geometry, which double-double cannot
// settle, are mostly of this kind).  r = p - e0 and e = e1 - e0 must be
// exact in FP64.  Every component of r x e is the sum of the two error-free
// products' four parts t_a, so |r x e|^2 is the sum of the error-free
// products t_a t_b; T |e|^2 likewise from e_x^2 and T = T.hi + T.lo.  Each of
// these doubles, an integer m < 2^53 times a power of two, is added into the
// accumulator at its bit position.  The accumulator's lowest bit is 2^-224
// of the largest term, which leaves every product's low part inside; a term
// outside the window returns 2, as does a difference that is not exact or a
// zero |e| (the caller then takes its other exact path).
struct FixAcc {
  unsigned long long w[4];
  int lsb;  // exponent of bit 0
  bool ok;
};
BFC_GD void fix_add(FixAcc& A, double d) {
  if (d == 0.0) return;
  unsigned long long bits;
  memcpy(&bits, &d, sizeof(bits));
  const bool neg = (bits >> 63) != 0;
  const int E = (int)((bits >> 52) & 0x7ff);
  unsigned long long m = bits & ((1ull << 52) - 1);
  int ex;
  if (E == 0) {
    ex = -1074;
  } else {
    m |= 1ull << 52;
    ex = E - 1075;
  }
  const int pos = ex - A.lsb;
  if (E == 0x7ff || pos < 0 || pos > 192) {  // not finite, below the window, or too close to its top
    A.ok = false;
    return;
  }
  unsigned long long t[4] = {0, 0, 0, 0};
  const int L = pos >> 6, sh = pos & 63;
  t[L] = m << sh;
  if (sh != 0) t[L + 1] = m >> (64 - sh);  // L <= 3 and, for sh != 0, L + 1 <= 3 since pos <= 192
  if (!neg) {
    unsigned long long c = 0;
    for (int i = 0; i < 4; ++i) {
      const unsigned long long x = A.w[i], s1 = x + t[i], c1 = s1 < x, s2 = s1 + c, c2 = s2 < s1;
      A.w[i] = s2;
      c = c1 | c2;
    }
  } else {
    unsigned long long b = 0;
    for (int i = 0; i < 4; ++i) {
      const unsigned long long x = A.w[i], d1 = x - t[i], b1 = x < t[i], d2 = d1 - b, b2 = d1 < b;
      A.w[i] = d2;
      b = b1 | b2;
    }
  }
}
BFC_GD void fix_prod(FixAcc& A, double a, double b, bool neg) {  // add (or subtract) a b exactly
#pragma clang fp contract(off)
  const double p = a * b, e = fma(a, b, -p);
  fix_add(A, neg ? -p : p);
  fix_add(A, neg ? -e : e);
}
__host__ __device__ __noinline__ int pe_sign_fixed(d3 p, d3 e0, d3 e1, dd T) {
#pragma clang fp contract(off)
  ExactD X{true};
  const d3 r = X.sub3(p, e0), e = X.sub3(e1, e0);
  if (!X.ok) return 2;
  const double rv[3] = {r.x, r.y, r.z}, ev[3] = {e.x, e.y, e.z};
  // the four parts of each component of r x e: p1 + q1 - p2 - q2
  double tp[3][4];
  double big = 0.0;
  for (int c = 0; c < 3; ++c) {
    const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
    const double p1 = rv[c1] * ev[c2], q1 = fma(rv[c1], ev[c2], -p1);
    const double p2 = rv[c2] * ev[c1], q2 = fma(rv[c2], ev[c1], -p2);
    tp[c][0] = p1; tp[c][1] = q1; tp[c][2] = -p2; tp[c][3] = -q2;
    big = fmax(big, fmax(fabs(p1), fabs(p2)));
  }
  const double ee = ev[0] * ev[0] + ev[1] * ev[1] + ev[2] * ev[2];
  if (!(ee > 0.0)) return 2;
  const double top = fmax(big * big, fabs(T.hi) * ee * 2.0);
  if (!(top > 0.0) || !(top < 1e300)) return 2;
  int etop;
  frexp(top, &etop);
  FixAcc A{{0, 0, 0, 0}, etop + 8 - 248, true};  // bit 255: sign; headroom for 120 terms and rounding of top
  for (int c = 0; c < 3; ++c)
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) fix_prod(A, tp[c][a], tp[c][b], false);
  for (int c = 0; c < 3; ++c) {
    const double h = ev[c] * ev[c], l = fma(ev[c], ev[c], -h);  // e_c^2 = h + l exactly
    fix_prod(A, T.hi, h, true);
    fix_prod(A, T.hi, l, true);
    fix_prod(A, T.lo, h, true);
    fix_prod(A, T.lo, l, true);
  }
  if (!A.ok) return 2;
  if (A.w[3] >> 63) return -1;
  return (A.w[0] | A.w[1] | A.w[2] | A.w[3]) ? 1 : 0;
}

// pe_sign_fixed for sub-case `code` (point-edge only; 2 for the others).
BFC_GD int pe_sign_code(int code, const d3* P, dd T) {
  if (case_kind(code) != K_PE) return 2;
  int s0, s1, s2;
  case_slots(code, s0, s1, s2);
  return pe_sign_fixed(pick(P, s0), pick(P, s1), pick(P, s2), T);
}

// D (FP64 value of sub-case `code`) against an exact squared threshold given
// as a double-double T: lt -> d < thr, else d <= thr.  Outside a relative
// band of 1e-9 the FP64 value decides.  Inside it the formula is tried in
// FP64 with exactness checks (lattice geometry: exact ties at d_min or h),
// then in double-double; within 1e-20 of T, where double-double rounding
// could still flip the answer, a point-edge pair is decided in fixed point
// (pe_sign_fixed) when its difference vectors are exact in FP64, and
// otherwise *amb is set and the narrow phase defers the pair to k_exact
// (decide_sq_exact).  Without amb (the line-search and
// core-set kernels) the band is decided in double-double.
BFC_GD bool decide_sq(int code, const d3* P, double D, dd T, bool lt, bool* amb) {
  double Th = T.hi;
  if (fabs(D - Th) > 1e-9 * Th) return lt ? (D < Th) : (D <= Th);
  if (amb) {
    const int sg = exact_in_double(code, P, T);
    if (sg != 2) return lt ? sg < 0 : sg <= 0;
  }
  q3 Q[4] = {q3_of(P[0]), q3_of(P[1]), q3_of(P[2]), q3_of(P[3])};
  const dd Dq = sqd_case<dd>(code, Q);
  if (amb && !(fabs((Dq - T).hi) > 1e-20 * Th)) {  // point-edge in fixed point, else the expansions
    const int sg = pe_sign_code(code, P, T);
    if (sg != 2) return lt ? sg < 0 : sg <= 0;
    *amb = true;
  }
  return lt ? dd_lt(Dq, T) : dd_le(Dq, T);
}

// The same decision, exact (k_exact): FP64 outside the 1e-9 band; inside
// it, exact FP64 evaluation when no operation rounds, else double-double,
// and within 1e-20 of T, where double-double rounding could still flip the
// answer, the exact sign on expansions (xp_sign_sq_minus, slab ws).  *limit
// is set when the expansions outgrow their room (the double-double decision
// is kept).
BFC_GD bool decide_sq_exact(int code, const d3* P, double D, dd T, bool lt, double* ws,
                                                bool* limit) {
  double Th = T.hi;
  if (fabs(D - Th) > 1e-9 * Th) return lt ? (D < Th) : (D <= Th);
  int sg = exact_in_double(code, P, T);
  if (sg != 2) return lt ? sg < 0 : sg <= 0;
  q3 Q[4] = {q3_of(P[0]), q3_of(P[1]), q3_of(P[2]), q3_of(P[3])};
  const dd Dq = sqd_case<dd>(code, Q);
  const bool r = lt ? dd_lt(Dq, T) : dd_le(Dq, T);
  if (fabs((Dq - T).hi) > 1e-20 * Th) return r;
  sg = pe_sign_code(code, P, T);
  if (sg != 2) return lt ? sg < 0 : sg <= 0;
  sg = xp_sign_sq_minus(code, P[0], P[1], P[2], P[3], T, ws);
  if (sg == 2) {
    *limit = true;
    return r;
  }
  return lt ? sg < 0 : sg <= 0;
}

// ---------------------------------------------------------------------------
// Reference distance in 2D rest coordinates (shell filter, Sec. 3.2)
// ---------------------------------------------------------------------------
template <class T> struct V2 {
  T x, y;
};
template <class T> BFC_GD T seg2(V2<T> p, V2<T> a, V2<T> b) {
  T ex = b.x - a.x, ey = b.y - a.y, rx = p.x - a.x, ry = p.y - a.y;
  T ee = ex * ex + ey * ey, re = rx * ex + ry * ey;
  if (!(re > T(0))) return rx * rx + ry * ry;
  if (!(re < ee)) {
    T qx = p.x - b.x, qy = p.y - b.y;
    return qx * qx + qy * qy;
  }
  T c = rx * ey - ry * ex;
  return c * c / ee;
}
template <class T> BFC_GD T orient(V2<T> a, V2<T> b, V2<T> c) {
  return (b.x - a.x) * (c.y - a.y) - (b.y - a.y) * (c.x - a.x);
}

// ---------------------------------------------------------------------------
// Offset barrier (Eq. 2, Eq. 3): u = d - a, w = d - eta, L = ln(w/(a-eta)).
// b = -u^2 L, b' = -2uL - u^2/w, b'' = -2L - 4u/w + u^2/w^2.
// ---------------------------------------------------------------------------
template <class T> BFC_GD void barrier3(T d, T a, T eta, T& b, T& b1, T& b2) {
  T u = d - a, w = d - eta;
  T L = log1p(u / (a - eta));
  T uw = u / w;
  b = -u * u * L;
  b1 = -2 * u * L - u * uw;
  b2 = -2 * L - 4 * uw + uw * uw;
}

}  // namespace bfc
