// Plain CPU oracle for barrier-filtered contact evaluation of thickened rods
// and shells (Gomez-Nogales et al., "Unlocking Thickness Modeling for
// Codimensional Contact Simulation", Sec. 3 and App. A).
//
// TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
// benchmark's CPU-baseline leg may load this library.  It shares no code with
// the GPU library: it has its own geometry, its own classification, forward
// automatic differentiation instead of hand-derived derivatives, and its own
// eigen-solver.
//
// Everything is the plain definition, evaluated slowly:
//   * pair universe: every non-incident point-triangle and edge-edge pair
//     (rods: edge-edge only), across components too (Sec. 3, primitives and
//     stencil pairings);
//   * components and reference distances in parametric space, d_min per
//     connected component (Sec. 3.2; Sec. 1 says "parametric space, 1D for
//     rods and 2D for shells");
//   * per-pair barrier parameters of the double-filtered barrier (Eq. 4;
//     Eq. 1 when eta = 0);
//   * IPC log barrier with biphasic offset (Eq. 2, Eq. 3);
//   * energy gradient and Hessian by hyper-dual forward differentiation of
//     E(x) = kappa * b(sqrt(D(x)), a, eta);
//   * projection of each pair Hessian onto the PSD cone by clamping its
//     eigenvalues at zero (the projected Newton solver of App. A; the paper
//     does not spell out the projection, this is the reading used);
//   * decisions "d < a", "d <= eta" and "dbar < h" made in double precision
//     and, inside a relative guard band of 1e-9, re-made in binary128
//     (__float128) from the same formula, and within 1e-20 of the threshold
//     in exact integer arithmetic: every decision is that of the exact
//     distance of the double inputs;
//   * line search (Sec. 3.3, last paragraph; App. A): additive CCD (ACCD, Li
//     et al. 2021) per pair with the offset of Eq. 4 (eta for ordinary pairs,
//     0 for filtered stencils), over the pairs whose boxes swept from x to
//     x + p come within h.  The energy-only evaluation at a trial point is
//     orc_evaluate without derivatives;
//   * temporary zero offset (Sec. 3.4): non-stencil pairs found inside the
//     core (d <= eta) at a configuration get eta = 0 (activation h) until
//     they are seen with d > eta, then the ordinary (h, eta) again;
//   * lagged friction (App. A: IPC energies for contact and friction; the
//     lagged model of IPC, Li et al. 2020): per active pair, from the lagged
//     positions, the normal force kappa |b'(d)|, the closest-point weights and
//     the contact normal; the friction energy mu lambda f0(|tangential
//     relative displacement|) with IPC's smoothed Coulomb f0, differentiated
//     by hyper-dual sweeps.
//
// Build: g++ -O2 -std=c++17 -fopenmp -ffp-contract=off -shared -fPIC
//        oracle.cpp -o liboracle.so -lquadmath

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <unordered_set>
#include <vector>
#include <omp.h>
#include <quadmath.h>

typedef __float128 f128;


namespace {

// ---------------------------------------------------------------------------
// Small vector helpers, templated on the scalar type.
// ---------------------------------------------------------------------------
template <class S> inline void sub3(const S* a, const S* b, S* c) {
  c[0] = a[0] - b[0]; c[1] = a[1] - b[1]; c[2] = a[2] - b[2];
}
template <class S> inline S dot3(const S* a, const S* b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
template <class S> inline void cross3(const S* a, const S* b, S* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// ---------------------------------------------------------------------------
// Hyper-dual numbers a + b e1 + c e2 + d e1 e2 (e1^2 = e2^2 = 0): evaluating
// f at x + e1 u + e2 v gives f, f'.u, f'.v and u^T f'' v exactly (no step).
// ---------------------------------------------------------------------------
template <class T> struct HD {
  T a, b, c, d;
  HD() : a(0), b(0), c(0), d(0) {}
  HD(T v) : a(v), b(0), c(0), d(0) {}
  HD(T a_, T b_, T c_, T d_) : a(a_), b(b_), c(c_), d(d_) {}
};
template <class T> HD<T> operator+(HD<T> x, HD<T> y) { return HD<T>(x.a + y.a, x.b + y.b, x.c + y.c, x.d + y.d); }
template <class T> HD<T> operator-(HD<T> x, HD<T> y) { return HD<T>(x.a - y.a, x.b - y.b, x.c - y.c, x.d - y.d); }
template <class T> HD<T> operator-(HD<T> x) { return HD<T>(-x.a, -x.b, -x.c, -x.d); }
template <class T> HD<T> operator*(HD<T> x, HD<T> y) {
  return HD<T>(x.a * y.a, x.a * y.b + x.b * y.a, x.a * y.c + x.c * y.a,
               x.a * y.d + x.b * y.c + x.c * y.b + x.d * y.a);
}
// apply a scalar function with value f0, first derivative f1, second f2
template <class T> HD<T> chain(HD<T> x, T f0, T f1, T f2) {
  return HD<T>(f0, f1 * x.b, f1 * x.c, f1 * x.d + f2 * x.b * x.c);
}
template <class T> HD<T> inv(HD<T> x) {
  T i = T(1) / x.a;
  return chain(x, i, -i * i, T(2) * i * i * i);
}
template <class T> HD<T> operator/(HD<T> x, HD<T> y) { return x * inv(y); }

inline double sqrt_(double v) { return std::sqrt(v); }
inline f128 sqrt_(f128 v) { return sqrtq(v); }
inline double log1p_(double v) { return std::log1p(v); }
inline f128 log1p_(f128 v) { return log1pq(v); }

template <class T> HD<T> hsqrt(HD<T> x) {
  T s = sqrt_(x.a);
  return chain(x, s, T(0.5) / s, T(-0.25) / (s * x.a));
}
template <class T> HD<T> hlog1p(HD<T> x) {
  T o = T(1) + x.a;
  return chain(x, log1p_(x.a), T(1) / o, T(-1) / (o * o));
}

// ---------------------------------------------------------------------------
// Squared distance formulas of the four distance types.  Local vertex slots:
// point-triangle pair (p, t0, t1, t2); edge-edge pair (a0, a1, b0, b1).
// ---------------------------------------------------------------------------
template <class S> S D_pp(const S* p, const S* q) {
  S r[3]; sub3(p, q, r);
  return dot3(r, r);
}
// distance from p to the line through e0, e1: |(p - e0) x (e1 - e0)|^2 / |e1 - e0|^2
template <class S> S D_pe(const S* p, const S* e0, const S* e1) {
  S r[3], e[3], c[3];
  sub3(p, e0, r); sub3(e1, e0, e); cross3(r, e, c);
  return dot3(c, c) / dot3(e, e);
}
// distance from p to the plane of (t0, t1, t2): ((p - t0) . n)^2 / |n|^2
template <class S> S D_pt(const S* p, const S* t0, const S* t1, const S* t2) {
  S u[3], v[3], n[3], r[3];
  sub3(t1, t0, u); sub3(t2, t0, v); cross3(u, v, n); sub3(p, t0, r);
  S s = dot3(r, n);
  return s * s / dot3(n, n);
}
// distance between the lines (a0, a1) and (b0, b1): ((a0 - b0) . n)^2 / |n|^2
template <class S> S D_ee(const S* a0, const S* a1, const S* b0, const S* b1) {
  S u[3], v[3], n[3], r[3];
  sub3(a1, a0, u); sub3(b1, b0, v); cross3(u, v, n); sub3(a0, b0, r);
  S s = dot3(r, n);
  return s * s / dot3(n, n);
}

// Distance sub-case codes.  Each names the formula and the local slots used.
//   point-triangle: 0 PP(0,1) 1 PP(0,2) 2 PP(0,3) 3 PE(0;1,2) 4 PE(0;2,3) 5 PE(0;3,1) 6 PT
//   edge-edge:      7 PP(0,2) 8 PP(0,3) 9 PP(1,2) 10 PP(1,3)
//                   11 PE(0;2,3) 12 PE(1;2,3) 13 PE(2;0,1) 14 PE(3;0,1) 15 EE
struct Case { int kind; int s0, s1, s2, s3; };  // kind 0 PP, 1 PE, 2 PT, 3 EE
const Case kCases[16] = {
  {0, 0, 1, -1, -1}, {0, 0, 2, -1, -1}, {0, 0, 3, -1, -1},
  {1, 0, 1, 2, -1}, {1, 0, 2, 3, -1}, {1, 0, 3, 1, -1}, {2, 0, 1, 2, 3},
  {0, 0, 2, -1, -1}, {0, 0, 3, -1, -1}, {0, 1, 2, -1, -1}, {0, 1, 3, -1, -1},
  {1, 0, 2, 3, -1}, {1, 1, 2, 3, -1}, {1, 2, 0, 1, -1}, {1, 3, 0, 1, -1}, {3, 0, 1, 2, 3},
};

// ---------------------------------------------------------------------------
// Exact rationals (numerator and denominator as sign-magnitude integers with
// 32-bit limbs, schoolbook arithmetic, no reduction): the last resort of the
// threshold decisions.  Every double is an exact rational, so the same
// formulas evaluated on Rat give the exact value of the double inputs.
// ---------------------------------------------------------------------------
struct Big {
  bool neg = false;
  std::vector<uint32_t> m;  // magnitude, least significant limb first, no leading zero limbs
};
inline void trim(std::vector<uint32_t>& a) { while (!a.empty() && a.back() == 0) a.pop_back(); }
inline int cmp_mag(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b) {
  if (a.size() != b.size()) return a.size() < b.size() ? -1 : 1;
  for (size_t k = a.size(); k-- > 0;)
    if (a[k] != b[k]) return a[k] < b[k] ? -1 : 1;
  return 0;
}
inline std::vector<uint32_t> add_mag(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b) {
  std::vector<uint32_t> r(std::max(a.size(), b.size()) + 1, 0);
  uint64_t carry = 0;
  for (size_t k = 0; k < r.size(); ++k) {
    uint64_t t = carry + (k < a.size() ? a[k] : 0) + (k < b.size() ? b[k] : 0);
    r[k] = (uint32_t)t;
    carry = t >> 32;
  }
  trim(r);
  return r;
}
inline std::vector<uint32_t> sub_mag(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b) {  // a >= b
  std::vector<uint32_t> r(a.size(), 0);
  int64_t borrow = 0;
  for (size_t k = 0; k < a.size(); ++k) {
    int64_t t = (int64_t)a[k] - (k < b.size() ? b[k] : 0) - borrow;
    borrow = t < 0;
    r[k] = (uint32_t)(t + (borrow ? (int64_t)1 << 32 : 0));
  }
  trim(r);
  return r;
}
inline Big big_add(const Big& a, const Big& b) {
  Big r;
  if (a.neg == b.neg) {
    r.m = add_mag(a.m, b.m);
    r.neg = a.neg;
  } else if (cmp_mag(a.m, b.m) >= 0) {
    r.m = sub_mag(a.m, b.m);
    r.neg = a.neg;
  } else {
    r.m = sub_mag(b.m, a.m);
    r.neg = b.neg;
  }
  if (r.m.empty()) r.neg = false;
  return r;
}
inline Big big_neg(Big a) {
  if (!a.m.empty()) a.neg = !a.neg;
  return a;
}
inline Big big_mul(const Big& a, const Big& b) {
  Big r;
  if (a.m.empty() || b.m.empty()) return r;
  r.m.assign(a.m.size() + b.m.size(), 0);
  for (size_t i = 0; i < a.m.size(); ++i) {
    uint64_t carry = 0;
    for (size_t j = 0; j < b.m.size(); ++j) {
      uint64_t t = (uint64_t)a.m[i] * b.m[j] + r.m[i + j] + carry;
      r.m[i + j] = (uint32_t)t;
      carry = t >> 32;
    }
    r.m[i + b.m.size()] = (uint32_t)carry;
  }
  trim(r.m);
  r.neg = a.neg != b.neg;
  return r;
}
inline Big big_pow2(int k) {  // 2^k, k >= 0
  Big r;
  r.m.assign(k / 32 + 1, 0);
  r.m[k / 32] = 1u << (k % 32);
  return r;
}
inline Big big_u64(uint64_t v) {
  Big r;
  r.m = {(uint32_t)v, (uint32_t)(v >> 32)};
  trim(r.m);
  return r;
}
inline int big_sign(const Big& a) { return a.m.empty() ? 0 : (a.neg ? -1 : 1); }

struct Rat {
  Big n, d;  // value n / d, d > 0
  Rat() { d = big_u64(1); }
  Rat(int v) {  // small integers (the constants of the formulas)
    n = big_u64((uint64_t)(v < 0 ? -(int64_t)v : v));
    n.neg = v < 0 && !n.m.empty();
    d = big_u64(1);
  }
  explicit Rat(double v) {  // exact value of a finite double: M 2^e
    d = big_u64(1);
    if (v == 0.0) return;
    int E;
    const double f = std::frexp(std::fabs(v), &E);   // |v| = f 2^E, f in [0.5, 1)
    n = big_u64((uint64_t)std::ldexp(f, 53));         // |v| = n 2^(E - 53)
    const int e = E - 53;
    if (e >= 0) n = big_mul(n, big_pow2(e));
    else d = big_pow2(-e);
    n.neg = v < 0.0;
  }
};
inline Rat operator+(const Rat& a, const Rat& b) {
  Rat r;
  r.n = big_add(big_mul(a.n, b.d), big_mul(b.n, a.d));
  r.d = big_mul(a.d, b.d);
  return r;
}
inline Rat operator-(const Rat& a) {
  Rat r = a;
  r.n = big_neg(a.n);
  return r;
}
inline Rat operator-(const Rat& a, const Rat& b) { return a + (-b); }
inline Rat operator*(const Rat& a, const Rat& b) {
  Rat r;
  r.n = big_mul(a.n, b.n);
  r.d = big_mul(a.d, b.d);
  return r;
}
inline Rat operator/(const Rat& a, const Rat& b) {  // b != 0
  Rat r;
  r.n = big_mul(a.n, b.d);
  r.d = big_mul(a.d, b.n);
  if (r.d.neg) {
    r.d.neg = false;
    r.n = big_neg(r.n);
  }
  return r;
}
inline int rat_cmp(const Rat& a, const Rat& b) { return big_sign(big_add(big_mul(a.n, b.d), big_neg(big_mul(b.n, a.d)))); }
inline bool operator<(const Rat& a, const Rat& b) { return rat_cmp(a, b) < 0; }
inline bool operator>(const Rat& a, const Rat& b) { return rat_cmp(a, b) > 0; }
inline bool operator<=(const Rat& a, const Rat& b) { return rat_cmp(a, b) <= 0; }
inline bool operator>=(const Rat& a, const Rat& b) { return rat_cmp(a, b) >= 0; }
inline bool operator==(const Rat& a, const Rat& b) { return rat_cmp(a, b) == 0; }
inline bool operator<(const Rat& a, int b) { return a < Rat(b); }
inline bool operator>(const Rat& a, int b) { return a > Rat(b); }
inline bool operator<=(const Rat& a, int b) { return a <= Rat(b); }
inline bool operator>=(const Rat& a, int b) { return a >= Rat(b); }

// Squared distance of sub-case `code` evaluated on 4 local vertices X[12].
template <class S> S D_case(int code, const S* X) {
  const Case& c = kCases[code];
  switch (c.kind) {
    case 0: return D_pp(X + 3 * c.s0, X + 3 * c.s1);
    case 1: return D_pe(X + 3 * c.s0, X + 3 * c.s1, X + 3 * c.s2);
    case 2: return D_pt(X + 3 * c.s0, X + 3 * c.s1, X + 3 * c.s2, X + 3 * c.s3);
    default: return D_ee(X + 3 * c.s0, X + 3 * c.s1, X + 3 * c.s2, X + 3 * c.s3);
  }
}

// ---------------------------------------------------------------------------
// Classification: the unsigned distance between two primitives is the minimum
// over their features; the closest feature pair fixes the formula.  Ties keep
// the first candidate in the order listed.
// ---------------------------------------------------------------------------
struct Dist { double D; int code; };

// point p vs segment (e0, e1), with the sub-case codes to report for the
// vertex-vertex (at e0, at e1) and interior outcomes.
inline Dist point_segment(const double* p, const double* e0, const double* e1,
                          int code_pp0, int code_pp1, int code_pe) {
  double e[3], r[3];
  sub3(e1, e0, e); sub3(p, e0, r);
  double t = dot3(r, e) / dot3(e, e);
  if (t <= 0.0) return {D_pp(p, e0), code_pp0};
  if (t >= 1.0) return {D_pp(p, e1), code_pp1};
  return {D_pe(p, e0, e1), code_pe};
}

// A later candidate replaces the current one only when it is closer by more
// than a relative 1e-12: candidates that tie (up to rounding) keep the first
// listed, so the choice of formula at region boundaries (e.g. exactly
// parallel edges, where several point-segment sub-cases give the same
// distance) is fixed by the listing order.
inline void keep_min(Dist& best, Dist c) { if (c.D < best.D * (1.0 - 1e-12)) best = c; }

Dist classify_pt(const double* X) {
  const double *p = X, *t0 = X + 3, *t1 = X + 6, *t2 = X + 9;
  double u[3], v[3], n[3];
  sub3(t1, t0, u); sub3(t2, t0, v); cross3(u, v, n);
  // the projection of p lies strictly inside the triangle iff p is strictly on
  // the inner side of all three edge planes (edge x n . (p - edge start) > 0)
  const double* T[3] = {t0, t1, t2};
  bool inside = true;
  for (int k = 0; k < 3; ++k) {
    double e[3], w[3], en[3];
    sub3(T[(k + 1) % 3], T[k], e); sub3(p, T[k], w); cross3(n, e, en);
    if (!(dot3(en, w) > 0.0)) inside = false;
  }
  if (inside) return {D_pt(p, t0, t1, t2), 6};
  Dist best = point_segment(p, t0, t1, 0, 1, 3);
  keep_min(best, point_segment(p, t1, t2, 1, 2, 4));
  keep_min(best, point_segment(p, t2, t0, 2, 0, 5));
  return best;
}

// Edges closer to parallel than this (|ea x eb|^2 < tol |ea|^2 |eb|^2) use the
// four point-segment sub-cases; the distance they give differs from the exact
// segment distance by at most ~tol * L^2 / d, far below the parity tolerance.
const double kParallelTol = 1e-10;

Dist classify_ee(const double* X) {
  const double *a0 = X, *a1 = X + 3, *b0 = X + 6, *b1 = X + 9;
  double ea[3], eb[3], n[3], r[3];
  sub3(a1, a0, ea); sub3(b1, b0, eb); cross3(ea, eb, n); sub3(a0, b0, r);
  double A = dot3(ea, ea), B = dot3(ea, eb), C = dot3(eb, eb);
  double nn = dot3(n, n);
  if (!(nn < kParallelTol * A * C)) {
    double Dd = dot3(ea, r), Ee = dot3(eb, r);
    double den = A * C - B * B;
    double s = (B * Ee - C * Dd) / den;
    double t = (A * Ee - B * Dd) / den;
    if (s > 0.0 && s < 1.0 && t > 0.0 && t < 1.0) return {D_ee(a0, a1, b0, b1), 15};
  }
  Dist best = point_segment(a0, b0, b1, 7, 8, 11);
  keep_min(best, point_segment(a1, b0, b1, 9, 10, 12));
  keep_min(best, point_segment(b0, a0, a1, 7, 9, 13));
  keep_min(best, point_segment(b1, a0, a1, 8, 10, 14));
  return best;
}

inline Dist classify(int ptype, const double* X) { return ptype == 0 ? classify_pt(X) : classify_ee(X); }

// Decide D < T (lt=true) or D <= T (lt=false) for the exact squared distance
// of sub-case `code` at the double inputs X, where T is an exact squared
// threshold (Tq, with Td its double approximation).  Outside a 1e-9 relative
// band the double value D decides; inside it, the formula is re-evaluated in
// binary128 (relative error far below 1e-28 for the formulas at the edge
// angles they are used for); within 1e-20 of T, where that rounding could
// still flip the answer (exact ties of lattice geometry land there), the
// decision is taken in exact integer arithmetic.
bool decide(int code, const double* X, double D, double Td, f128 Tq, bool lt, bool* used_ext) {
  if (std::fabs(D - Td) > 1e-9 * Td) return lt ? (D < Td) : (D <= Td);
  if (used_ext) *used_ext = true;
  f128 Xq[12];
  for (int k = 0; k < 12; ++k) Xq[k] = (f128)X[k];
  f128 Dq = D_case<f128>(code, Xq);
  f128 gap = Dq - Tq;
  if (gap < 0) gap = -gap;
  if (gap > Tq * (f128)1e-20) return lt ? (Dq < Tq) : (Dq <= Tq);
  // exact: T is the square of a double, or a double (at most 106 bits: two doubles)
  const double Th = (double)Tq, Tl = (double)(Tq - (f128)Th);
  Rat Xr[12];
  for (int k = 0; k < 12; ++k) Xr[k] = Rat(X[k]);
  const int sg = rat_cmp(D_case<Rat>(code, Xr), Rat(Th) + Rat(Tl));
  return lt ? sg < 0 : sg <= 0;
}
inline f128 sq(double v) { return (f128)v * (f128)v; }  // exact square of a double

// ---------------------------------------------------------------------------
// Barrier (Eq. 2 with the offset of Eq. 3): b(d, a, eta) = -(d-a)^2 ln((d-eta)/(a-eta))
// for eta < d < a, 0 for d >= a.  ln((d-eta)/(a-eta)) = log1p((d-a)/(a-eta)).
// ---------------------------------------------------------------------------
template <class T> HD<T> barrier_hd(HD<T> d, T a, T eta) {
  HD<T> u = d - HD<T>(a);
  HD<T> L = hlog1p(u * HD<T>(T(1) / (a - eta)));
  return -(u * u) * L;
}

// E(x), grad and Hessian of kappa * b(sqrt(D_code(x))) by hyper-dual sweeps.
template <class T>
void energy_derivs(int code, const double* X, double a, double eta, double kappa,
                   double* E, double* G, double* H) {
  // Eq. 2: the barrier and its derivatives are zero for d >= a (this can
  // happen for pairs decided active on the exact squared threshold whose
  // rounded distance lands on or above a)
  if (!(std::sqrt(D_case<double>(code, X)) < a)) {
    *E = 0.0;
    for (int i = 0; i < 12; ++i) G[i] = 0.0;
    for (int i = 0; i < 144; ++i) H[i] = 0.0;
    return;
  }
  for (int i = 0; i < 12; ++i) {
    for (int j = i; j < 12; ++j) {
      HD<T> Xh[12];
      for (int k = 0; k < 12; ++k) Xh[k] = HD<T>((T)X[k]);
      Xh[i].b = T(1);
      Xh[j].c = T(1);
      HD<T> D = D_case<HD<T>>(code, Xh);
      HD<T> e = barrier_hd(hsqrt(D), (T)a, (T)eta) * HD<T>((T)kappa);
      if (i == 0 && j == 0) *E = (double)e.a;
      if (j == i) G[i] = (double)e.b;
      H[i * 12 + j] = (double)e.d;
      H[j * 12 + i] = (double)e.d;
    }
  }
}

// ---------------------------------------------------------------------------
// PSD projection: cyclic Jacobi eigen-decomposition of a symmetric n x n
// matrix, eigenvalues clamped at 0, H+ = Q max(L, 0) Q^T.
// ---------------------------------------------------------------------------
void jacobi_eig(int n, const double* Ain, double* evals, double* Q) {
  std::vector<double> A(Ain, Ain + n * n);
  for (int i = 0; i < n * n; ++i) Q[i] = 0.0;
  for (int i = 0; i < n; ++i) Q[i * n + i] = 1.0;
  double fro = 0.0;
  for (int i = 0; i < n * n; ++i) fro += A[i] * A[i];
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        if (i != j) off += A[i * n + j] * A[i * n + j];
    if (off <= 1e-34 * fro || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p) {
      for (int q = p + 1; q < n; ++q) {
        double apq = A[p * n + q];
        if (apq == 0.0) continue;
        double app = A[p * n + p], aqq = A[q * n + q];
        // rotation angle that zeroes A[p][q] (Golub & Van Loan, sym. Schur 2x2)
        double tau = (aqq - app) / (2.0 * apq);
        double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < n; ++k) {  // A <- A J (columns p, q)
          double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // A <- J^T A (rows p, q)
          double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {  // Q <- Q J
          double qkp = Q[k * n + p], qkq = Q[k * n + q];
          Q[k * n + p] = c * qkp - s * qkq;
          Q[k * n + q] = s * qkp + c * qkq;
        }
      }
    }
  }
  for (int i = 0; i < n; ++i) evals[i] = A[i * n + i];
}

void psd_project(int n, const double* A, double* Ap, double* evals_out) {
  std::vector<double> ev(n), Q(n * n);
  jacobi_eig(n, A, ev.data(), Q.data());
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int k = 0; k < n; ++k)
        if (ev[k] > 0.0) s += Q[i * n + k] * ev[k] * Q[j * n + k];
      Ap[i * n + j] = s;
    }
  // exact symmetry
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      double m = 0.5 * (Ap[i * n + j] + Ap[j * n + i]);
      Ap[i * n + j] = m; Ap[j * n + i] = m;
    }
  if (evals_out)
    for (int i = 0; i < n; ++i) evals_out[i] = ev[i];
}

// ---------------------------------------------------------------------------
// Mesh-side data: components and reference distances (Sec. 3.2).
// ---------------------------------------------------------------------------
int find_root(std::vector<int>& par, int v) {
  while (par[v] != v) { par[v] = par[par[v]]; v = par[v]; }
  return v;
}

// Components numbered in order of their smallest vertex index.
int components(int64_t nv, int64_t ne, const int32_t* edges, const int32_t* tris, int64_t nt,
               int32_t* comp) {
  std::vector<int> par(nv);
  for (int64_t v = 0; v < nv; ++v) par[v] = (int)v;
  auto unite = [&](int a, int b) {
    a = find_root(par, a); b = find_root(par, b);
    if (a != b) par[std::max(a, b)] = std::min(a, b);
  };
  for (int64_t e = 0; e < ne; ++e) unite(edges[2 * e], edges[2 * e + 1]);
  for (int64_t t = 0; t < nt; ++t) { unite(tris[3 * t], tris[3 * t + 1]); unite(tris[3 * t], tris[3 * t + 2]); }
  std::vector<int> label(nv, -1);
  int nc = 0;
  for (int64_t v = 0; v < nv; ++v) {
    int r = find_root(par, (int)v);
    if (label[r] < 0) label[r] = nc++;
    comp[v] = label[r];
  }
  return nc;
}

// 2D squared distance from point p to segment (e0, e1).
template <class S> S seg_dist2_2d(const S* p, const S* e0, const S* e1) {
  S ex = e1[0] - e0[0], ey = e1[1] - e0[1];
  S rx = p[0] - e0[0], ry = p[1] - e0[1];
  S ee = ex * ex + ey * ey;
  S t = rx * ex + ry * ey;
  if (t <= 0) return rx * rx + ry * ry;
  if (t >= ee) { S qx = p[0] - e1[0], qy = p[1] - e1[1]; return qx * qx + qy * qy; }
  S c = rx * ey - ry * ex;
  return c * c / ee;
}
template <class S> S orient2(const S* a, const S* b, const S* c) {
  return (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]);
}

struct Mesh {
  int kind;  // 0 rod, 1 shell
  int64_t nv, ne, nt;
  const int32_t* edges;
  const int32_t* tris;
  const double* ref;
  double h, eta, kappa;
  int filter_mode;  // 0 paper (Eq. 4), 1 none (plain offset barrier everywhere), 2 cull (rods)
  // reference distance: 0 parametric (rest-space parameters), 1 Euclidean
  // distance between the primitives at the rest pose xrest [V,3]
  int refdist;
  const double* xrest;
  int cull_radius;  // mode 2: edges of one polyline at most this many elements apart are ignored
  std::vector<int> edge_pos;   // mode 2: index of each edge along its polyline
  std::vector<int> loop_len;   // mode 2: edge count of the edge's polyline if it is closed, else 0
  std::vector<int32_t> comp;
  std::vector<double> dmin2, dmin;  // per component; +inf when nothing is filtered
  // exact squared activation threshold of filtered pairs per component: the
  // canonical d_min^2 (shells) or the exact square of the minimum gap (rods)
  std::vector<f128> thr2;
  // pairs under the temporary zero offset of Sec. 3.4 (not yet released)
  std::unordered_set<uint64_t> core;
};

inline uint64_t pair_key(int ptype, int i, int j) {
  return ((uint64_t)ptype << 62) | ((uint64_t)(uint32_t)i << 31) | (uint64_t)(uint32_t)j;
}

// Reference (parametric-space) distance of a pair, as the value that the
// filter compares with h.  Rods: 1D gap between the two edges' arc-length
// intervals, one double subtraction.  Shells: squared 2D distance in rest
// coordinates (evaluated in scalar type S).  Returns false for pairs in
// different components (never stencils).  For rods *q holds dbar, for shells
// dbar^2.
template <class S>
bool ref_dist(const Mesh& m, int ptype, int i, int j, S* q, double* dbar_rod) {
  if (m.kind == 0) {
    const int32_t* ea = m.edges + 2 * i; const int32_t* eb = m.edges + 2 * j;
    if (m.comp[ea[0]] != m.comp[eb[0]]) return false;
    double sa0 = m.ref[ea[0]], sa1 = m.ref[ea[1]], sb0 = m.ref[eb[0]], sb1 = m.ref[eb[1]];
    double loa = std::min(sa0, sa1), hia = std::max(sa0, sa1);
    double lob = std::min(sb0, sb1), hib = std::max(sb0, sb1);
    double g = std::max(lob - hia, loa - hib);
    *dbar_rod = g;
    *q = (S)g;
    return true;
  }
  auto U = [&](int v, S* o) { o[0] = (S)m.ref[2 * v]; o[1] = (S)m.ref[2 * v + 1]; };
  if (ptype == 0) {
    int v = i; const int32_t* t = m.tris + 3 * j;
    if (m.comp[v] != m.comp[t[0]]) return false;
    S p[2], a[2], b[2], c[2];
    U(v, p); U(t[0], a); U(t[1], b); U(t[2], c);
    S o1 = orient2(a, b, p), o2 = orient2(b, c, p), o3 = orient2(c, a, p);
    bool in = (o1 >= 0 && o2 >= 0 && o3 >= 0) || (o1 <= 0 && o2 <= 0 && o3 <= 0);
    if (in) { *q = 0; return true; }
    S d = seg_dist2_2d(p, a, b);
    d = std::min(d, seg_dist2_2d(p, b, c));
    d = std::min(d, seg_dist2_2d(p, c, a));
    *q = d;
    return true;
  }
  const int32_t* ea = m.edges + 2 * i; const int32_t* eb = m.edges + 2 * j;
  if (m.comp[ea[0]] != m.comp[eb[0]]) return false;
  S a0[2], a1[2], b0[2], b1[2];
  U(ea[0], a0); U(ea[1], a1); U(eb[0], b0); U(eb[1], b1);
  S o1 = orient2(a0, a1, b0), o2 = orient2(a0, a1, b1);
  S o3 = orient2(b0, b1, a0), o4 = orient2(b0, b1, a1);
  if (((o1 > 0 && o2 < 0) || (o1 < 0 && o2 > 0)) && ((o3 > 0 && o4 < 0) || (o3 < 0 && o4 > 0))) {
    *q = 0; return true;
  }
  S d = seg_dist2_2d(a0, b0, b1);
  d = std::min(d, seg_dist2_2d(a1, b0, b1));
  d = std::min(d, seg_dist2_2d(b0, a0, a1));
  d = std::min(d, seg_dist2_2d(b1, a0, a1));
  *q = d;
  return true;
}

// Is the pair in the stencil set with reference distance below h (filtered)?
// Shells: decided on dbar^2 in double outside a 1e-9 relative band around
// h^2 (and away from 0), in binary128 inside it, exactly within 1e-20 of h^2.
bool is_filtered_euclid(const Mesh& m, int ptype, int i, int j);
bool is_filtered(const Mesh& m, int ptype, int i, int j) {
  if (m.filter_mode != 0) return false;
  if (m.refdist == 1) return is_filtered_euclid(m, ptype, i, j);
  double g;
  if (m.kind == 0) {
    double q;
    if (!ref_dist<double>(m, ptype, i, j, &q, &g)) return false;
    return g > 0.0 && g < m.h;
  }
  double qd;
  if (!ref_dist<double>(m, ptype, i, j, &qd, &g)) return false;
  double h2 = m.h * m.h;
  if (std::fabs(qd - h2) > 1e-9 * h2 && qd > 1e-9 * h2) return qd < h2;
  f128 q;
  ref_dist<f128>(m, ptype, i, j, &q, &g);
  f128 hq = (f128)m.h * (f128)m.h;
  // binary128 is exact for every branch test and for zero (differences and
  // 2D cross products of doubles fit its mantissa); only the division c^2/ee
  // rounds, which matters within 1e-20 of h^2: decide that band exactly
  f128 gap = q - hq;
  if (gap < 0) gap = -gap;
  if (gap > hq * (f128)1e-20) return q > 0 && q < hq;
  Rat qr;
  ref_dist<Rat>(m, ptype, i, j, &qr, &g);
  return qr > 0 && qr < Rat(m.h) * Rat(m.h);
}

// Culling comparison mode (Kaldor et al.): two edges of the same polyline
// whose positions along it differ by at most the radius (the shorter way
// round a closed loop) are not contact pairs.
bool is_culled(const Mesh& m, int ptype, int i, int j) {
  if (m.filter_mode != 2 || ptype != 1) return false;
  if (m.comp[m.edges[2 * i]] != m.comp[m.edges[2 * j]]) return false;
  int d = std::abs(m.edge_pos[i] - m.edge_pos[j]);
  if (m.loop_len[i] > 0) d = std::min(d, m.loop_len[i] - d);
  return d <= m.cull_radius;
}

// Positions of the edges along each polyline: walk every open polyline from
// its lower-numbered end, then every closed loop from its smallest vertex.
void order_polylines(Mesh& m) {
  std::vector<std::vector<int>> inc(m.nv);
  for (int64_t e = 0; e < m.ne; ++e) {
    inc[m.edges[2 * e]].push_back((int)e);
    inc[m.edges[2 * e + 1]].push_back((int)e);
  }
  m.edge_pos.assign(m.ne, -1);
  m.loop_len.assign(m.ne, 0);
  auto walk = [&](int v) {
    std::vector<int> seq;
    int prev = -1;
    for (;;) {
      int next = -1;
      for (int e : inc[v])
        if (e != prev && m.edge_pos[e] < 0) { next = e; break; }
      if (next < 0) break;
      m.edge_pos[next] = (int)seq.size();
      seq.push_back(next);
      v = m.edges[2 * next] == v ? m.edges[2 * next + 1] : m.edges[2 * next];
      prev = next;
    }
    return seq;
  };
  for (int64_t v = 0; v < m.nv; ++v)
    if (inc[v].size() == 1 && m.edge_pos[inc[v][0]] < 0) walk((int)v);
  for (int64_t v = 0; v < m.nv; ++v)
    if (inc[v].size() == 2 && m.edge_pos[inc[v][0]] < 0) {
      std::vector<int> seq = walk((int)v);
      for (int e : seq) m.loop_len[e] = (int)seq.size();
    }
}

// Incident pairs share a vertex and are not in the pair universe.
bool incident(const Mesh& m, int ptype, int i, int j) {
  if (ptype == 0) {
    const int32_t* t = m.tris + 3 * j;
    return i == t[0] || i == t[1] || i == t[2];
  }
  const int32_t* a = m.edges + 2 * i; const int32_t* b = m.edges + 2 * j;
  return a[0] == b[0] || a[0] == b[1] || a[1] == b[0] || a[1] == b[1];
}

// d_min per component: the minimum reference distance over the stencil pairs
// with 0 < dbar < h (Sec. 3.2).  Shells: the binary128 minimum of dbar^2,
// rounded once to double; d_min = sqrt of that double.  Rods: the minimum
// gap itself, and d_min2 its square rounded to double.  Components with no
// stencil pair closer than h are not filtered (d_min = +inf, unused).
// Stencil pairs are enumerated with a conservative sweep over the reference
// bounding boxes (pairs whose boxes are h apart cannot have dbar < h).
void compute_dmin(Mesh& m, int nc) {
  m.dmin2.assign(nc, std::numeric_limits<double>::infinity());
  m.dmin.assign(nc, std::numeric_limits<double>::infinity());
  int T = omp_get_max_threads();
  std::vector<std::vector<f128>> best(T, std::vector<f128>(nc, (f128)INFINITY));
  std::vector<std::vector<double>> best_rod(T, std::vector<double>(nc, std::numeric_limits<double>::infinity()));
  struct Box { double lo0, hi0, lo1, hi1; int id; };
  double rmax = 0.0;
  for (int64_t k = 0; k < (m.kind == 0 ? m.nv : 2 * m.nv); ++k) rmax = std::max(rmax, std::fabs(m.ref[k]));
  const double lim = m.h * (1.0 + 1e-12) + 1e-14 * rmax;
  auto R0 = [&](int v) { return m.kind == 0 ? m.ref[v] : m.ref[2 * v]; };
  auto R1 = [&](int v) { return m.kind == 0 ? 0.0 : m.ref[2 * v + 1]; };
  auto make_box = [&](const int32_t* vs, int n, int id) {
    Box b{INFINITY, -INFINITY, INFINITY, -INFINITY, id};
    for (int k = 0; k < n; ++k) {
      b.lo0 = std::min(b.lo0, R0(vs[k])); b.hi0 = std::max(b.hi0, R0(vs[k]));
      b.lo1 = std::min(b.lo1, R1(vs[k])); b.hi1 = std::max(b.hi1, R1(vs[k]));
    }
    return b;
  };
  auto gap_ok = [&](const Box& a, const Box& b) {
    return std::max(b.lo0 - a.hi0, a.lo0 - b.hi0) < lim && std::max(b.lo1 - a.hi1, a.lo1 - b.hi1) < lim;
  };
  auto by_lo0 = [](const Box& a, const Box& b) { return a.lo0 < b.lo0 || (a.lo0 == b.lo0 && a.id < b.id); };
  auto consider = [&](int ptype, int i, int j) {
    if (incident(m, ptype, i, j)) return;
    f128 q; double g;
    if (!ref_dist<f128>(m, ptype, i, j, &q, &g)) return;
    int t = omp_get_thread_num();
    int c = ptype == 0 ? m.comp[i] : m.comp[m.edges[2 * i]];
    if (m.kind == 0) {
      if (g > 0.0 && g < m.h && g < best_rod[t][c]) best_rod[t][c] = g;
    } else {
      f128 hq = (f128)m.h * (f128)m.h;
      if (q > 0 && q < hq && q < best[t][c]) best[t][c] = q;
    }
  };
  std::vector<Box> eb(m.ne);
  for (int64_t e = 0; e < m.ne; ++e) eb[e] = make_box(m.edges + 2 * e, 2, (int)e);
  std::sort(eb.begin(), eb.end(), by_lo0);
  #pragma omp parallel for schedule(dynamic, 64)
  for (int64_t a = 0; a < (int64_t)eb.size(); ++a)
    for (size_t b = a + 1; b < eb.size(); ++b) {
      if (eb[b].lo0 - eb[a].hi0 >= lim) break;
      if (!gap_ok(eb[a], eb[b])) continue;
      consider(1, std::min(eb[a].id, eb[b].id), std::max(eb[a].id, eb[b].id));
    }
  if (m.kind == 1) {
    std::vector<Box> tb(m.nt);
    for (int64_t t = 0; t < m.nt; ++t) tb[t] = make_box(m.tris + 3 * t, 3, (int)t);
    std::sort(tb.begin(), tb.end(), by_lo0);
    double wmax = 0.0;
    for (const Box& b : tb) wmax = std::max(wmax, b.hi0 - b.lo0);
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t v = 0; v < m.nv; ++v) {
      int32_t vv = (int32_t)v;
      Box P = make_box(&vv, 1, (int)v);
      size_t l = std::lower_bound(tb.begin(), tb.end(), P.lo0 - lim - wmax,
                                  [](const Box& b, double val) { return b.lo0 < val; }) - tb.begin();
      for (; l < tb.size(); ++l) {
        if (tb[l].lo0 - P.hi0 >= lim) break;
        if (!gap_ok(P, tb[l])) continue;
        consider(0, (int)v, tb[l].id);
      }
    }
  }
  m.thr2.assign(nc, (f128)INFINITY);
  for (int c = 0; c < nc; ++c) {
    if (m.kind == 0) {
      double g = std::numeric_limits<double>::infinity();
      for (int t = 0; t < T; ++t) g = std::min(g, best_rod[t][c]);
      if (g < INFINITY) { m.dmin[c] = g; m.dmin2[c] = g * g; m.thr2[c] = sq(g); }
    } else {
      f128 q = (f128)INFINITY;
      for (int t = 0; t < T; ++t) q = std::min(q, best[t][c]);
      if (q < (f128)INFINITY) {
        m.dmin2[c] = (double)q;
        m.dmin[c] = std::sqrt(m.dmin2[c]);
        m.thr2[c] = (f128)m.dmin2[c];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Per-pair record.
// ---------------------------------------------------------------------------
enum { F_FILTERED = 1, F_ACTIVE = 2, F_INFEASIBLE = 4, F_EXTENDED = 8, F_CORE = 16 };

struct Deriv {
  double G[12];
  double Hraw[144];
  double Hpsd[144];
};

struct Rec {
  int ptype, i, j;
  int verts[4];
  int code, flags;
  double d, a, eta;
  double E;
  Deriv* der;  // only for active, feasible pairs evaluated with derivatives
};

void gather(const Mesh& m, const double* x, int ptype, int i, int j, int* verts, double* X) {
  if (ptype == 0) {
    verts[0] = i;
    verts[1] = m.tris[3 * j]; verts[2] = m.tris[3 * j + 1]; verts[3] = m.tris[3 * j + 2];
  } else {
    verts[0] = m.edges[2 * i]; verts[1] = m.edges[2 * i + 1];
    verts[2] = m.edges[2 * j]; verts[3] = m.edges[2 * j + 1];
  }
  for (int k = 0; k < 4; ++k)
    for (int c = 0; c < 3; ++c) X[3 * k + c] = x[3 * verts[k] + c];
}

// The literal reading of the reference distance (Eq. 1 with dbar measured on
// the rest pose): dbar = the Euclidean distance between the two primitives at
// the rest positions xrest, the same distance function as d(x).  A stencil
// pair (same component, not incident) is filtered iff 0 < dbar < h; the
// comparison with h is the exact decision used for d(x) < h, and dbar > 0 is
// read on the double value (rest poses whose non-incident primitives touch
// are outside the model).
bool is_filtered_euclid(const Mesh& m, int ptype, int i, int j) {
  const int ca = ptype == 0 ? m.comp[i] : m.comp[m.edges[2 * i]];
  const int cb = ptype == 0 ? m.comp[m.tris[3 * j]] : m.comp[m.edges[2 * j]];
  if (ca != cb) return false;
  int verts[4];
  double X[12];
  gather(m, m.xrest, ptype, i, j, verts, X);
  const Dist ds = classify(ptype, X);
  if (!(ds.D > 0.0)) return false;
  return decide(ds.code, X, ds.D, m.h * m.h, sq(m.h), true, nullptr);
}

// d_min per component under the Euclidean reading: the binary128 minimum of
// dbar^2 over the filtered stencil pairs (0 < dbar < h), rounded once to
// double, found by a sweep over the rest-pose bounding boxes (boxes h or more
// apart on some axis hold no pair with dbar < h).
void compute_dmin_euclid(Mesh& m, int nc) {
  m.dmin2.assign(nc, std::numeric_limits<double>::infinity());
  m.dmin.assign(nc, std::numeric_limits<double>::infinity());
  m.thr2.assign(nc, (f128)INFINITY);
  struct Box { double lo[3], hi[3]; int id; };
  double rmax = 0.0;
  for (int64_t k = 0; k < 3 * m.nv; ++k) rmax = std::max(rmax, std::fabs(m.xrest[k]));
  const double lim = m.h * (1.0 + 1e-12) + 1e-14 * rmax;
  auto make_box = [&](const int32_t* vs, int n, int id) {
    Box b;
    for (int a = 0; a < 3; ++a) { b.lo[a] = INFINITY; b.hi[a] = -INFINITY; }
    b.id = id;
    for (int k = 0; k < n; ++k)
      for (int a = 0; a < 3; ++a) {
        b.lo[a] = std::min(b.lo[a], m.xrest[3 * vs[k] + a]);
        b.hi[a] = std::max(b.hi[a], m.xrest[3 * vs[k] + a]);
      }
    return b;
  };
  auto near = [&](const Box& a, const Box& b) {
    for (int k = 0; k < 3; ++k)
      if (!(std::max(b.lo[k] - a.hi[k], a.lo[k] - b.hi[k]) < lim)) return false;
    return true;
  };
  auto by_lo = [](const Box& a, const Box& b) { return a.lo[0] < b.lo[0] || (a.lo[0] == b.lo[0] && a.id < b.id); };
  int T = omp_get_max_threads();
  std::vector<std::vector<f128>> best(T, std::vector<f128>(nc, (f128)INFINITY));
  auto consider = [&](int ptype, int i, int j) {
    if (incident(m, ptype, i, j) || !is_filtered_euclid(m, ptype, i, j)) return;
    int verts[4];
    double X[12];
    gather(m, m.xrest, ptype, i, j, verts, X);
    const Dist ds = classify(ptype, X);
    f128 Xq[12];
    for (int k = 0; k < 12; ++k) Xq[k] = (f128)X[k];
    const f128 q = D_case<f128>(ds.code, Xq);
    const int c = ptype == 0 ? m.comp[i] : m.comp[m.edges[2 * i]];
    const int t = omp_get_thread_num();
    if (q < best[t][c]) best[t][c] = q;
  };
  std::vector<Box> eb(m.ne);
  for (int64_t e = 0; e < m.ne; ++e) eb[e] = make_box(m.edges + 2 * e, 2, (int)e);
  std::sort(eb.begin(), eb.end(), by_lo);
  #pragma omp parallel for schedule(dynamic, 64)
  for (int64_t a = 0; a < (int64_t)eb.size(); ++a)
    for (size_t b = a + 1; b < eb.size(); ++b) {
      if (eb[b].lo[0] - eb[a].hi[0] >= lim) break;
      if (!near(eb[a], eb[b])) continue;
      consider(1, std::min(eb[a].id, eb[b].id), std::max(eb[a].id, eb[b].id));
    }
  if (m.kind == 1) {
    std::vector<Box> tb(m.nt);
    for (int64_t t = 0; t < m.nt; ++t) tb[t] = make_box(m.tris + 3 * t, 3, (int)t);
    std::sort(tb.begin(), tb.end(), by_lo);
    double wmax = 0.0;
    for (const Box& b : tb) wmax = std::max(wmax, b.hi[0] - b.lo[0]);
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t v = 0; v < m.nv; ++v) {
      int32_t vv = (int32_t)v;
      Box P = make_box(&vv, 1, (int)v);
      size_t l = std::lower_bound(tb.begin(), tb.end(), P.lo[0] - lim - wmax,
                                  [](const Box& b, double val) { return b.lo[0] < val; }) - tb.begin();
      for (; l < tb.size(); ++l) {
        if (tb[l].lo[0] - P.hi[0] >= lim) break;
        if (!near(P, tb[l])) continue;
        consider(0, (int)v, tb[l].id);
      }
    }
  }
  for (int c = 0; c < nc; ++c) {
    f128 q = (f128)INFINITY;
    for (int t = 0; t < T; ++t) q = std::min(q, best[t][c]);
    if (q < (f128)INFINITY) {
      m.dmin2[c] = (double)q;
      m.dmin[c] = std::sqrt(m.dmin2[c]);
      m.thr2[c] = (f128)m.dmin2[c];
    }
  }
}

// Evaluate one pair of the universe; returns false if d >= h (not a contact
// candidate at the full activation distance).
bool eval_pair(const Mesh& m, const double* x, int ptype, int i, int j, bool derivs, Rec& r) {
  if (is_culled(m, ptype, i, j)) return false;  // culling mode: not a contact pair
  double X[12];
  gather(m, x, ptype, i, j, r.verts, X);
  Dist ds = classify(ptype, X);
  bool ext = false;
  // contact candidate at the full activation distance: d < h
  if (!decide(ds.code, X, ds.D, m.h * m.h, sq(m.h), true, &ext)) return false;
  r.ptype = ptype; r.i = i; r.j = j; r.code = ds.code;
  r.d = std::sqrt(ds.D);
  r.flags = 0;
  bool filt = is_filtered(m, ptype, i, j);
  // Sec. 3.4: a non-stencil pair initialised inside the core keeps a zero
  // offset (activation h) until it is released
  bool core = !filt && !m.core.empty() && m.core.count(pair_key(ptype, i, j)) != 0;
  int c = ptype == 0 ? m.comp[i] : m.comp[m.edges[2 * i]];
  double Td; f128 Tq;
  if (filt) {  // Eq. 4, second case: activation d_min, no offset
    r.a = m.dmin[c]; r.eta = 0.0; r.flags |= F_FILTERED;
    Tq = m.thr2[c]; Td = (double)Tq;
  } else {     // Eq. 4, first case: activation h, offset eta (0 while in the core set)
    r.a = m.h; r.eta = core ? 0.0 : m.eta;
    if (core) r.flags |= F_CORE;
    Tq = sq(m.h); Td = m.h * m.h;
  }
  // Eq. 2: active iff d < a; Eq. 3: the barrier diverges at d = eta
  bool active = decide(ds.code, X, ds.D, Td, Tq, true, &ext);
  bool infeas = false;
  if (active) infeas = r.eta > 0.0 ? decide(ds.code, X, ds.D, r.eta * r.eta, sq(r.eta), false, &ext) : !(ds.D > 0.0);
  if (active) r.flags |= F_ACTIVE;
  if (infeas) r.flags |= F_INFEASIBLE;
  if (ext) r.flags |= F_EXTENDED;
  r.E = 0.0;
  r.der = nullptr;
  if (active && infeas) { r.E = std::numeric_limits<double>::infinity(); return true; }
  if (active && derivs) {
    // near-parallel edge-edge interior: differentiate in binary128
    bool hi = false;
    if (kCases[ds.code].kind == 3) {
      double ea[3], eb[3], n[3];
      sub3(X + 3, X, ea); sub3(X + 9, X + 6, eb); cross3(ea, eb, n);
      hi = dot3(n, n) < 1e-4 * dot3(ea, ea) * dot3(eb, eb);
    }
    r.der = new Deriv;
    if (hi) energy_derivs<f128>(ds.code, X, r.a, r.eta, m.kappa, &r.E, r.der->G, r.der->Hraw);
    else energy_derivs<double>(ds.code, X, r.a, r.eta, m.kappa, &r.E, r.der->G, r.der->Hraw);
    psd_project(12, r.der->Hraw, r.der->Hpsd, nullptr);
  } else if (active) {
    HD<double> dd(r.d);
    r.E = r.d < r.a ? m.kappa * barrier_hd(dd, r.a, r.eta).a : 0.0;
  }
  return true;
}

struct Result {
  std::vector<Rec> recs;
  ~Result() { for (Rec& r : recs) delete r.der; }
};

void prim_box(const Mesh& m, const double* x, int role, int id, double* lo, double* hi) {
  int vs[3]; int nvs;
  if (role == 0) { vs[0] = id; nvs = 1; }
  else if (role == 1) { vs[0] = m.edges[2 * id]; vs[1] = m.edges[2 * id + 1]; nvs = 2; }
  else { vs[0] = m.tris[3 * id]; vs[1] = m.tris[3 * id + 1]; vs[2] = m.tris[3 * id + 2]; nvs = 3; }
  for (int c = 0; c < 3; ++c) { lo[c] = INFINITY; hi[c] = -INFINITY; }
  for (int k = 0; k < nvs; ++k)
    for (int c = 0; c < 3; ++c) {
      lo[c] = std::min(lo[c], x[3 * vs[k] + c]);
      hi[c] = std::max(hi[c], x[3 * vs[k] + c]);
    }
}

// ---------------------------------------------------------------------------
// Line search: additive CCD with the filtered offsets.
//
// ACCD (Li, Kaufman and Jiang 2021, "Codimensional Incremental Potential
// Contact", additive CCD) advances the stencil along its displacement in
// steps that cannot close more than a fixed fraction of the remaining gap
// d - xi: the distance between the two primitives shrinks at most at the rate
// lp (the largest displacement on one side plus the largest on the other,
// after removing the stencil's mean displacement, which does not change any
// distance).  The first step closes (1 - s) of the gap, every later one 0.9
// of the current gap; the search stops before the step after which the gap
// fell below s times the initial gap, or when the accumulated step passes the
// full step 1.  The gap is written (D - xi^2) / (sqrt(D) + xi) (no
// cancellation when xi is close to d).
// ---------------------------------------------------------------------------
inline double accd_gap(double D, double xi) { return (D - xi * xi) / (std::sqrt(D) + xi); }

double accd_pair(int ptype, const double* X0, const double* P0, double xi, double s, int max_iter, int* iters) {
  double X[12], P[12], pm[3] = {0.0, 0.0, 0.0};
  for (int v = 0; v < 4; ++v)
    for (int c = 0; c < 3; ++c) pm[c] += P0[3 * v + c];
  for (int c = 0; c < 3; ++c) pm[c] /= 4.0;
  for (int k = 0; k < 12; ++k) { X[k] = X0[k]; P[k] = P0[k] - pm[k % 3]; }
  double nrm[4];
  for (int v = 0; v < 4; ++v) nrm[v] = std::sqrt(dot3(P + 3 * v, P + 3 * v));
  // point-triangle: the point against the triangle's vertices; edge-edge: one
  // edge's endpoints against the other's
  const double lp = ptype == 0 ? nrm[0] + std::max(nrm[1], std::max(nrm[2], nrm[3]))
                               : std::max(nrm[0], nrm[1]) + std::max(nrm[2], nrm[3]);
  *iters = 0;
  if (lp == 0.0) return 1.0;
  const double gap0 = accd_gap(classify(ptype, X).D, xi);
  if (!(gap0 > 0.0)) return 0.0;  // already at or inside the offset: no step is safe
  const double g = s * gap0;
  double t = 0.0, tl = (1.0 - s) * gap0 / lp;
  for (int it = 0; it < max_iter; ++it) {
    *iters = it + 1;
    for (int k = 0; k < 12; ++k) X[k] = X[k] + tl * P[k];
    const double gap = accd_gap(classify(ptype, X).D, xi);
    if (t > 0.0 && gap < g) break;
    t += tl;
    if (t > 1.0) return 1.0;
    tl = 0.9 * gap / lp;
  }
  return t;
}

// Box of a primitive's vertices at x and at x + p (the straight-line sweep).
void swept_box(const Mesh& m, const double* x, const double* p, int role, int id, double* lo, double* hi) {
  int vs[3]; int nvs;
  if (role == 0) { vs[0] = id; nvs = 1; }
  else if (role == 1) { vs[0] = m.edges[2 * id]; vs[1] = m.edges[2 * id + 1]; nvs = 2; }
  else { vs[0] = m.tris[3 * id]; vs[1] = m.tris[3 * id + 1]; vs[2] = m.tris[3 * id + 2]; nvs = 3; }
  for (int c = 0; c < 3; ++c) { lo[c] = INFINITY; hi[c] = -INFINITY; }
  for (int k = 0; k < nvs; ++k)
    for (int c = 0; c < 3; ++c) {
      const double a = x[3 * vs[k] + c], b = a + p[3 * vs[k] + c];
      lo[c] = std::min(lo[c], std::min(a, b));
      hi[c] = std::max(hi[c], std::max(a, b));
    }
}

// ---------------------------------------------------------------------------
// Lagged friction.  The relative displacement of the two closest points of a
// pair is sum_s w[s] dX_s (first primitive minus second), with the weights of
// the distance sub-case at the lagged positions: PP (1, -1); PE the point
// against the edge point at parameter beta; PT the point against its
// projection's barycentric combination; EE the two line points at (alpha,
// beta).  Its tangential part (orthogonal to the lagged contact normal n)
// has length y, and the pair's friction energy is mu lambda f0(y) with
// f0(y) = y for y >= eh and -y^3/(3 eh^2) + y^2/eh + eh/3 below (eh: the
// sliding threshold eps_v times the time step).
// ---------------------------------------------------------------------------
void closest_weights(int code, const double* X, double* w) {
  for (int s = 0; s < 4; ++s) w[s] = 0.0;
  const Case& c = kCases[code];
  if (c.kind == 0) {
    w[c.s0] = 1.0; w[c.s1] = -1.0;
  } else if (c.kind == 1) {
    double e[3], r[3];
    sub3(X + 3 * c.s2, X + 3 * c.s1, e); sub3(X + 3 * c.s0, X + 3 * c.s1, r);
    const double beta = dot3(r, e) / dot3(e, e);
    w[c.s0] = 1.0; w[c.s1] = -(1.0 - beta); w[c.s2] = -beta;
  } else if (c.kind == 2) {
    double u[3], v[3], r[3];
    sub3(X + 6, X + 3, u); sub3(X + 9, X + 3, v); sub3(X, X + 3, r);
    const double uu = dot3(u, u), uv = dot3(u, v), vv = dot3(v, v), ru = dot3(r, u), rv = dot3(r, v);
    const double det = uu * vv - uv * uv;
    const double b1 = (vv * ru - uv * rv) / det, b2 = (uu * rv - uv * ru) / det;
    w[0] = 1.0; w[1] = -(1.0 - b1 - b2); w[2] = -b1; w[3] = -b2;
  } else {
    // in binary128: for nearly parallel edges the 2 x 2 system loses about
    // log10(1 / sin^2) digits, more than double precision can spare
    f128 Q[12], ea[3], eb[3], r[3];
    for (int k = 0; k < 12; ++k) Q[k] = (f128)X[k];
    sub3(Q + 3, Q, ea); sub3(Q + 9, Q + 6, eb); sub3(Q, Q + 6, r);
    const f128 A = dot3(ea, ea), B = dot3(ea, eb), C = dot3(eb, eb), D = dot3(ea, r), E = dot3(eb, r);
    const f128 den = A * C - B * B;
    const f128 al = (B * E - C * D) / den, be = (A * E - B * D) / den;
    w[0] = (double)(1 - al); w[1] = (double)al; w[2] = (double)(-(1 - be)); w[3] = (double)(-be);
  }
}

template <class T> HD<T> f0_hd(HD<T> y, T eh) {
  if (y.a >= eh) return y;
  return -(y * y * y) * HD<T>(T(1) / (T(3) * eh * eh)) + y * y * HD<T>(T(1) / eh) + HD<T>(eh / T(3));
}

// mu lambda f0(|tangential part of sum_s w_s (X_s - Xlag_s)|) in scalar type T
template <class T> HD<T> friction_hd(const HD<T>* Xh, const double* Xlag, const double* w, const double* n,
                                     double lam, double mu, double eh) {
  HD<T> dl[3];
  for (int c = 0; c < 3; ++c) {
    dl[c] = HD<T>(T(0));
    for (int s = 0; s < 4; ++s) dl[c] = dl[c] + HD<T>((T)w[s]) * (Xh[3 * s + c] - HD<T>((T)Xlag[3 * s + c]));
  }
  HD<T> dn = dl[0] * HD<T>((T)n[0]) + dl[1] * HD<T>((T)n[1]) + dl[2] * HD<T>((T)n[2]);
  HD<T> y2(T(0));
  for (int c = 0; c < 3; ++c) {
    HD<T> t = dl[c] - HD<T>((T)n[c]) * dn;
    y2 = y2 + t * t;
  }
  return f0_hd(hsqrt(y2), (T)eh) * HD<T>((T)(mu * lam));
}

struct StepRec { int ptype, i, j, filtered, iters; double xi, t; };
struct StepResult { std::vector<StepRec> recs; };

}  // namespace

// ===========================================================================
// C API
// ===========================================================================
extern "C" {

typedef struct {
  int32_t kind;
  int64_t nv, ne, nt;
  const int32_t* edges;
  const int32_t* tris;
  const double* ref;
  double h, eta, kappa;
  int32_t filter_mode;
  int64_t n_core;  // pairs under the temporary zero offset (Sec. 3.4), may be 0
  const int32_t* core_ptype;
  const int32_t* core_i;
  const int32_t* core_j;
  int32_t cull_radius;  // filter_mode 2 (rods): radius in elements
  int32_t refdist;      // 0 parametric reference distance, 1 Euclidean at the rest pose
  const double* xrest;  // [V,3] rest pose (refdist 1)
} orc_scene;

static Mesh make_mesh(const orc_scene* s) {
  Mesh m;
  m.kind = s->kind; m.nv = s->nv; m.ne = s->ne; m.nt = s->kind == 1 ? s->nt : 0;
  m.edges = s->edges; m.tris = s->tris; m.ref = s->ref;
  m.h = s->h; m.eta = s->eta; m.kappa = s->kappa; m.filter_mode = s->filter_mode;
  m.refdist = s->refdist;
  m.xrest = s->xrest;
  m.comp.resize(m.nv);
  int nc = components(m.nv, m.ne, m.edges, m.tris, m.nt, m.comp.data());
  if (m.refdist == 1) compute_dmin_euclid(m, nc);
  else compute_dmin(m, nc);
  for (int64_t k = 0; k < s->n_core; ++k) m.core.insert(pair_key(s->core_ptype[k], s->core_i[k], s->core_j[k]));
  m.cull_radius = s->cull_radius;
  if (m.filter_mode == 2) order_polylines(m);
  return m;
}

// Connected components (numbered by smallest vertex) and per-component d_min.
int32_t orc_precompute(const orc_scene* s, int32_t* comp, double* dmin2, double* dmin, int32_t cap) {
  Mesh m = make_mesh(s);
  std::copy(m.comp.begin(), m.comp.end(), comp);
  int nc = (int)m.dmin.size();
  for (int c = 0; c < nc && c < cap; ++c) { dmin2[c] = m.dmin2[c]; dmin[c] = m.dmin[c]; }
  return nc;
}

// Evaluate every pair of the universe with d < h.
//   mode 0: all pairs (the definition); mode 1: the same pairs, pruned by a
//   conservative sweep over bounding boxes inflated by h (a pair whose boxes
//   are h or more apart along some axis has d >= h).
void* orc_evaluate(const orc_scene* s, const double* x, int32_t mode, int32_t derivs, int32_t nthreads) {
  Mesh m = make_mesh(s);
  if (nthreads > 0) omp_set_num_threads(nthreads);
  int T = omp_get_max_threads();
  std::vector<std::vector<Rec>> recs(T);
  struct P { int id; double lo[3], hi[3]; };
  std::vector<P> pts, egs, trs;
  if (m.kind == 1)
    for (int64_t v = 0; v < m.nv; ++v) { P p; p.id = (int)v; prim_box(m, x, 0, (int)v, p.lo, p.hi); pts.push_back(p); }
  for (int64_t e = 0; e < m.ne; ++e) { P p; p.id = (int)e; prim_box(m, x, 1, (int)e, p.lo, p.hi); egs.push_back(p); }
  if (m.kind == 1)
    for (int64_t t = 0; t < m.nt; ++t) { P p; p.id = (int)t; prim_box(m, x, 2, (int)t, p.lo, p.hi); trs.push_back(p); }
  // pruning slack: the gaps are rounded double differences, so allow a few
  // ulps of the largest coordinate beyond h
  double amax = 0.0;
  for (int64_t k = 0; k < 3 * m.nv; ++k) amax = std::max(amax, std::fabs(x[k]));
  const double lim = m.h * (1.0 + 1e-12) + 1e-14 * amax;
  auto near = [&](const P& a, const P& b) {
    for (int c = 0; c < 3; ++c)
      if (std::max(b.lo[c] - a.hi[c], a.lo[c] - b.hi[c]) >= lim) return false;
    return true;
  };
  auto by_lo0 = [](const P& a, const P& b) { return a.lo[0] < b.lo[0] || (a.lo[0] == b.lo[0] && a.id < b.id); };
  auto visit = [&](int ptype, int i, int j) {
    if (incident(m, ptype, i, j)) return;
    Rec r;
    if (eval_pair(m, x, ptype, i, j, derivs != 0, r)) recs[omp_get_thread_num()].push_back(r);
  };
  // edge-edge pairs
  if (mode == 0) {
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t a = 0; a < m.ne; ++a)
      for (int64_t b = a + 1; b < m.ne; ++b) visit(1, (int)a, (int)b);
  } else {
    std::vector<P> es = egs;
    std::sort(es.begin(), es.end(), by_lo0);
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < (int64_t)es.size(); ++k) {
      const P& A = es[k];
      for (size_t l = k + 1; l < es.size(); ++l) {
        const P& B = es[l];
        if (B.lo[0] - A.hi[0] >= lim) break;
        if (!near(A, B)) continue;
        visit(1, std::min(A.id, B.id), std::max(A.id, B.id));
      }
    }
  }
  // point-triangle pairs
  if (m.kind == 1) {
    if (mode == 0) {
      #pragma omp parallel for schedule(dynamic, 16)
      for (int64_t v = 0; v < m.nv; ++v)
        for (int64_t t = 0; t < m.nt; ++t) visit(0, (int)v, (int)t);
    } else {
      std::vector<P> ts = trs;
      std::sort(ts.begin(), ts.end(), by_lo0);
      double wmax = 0.0;
      for (const P& t : ts) wmax = std::max(wmax, t.hi[0] - t.lo[0]);
      #pragma omp parallel for schedule(dynamic, 64)
      for (int64_t v = 0; v < m.nv; ++v) {
        const P& A = pts[v];
        // every triangle with hi0 > A.lo0 - lim has lo0 > A.lo0 - lim - wmax
        double lo_bound = A.lo[0] - lim - wmax;
        size_t l = std::lower_bound(ts.begin(), ts.end(), lo_bound,
                                    [](const P& p, double val) { return p.lo[0] < val; }) - ts.begin();
        for (; l < ts.size(); ++l) {
          const P& B = ts[l];
          if (B.lo[0] - A.hi[0] >= lim) break;
          if (!near(A, B)) continue;
          visit(0, (int)v, B.id);
        }
      }
    }
  }
  Result* res = new Result;
  for (auto& v : recs) { res->recs.insert(res->recs.end(), v.begin(), v.end()); std::vector<Rec>().swap(v); }
  std::sort(res->recs.begin(), res->recs.end(), [](const Rec& a, const Rec& b) {
    if (a.ptype != b.ptype) return a.ptype < b.ptype;
    if (a.i != b.i) return a.i < b.i;
    return a.j < b.j;
  });
  return res;
}

int64_t orc_count(void* h) { return (int64_t)((Result*)h)->recs.size(); }

void orc_get(void* h, int32_t* ptype, int32_t* pi, int32_t* pj, int32_t* verts, int32_t* code,
             int32_t* flags, double* d, double* a, double* eta, double* E, double* G,
             double* Hraw, double* Hpsd) {
  const auto& R = ((Result*)h)->recs;
  for (size_t k = 0; k < R.size(); ++k) {
    const Rec& r = R[k];
    if (ptype) ptype[k] = r.ptype;
    if (pi) pi[k] = r.i;
    if (pj) pj[k] = r.j;
    if (verts) for (int q = 0; q < 4; ++q) verts[4 * k + q] = r.verts[q];
    if (code) code[k] = r.code;
    if (flags) flags[k] = r.flags;
    if (d) d[k] = r.d;
    if (a) a[k] = r.a;
    if (eta) eta[k] = r.eta;
    if (E) E[k] = r.E;
    if (r.der) {
      if (G) std::memcpy(G + 12 * k, r.der->G, sizeof(r.der->G));
      if (Hraw) std::memcpy(Hraw + 144 * k, r.der->Hraw, sizeof(r.der->Hraw));
      if (Hpsd) std::memcpy(Hpsd + 144 * k, r.der->Hpsd, sizeof(r.der->Hpsd));
    }
  }
}

void orc_free(void* h) { delete (Result*)h; }

// ---- single-pair utilities (for pins) -------------------------------------

// Classify and return the squared distance of one pair of 4 local vertices.
void orc_pair_distance(int32_t ptype, const double* X, double* D, int32_t* code) {
  Dist d = classify(ptype, X);
  *D = d.D; *code = d.code;
}

// Squared distance of a given sub-case formula, in double and in binary128.
void orc_case_distance(int32_t code, const double* X, double* Dd, double* Dq_hi, double* Dq_lo) {
  *Dd = D_case<double>(code, X);
  f128 Xq[12];
  for (int k = 0; k < 12; ++k) Xq[k] = (f128)X[k];
  f128 q = D_case<f128>(code, Xq);
  double hi = (double)q;
  *Dq_hi = hi;
  *Dq_lo = (double)(q - (f128)hi);
}

// Energy, gradient, raw and projected Hessian of one pair (given a, eta).
void orc_pair_barrier(int32_t ptype, const double* X, double a, double eta, double kappa,
                      double* E, double* G, double* Hraw, double* Hpsd, int32_t* code, int32_t quad) {
  Dist d = classify(ptype, X);
  *code = d.code;
  if (quad) energy_derivs<f128>(d.code, X, a, eta, kappa, E, G, Hraw);
  else energy_derivs<double>(d.code, X, a, eta, kappa, E, G, Hraw);
  psd_project(12, Hraw, Hpsd, nullptr);
}

// The same with the distance sub-case given: at a region boundary, where
// several sub-cases give the same distance, each one's formula is a valid
// one-sided derivative (the tests accept the one the GPU took there).
void orc_pair_barrier_code(int32_t code, const double* X, double a, double eta, double kappa,
                           double* E, double* G, double* Hraw, double* Hpsd, int32_t quad) {
  if (quad) energy_derivs<f128>(code, X, a, eta, kappa, E, G, Hraw);
  else energy_derivs<double>(code, X, a, eta, kappa, E, G, Hraw);
  psd_project(12, Hraw, Hpsd, nullptr);
}

// b, b', b'' of the offset barrier at scalar d (Eq. 2 and Eq. 3).
void orc_barrier_scalar(double d, double a, double eta, double* b, double* b1, double* b2) {
  HD<double> x(d, 1.0, 1.0, 0.0);
  HD<double> r = barrier_hd(x, a, eta);
  *b = r.a; *b1 = r.b; *b2 = r.d;
}

// Threshold decision used for "d < thr" (lt = 1) and "d <= thr" (lt = 0) on
// sub-case `code`; *ext reports whether binary128 was needed.
int32_t orc_decide(int32_t code, const double* X, double thr, int32_t lt, int32_t* ext) {
  double D = D_case<double>(code, X);
  bool e = false;
  bool r = decide(code, X, D, thr * thr, sq(thr), lt != 0, &e);
  *ext = e ? 1 : 0;
  return r ? 1 : 0;
}

// PSD projection of a symmetric n x n matrix (eigenvalue clamp at zero).
void orc_psd_project(int32_t n, const double* A, double* Ap, double* evals) {
  psd_project(n, A, Ap, evals);
}

// ACCD of one pair of 4 local vertices X with displacements P and offset xi.
void orc_accd_pair(int32_t ptype, const double* X, const double* P, double xi, double s, int32_t max_iter,
                   double* t, int32_t* iters) {
  int it = 0;
  *t = accd_pair(ptype, X, P, xi, s, max_iter, &it);
  *iters = it;
}

// ACCD over the pairs of the universe whose swept boxes are within h on every
// axis (gap max(lo_b - hi_a, lo_a - hi_b) < h in double), each with its
// filtered offset; records sorted by (ptype, i, j).  The step is the minimum
// of their t.  mode 0: all pairs (the definition); mode 1: the same pairs,
// pruned first by a sweep along x with a few ulps of slack.
void* orc_max_step(const orc_scene* s, const double* x, const double* p, double sfac, int32_t max_iter,
                   int32_t mode, int32_t nthreads) {
  Mesh m = make_mesh(s);
  if (nthreads > 0) omp_set_num_threads(nthreads);
  int T = omp_get_max_threads();
  std::vector<std::vector<StepRec>> recs(T);
  struct B { int id; double lo[3], hi[3]; };
  std::vector<B> pts, egs, trs;
  if (m.kind == 1)
    for (int64_t v = 0; v < m.nv; ++v) { B b; b.id = (int)v; swept_box(m, x, p, 0, (int)v, b.lo, b.hi); pts.push_back(b); }
  for (int64_t e = 0; e < m.ne; ++e) { B b; b.id = (int)e; swept_box(m, x, p, 1, (int)e, b.lo, b.hi); egs.push_back(b); }
  if (m.kind == 1)
    for (int64_t t = 0; t < m.nt; ++t) { B b; b.id = (int)t; swept_box(m, x, p, 2, (int)t, b.lo, b.hi); trs.push_back(b); }
  double amax = 0.0;
  for (int64_t k = 0; k < 3 * m.nv; ++k) amax = std::max(amax, std::fabs(x[k]) + std::fabs(p[k]));
  const double lim = m.h * (1.0 + 1e-12) + 1e-14 * amax;  // pruning only
  auto within_h = [&](const B& a, const B& b) {  // the definition of the pair set
    for (int c = 0; c < 3; ++c)
      if (!(std::max(b.lo[c] - a.hi[c], a.lo[c] - b.hi[c]) < m.h)) return false;
    return true;
  };
  auto visit = [&](int ptype, int i, int j, const B& A, const B& Bb) {
    if (incident(m, ptype, i, j) || is_culled(m, ptype, i, j) || !within_h(A, Bb)) return;
    int verts[4];
    double X[12], P[12];
    gather(m, x, ptype, i, j, verts, X);
    for (int k = 0; k < 4; ++k)
      for (int c = 0; c < 3; ++c) P[3 * k + c] = p[3 * verts[k] + c];
    StepRec r;
    r.ptype = ptype; r.i = i; r.j = j;
    r.filtered = is_filtered(m, ptype, i, j) ? 1 : 0;
    // Eq. 4: filtered stencils have no offset; nor do pairs in the core set (Sec. 3.4)
    const bool core = !r.filtered && !m.core.empty() && m.core.count(pair_key(ptype, i, j)) != 0;
    r.xi = r.filtered || core ? 0.0 : m.eta;
    r.t = accd_pair(ptype, X, P, r.xi, sfac, max_iter, &r.iters);
    recs[omp_get_thread_num()].push_back(r);
  };
  auto by_lo0 = [](const B& a, const B& b) { return a.lo[0] < b.lo[0] || (a.lo[0] == b.lo[0] && a.id < b.id); };
  if (mode == 0) {
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t a = 0; a < m.ne; ++a)
      for (int64_t b = a + 1; b < m.ne; ++b) visit(1, (int)a, (int)b, egs[a], egs[b]);
    if (m.kind == 1) {
      #pragma omp parallel for schedule(dynamic, 16)
      for (int64_t v = 0; v < m.nv; ++v)
        for (int64_t t = 0; t < m.nt; ++t) visit(0, (int)v, (int)t, pts[v], trs[t]);
    }
  } else {
    std::vector<B> es = egs;
    std::sort(es.begin(), es.end(), by_lo0);
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < (int64_t)es.size(); ++k)
      for (size_t l = k + 1; l < es.size(); ++l) {
        if (es[l].lo[0] - es[k].hi[0] >= lim) break;
        const B& A = es[k].id < es[l].id ? es[k] : es[l];
        const B& Bb = es[k].id < es[l].id ? es[l] : es[k];
        visit(1, A.id, Bb.id, A, Bb);
      }
    if (m.kind == 1) {
      std::vector<B> ts = trs;
      std::sort(ts.begin(), ts.end(), by_lo0);
      double wmax = 0.0;
      for (const B& t : ts) wmax = std::max(wmax, t.hi[0] - t.lo[0]);
      #pragma omp parallel for schedule(dynamic, 64)
      for (int64_t v = 0; v < m.nv; ++v) {
        const B& A = pts[v];
        double lo_bound = A.lo[0] - lim - wmax;
        size_t l = std::lower_bound(ts.begin(), ts.end(), lo_bound,
                                    [](const B& q, double val) { return q.lo[0] < val; }) - ts.begin();
        for (; l < ts.size(); ++l) {
          if (ts[l].lo[0] - A.hi[0] >= lim) break;
          visit(0, (int)v, ts[l].id, A, ts[l]);
        }
      }
    }
  }
  StepResult* res = new StepResult;
  for (auto& v : recs) res->recs.insert(res->recs.end(), v.begin(), v.end());
  std::sort(res->recs.begin(), res->recs.end(), [](const StepRec& a, const StepRec& b) {
    if (a.ptype != b.ptype) return a.ptype < b.ptype;
    if (a.i != b.i) return a.i < b.i;
    return a.j < b.j;
  });
  return res;
}

// Lagged friction data of one active pair of sub-case `code` at the lagged
// local positions X (distance d, barrier parameters a, eta): the normal force
// lambda = kappa |b'(d)| (0 when d >= a or d <= eta), the closest-point
// weights w[4] and the contact normal n[3].
void orc_friction_lag(int32_t code, const double* X, double d, double a, double eta, double kappa, double* lam,
                      double* w, double* n) {
  closest_weights(code, X, w);
  double c[3] = {0.0, 0.0, 0.0};
  for (int s = 0; s < 4; ++s)
    for (int k = 0; k < 3; ++k) c[k] += w[s] * X[3 * s + k];
  const double nc = std::sqrt(dot3(c, c));
  for (int k = 0; k < 3; ++k) n[k] = c[k] / nc;
  *lam = 0.0;
  if (d < a && d > eta) {
    HD<double> x(d, 1.0, 1.0, 0.0);
    *lam = kappa * std::fabs(barrier_hd(x, a, eta).b);
  }
}

// Friction energy, gradient and Hessian (then its PSD projection, which the
// exact Hessian does not need) of one pair at local positions X.
void orc_friction_pair(const double* X, const double* Xlag, const double* w, const double* n, double lam, double mu,
                       double eh, double* E, double* G, double* H, double* Hpsd) {
  for (int i = 0; i < 12; ++i)
    for (int j = i; j < 12; ++j) {
      HD<double> Xh[12];
      for (int k = 0; k < 12; ++k) Xh[k] = HD<double>(X[k]);
      Xh[i].b = 1.0;
      Xh[j].c = 1.0;
      HD<double> e = friction_hd<double>(Xh, Xlag, w, n, lam, mu, eh);
      if (i == 0 && j == 0) *E = e.a;
      if (j == i) G[i] = e.b;
      H[i * 12 + j] = e.d;
      H[j * 12 + i] = e.d;
    }
  psd_project(12, H, Hpsd, nullptr);
}

// The same for n pairs at once (local positions and lagged data stacked),
// over OpenMP threads.
void orc_friction_batch(int64_t n, const double* X, const double* Xlag, const double* w, const double* nrm,
                        const double* lam, double mu, double eh, double* E, double* G, double* H, double* Hpsd,
                        int32_t nthreads) {
  if (nthreads > 0) omp_set_num_threads(nthreads);
  #pragma omp parallel for schedule(dynamic, 64)
  for (int64_t k = 0; k < n; ++k)
    orc_friction_pair(X + 12 * k, Xlag + 12 * k, w + 4 * k, nrm + 3 * k, lam[k], mu, eh, E + k, G + 12 * k,
                      H + 144 * k, Hpsd + 144 * k);
}

// Friction energy alone (no derivatives; defined at zero sliding too).
double orc_friction_energy(const double* X, const double* Xlag, const double* w, const double* n, double lam,
                           double mu, double eh) {
  HD<double> Xh[12];
  for (int k = 0; k < 12; ++k) Xh[k] = HD<double>(X[k]);
  double dl[3] = {0.0, 0.0, 0.0};
  for (int c = 0; c < 3; ++c)
    for (int s = 0; s < 4; ++s) dl[c] += w[s] * (X[3 * s + c] - Xlag[3 * s + c]);
  const double dn = dot3(dl, n);
  double y2 = 0.0;
  for (int c = 0; c < 3; ++c) y2 += (dl[c] - n[c] * dn) * (dl[c] - n[c] * dn);
  const double y = std::sqrt(y2);
  const double f0 = y >= eh ? y : -y * y * y / (3.0 * eh * eh) + y * y / eh + eh / 3.0;
  return mu * lam * f0;
}

int64_t orc_ms_count(void* h) { return (int64_t)((StepResult*)h)->recs.size(); }

void orc_ms_get(void* h, int32_t* ptype, int32_t* pi, int32_t* pj, int32_t* filtered, int32_t* iters, double* xi,
                double* t) {
  const auto& R = ((StepResult*)h)->recs;
  for (size_t k = 0; k < R.size(); ++k) {
    ptype[k] = R[k].ptype; pi[k] = R[k].i; pj[k] = R[k].j; filtered[k] = R[k].filtered;
    iters[k] = R[k].iters; xi[k] = R[k].xi; t[k] = R[k].t;
  }
}

void orc_ms_free(void* h) { delete (StepResult*)h; }

// Release test of the temporary zero offset (Sec. 3.4): released[k] = 1 when
// pair k is at d > eta at x (decided as the filter decides d <= eta).
void orc_core_release(const orc_scene* s, const double* x, int64_t n, const int32_t* ptype, const int32_t* pi,
                      const int32_t* pj, int32_t* released) {
  Mesh m = make_mesh(s);
  for (int64_t k = 0; k < n; ++k) {
    int verts[4];
    double X[12];
    gather(m, x, ptype[k], pi[k], pj[k], verts, X);
    Dist ds = classify(ptype[k], X);
    bool ext = false;
    released[k] = decide(ds.code, X, ds.D, m.eta * m.eta, sq(m.eta), false, &ext) ? 0 : 1;
  }
}

}  // extern "C"
