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

namespace bfc {

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
__device__ __forceinline__ dd dd_two_sum(double a, double b) {
#pragma clang fp contract(off)
  double s = a + b;
  double bb = s - a;
  double e = (a - (s - bb)) + (b - bb);
  return {s, e};
}
__device__ __forceinline__ dd dd_fast(double a, double b) {
#pragma clang fp contract(off)
  double s = a + b;
  return {s, b - (s - a)};
}
__device__ __forceinline__ dd operator+(dd a, dd b) {
#pragma clang fp contract(off)
  dd s = dd_two_sum(a.hi, b.hi);
  dd t = dd_two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = dd_fast(s.hi, s.lo);
  s.lo += t.lo;
  return dd_fast(s.hi, s.lo);
}
__device__ __forceinline__ dd operator-(dd a) { return {-a.hi, -a.lo}; }
__device__ __forceinline__ dd operator-(dd a, dd b) { return a + (-b); }
__device__ __forceinline__ dd operator*(dd a, dd b) {
#pragma clang fp contract(off)
  double p = a.hi * b.hi;
  double e = __fma_rn(a.hi, b.hi, -p);
  e += a.hi * b.lo + a.lo * b.hi;
  return dd_fast(p, e);
}
__device__ __forceinline__ dd operator/(dd a, dd b) {
#pragma clang fp contract(off)
  double q1 = a.hi / b.hi;
  dd r = a - dd{q1, 0.0} * b;
  double q2 = r.hi / b.hi;
  r = r - dd{q2, 0.0} * b;
  double q3 = r.hi / b.hi;
  dd q = dd_fast(q1, q2);
  return q + dd{q3, 0.0};
}
__device__ __forceinline__ bool dd_lt(dd a, dd b) { return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo); }
__device__ __forceinline__ bool dd_le(dd a, dd b) { return a.hi < b.hi || (a.hi == b.hi && a.lo <= b.lo); }
__device__ __forceinline__ dd dd_of(double v) { return {v, 0.0}; }
// exact square of a double
__device__ __forceinline__ dd dd_sq(double v) {
#pragma clang fp contract(off)
  double p = v * v;
  return {p, __fma_rn(v, v, -p)};
}

// ---------------------------------------------------------------------------
// 3-vectors over a scalar type (double, float or dd)
// ---------------------------------------------------------------------------
template <class T> struct V3 {
  T x, y, z;
};
template <class T> __device__ __forceinline__ V3<T> operator-(V3<T> a, V3<T> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class T> __device__ __forceinline__ V3<T> operator+(V3<T> a, V3<T> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class T> __device__ __forceinline__ V3<T> operator*(T s, V3<T> a) { return {s * a.x, s * a.y, s * a.z}; }
template <class T> __device__ __forceinline__ T dot(V3<T> a, V3<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class T> __device__ __forceinline__ V3<T> cross(V3<T> a, V3<T> b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
typedef V3<double> d3;
typedef V3<dd> q3;

__device__ __forceinline__ q3 q3_of(d3 a) { return {dd_of(a.x), dd_of(a.y), dd_of(a.z)}; }

// ---------------------------------------------------------------------------
// Sub-case table
// ---------------------------------------------------------------------------
enum { K_PP = 0, K_PE = 1, K_PT = 2, K_EE = 3 };
__device__ __forceinline__ int case_kind(int code) {
  // 0-2 PP, 3-5 PE, 6 PT, 7-10 PP, 11-14 PE, 15 EE
  return code <= 2 ? K_PP : code <= 5 ? K_PE : code == 6 ? K_PT : code <= 10 ? K_PP : code <= 14 ? K_PE : K_EE;
}
// participating slots; PP: (s0, s1); PE: point s0, edge (s1, s2); PT/EE: all four
__device__ __forceinline__ void case_slots(int code, int& s0, int& s1, int& s2) {
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
template <class T> __device__ __forceinline__ T sqd_pp(V3<T> p, V3<T> q) {
  V3<T> r = p - q;
  return dot(r, r);
}
template <class T> __device__ __forceinline__ T sqd_pe(V3<T> p, V3<T> e0, V3<T> e1) {
  V3<T> e = e1 - e0;
  V3<T> c = cross(p - e0, e);
  return dot(c, c) / dot(e, e);
}
// plane / line-line form shared by PT and EE: (r . (u x v))^2 / |u x v|^2
template <class T> __device__ __forceinline__ T sqd_tri(V3<T> r, V3<T> u, V3<T> v) {
  V3<T> n = cross(u, v);
  T s = dot(r, n);
  return s * s / dot(n, n);
}
// one of four vertices, chosen by value selects (indexing the array with a
// run-time slot, or selecting between element addresses, would keep the
// array in scratch memory)
template <class T> __device__ __forceinline__ T sel4(int s, T a, T b, T c, T d) {
  T lo = s == 0 ? a : b;
  T hi = s == 2 ? c : d;
  return s < 2 ? lo : hi;
}
template <class T> __device__ __forceinline__ V3<T> pick(const V3<T>* P, int s) {
  const V3<T> p0 = P[0], p1 = P[1], p2 = P[2], p3 = P[3];
  return {sel4(s, p0.x, p1.x, p2.x, p3.x), sel4(s, p0.y, p1.y, p2.y, p3.y), sel4(s, p0.z, p1.z, p2.z, p3.z)};
}
template <class T> __device__ __forceinline__ T sqd_case(int code, const V3<T>* P) {
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
__device__ __forceinline__ Near near_pseg(d3 p, d3 e0, d3 e1, int c0, int c1, int ce) {
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
__device__ __forceinline__ void take_min(Near& best, Near c) {
  if (c.D < best.D * (1.0 - 1e-12)) best = c;
}
__device__ __forceinline__ Near classify_pt(const d3* P) {
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
__device__ __forceinline__ Near classify_ee(const d3* P) {
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

// Relative width of a tie in the re-evaluated threshold decisions: exact ties
// of the geometry (e.g. lattice-aligned primitives exactly h apart) reach the
// division in a distance formula as rounding noise of about this size, so a
// re-evaluated D within this margin of T counts as D = T.
#define BFC_TIE 1e-24

// D (FP64 value of sub-case `code`) against an exact squared threshold given
// as a double-double T: lt -> d < thr, else d <= thr.  Outside a relative band
// of 1e-9 the FP64 value decides; inside, D is re-evaluated in double-double
// and a tie counts as d = thr.
__device__ __forceinline__ bool decide_sq(int code, const d3* P, double D, dd T, bool lt) {
  double Th = T.hi;
  if (fabs(D - Th) > 1e-9 * Th) return lt ? (D < Th) : (D <= Th);
  q3 Q[4] = {q3_of(P[0]), q3_of(P[1]), q3_of(P[2]), q3_of(P[3])};
  dd Dq = sqd_case<dd>(code, Q);
  dd m = dd_of(Th * BFC_TIE);
  return lt ? dd_lt(Dq, T - m) : dd_le(Dq, T + m);
}

// ---------------------------------------------------------------------------
// Reference distance in 2D rest coordinates (shell filter, Sec. 3.2)
// ---------------------------------------------------------------------------
template <class T> struct V2 {
  T x, y;
};
template <class T> __device__ __forceinline__ T seg2(V2<T> p, V2<T> a, V2<T> b) {
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
template <class T> __device__ __forceinline__ T orient(V2<T> a, V2<T> b, V2<T> c) {
  return (b.x - a.x) * (c.y - a.y) - (b.y - a.y) * (c.x - a.x);
}

// ---------------------------------------------------------------------------
// Offset barrier (Eq. 2, Eq. 3): u = d - a, w = d - eta, L = ln(w/(a-eta)).
// b = -u^2 L, b' = -2uL - u^2/w, b'' = -2L - 4u/w + u^2/w^2.
// ---------------------------------------------------------------------------
template <class T> __device__ __forceinline__ void barrier3(T d, T a, T eta, T& b, T& b1, T& b2) {
  T u = d - a, w = d - eta;
  T L = log1p(u / (a - eta));
  T uw = u / w;
  b = -u * u * L;
  b1 = -2 * u * L - u * uw;
  b2 = -2 * L - 4 * uw + uw * uw;
}

}  // namespace bfc
