// Kernels of libbfc (gfx950, wave64).
//
//   broad phase   : k_begin, k_bounds, k_grid, k_zero_i, k_count, scan, k_scatter, k_pairs
//   narrow phase  : k_narrow      (distance, filter of Eq. 4, exact thresholds, ballot compaction)
//   evaluation    : k_eval        (Eq. 2/3 barrier, derivatives, PSD projection)
//   assembly      : k_esum*, k_grad, k_asm_*
//   precompute    : k_cc_*, k_refmin (components and d_min, Sec. 3.2)
#include "bfc_kernels.h"
#include "bfc_eval.h"

namespace bfc {

// ---------------------------------------------------------------------------
// small utilities
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned f2ord(float f) {
  unsigned u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ord2f(unsigned u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}
__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int lanes_below(unsigned long long mask) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}
__device__ __forceinline__ d3 load3(const double* x, int v) {
  return {x[3 * v], x[3 * v + 1], x[3 * v + 2]};
}
__device__ __forceinline__ int grid_stride() { return gridDim.x * blockDim.x; }

// inclusive scan across the 64 lanes of a wave
template <class T> __device__ __forceinline__ T wave_incl_scan(T v) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    T y = __shfl_up(v, o, 64);
    if (lane_id() >= o) v += y;
  }
  return v;
}
template <class T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// exclusive scan across a block of 256 threads (4 waves)
__device__ __forceinline__ int block_excl_scan256(int v, int* total) {
  __shared__ int ws[4];
  int x = wave_incl_scan(v);
  int w = threadIdx.x >> 6;
  if (lane_id() == 63) ws[w] = x;
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    int t = ws[k];
    if (k < w) off += t;
    tot += t;
  }
  __syncthreads();
  if (total) *total = tot;
  return off + x - v;
}

// ---------------------------------------------------------------------------
// device-wide exclusive scan of int32 (3 kernels); n = n_dev ? *n_dev : n_const
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_scan_reduce(const int* in, const int* n_dev, int n_const, int* part) {
  int n = n_dev ? *n_dev : n_const;
  int base = blockIdx.x * SCAN_TILE;
  if (base >= n) return;
  int s = 0;
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    int i = base + threadIdx.x * SCAN_ITEMS + k;
    if (i < n) s += in[i];
  }
  int tot;
  block_excl_scan256(s, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_scan_partials(int* part, const int* n_dev, int n_const) {
  int n = n_dev ? *n_dev : n_const;
  int nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  __shared__ int ws[16];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < nb; base += 1024) {
    int i = base + threadIdx.x;
    int v = i < nb ? part[i] : 0;
    int x = wave_incl_scan(v);
    int w = threadIdx.x >> 6;
    if (lane_id() == 63) ws[w] = x;
    __syncthreads();
    int off = 0, tot = 0;
    for (int k = 0; k < 16; ++k) {
      if (k < w) off += ws[k];
      tot += ws[k];
    }
    int c = carry;
    if (i < nb) part[i] = c + off + x - v;
    __syncthreads();
    if (threadIdx.x == 0) carry = c + tot;
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_scan_down(const int* in, int* out, const int* n_dev, int n_const,
                                                   const int* part) {
  int n = n_dev ? *n_dev : n_const;
  int base = blockIdx.x * SCAN_TILE;
  if (base >= n) return;
  int v[SCAN_ITEMS];
  int s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    int i = base + threadIdx.x * SCAN_ITEMS + k;
    v[k] = i < n ? in[i] : 0;
    s += v[k];
  }
  int run = block_excl_scan256(s, nullptr) + part[blockIdx.x];
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    int i = base + threadIdx.x * SCAN_ITEMS + k;
    if (i < n) out[i] = run;
    run += v[k];
  }
}

void scan_excl(const int* in, int* out, const int* n_dev, int n_max, int* tmp, hipStream_t st) {
  int nb = (n_max + SCAN_TILE - 1) / SCAN_TILE;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(256), 0, st, in, n_dev, n_max, tmp);
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, st, tmp, n_dev, n_max);
  hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(256), 0, st, in, out, n_dev, n_max, tmp);
}

__global__ void k_zero_i(int* a, const int* n_dev, long long n_const) {
  long long n = n_dev ? (long long)*n_dev : n_const;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += grid_stride()) a[i] = 0;
}
__global__ void k_fill_u64(unsigned long long* a, long long n, unsigned long long v) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += grid_stride()) a[i] = v;
}
__global__ void k_zero_d(double* a, const long long* n_dev, long long n_const, long long mul, long long cap) {
  long long n = n_dev ? *n_dev : n_const;
  if (n > cap) n = cap;
  n *= mul;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += grid_stride()) a[i] = 0.0;
}

// ---------------------------------------------------------------------------
// Broad phase at the full activation distance (Sec. 3.3, last paragraph)
// ---------------------------------------------------------------------------
// Primitive numbering: [0, E) edges, [E, E+F) triangles, [E+F, E+F+V) points
// (shells only).  Edges and triangles are stored in the grid; points and
// edges query it.
__global__ void k_begin(unsigned* bounds, long long* cand_count) {
  if (threadIdx.x < 3) bounds[threadIdx.x] = 0xffffffffu;      // min: largest key
  else if (threadIdx.x < 7) bounds[threadIdx.x] = 0u;           // max / extent: smallest key
  if (threadIdx.x == 0 && cand_count) *cand_count = 0;
}

__device__ __forceinline__ int prim_verts(const SceneDev& S, int p, int* v) {
  if (p < S.ne) { v[0] = S.edges[2 * p]; v[1] = S.edges[2 * p + 1]; return 2; }
  if (p < S.ne + S.nt) {
    int t = p - S.ne;
    v[0] = S.tris[3 * t]; v[1] = S.tris[3 * t + 1]; v[2] = S.tris[3 * t + 2];
    return 3;
  }
  v[0] = p - S.ne - S.nt;
  return 1;
}

__global__ __launch_bounds__(256) void k_bounds(SceneDev S, const double* x, int np, Box* box, unsigned* bounds) {
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY}, ext = 0.0f;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < np; p += grid_stride()) {
    int v[3];
    int nvx = prim_verts(S, p, v);
    double l[3] = {INFINITY, INFINITY, INFINITY}, h[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int k = 0; k < nvx; ++k)
      for (int a = 0; a < 3; ++a) {
        double c = x[3 * v[k] + a];
        l[a] = fmin(l[a], c);
        h[a] = fmax(h[a], c);
      }
    Box b;
    for (int a = 0; a < 3; ++a) {
      b.lo[a] = __double2float_rd(l[a]);
      b.hi[a] = __double2float_ru(h[a]);
      lo[a] = fminf(lo[a], b.lo[a]);
      hi[a] = fmaxf(hi[a], b.hi[a]);
      ext = fmaxf(ext, __double2float_ru((double)b.hi[a] - (double)b.lo[a]));
    }
    box[p] = b;
  }
  // wave reduction, then one atomic per wave
  for (int o = 32; o > 0; o >>= 1) {
    for (int a = 0; a < 3; ++a) {
      lo[a] = fminf(lo[a], __shfl_xor(lo[a], o, 64));
      hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], o, 64));
    }
    ext = fmaxf(ext, __shfl_xor(ext, o, 64));
  }
  if (lane_id() == 0) {
    for (int a = 0; a < 3; ++a) {
      if (lo[a] <= hi[a]) {
        atomicMin(&bounds[a], f2ord(lo[a]));
        atomicMax(&bounds[3 + a], f2ord(hi[a]));
      }
    }
    atomicMax(&bounds[6], f2ord(ext));
  }
}

__global__ void k_grid(const unsigned* bounds, double h, int max_cells, Grid* g) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double lo[3], hi[3], span[3], amax = 0.0;
  for (int a = 0; a < 3; ++a) {
    lo[a] = (double)ord2f(bounds[a]);
    hi[a] = (double)ord2f(bounds[3 + a]);
    if (!(hi[a] >= lo[a])) { lo[a] = 0.0; hi[a] = 0.0; }
    span[a] = hi[a] - lo[a];
    amax = fmax(amax, fmax(fabs(lo[a]), fabs(hi[a])));
  }
  double ext = (double)ord2f(bounds[6]);
  if (!(ext >= 0.0)) ext = 0.0;
  double cell = (ext + h) * 1.001 + 1e-6 * (1.0 + amax);
  int coarse = 0;
  long long n[3], tot = 1;
  for (int it = 0; it < 64; ++it) {
    tot = 1;
    for (int a = 0; a < 3; ++a) {
      double q = floor(span[a] / cell) + 1.0;
      n[a] = q > 1048576.0 ? 1048576 : (long long)q;
      tot *= n[a];
    }
    if (tot <= max_cells) break;
    cell *= cbrt((double)tot / (double)max_cells) * 1.01;
    coarse = 1;
  }
  if (!(tot <= max_cells) || !(cell > 0.0) || !(cell < INFINITY)) {  // non-finite input: one cell
    n[0] = n[1] = n[2] = 1;
    tot = 1;
    cell = 1.0;
    coarse = 1;
  }
  g->cell = cell;
  g->inv_cell = 1.0 / cell;
  for (int a = 0; a < 3; ++a) { g->n[a] = (int)n[a]; g->orgd[a] = lo[a]; }
  g->ncells = (int)tot;
  g->nscan = 2 * (int)tot + 1;
  g->coarsened = coarse;
}

__device__ __forceinline__ void cell_coords(const Grid& g, const Box& b, int* c) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double ctr = 0.5 * ((double)b.lo[a] + (double)b.hi[a]);
    double q = floor((ctr - g.orgd[a]) / g.cell);
    // clamp (NaN lands in cell 0): clamping keeps adjacent cells adjacent
    int ci = q >= 0.0 ? (q < (double)g.n[a] ? (int)q : g.n[a] - 1) : 0;
    c[a] = ci;
  }
}
__device__ __forceinline__ int cell_lin(const Grid& g, int cx, int cy, int cz) {
  return (cz * g.n[1] + cy) * g.n[0] + cx;
}

__global__ __launch_bounds__(256) void k_count(int nstored, int ne, const Box* box, const Grid* gp, int* cell_cnt,
                                               int* cell_of) {
  Grid g = *gp;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < nstored; p += grid_stride()) {
    int c[3];
    cell_coords(g, box[p], c);
    int sub = 2 * cell_lin(g, c[0], c[1], c[2]) + (p >= ne ? 1 : 0);
    cell_of[p] = sub;
    atomicAdd(&cell_cnt[sub], 1);
  }
}

__global__ __launch_bounds__(256) void k_scatter(int nstored, const Box* box, const int* cell_of, int* cell_cnt,
                                                 const int* cell_start, int* sorted_id, Box* sorted_box) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < nstored; p += grid_stride()) {
    int sub = cell_of[p];
    int pos = cell_start[sub] + atomicSub(&cell_cnt[sub], 1) - 1;
    sorted_id[pos] = p;
    sorted_box[pos] = box[p];
  }
}

// Box gap below h on every axis.  The gap is a double difference of two
// floats, which rounds when their magnitudes are far apart; the slack (a
// few ulps of the operands) keeps the test conservative.
__device__ __forceinline__ bool boxes_near(const Box& a, const Box& b, double h) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double g1 = (double)b.lo[k] - (double)a.hi[k], g2 = (double)a.lo[k] - (double)b.hi[k];
    double mag = fmax(fmax(fabs((double)b.lo[k]), fabs((double)a.hi[k])),
                      fmax(fabs((double)a.lo[k]), fabs((double)b.hi[k])));
    if (!(fmax(g1, g2) < h + 1e-15 * mag)) return false;
  }
  return true;
}

// Visit every stored primitive of sub-list `sub` (0 edges, 1 triangles) in the
// cells adjacent to the query's cell whose box is within h of the query box
// and that forms a non-incident pair; emit (or count) it.
template <bool EMIT>
__device__ __forceinline__ int visit_pairs(const SceneDev& S, const Grid& g, const int* cell_start,
                                           const int* sorted_id, const Box* sorted_box, double hf, int qtype,
                                           int qid, const Box& qb, const int* qv, long long pos, long long cap,
                                           int* oi, int* oj, unsigned char* ot, unsigned* status) {
  int c[3];
  cell_coords(g, qb, c);
  int cnt = 0;
  int sub_type = qtype == BF_PT ? 1 : 0;
  int z0 = max(c[2] - 1, 0), z1 = min(c[2] + 1, g.n[2] - 1);
  int y0 = max(c[1] - 1, 0), y1 = min(c[1] + 1, g.n[1] - 1);
  int x0 = max(c[0] - 1, 0), x1 = min(c[0] + 1, g.n[0] - 1);
  for (int cz = z0; cz <= z1; ++cz)
    for (int cy = y0; cy <= y1; ++cy)
      for (int cx = x0; cx <= x1; ++cx) {
        int sub = 2 * cell_lin(g, cx, cy, cz) + sub_type;
        int b = cell_start[sub], e = cell_start[sub + 1];
        for (int k = b; k < e; ++k) {
          Box rb = sorted_box[k];
          if (!boxes_near(qb, rb, hf)) continue;
          int r = sorted_id[k];
          if (qtype == BF_EE) {
            if (r <= qid) continue;
            int r0 = S.edges[2 * r], r1 = S.edges[2 * r + 1];
            if (r0 == qv[0] || r0 == qv[1] || r1 == qv[0] || r1 == qv[1]) continue;
          } else {
            int t = r - S.ne;
            int t0 = S.tris[3 * t], t1 = S.tris[3 * t + 1], t2 = S.tris[3 * t + 2];
            if (t0 == qid || t1 == qid || t2 == qid) continue;
            r = t;
          }
          if (EMIT) {
            long long p = pos + cnt;
            if (p < cap) {
              oi[p] = qid;
              oj[p] = r;
              ot[p] = (unsigned char)qtype;
            } else {
              atomicOr(status, (unsigned)BF_S_CAND_OVERFLOW);
            }
          }
          ++cnt;
        }
      }
  return cnt;
}

__global__ __launch_bounds__(256) void k_pairs(SceneDev S, int nquery, const Box* box, const Grid* gp,
                                               const int* cell_start, const int* sorted_id, const Box* sorted_box,
                                               double hf, int* oi, int* oj, unsigned char* ot, long long cap,
                                               unsigned long long* count, unsigned* status) {
  Grid g = *gp;
  // wave-uniform loop so that all lanes take part in the scans
  for (int base = blockIdx.x * blockDim.x; base < nquery; base += grid_stride()) {
    int q = base + threadIdx.x;
    int qtype = BF_EE, qid = 0, qv[2] = {-1, -1};
    Box qb;
    bool valid = q < nquery;
    if (valid) {
      if (S.kind == 1 && q < S.nv) {  // point query against triangles
        qtype = BF_PT;
        qid = q;
        qb = box[S.ne + S.nt + q];
      } else {                         // edge query against edges with larger id
        qid = S.kind == 1 ? q - S.nv : q;
        qb = box[qid];
        qv[0] = S.edges[2 * qid];
        qv[1] = S.edges[2 * qid + 1];
      }
    }
    int cnt = valid ? visit_pairs<false>(S, g, cell_start, sorted_id, sorted_box, hf, qtype, qid, qb, qv, 0, 0,
                                         nullptr, nullptr, nullptr, nullptr)
                    : 0;
    long long incl = wave_incl_scan((long long)cnt);
    long long tot = __shfl(incl, 63, 64);
    long long wbase = 0;
    if (lane_id() == 63 && tot > 0) wbase = (long long)atomicAdd(count, (unsigned long long)tot);
    wbase = __shfl(wbase, 63, 64);
    if (valid && cnt > 0)
      visit_pairs<true>(S, g, cell_start, sorted_id, sorted_box, hf, qtype, qid, qb, qv, wbase + incl - cnt, cap,
                        oi, oj, ot, status);
  }
}

// ---------------------------------------------------------------------------
// Narrow phase + filter (Eq. 4) + compaction
// ---------------------------------------------------------------------------
__device__ __forceinline__ void pair_verts(const SceneDev& S, int type, int i, int j, int* v) {
  if (type == BF_PT) {
    v[0] = i;
    v[1] = S.tris[3 * j]; v[2] = S.tris[3 * j + 1]; v[3] = S.tris[3 * j + 2];
  } else {
    v[0] = S.edges[2 * i]; v[1] = S.edges[2 * i + 1];
    v[2] = S.edges[2 * j]; v[3] = S.edges[2 * j + 1];
  }
}

// 2D rest-space squared distance between the pair's primitives (shells).
__device__ __forceinline__ V2<double> ref2(const SceneDev& S, int v) { return {S.ref[2 * v], S.ref[2 * v + 1]}; }

__device__ double ref_sqdist_d(const SceneDev& S, int type, const int* v) {
  V2<double> P[4] = {ref2(S, v[0]), ref2(S, v[1]), ref2(S, v[2]), ref2(S, v[3])};
  if (type == BF_PT) {
    double o1 = orient(P[1], P[2], P[0]), o2 = orient(P[2], P[3], P[0]), o3 = orient(P[3], P[1], P[0]);
    if ((o1 >= 0 && o2 >= 0 && o3 >= 0) || (o1 <= 0 && o2 <= 0 && o3 <= 0)) return 0.0;
    return fmin(fmin(seg2(P[0], P[1], P[2]), seg2(P[0], P[2], P[3])), seg2(P[0], P[3], P[1]));
  }
  double o1 = orient(P[0], P[1], P[2]), o2 = orient(P[0], P[1], P[3]);
  double o3 = orient(P[2], P[3], P[0]), o4 = orient(P[2], P[3], P[1]);
  if (((o1 > 0 && o2 < 0) || (o1 < 0 && o2 > 0)) && ((o3 > 0 && o4 < 0) || (o3 < 0 && o4 > 0))) return 0.0;
  return fmin(fmin(seg2(P[0], P[2], P[3]), seg2(P[1], P[2], P[3])), fmin(seg2(P[2], P[0], P[1]), seg2(P[3], P[0], P[1])));
}

__device__ __forceinline__ dd dd_min(dd a, dd b) { return dd_lt(b, a) ? b : a; }
__device__ __forceinline__ dd seg2q(V2<dd> p, V2<dd> a, V2<dd> b) {
  dd ex = b.x - a.x, ey = b.y - a.y, rx = p.x - a.x, ry = p.y - a.y;
  dd ee = ex * ex + ey * ey, re = rx * ex + ry * ey;
  if (!dd_lt(dd_of(0.0), re)) return rx * rx + ry * ry;
  if (!dd_lt(re, ee)) {
    dd qx = p.x - b.x, qy = p.y - b.y;
    return qx * qx + qy * qy;
  }
  dd c = rx * ey - ry * ex;
  return c * c / ee;
}
__device__ __forceinline__ int sgn_dd(dd a) { return a.hi > 0.0 ? 1 : (a.hi < 0.0 ? -1 : (a.lo > 0.0 ? 1 : (a.lo < 0.0 ? -1 : 0))); }
__device__ __forceinline__ dd orientq(V2<dd> a, V2<dd> b, V2<dd> c) {
  return (b.x - a.x) * (c.y - a.y) - (b.y - a.y) * (c.x - a.x);
}

__device__ dd ref_sqdist_q(const SceneDev& S, int type, const int* v) {
  V2<dd> P[4];
  for (int k = 0; k < 4; ++k) P[k] = {dd_of(S.ref[2 * v[k]]), dd_of(S.ref[2 * v[k] + 1])};
  if (type == BF_PT) {
    int o1 = sgn_dd(orientq(P[1], P[2], P[0])), o2 = sgn_dd(orientq(P[2], P[3], P[0])), o3 = sgn_dd(orientq(P[3], P[1], P[0]));
    if ((o1 >= 0 && o2 >= 0 && o3 >= 0) || (o1 <= 0 && o2 <= 0 && o3 <= 0)) return dd_of(0.0);
    return dd_min(dd_min(seg2q(P[0], P[1], P[2]), seg2q(P[0], P[2], P[3])), seg2q(P[0], P[3], P[1]));
  }
  int o1 = sgn_dd(orientq(P[0], P[1], P[2])), o2 = sgn_dd(orientq(P[0], P[1], P[3]));
  int o3 = sgn_dd(orientq(P[2], P[3], P[0])), o4 = sgn_dd(orientq(P[2], P[3], P[1]));
  if (o1 * o2 < 0 && o3 * o4 < 0) return dd_of(0.0);
  return dd_min(dd_min(seg2q(P[0], P[2], P[3]), seg2q(P[1], P[2], P[3])), dd_min(seg2q(P[2], P[0], P[1]), seg2q(P[3], P[0], P[1])));
}

// Stencil pair with 0 < dbar < h in the same component (Sec. 3.2)?
__device__ __forceinline__ bool is_filtered(const SceneDev& S, int type, const int* v) {
  if (S.filter != 0) return false;
  if (S.comp[v[0]] != S.comp[v[2]]) return false;
  if (S.kind == 0) {
    double sa0 = S.ref[v[0]], sa1 = S.ref[v[1]], sb0 = S.ref[v[2]], sb1 = S.ref[v[3]];
    double gap = fmax(fmin(sb0, sb1) - fmax(sa0, sa1), fmin(sa0, sa1) - fmax(sb0, sb1));
    return gap > 0.0 && gap < S.h;
  }
  double h2 = S.h * S.h;
  double q = ref_sqdist_d(S, type, v);
  if (fabs(q - h2) > 1e-9 * h2 && q > 1e-9 * h2) return q < h2;
  dd qq = ref_sqdist_q(S, type, v);
  dd hh = dd_sq(S.h), m = dd_of(h2 * BFC_TIE);
  return dd_lt(m, qq) && dd_lt(qq, hh - m);
}

__global__ __launch_bounds__(256) void k_narrow(SceneDev S, const double* x, const int* ci, const int* cj,
                                                const unsigned char* ct, const long long* cand_count, long long ccap,
                                                int* ai, int* aj, unsigned char* at, unsigned char* acode,
                                                unsigned char* aflags, double* adist, long long acap,
                                                unsigned long long* act_count, unsigned long long* counters,
                                                unsigned* status) {
  long long n = *cand_count;
  if (n > ccap) n = ccap;
  const dd h2 = dd_sq(S.h), e2 = dd_sq(S.eta);
  for (long long base = (long long)blockIdx.x * blockDim.x; base < n; base += grid_stride()) {
    long long k = base + threadIdx.x;
    bool nc = false, filt = false, active = false, infeas = false;
    int type = 0, i = 0, j = 0, code = 0;
    double D = 0.0;
    if (k < n) {
      type = ct[k]; i = ci[k]; j = cj[k];
      int v[4];
      pair_verts(S, type, i, j, v);
      d3 P[4] = {load3(x, v[0]), load3(x, v[1]), load3(x, v[2]), load3(x, v[3])};
      Near nr = type == BF_PT ? classify_pt(P) : classify_ee(P);
      code = nr.code;
      D = nr.D;
      nc = decide_sq(code, P, D, h2, true);  // d < h
      if (nc) {
        filt = is_filtered(S, type, v);
        dd T;
        double eta;
        if (filt) {  // Eq. 4 second case: (d_min, 0)
          int c = S.comp[v[0]];
          T = dd{S.thr2[2 * c], S.thr2[2 * c + 1]};
          eta = 0.0;
        } else {     // Eq. 4 first case: (h, eta)
          T = h2;
          eta = S.eta;
        }
        active = decide_sq(code, P, D, T, true);  // Eq. 2: d < a
        if (active) infeas = eta > 0.0 ? decide_sq(code, P, D, e2, false) : !(D > 0.0);
      }
    }
    unsigned long long m_nc = __ballot(nc), m_f = __ballot(nc && filt), m_a = __ballot(active),
                       m_i = __ballot(infeas);
    if (lane_id() == 0) {
      if (m_nc) atomicAdd(&counters[0], (unsigned long long)__popcll(m_nc));
      if (m_f) atomicAdd(&counters[1], (unsigned long long)__popcll(m_f));
      if (m_a) atomicAdd(&counters[2], (unsigned long long)__popcll(m_a));
      if (m_i) {
        atomicAdd(&counters[3], (unsigned long long)__popcll(m_i));
        atomicOr(status, (unsigned)BF_S_INFEASIBLE);
      }
    }
    if (m_a) {
      int leader = __ffsll((long long)m_a) - 1;
      unsigned long long wb = 0;
      if (lane_id() == leader) wb = atomicAdd(act_count, (unsigned long long)__popcll(m_a));
      wb = __shfl(wb, leader, 64);
      if (active) {
        long long pos = (long long)wb + lanes_below(m_a);
        if (pos < acap) {
          ai[pos] = i; aj[pos] = j; at[pos] = (unsigned char)type;
          acode[pos] = (unsigned char)code;
          aflags[pos] = (unsigned char)((filt ? BF_F_FILTERED : 0) | (infeas ? BF_F_INFEASIBLE : 0));
          adist[pos] = sqrt(D);
        } else {
          atomicOr(status, (unsigned)BF_S_ACT_OVERFLOW);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Barrier evaluation (Eq. 2, Eq. 3) and PSD projection
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(128) void k_eval(SceneDev S, const double* x, const int* ai, const int* aj,
                                              const unsigned char* at, const unsigned char* acode,
                                              const unsigned char* aflags, const unsigned long long* act_count,
                                              long long acap, double* E, double* G, double* H) {
  long long n = (long long)*act_count;
  if (n > acap) n = acap;
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n; k += grid_stride()) {
    int type = at[k], code = acode[k], fl = aflags[k];
    int v[4];
    pair_verts(S, type, ai[k], aj[k], v);
    PairOut o;
    if (fl & BF_F_INFEASIBLE) {
      o.E = INFINITY;
#pragma unroll
      for (int q = 0; q < 12; ++q) o.G[q] = 0.0;
#pragma unroll
      for (int q = 0; q < 78; ++q) o.H[q] = 0.0;
    } else {
      d3 P[4] = {load3(x, v[0]), load3(x, v[1]), load3(x, v[2]), load3(x, v[3])};
      double a, eta;
      if (fl & BF_F_FILTERED) { a = S.dmin[S.comp[v[0]]]; eta = 0.0; }
      else { a = S.h; eta = S.eta; }
      eval_pair(P, code, a, eta, S.kappa, o);
    }
    E[k] = o.E;
#pragma unroll
    for (int q = 0; q < 12; ++q) G[12 * k + q] = o.G[q];
#pragma unroll
    for (int q = 0; q < 78; ++q) H[78 * k + q] = o.H[q];
  }
}

// ---------------------------------------------------------------------------
// Assembly
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_esum(const double* E, const unsigned long long* act_count, long long acap,
                                              double* part) {
  long long n = (long long)*act_count;
  if (n > acap) n = acap;
  double s = 0.0;
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n; k += grid_stride()) s += E[k];
  s = wave_sum(s);
  __shared__ double ws[4];
  if (lane_id() == 0) ws[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
}
__global__ __launch_bounds__(256) void k_esum_final(const double* part, int nparts, double* out) {
  double s = 0.0;
  for (int k = threadIdx.x; k < nparts; k += blockDim.x) s += part[k];
  s = wave_sum(s);
  __shared__ double ws[4];
  if (lane_id() == 0) ws[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *out = (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

__global__ __launch_bounds__(256) void k_grad(SceneDev S, const int* ai, const int* aj, const unsigned char* at,
                                              const unsigned char* aflags, const unsigned long long* act_count,
                                              long long acap, const double* G, double* g) {
  long long n = (long long)*act_count;
  if (n > acap) n = acap;
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n; k += grid_stride()) {
    if (aflags[k] & BF_F_INFEASIBLE) continue;
    int v[4];
    pair_verts(S, at[k], ai[k], aj[k], v);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        double val = G[12 * k + 3 * s + a];
        if (val != 0.0) unsafeAtomicAdd(&g[3 * v[s] + a], val);
      }
  }
}

__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
  z ^= z >> 33; z *= 0xff51afd7ed558ccdull;
  z ^= z >> 33; z *= 0xc4ceb9fe1a85ec53ull;
  z ^= z >> 33;
  return z;
}

// Insert the 16 (row, col) blocks of every feasible active pair; count new
// keys per row.
__global__ __launch_bounds__(256) void k_asm_insert(SceneDev S, const int* ai, const int* aj, const unsigned char* at,
                                                    const unsigned char* aflags,
                                                    const unsigned long long* act_count, long long acap,
                                                    unsigned long long* keys, long long hsize, int* entry_slot,
                                                    int* rowcnt, unsigned* status) {
  long long n = (long long)*act_count;
  if (n > acap) n = acap;
  unsigned long long mask = (unsigned long long)hsize - 1;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < 16 * n; e += grid_stride()) {
    long long k = e >> 4;
    int b = (int)(e & 15);
    if (aflags[k] & BF_F_INFEASIBLE) { entry_slot[e] = -1; continue; }
    int v[4];
    pair_verts(S, at[k], ai[k], aj[k], v);
    unsigned long long key = ((unsigned long long)(unsigned)v[b >> 2] << 32) | (unsigned)v[b & 3];
    unsigned long long h = mix64(key) & mask;
    int slot = -1;
    for (long long probe = 0; probe < hsize; ++probe) {
      unsigned long long prev = atomicCAS(&keys[h], kEmpty, key);
      if (prev == kEmpty) { slot = (int)h; atomicAdd(&rowcnt[v[b >> 2]], 1); break; }
      if (prev == key) { slot = (int)h; break; }
      h = (h + 1) & mask;
    }
    if (slot < 0) atomicOr(status, (unsigned)BF_S_HASH_OVERFLOW);
    entry_slot[e] = slot;
  }
}

__global__ void k_asm_nnzb(const int* row_ptr, int nv, long long* nnzb, long long cap, unsigned* status) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    long long t = row_ptr[nv];
    *nnzb = t;
    if (t > cap) atomicOr(status, (unsigned)BF_S_BSR_OVERFLOW);
  }
}

__global__ __launch_bounds__(256) void k_asm_fillseg(const unsigned long long* keys, long long hsize, const int* row_ptr,
                                                     int* rowfill, int* tmpcol, long long cap) {
  for (long long s = blockIdx.x * (long long)blockDim.x + threadIdx.x; s < hsize; s += grid_stride()) {
    unsigned long long key = keys[s];
    if (key == kEmpty) continue;
    int row = (int)(key >> 32);
    int pos = row_ptr[row] + atomicAdd(&rowfill[row], 1);
    if (pos < cap) tmpcol[pos] = (int)(key & 0xffffffffu);
  }
}

__global__ __launch_bounds__(256) void k_asm_rank(const unsigned long long* keys, long long hsize, const int* row_ptr,
                                                  const int* tmpcol, int* slot_pos, int* col_out, long long cap) {
  for (long long s = blockIdx.x * (long long)blockDim.x + threadIdx.x; s < hsize; s += grid_stride()) {
    unsigned long long key = keys[s];
    if (key == kEmpty) continue;
    int row = (int)(key >> 32), col = (int)(key & 0xffffffffu);
    int lo = row_ptr[row], hi = row_ptr[row + 1];
    if (hi > cap) { slot_pos[s] = -1; continue; }
    int rank = 0;
    for (int q = lo; q < hi; ++q) rank += tmpcol[q] < col ? 1 : 0;
    slot_pos[s] = lo + rank;
    col_out[lo + rank] = col;
  }
}

__global__ __launch_bounds__(256) void k_asm_vals(const unsigned long long* act_count, long long acap,
                                                  const unsigned char* aflags, const int* entry_slot,
                                                  const int* slot_pos, const double* H, double* val) {
  long long n = (long long)*act_count;
  if (n > acap) n = acap;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < 16 * n; e += grid_stride()) {
    int slot = entry_slot[e];
    if (slot < 0) continue;
    int pos = slot_pos[slot];
    if (pos < 0) continue;
    long long k = e >> 4;
    int b = (int)(e & 15), sr = b >> 2, sc = b & 3;
    const double* Hk = H + 78 * k;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        int I = 3 * sr + i, J = 3 * sc + j;
        double hv = I <= J ? Hk[hix(I, J)] : Hk[hix(J, I)];
        if (hv != 0.0) unsafeAtomicAdd(&val[9 * (long long)pos + 3 * i + j], hv);
      }
  }
}

// ---------------------------------------------------------------------------
// Precompute (Sec. 3.2): connected components and d_min
// ---------------------------------------------------------------------------
__global__ void k_cc_init(int* lab, int nv) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += grid_stride()) lab[v] = v;
}
__device__ __forceinline__ int cc_root(const int* lab, int v) {
  int r = lab[v];
  while (true) {
    int q = lab[r];
    if (q == r) return r;
    r = q;
  }
}
__device__ __forceinline__ void cc_link(int* lab, int a, int b, int* changed) {
  int ra = cc_root(lab, a), rb = cc_root(lab, b);
  if (ra == rb) return;
  int hi = max(ra, rb), lo = min(ra, rb);
  int old = atomicMin(&lab[hi], lo);
  if (old != lo) *changed = 1;
}
// link the roots of the endpoints of every edge and triangle (smaller root wins)
__global__ void k_cc_hook(const int* edges, int ne, const int* tris, int nt, int* lab, int* changed) {
  int total = ne + nt;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < total; k += grid_stride()) {
    if (k < ne) {
      cc_link(lab, edges[2 * k], edges[2 * k + 1], changed);
    } else {
      const int* t = tris + 3 * (k - ne);
      cc_link(lab, t[0], t[1], changed);
      cc_link(lab, t[0], t[2], changed);
    }
  }
}
__global__ void k_cc_compress(int* lab, int nv) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += grid_stride()) lab[v] = cc_root(lab, v);
}
__global__ void k_cc_isroot(const int* lab, int nv, int* flag) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += grid_stride()) flag[v] = lab[v] == v ? 1 : 0;
}
__global__ void k_cc_label(const int* lab, const int* scan, int nv, int* comp) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += grid_stride()) comp[v] = scan[lab[v]];
}

// Minimum reference distance per component over stencil pairs with 0 < dbar < h.
// Rods: the gap (one double subtraction); shells: dbar^2 in double-double,
// rounded to double.  Non-negative doubles order like their bit patterns.
__global__ __launch_bounds__(256) void k_refmin(SceneDev S, const int* ci, const int* cj, const unsigned char* ct,
                                                const long long* count, long long cap, unsigned long long* best) {
  long long n = *count;
  if (n > cap) n = cap;
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n; k += grid_stride()) {
    int v[4];
    pair_verts(S, ct[k], ci[k], cj[k], v);
    if (S.comp[v[0]] != S.comp[v[2]]) continue;
    double val;
    if (S.kind == 0) {
      double sa0 = S.ref[v[0]], sa1 = S.ref[v[1]], sb0 = S.ref[v[2]], sb1 = S.ref[v[3]];
      double gap = fmax(fmin(sb0, sb1) - fmax(sa0, sa1), fmin(sa0, sa1) - fmax(sb0, sb1));
      if (!(gap > 0.0 && gap < S.h)) continue;
      val = gap;
    } else {
      dd q = ref_sqdist_q(S, ct[k], v);
      if (!(dd_lt(dd_of(0.0), q) && dd_lt(q, dd_sq(S.h)))) continue;
      val = q.hi + q.lo;  // round to nearest double
    }
    atomicMin(&best[S.comp[v[0]]], (unsigned long long)__double_as_longlong(val));
  }
}

}  // namespace bfc

// ===========================================================================
// Host-side launchers
// ===========================================================================
namespace bfc {

static inline int nblocks(long long n, int bs = 256, int cap = 8192) {
  long long b = (n + bs - 1) / bs;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

__global__ void k_lift_ref(SceneDev S, double* xr) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < S.nv; v += grid_stride()) {
    if (S.kind == 0) { xr[3 * v] = S.ref[v]; xr[3 * v + 1] = 0.0; }
    else { xr[3 * v] = S.ref[2 * v]; xr[3 * v + 1] = S.ref[2 * v + 1]; }
    xr[3 * v + 2] = 0.0;
  }
}

__global__ void k_zero_ll(long long* a, int n, long long* b, int m) {
  if (threadIdx.x < n) a[threadIdx.x] = 0;
  if (b && threadIdx.x < m) b[threadIdx.x] = 0;
}

void run_lift_ref(const SceneDev& S, double* xref, hipStream_t st) {
  hipLaunchKernelGGL(k_lift_ref, dim3(nblocks(S.nv)), dim3(256), 0, st, S, xref);
}

void run_broad(const SceneDev& S, const double* x, const BroadWs& W, int* oi, int* oj, unsigned char* ot,
               long long cap, long long* count, unsigned* status, hipStream_t st) {
  int np = S.ne + S.nt + (S.kind == 1 ? S.nv : 0);
  int nstored = S.ne + S.nt;
  int nquery = S.kind == 1 ? S.nv + S.ne : S.ne;
  int nscan_max = 2 * W.max_cells + 1;
  const int* nscan_dev = &W.grid->nscan;
  hipLaunchKernelGGL(k_begin, dim3(1), dim3(64), 0, st, W.bounds, count);
  hipLaunchKernelGGL(k_bounds, dim3(nblocks(np)), dim3(256), 0, st, S, x, np, W.box, W.bounds);
  hipLaunchKernelGGL(k_grid, dim3(1), dim3(64), 0, st, W.bounds, S.h, W.max_cells, W.grid);
  hipLaunchKernelGGL(k_zero_i, dim3(nblocks(nscan_max)), dim3(256), 0, st, W.cell_cnt, nscan_dev, 0LL);
  hipLaunchKernelGGL(k_count, dim3(nblocks(nstored)), dim3(256), 0, st, nstored, S.ne, W.box, W.grid, W.cell_cnt,
                     W.cell_of);
  scan_excl(W.cell_cnt, W.cell_start, nscan_dev, nscan_max, W.scan_tmp, st);
  hipLaunchKernelGGL(k_scatter, dim3(nblocks(nstored)), dim3(256), 0, st, nstored, W.box, W.cell_of, W.cell_cnt,
                     W.cell_start, W.sorted_id, W.sorted_box);
  hipLaunchKernelGGL(k_pairs, dim3(nblocks(nquery)), dim3(256), 0, st, S, nquery, W.box, W.grid, W.cell_start,
                     W.sorted_id, W.sorted_box, S.h, oi, oj, ot, cap, (unsigned long long*)count,
                     status);
}

void run_narrow(const SceneDev& S, const double* x, const int* ci, const int* cj, const unsigned char* ct,
                const long long* ccount, long long ccap, int* ai, int* aj, unsigned char* at, unsigned char* acode,
                unsigned char* aflags, double* adist, long long acap, long long* act_count, long long* counters,
                unsigned* status, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_ll, dim3(1), dim3(64), 0, st, act_count, 1, counters, 4);
  hipLaunchKernelGGL(k_narrow, dim3(nblocks(ccap)), dim3(256), 0, st, S, x, ci, cj, ct, ccount, ccap, ai, aj, at,
                     acode, aflags, adist, acap, (unsigned long long*)act_count, (unsigned long long*)counters,
                     status);
}

void run_eval(const SceneDev& S, const double* x, const int* ai, const int* aj, const unsigned char* at,
              const unsigned char* acode, const unsigned char* aflags, const long long* act_count, long long acap,
              double* E, double* G, double* H, hipStream_t st) {
  hipLaunchKernelGGL(k_eval, dim3(nblocks(acap, 128, 16384)), dim3(128), 0, st, S, x, ai, aj, at, acode, aflags,
                     (const unsigned long long*)act_count, acap, E, G, H);
}

void run_assemble(const SceneDev& S, const int* ai, const int* aj, const unsigned char* at,
                  const unsigned char* aflags, const long long* act_count, long long acap, const double* E,
                  const double* G, const double* H, double* E_out, double* g, int* row_ptr, int* col, double* val,
                  long long bsr_cap, long long* nnzb, const AsmWs& A, long long act_cap_ws, unsigned* status,
                  hipStream_t st) {
  const unsigned long long* nact = (const unsigned long long*)act_count;
  long long n16 = 16 * acap;
  hipLaunchKernelGGL(k_esum, dim3(256), dim3(256), 0, st, E, nact, acap, A.epart);
  hipLaunchKernelGGL(k_esum_final, dim3(1), dim3(256), 0, st, A.epart, 256, E_out);
  hipLaunchKernelGGL(k_zero_d, dim3(nblocks(3LL * S.nv)), dim3(256), 0, st, g, (const long long*)nullptr,
                     3LL * S.nv, 1LL, 3LL * S.nv);
  hipLaunchKernelGGL(k_grad, dim3(nblocks(acap)), dim3(256), 0, st, S, ai, aj, at, aflags, nact, acap, G, g);
  hipLaunchKernelGGL(k_fill_u64, dim3(nblocks(A.hash_size)), dim3(256), 0, st, A.keys, A.hash_size, kEmpty);
  hipLaunchKernelGGL(k_zero_i, dim3(nblocks(S.nv + 1)), dim3(256), 0, st, A.rowcnt, (const int*)nullptr,
                     (long long)S.nv + 1);
  hipLaunchKernelGGL(k_zero_i, dim3(nblocks(S.nv)), dim3(256), 0, st, A.rowfill, (const int*)nullptr,
                     (long long)S.nv);
  hipLaunchKernelGGL(k_asm_insert, dim3(nblocks(n16)), dim3(256), 0, st, S, ai, aj, at, aflags, nact, acap, A.keys,
                     A.hash_size, A.entry_slot, A.rowcnt, status);
  scan_excl(A.rowcnt, row_ptr, nullptr, S.nv + 1, A.scan_tmp, st);
  hipLaunchKernelGGL(k_asm_nnzb, dim3(1), dim3(64), 0, st, row_ptr, S.nv, nnzb, bsr_cap, status);
  hipLaunchKernelGGL(k_asm_fillseg, dim3(nblocks(A.hash_size)), dim3(256), 0, st, A.keys, A.hash_size, row_ptr,
                     A.rowfill, A.tmpcol, 16 * act_cap_ws);
  hipLaunchKernelGGL(k_asm_rank, dim3(nblocks(A.hash_size)), dim3(256), 0, st, A.keys, A.hash_size, row_ptr,
                     A.tmpcol, A.slot_pos, col, bsr_cap);
  hipLaunchKernelGGL(k_zero_d, dim3(nblocks(9 * bsr_cap)), dim3(256), 0, st, val, (const long long*)nnzb, 0LL, 9LL,
                     bsr_cap);
  hipLaunchKernelGGL(k_asm_vals, dim3(nblocks(n16)), dim3(256), 0, st, nact, acap, aflags, A.entry_slot, A.slot_pos,
                     H, val);
}

int run_components(const SceneDev& S, int* lab, int* flag, int* scan, int* comp, int* scan_tmp, int* d_changed,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_cc_init, dim3(nblocks(S.nv)), dim3(256), 0, st, lab, S.nv);
  for (int it = 0; it < 4096; ++it) {
    hipLaunchKernelGGL(k_zero_i, dim3(1), dim3(64), 0, st, d_changed, (const int*)nullptr, 1LL);
    hipLaunchKernelGGL(k_cc_hook, dim3(nblocks(S.ne + S.nt)), dim3(256), 0, st, S.edges, S.ne, S.tris, S.nt, lab,
                       d_changed);
    hipLaunchKernelGGL(k_cc_compress, dim3(nblocks(S.nv)), dim3(256), 0, st, lab, S.nv);
    int h_changed = 0;
    if (hipMemcpyAsync(&h_changed, d_changed, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess) return -1;
    if (hipStreamSynchronize(st) != hipSuccess) return -1;
    if (!h_changed) break;
  }
  hipLaunchKernelGGL(k_cc_isroot, dim3(nblocks(S.nv)), dim3(256), 0, st, lab, S.nv, flag);
  scan_excl(flag, scan, nullptr, S.nv, scan_tmp, st);
  hipLaunchKernelGGL(k_cc_label, dim3(nblocks(S.nv)), dim3(256), 0, st, lab, scan, S.nv, comp);
  int last_scan = 0, last_flag = 0;
  if (hipMemcpyAsync(&last_scan, scan + S.nv - 1, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess) return -1;
  if (hipMemcpyAsync(&last_flag, flag + S.nv - 1, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess) return -1;
  if (hipStreamSynchronize(st) != hipSuccess) return -1;
  return last_scan + last_flag;
}

void run_refmin(const SceneDev& S, const int* ci, const int* cj, const unsigned char* ct, const long long* count,
                long long cap, unsigned long long* best, hipStream_t st) {
  hipLaunchKernelGGL(k_refmin, dim3(nblocks(cap)), dim3(256), 0, st, S, ci, cj, ct, count, cap, best);
}

}  // namespace bfc
