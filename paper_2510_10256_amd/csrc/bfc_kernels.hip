// Kernels of libbfc (gfx950, wave64).
//
//   broad phase   : k_bounds, k_count, scan, k_scatter, k_cell_order, k_pair_count, k_pair_emit
//   narrow phase  : k_narrow, scan, k_compact (distance, filter of Eq. 4, exact thresholds,
//                   ballot compaction by distance kind)
//   evaluation    : k_eval        (Eq. 2/3 barrier, derivatives, PSD projection)
//   assembly      : k_inc_count (with the energy partials), scan, k_inc_fill,
//                   k_row_a / k_row_a_big, scan, k_row_b / k_row_b_big
//   precompute    : k_cc_*, k_refmin (components and d_min, Sec. 3.2)
#include <algorithm>
#include <type_traits>

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

// Sum across the wave in a fixed order (lane i adds lane i + o); lane 0 has the total.
__device__ __forceinline__ void wave_ordered_sum3(double& x, double& y, double& z) {
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    double tx = __shfl_down(x, o, 64), ty = __shfl_down(y, o, 64), tz = __shfl_down(z, o, 64);
    if ((lane & (2 * o - 1)) == 0) { x += tx; y += ty; z += tz; }
  }
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

// sum across a block of 256 threads (4 waves); every thread gets the total
__device__ __forceinline__ long long block_sum256(long long v) {
  __shared__ long long ws[4];
  v = wave_sum(v);
  if (lane_id() == 0) ws[threadIdx.x >> 6] = v;
  __syncthreads();
  long long t = (ws[0] + ws[1]) + (ws[2] + ws[3]);
  __syncthreads();
  return t;
}

// ---------------------------------------------------------------------------
// device-wide exclusive scan of int32; n = n_dev ? *n_dev : n_const: one
// work-group (k_scan1), one pass (k_scan_lb) or, for more than SCAN_LB_TILES
// tiles, three kernels (tile totals, their scan, down-sweep)
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

// Single-pass exclusive scan of at most SCAN_LB_TILES tiles.  A work-group
// takes its tile from a ticket when it starts, publishes the tile's total,
// then reads the totals of all earlier tiles at once (one thread a tile) and
// adds them.  It only ever waits on tiles whose work-groups started before
// it, and those publish before they wait on anything: every wait ends.  The
// total and its "published" flag share one 64-bit word, written and read
// with device-scope atomics (no other data passes between work-groups, so
// no release or acquire is needed).  The last work-group to finish clears the
// words and the counters for the next scan.  The poll is bounded all the
// same (max_polls loads): a total still missing then is summed from the
// input tile by the waiting thread itself, so the scan stays exact, and
// BF_S_SCAN_SLOW is raised in the status word.
__global__ __launch_bounds__(256) void k_scan_lb(const int* in, int* out, const int* n_dev, int n_const,
                                                 int* state, int max_polls, unsigned* status) {
  unsigned long long* word = (unsigned long long*)state;  // [SCAN_LB_TILES] 1 << 32 | total
  unsigned* ctr = (unsigned*)(state + 2 * SCAN_LB_TILES);  // ticket, done
  __shared__ int s_tile;
  const int n = n_dev ? *n_dev : n_const;
  if (threadIdx.x == 0) s_tile = (int)atomicAdd(&ctr[0], 1u);
  __syncthreads();
  const int tile = s_tile, base = tile * SCAN_TILE;
  int v[SCAN_ITEMS];
  int s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    int i = base + threadIdx.x * SCAN_ITEMS + k;
    v[k] = i < n ? in[i] : 0;
    s += v[k];
  }
  int tot;
  const int excl = block_excl_scan256(s, &tot);
  if (threadIdx.x == 0)
    __hip_atomic_store(&word[tile], (1ull << 32) | (unsigned)tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  int earlier = 0;
  if ((int)threadIdx.x < tile) {
    unsigned long long w = 0;
    for (int polls = 0; polls < max_polls; ++polls) {
      w = __hip_atomic_load(&word[threadIdx.x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if ((w >> 32) != 0) break;
    }
    if ((w >> 32) != 0) {
      earlier = (int)(unsigned)w;
    } else {  // not published within the bound: sum that tile of the input here
      const int b0 = threadIdx.x * SCAN_TILE, b1 = min(n, b0 + SCAN_TILE);
      for (int i = b0; i < b1; ++i) earlier += in[i];
      if (status) atomicOr(status, (unsigned)BF_S_SCAN_SLOW);
    }
  }
  int run = excl + (int)block_sum256(earlier);
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    int i = base + threadIdx.x * SCAN_ITEMS + k;
    if (i < n) out[i] = run;
    run += v[k];
  }
  if (threadIdx.x == 0) {  // after the block sum: this work-group has read every word it needs
    const unsigned d = __hip_atomic_fetch_add(&ctr[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (d == gridDim.x - 1) {
      for (int j = 0; j < (int)gridDim.x; ++j) word[j] = 0ull;
      ctr[0] = 0u;
      ctr[1] = 0u;
    }
  }
}

// one work-group scan for short arrays (n <= SCAN1_MAX)
__global__ __launch_bounds__(1024) void k_scan1(const int* in, int* out, const int* n_dev, int n_const) {
  int n = n_dev ? *n_dev : n_const;
  __shared__ int ws[16];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < n; base += 1024 * SCAN_ITEMS) {
    int v[SCAN_ITEMS];
    int s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
      int i = base + threadIdx.x * SCAN_ITEMS + k;
      v[k] = i < n ? in[i] : 0;
      s += v[k];
    }
    int x = wave_incl_scan(s);
    int w = threadIdx.x >> 6;
    if (lane_id() == 63) ws[w] = x;
    __syncthreads();
    int off = 0, tot = 0;
    for (int k = 0; k < 16; ++k) {
      if (k < w) off += ws[k];
      tot += ws[k];
    }
    int run = carry + off + x - s;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
      int i = base + threadIdx.x * SCAN_ITEMS + k;
      if (i < n) out[i] = run;
      run += v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) carry += tot;
    __syncthreads();
  }
}

int g_scan_polls = 1 << 22;

void scan_excl(const int* in, int* out, const int* n_dev, int n_max, int* tmp, unsigned* status, hipStream_t st) {
  if (n_max <= SCAN1_MAX) {
    hipLaunchKernelGGL(k_scan1, dim3(1), dim3(1024), 0, st, in, out, n_dev, n_max);
    return;
  }
  int nb = (n_max + SCAN_TILE - 1) / SCAN_TILE;
  if (nb < 1) nb = 1;
  if (nb <= SCAN_LB_TILES) {
    hipLaunchKernelGGL(k_scan_lb, dim3(nb), dim3(256), 0, st, in, out, n_dev, n_max, tmp, g_scan_polls, status);
    return;
  }
  int* part = tmp + SCAN_LB_STATE;
  hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(256), 0, st, in, n_dev, n_max, part);
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, st, part, n_dev, n_max);
  hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(256), 0, st, in, out, n_dev, n_max, part);
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

// Grid parameters from the scene bounds and the largest primitive box side.
__device__ void make_grid(const float* lo_f, const float* hi_f, float ext_f, double h, int max_cells, Grid* g) {
  double lo[3], hi[3], span[3], amax = 0.0;
  for (int a = 0; a < 3; ++a) {
    lo[a] = (double)lo_f[a];
    hi[a] = (double)hi_f[a];
    if (!(hi[a] >= lo[a])) { lo[a] = 0.0; hi[a] = 0.0; }
    span[a] = hi[a] - lo[a];
    amax = fmax(amax, fmax(fabs(lo[a]), fabs(hi[a])));
  }
  double ext = (double)ext_f;
  if (!(ext >= 0.0)) ext = 0.0;
  // cell side 0.7 (largest side + h): measured against 0.25 to 2 (the
  // rows a query visits against the primitives it tests)
  double cell = 0.7 * (ext + h) + 1e-6 * (1.0 + amax);
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
  // centre reach: h (and the exact test's slack) + half the largest side
  g->reach = h + 0.5 * ext + 1e-9 * (1.0 + amax + ext + h);
  // float prefilter bound: a float gap g > gapf has an exact gap of at least
  // g (1 - 2^-24) > h + 1e-15 |coordinates|
  g->gapf = __double2float_ru(h * (1.0 + 1e-6) + 2e-15 * amax);
  for (int a = 0; a < 3; ++a) { g->n[a] = (int)n[a]; g->orgd[a] = lo[a]; }
  g->ncells = (int)tot;
  g->nscan = 2 * (int)tot + 1;
  g->coarsened = coarse;
}

// Boxes of all primitives (FP32, rounded outward; with pdisp, the boxes of
// the straight sweep from x to x + pdisp) and, in the last block to finish,
// the reduction of the per-block bounds and the grid parameters.
// The last block also clears the candidate counter of this step.
__global__ __launch_bounds__(256) void k_bounds(SceneDev S, const double* x, const double* pdisp, int np, Box* box,
                                                float* part, unsigned* done, double h, int max_cells, Grid* grid,
                                                long long* cand_count) {
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY}, ext = 0.0f;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < np; p += grid_stride()) {
    int v[3];
    int nvx = prim_verts(S, p, v);
    double l[3] = {INFINITY, INFINITY, INFINITY}, hh[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int k = 0; k < nvx; ++k)
      for (int a = 0; a < 3; ++a) {
        double c = x[3 * v[k] + a];
        l[a] = fmin(l[a], c);
        hh[a] = fmax(hh[a], c);
        if (pdisp) {  // swept box: the vertex at x and at x + p
          const double ce = c + pdisp[3 * v[k] + a];
          l[a] = fmin(l[a], ce);
          hh[a] = fmax(hh[a], ce);
        }
      }
    Box b;
    for (int a = 0; a < 3; ++a) {
      b.lo[a] = __double2float_rd(l[a]);
      b.hi[a] = __double2float_ru(hh[a]);
      lo[a] = fminf(lo[a], b.lo[a]);
      hi[a] = fmaxf(hi[a], b.hi[a]);
      ext = fmaxf(ext, __double2float_ru((double)b.hi[a] - (double)b.lo[a]));
    }
    box[p] = b;
  }
  __shared__ float red[4][7];
  __shared__ int last;
  for (int o = 32; o > 0; o >>= 1) {
    for (int a = 0; a < 3; ++a) {
      lo[a] = fminf(lo[a], __shfl_xor(lo[a], o, 64));
      hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], o, 64));
    }
    ext = fmaxf(ext, __shfl_xor(ext, o, 64));
  }
  int w = threadIdx.x >> 6;
  if (lane_id() == 0) {
    for (int a = 0; a < 3; ++a) { red[w][a] = lo[a]; red[w][3 + a] = hi[a]; }
    red[w][6] = ext;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float r[7];
    for (int a = 0; a < 7; ++a) r[a] = red[0][a];
    for (int k = 1; k < 4; ++k) {
      for (int a = 0; a < 3; ++a) { r[a] = fminf(r[a], red[k][a]); r[3 + a] = fmaxf(r[3 + a], red[k][3 + a]); }
      r[6] = fmaxf(r[6], red[k][6]);
    }
    for (int a = 0; a < 7; ++a) part[8 * blockIdx.x + a] = r[a];
    __threadfence();
    last = atomicAdd(done, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!last) return;
  // last block: reduce the partials of all blocks (one per thread, then a
  // wave reduction and a 4-wave combine)
  __threadfence();
  float r[7] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY, 0.0f};
  const volatile float* vp = part;
  for (unsigned b = threadIdx.x; b < gridDim.x; b += blockDim.x) {
    for (int a = 0; a < 3; ++a) { r[a] = fminf(r[a], vp[8 * b + a]); r[3 + a] = fmaxf(r[3 + a], vp[8 * b + 3 + a]); }
    r[6] = fmaxf(r[6], vp[8 * b + 6]);
  }
  for (int o = 32; o > 0; o >>= 1) {
    for (int a = 0; a < 3; ++a) {
      r[a] = fminf(r[a], __shfl_xor(r[a], o, 64));
      r[3 + a] = fmaxf(r[3 + a], __shfl_xor(r[3 + a], o, 64));
    }
    r[6] = fmaxf(r[6], __shfl_xor(r[6], o, 64));
  }
  __syncthreads();
  if (lane_id() == 0)
    for (int a = 0; a < 7; ++a) red[w][a] = r[a];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < 4; ++k) {
      for (int a = 0; a < 3; ++a) { r[a] = fminf(r[a], red[k][a]); r[3 + a] = fmaxf(r[3 + a], red[k][3 + a]); }
      r[6] = fmaxf(r[6], red[k][6]);
    }
    make_grid(r, r + 3, r[6], h, max_cells, grid);
    if (cand_count) *cand_count = 0;
    *done = 0u;
  }
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
__device__ __forceinline__ int clamp_cell(double q, int n) { return q >= 0.0 ? (q < (double)n ? (int)q : n - 1) : 0; }
// Cells of the box centres within reach of box b (the same rounding steps
// as cell_coords, which keeps the range a superset).
__device__ __forceinline__ void cell_range(const Grid& g, const Box& b, int* lo, int* hi) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lo[a] = clamp_cell(floor(((double)b.lo[a] - g.reach - g.orgd[a]) / g.cell), g.n[a]);
    hi[a] = max(lo[a], clamp_cell(floor(((double)b.hi[a] + g.reach - g.orgd[a]) / g.cell), g.n[a]));
  }
}

__global__ __launch_bounds__(256) void k_count(int nstored, int ne, const Box* box, const Grid* gp, int* cell_cnt,
                                               int* cell_of, unsigned long long* seg_count) {
  Grid g = *gp;
  if (blockIdx.x == 0 && threadIdx.x == 0) *seg_count = 0;  // segments of this step's count pass
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < nstored; p += grid_stride()) {
    int c[3];
    cell_coords(g, box[p], c);
    int sub = cell_lin(g, c[0], c[1], c[2]) + (p >= ne ? g.ncells : 0);
    cell_of[p] = sub;
    atomicAdd(&cell_cnt[sub], 1);
  }
}

__global__ __launch_bounds__(256) void k_scatter(int nstored, const Box* box, const int* cell_of, int* cell_cnt,
                                                 const int* cell_start, int* placed_id, Box* placed_box) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < nstored; p += grid_stride()) {
    int sub = cell_of[p];
    int pos = cell_start[sub] + atomicSub(&cell_cnt[sub], 1) - 1;
    placed_id[pos] = p;
    placed_box[pos] = box[p];
  }
}

// The scatter's atomics leave the entries of a cell in arbitrary order; each
// entry's rank among the cell's ids puts them in id order, so candidate
// lists, and every result downstream, are the same from run to run.
// Beside each entry go its vertex ids (edges: v0, v1, -1; triangles: t0, t1,
// t2), which the pair search's incidence test reads with the box instead of
// gathering them from the topology.
__global__ __launch_bounds__(256) void k_cell_order(SceneDev S, int nstored, const int* cell_of,
                                                    const int* cell_start, const int* placed_id,
                                                    const Box* placed_box, int* sorted_id, Box* sorted_box,
                                                    int4* sorted_vid) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nstored; k += grid_stride()) {
    const int p = placed_id[k], sub = cell_of[p];
    const int b = cell_start[sub], e = cell_start[sub + 1];
    int r = 0;
    for (int q = b; q < e; ++q) r += placed_id[q] < p;
    sorted_id[b + r] = p;
    sorted_box[b + r] = placed_box[k];
    if (p < S.ne) {
      sorted_vid[b + r] = make_int4(S.edges[2 * p], S.edges[2 * p + 1], -1, 0);
    } else {
      const int t = p - S.ne;
      sorted_vid[b + r] = make_int4(S.tris[3 * t], S.tris[3 * t + 1], S.tris[3 * t + 2], 0);
    }
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

// Euclidean distance between the boxes at or beyond h: the primitives they
// contain are at least that far apart, so the pair is not a candidate.  The
// gaps come from the float bounds in FP64 and their squares are summed there;
// the relative margin of 1e-9 covers every rounding, so a pair is rejected
// only when its boxes are truly h apart or more (boxes_near, the per-axis
// test, runs first).
__device__ __forceinline__ bool boxes_far_l2(const Box& a, const Box& b, double h) {
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double g = fmax(0.0, fmax((double)b.lo[k] - (double)a.hi[k], (double)a.lo[k] - (double)b.hi[k]));
    s += g * g;
  }
  return s > h * h * (1.0 + 1e-9);
}

// Float gap above gapf on some axis: the exact test below fails too.  (NaN
// gaps compare false and go on to the exact test.)
__device__ __forceinline__ bool boxes_far_f(const Box& a, const Box& b, float gapf) {
#pragma unroll
  for (int k = 0; k < 3; ++k)
    if (fmaxf(b.lo[k] - a.hi[k], a.lo[k] - b.hi[k]) > gapf) return true;
  return false;
}

// Visit the stored primitives of the sub-list for the query (triangles for a
// point, edges with a larger id for an edge) in the rows (y, z) = sub,
// sub + PQ, ... of the query's cell range, each row one contiguous run of
// cells along x; count every non-incident pair whose boxes are within h,
// and stage it (its stored id at stage[256 * n] while n < STAGE_K) or emit
// it at `pos`.
constexpr int VISIT_COUNT = 0, VISIT_STAGE = 1, VISIT_EMIT = 2;
constexpr int STAGE_K = 24;  // candidates a count-pass thread keeps in LDS (24 KiB a work-group: six waves per SIMD)
template <int PQ, int MODE>
__device__ __forceinline__ int visit_pairs(const SceneDev& S, const Grid& g, const int* cell_start,
                                           const int* sorted_id, const Box* sorted_box, const int4* sorted_vid,
                                           double hf, bool l2, int qtype,
                                           int qid, const Box& qb, const int* qv, int sub, long long pos,
                                           long long cap, int* oi, int* oj, unsigned char* ot, unsigned* status) {
  int lo[3], hi[3];
  cell_range(g, qb, lo, hi);
  const int ny = hi[1] - lo[1] + 1, nrow = ny * (hi[2] - lo[2] + 1);
  const int base = qtype == BF_PT ? g.ncells : 0;
  int cnt = 0;
  // the PQ threads of the query take the stored primitives of every row in
  // turn (thread sub: the row's sub-th, (sub + PQ)-th, ...), so that their
  // loads are neighbours and their work is even
  for (int row = 0; row < nrow; ++row) {
    const int cy = lo[1] + row % ny, cz = lo[2] + row / ny;
    const int l0 = base + cell_lin(g, lo[0], cy, cz);
    const int b = cell_start[l0], e = cell_start[l0 + hi[0] - lo[0] + 1];
    for (int k = b + sub; k < e; k += PQ) {
      int r = sorted_id[k];
      if (qtype == BF_EE && r <= qid) continue;
      const Box rb = sorted_box[k];
      if (boxes_far_f(qb, rb, g.gapf) || !boxes_near(qb, rb, hf) || (l2 && boxes_far_l2(qb, rb, hf))) continue;
      const int4 rv = sorted_vid[k];
      if (qtype == BF_EE) {
        if (rv.x == qv[0] || rv.x == qv[1] || rv.y == qv[0] || rv.y == qv[1]) continue;
      } else {
        if (rv.x == qid || rv.y == qid || rv.z == qid) continue;
        r -= S.ne;
      }
      if (MODE == VISIT_STAGE && cnt < STAGE_K) oi[256 * cnt] = r;
      if (MODE == VISIT_EMIT) {
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

__device__ __forceinline__ void query_of(const SceneDev& S, const Box* box, int q, int& qtype, int& qid, Box& qb,
                                         int* qv) {
  if (S.kind == 1 && q < S.nv) {  // point query against triangles
    qtype = BF_PT;
    qid = q;
    qb = box[S.ne + S.nt + q];
    qv[0] = qv[1] = -1;
  } else {                         // edge query against edges with a larger id
    qtype = BF_EE;
    qid = S.kind == 1 ? q - S.nv : q;
    qb = box[qid];
    qv[0] = S.edges[2 * qid];
    qv[1] = S.edges[2 * qid + 1];
  }
}

// (type, id) of query q: points first for shells, then edges
__device__ __forceinline__ void query_id(const SceneDev& S, int q, int& qtype, int& qid) {
  if (S.kind == 1 && q < S.nv) { qtype = BF_PT; qid = q; }
  else { qtype = BF_EE; qid = S.kind == 1 ? q - S.nv : q; }
}

// Pass 1: pair count of every (query, share of its cells) thread and the total of
// each work-group in bsum[block] (bsum[nblocks] = 0).  The pairs are staged
// in LDS; the group takes a segment of seg_r / seg_t (one atomic per group,
// in any order) and stores there, coalesced, the pairs of its threads that
// found at most STAGE_K: stored id, and thread | index << 8.  bseg[block] =
// the segment's start, or -1 when there was no room (pass 2 then visits
// the cells of every thread again, as it does for threads over STAGE_K).
template <int PQ>
__global__ __launch_bounds__(256) void k_pair_count(SceneDev S, int nquery, const Box* box, const Grid* gp,
                                                    const int* cell_start, const int* sorted_id, const Box* sorted_box,
                                                    const int4* sorted_vid,
                                                    double hf, bool l2, int* cnt, int* bsum, long long* bseg,
                                                    unsigned long long* seg_count, int* seg_r, unsigned* seg_t,
                                                    long long seg_cap) {
  __shared__ int stage[STAGE_K * 256];
  __shared__ int locs[256];
  __shared__ long long s_seg;
  Grid g = *gp;
  int nt = nquery * PQ;
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  int c = 0;
  if (t < nt) {
    int qtype, qid, qv[2];
    Box qb;
    query_of(S, box, t / PQ, qtype, qid, qb, qv);
    c = visit_pairs<PQ, VISIT_STAGE>(S, g, cell_start, sorted_id, sorted_box, sorted_vid, hf, l2, qtype, qid, qb, qv,
                                     t % PQ, 0, 0,
                                     stage + threadIdx.x, nullptr, nullptr, nullptr);
    cnt[t] = c;
  }
  int tot, stot;
  block_excl_scan256(c, &tot);
  const int ks = c <= STAGE_K ? c : 0;  // staged pairs of this thread
  locs[threadIdx.x] = block_excl_scan256(ks, &stot);
  if (threadIdx.x == 0) {
    long long sg = -1;
    if (stot == 0) {
      sg = 0;
    } else if (seg_r != nullptr) {
      const unsigned long long a = atomicAdd(seg_count, (unsigned long long)stot);
      if ((long long)a + stot <= seg_cap) sg = (long long)a;
    }
    s_seg = sg;
    bsum[blockIdx.x] = tot;
    bseg[blockIdx.x] = sg;
    if (blockIdx.x == 0) bsum[gridDim.x] = 0;
  }
  __syncthreads();
  const long long sg = s_seg;
  if (sg < 0) return;
  for (int q = threadIdx.x; q < stot; q += 256) {
    int lo = 0, hi = 255;  // the thread that staged pair q: the last u with locs[u] <= q
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (locs[mid] <= q) lo = mid; else hi = mid - 1;
    }
    const int k = q - locs[lo];
    seg_r[sg + q] = stage[256 * k + lo];
    seg_t[sg + q] = (unsigned)lo | ((unsigned)k << 8);
  }
}

// Pass 2: the group's offset (the scan of the count pass's group totals)
// plus, per thread, an in-group scan; output in query-major order (no
// atomics).  The
// group copies its segment (coalesced); threads whose pairs are not in it
// visit their cells again.
template <int PQ>
__global__ __launch_bounds__(256) void k_pair_emit(SceneDev S, int nquery, const Box* box, const Grid* gp,
                                                   const int* cell_start, const int* sorted_id, const Box* sorted_box,
                                                   const int4* sorted_vid,
                                                   double hf, bool l2, const int* cnt, const int* bofs,
                                                   const long long* bseg,
                                                   const int* seg_r, const unsigned* seg_t, int* oi, int* oj,
                                                   unsigned char* ot, long long cap, long long* count,
                                                   unsigned* status) {
  __shared__ int locs[256];
  Grid g = *gp;
  int nt = nquery * PQ;
  // this block's offset: the exclusive scan of the count pass's block totals
  // (its last entry, the candidate count, is written by block 0)
  if (blockIdx.x == 0 && threadIdx.x == 0) *count = bofs[gridDim.x];
  const long long base = bofs[blockIdx.x];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = t < nt ? cnt[t] : 0;
  const int loc = block_excl_scan256(c, nullptr);
  int stot;
  block_excl_scan256(c <= STAGE_K ? c : 0, &stot);
  locs[threadIdx.x] = loc;
  __syncthreads();
  const long long sg = bseg[blockIdx.x];
  if (sg >= 0) {
    for (int q = threadIdx.x; q < stot; q += 256) {
      const unsigned w = seg_t[sg + q];
      const int u = (int)(w & 255u);
      const long long p = base + locs[u] + (int)(w >> 8);
      if (p >= cap) {
        atomicOr(status, (unsigned)BF_S_CAND_OVERFLOW);
        continue;
      }
      int qtype, qid;
      query_id(S, (int)(((long long)blockIdx.x * 256 + u) / PQ), qtype, qid);
      oi[p] = qid;
      oj[p] = seg_r[sg + q];
      ot[p] = (unsigned char)qtype;
    }
  }
  if (c == 0 || (sg >= 0 && c <= STAGE_K)) return;
  int qtype, qid, qv[2];
  Box qb;
  query_of(S, box, t / PQ, qtype, qid, qb, qv);
  visit_pairs<PQ, VISIT_EMIT>(S, g, cell_start, sorted_id, sorted_box, sorted_vid, hf, l2, qtype, qid, qb, qv, t % PQ,
                              base + loc, cap,
                              oi, oj, ot, status);
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

// Pairs under the temporary zero offset (Sec. 3.4): key = type << 62 |
// i << 31 | j, open addressing with linear probing over a power-of-two
// table that is at most half full.
constexpr unsigned long long CORE_EMPTY = ~0ull;
__device__ __forceinline__ unsigned long long core_key_of(int type, int i, int j) {
  return ((unsigned long long)type << 62) | ((unsigned long long)(unsigned)i << 31) | (unsigned long long)(unsigned)j;
}
__device__ __forceinline__ unsigned core_hash(unsigned long long k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  return (unsigned)k;
}
__device__ __forceinline__ bool in_core(const SceneDev& S, int type, int i, int j) {
  if (!S.core_key) return false;
  const unsigned long long key = core_key_of(type, i, j);
  unsigned h = core_hash(key) & S.core_mask;
  for (unsigned p = 0; p <= S.core_mask; ++p) {
    const unsigned long long kk = S.core_key[h];
    if (kk == key) return S.core_live[h] != 0;
    if (kk == CORE_EMPTY) return false;
    h = (h + 1) & S.core_mask;
  }
  return false;
}

// Culling comparison mode (rods): edges of one polyline at most cull_r
// elements apart are left out of contact.
__device__ __forceinline__ bool is_culled(const SceneDev& S, int type, int i, int j) {
  if (S.filter != BF_FILTER_CULL || type != BF_EE) return false;
  if (S.comp[S.edges[2 * i]] != S.comp[S.edges[2 * j]]) return false;
  int d = abs(S.eidx[i] - S.eidx[j]);
  const int L = S.eloop[i];
  if (L > 0) d = min(d, L - d);
  return d <= S.cull_r;
}

// dbar^2 < h^2 for a shell pair whose rest distance is near h (not
// overlapping), exactly when the 2D formulas evaluate without rounding in
// FP64 (rest coordinates on a lattice): 1 / 0, or 2 when some operation
// rounds.  dbar^2 < h^2 iff one of the segment distances is.
__device__ __forceinline__ int seg2_below_exact_in_double(V2<double> p, V2<double> a, V2<double> b, dd hh, bool& ok) {
  ExactD E{true};
  const double ex = E.sub(b.x, a.x), ey = E.sub(b.y, a.y), rx = E.sub(p.x, a.x), ry = E.sub(p.y, a.y);
  const double ee = E.add(E.mul(ex, ex), E.mul(ey, ey)), re = E.add(E.mul(rx, ex), E.mul(ry, ey));
  double num, den = 1.0;
  if (!(re > 0.0)) {
    num = E.add(E.mul(rx, rx), E.mul(ry, ry));
  } else if (!(re < ee)) {
    const double qx = E.sub(p.x, b.x), qy = E.sub(p.y, b.y);
    num = E.add(E.mul(qx, qx), E.mul(qy, qy));
  } else {
    const double c = E.sub(E.mul(rx, ey), E.mul(ry, ex));
    num = E.mul(c, c);
    den = ee;
  }
  ok = ok && E.ok && den > 0.0;
  return sign_num_minus_tden(num, den, hh) < 0;
}
__device__ __forceinline__ int ref_below_h_exact_in_double(const SceneDev& S, int type, const int* v, dd hh) {
  const V2<double> P0 = ref2(S, v[0]), P1 = ref2(S, v[1]), P2 = ref2(S, v[2]), P3 = ref2(S, v[3]);
  bool ok = true;
  int below;
  if (type == BF_PT) {
    below = seg2_below_exact_in_double(P0, P1, P2, hh, ok) | seg2_below_exact_in_double(P0, P2, P3, hh, ok) |
            seg2_below_exact_in_double(P0, P3, P1, hh, ok);
  } else {
    below = seg2_below_exact_in_double(P0, P2, P3, hh, ok) | seg2_below_exact_in_double(P1, P2, P3, hh, ok) |
            seg2_below_exact_in_double(P2, P0, P1, hh, ok) | seg2_below_exact_in_double(P3, P0, P1, hh, ok);
  }
  return ok ? below : 2;
}

// Under the Euclidean reading (BF_REFDIST_EUCLID_REST) dbar is the distance
// between the pair's primitives at the rest pose, the same distance function
// as d(x); 0 < dbar holds for every pair of the scene (a rest pose with
// touching primitives is refused at creation), so the filter is dbar < h,
// decided like d < h: FP64, then (where amb is given) the exact-in-FP64
// check, then double-double, *amb set within 1e-20 of h^2.
__device__ __forceinline__ Near rest_near(const SceneDev& S, int type, const int* v, d3* P) {
#pragma unroll
  for (int k = 0; k < 4; ++k) P[k] = load3(S.xrest, v[k]);
  return type == BF_PT ? classify_pt(P) : classify_ee(P);
}
__device__ __forceinline__ bool euclid_below_h(const SceneDev& S, int type, const int* v, bool* amb) {
  d3 P[4];
  const Near nr = rest_near(S, type, v, P);
  return decide_sq(nr.code, P, nr.D, dd_sq(S.h), true, amb);
}

// Stencil pair with 0 < dbar < h in the same component (Sec. 3.2)?  Shells
// compare dbar^2 with h^2 in FP64 outside a relative band of 1e-9 and in
// double-double inside it; within 1e-20 of h^2 (*amb set, when amb is given)
// the narrow phase defers the pair to exact arithmetic (is_filtered_exact).
__device__ __forceinline__ bool is_filtered(const SceneDev& S, int type, const int* v, bool* amb) {
  if (S.filter != 0) return false;
  if (S.comp[v[0]] != S.comp[v[2]]) return false;
  if (S.refdist == BF_REFDIST_EUCLID_REST) return euclid_below_h(S, type, v, amb);
  if (S.kind == 0) {
    double sa0 = S.ref[v[0]], sa1 = S.ref[v[1]], sb0 = S.ref[v[2]], sb1 = S.ref[v[3]];
    double gap = fmax(fmin(sb0, sb1) - fmax(sa0, sa1), fmin(sa0, sa1) - fmax(sb0, sb1));
    return gap > 0.0 && gap < S.h;
  }
  const double h2 = S.h * S.h;
  const double q = ref_sqdist_d(S, type, v);
  if (fabs(q - h2) > 1e-9 * h2 && q > 1e-9 * h2) return q < h2;
  const dd hh = dd_sq(S.h);
  if (amb && fabs(q - h2) <= 1e-9 * h2) {  // near h: exact in FP64 on lattice rest coordinates
    const int r = ref_below_h_exact_in_double(S, type, v, hh);
    if (r != 2) return r == 1;
  }
  const dd qq = ref_sqdist_q(S, type, v);
  if (amb && !(fabs((qq - hh).hi) > 1e-20 * h2)) *amb = true;  // deferred to exact arithmetic
  return qq.hi > 0.0 && dd_lt(qq, hh);
}

// The narrow phase's first pass decides in FP64 alone: outside the relative
// band of 1e-9 around h^2 the FP64 value settles it; inside it *amb is set
// and the pair goes to k_exact, which takes the whole ladder (FP64, the
// exact-in-FP64 check, double-double, expansions).  Keeping the ladder out of
// this pass keeps its register footprint small.
__device__ __forceinline__ bool decide_fp64(double D, double Th, bool lt, bool* amb) {
  if (fabs(D - Th) > 1e-9 * Th) return lt ? (D < Th) : (D <= Th);
  *amb = true;
  return false;
}
__device__ __forceinline__ bool is_filtered_fp64(const SceneDev& S, int type, const int* v, bool* amb) {
  if (S.filter != 0) return false;
  if (S.comp[v[0]] != S.comp[v[2]]) return false;
  if (S.refdist == BF_REFDIST_EUCLID_REST) {
    d3 P[4];
    return decide_fp64(rest_near(S, type, v, P).D, S.h * S.h, true, amb);
  }
  if (S.kind == 0) {
    double sa0 = S.ref[v[0]], sa1 = S.ref[v[1]], sb0 = S.ref[v[2]], sb1 = S.ref[v[3]];
    double gap = fmax(fmin(sb0, sb1) - fmax(sa0, sa1), fmin(sa0, sa1) - fmax(sb0, sb1));
    return gap > 0.0 && gap < S.h;
  }
  const double h2 = S.h * S.h;
  const double q = ref_sqdist_d(S, type, v);
  if (fabs(q - h2) > 1e-9 * h2 && q > 1e-9 * h2) return q < h2;
  *amb = true;
  return false;
}

// The same decision, exact (k_exact): near h^2 the rest distance is below h
// iff one of its segment distances is (the pair does not overlap in rest
// space there), each decided on expansions (xp_seg2_below, slab ws).
__device__ bool is_filtered_exact(const SceneDev& S, int type, const int* v, double* ws, bool* limit) {
  if (S.filter == 0 && S.refdist == BF_REFDIST_EUCLID_REST && S.comp[v[0]] == S.comp[v[2]]) {
    d3 P[4];
    const Near nr = rest_near(S, type, v, P);
    return decide_sq_exact(nr.code, P, nr.D, dd_sq(S.h), true, ws, limit);
  }
  const bool r = is_filtered(S, type, v, nullptr);  // FP64, double-double in the band
  if (S.filter != 0 || S.kind == 0 || S.comp[v[0]] != S.comp[v[2]]) return r;
  const double h2 = S.h * S.h;
  if (fabs(ref_sqdist_d(S, type, v) - h2) > 1e-9 * h2) return r;
  const dd hh = dd_sq(S.h);
  const int ex = ref_below_h_exact_in_double(S, type, v, hh);
  if (ex != 2) return ex == 1;
  if (fabs((ref_sqdist_q(S, type, v) - hh).hi) > 1e-20 * h2) return r;
  const V2<double> P0 = ref2(S, v[0]), P1 = ref2(S, v[1]), P2 = ref2(S, v[2]), P3 = ref2(S, v[3]);
  int b[4];
  if (type == BF_PT) {
    b[0] = xp_seg2_below(P0.x, P0.y, P1.x, P1.y, P2.x, P2.y, hh, ws);
    b[1] = xp_seg2_below(P0.x, P0.y, P2.x, P2.y, P3.x, P3.y, hh, ws);
    b[2] = xp_seg2_below(P0.x, P0.y, P3.x, P3.y, P1.x, P1.y, hh, ws);
    b[3] = 0;
  } else {
    b[0] = xp_seg2_below(P0.x, P0.y, P2.x, P2.y, P3.x, P3.y, hh, ws);
    b[1] = xp_seg2_below(P1.x, P1.y, P2.x, P2.y, P3.x, P3.y, hh, ws);
    b[2] = xp_seg2_below(P2.x, P2.y, P0.x, P0.y, P1.x, P1.y, hh, ws);
    b[3] = xp_seg2_below(P3.x, P3.y, P0.x, P0.y, P1.x, P1.y, hh, ws);
  }
  if (b[0] == 2 || b[1] == 2 || b[2] == 2 || b[3] == 2) {
    *limit = true;
    return r;
  }
  return b[0] == 1 || b[1] == 1 || b[2] == 1 || b[3] == 1;
}

// Order of the active list by distance kind: 9 x 9 systems (PT, EE) first,
// then 6 x 6 (PE), then the closed form (PP), so the evaluation kernel's
// waves are uniform and the heaviest start first.
__device__ __forceinline__ int kind_rank(int code) {
  int k = case_kind(code);
  return (k == K_PT || k == K_EE) ? 0 : (k == K_PE ? 1 : 2);
}

// Decisions of one candidate pair: the distance sub-case and D = d^2, and
// d < h (a contact pair, N_c), the filter (Eq. 4: a stencil with
// 0 < dbar < h), the temporary zero offset (Sec. 3.4), active (Eq. 2: d < a)
// and infeasible (Eq. 3: d <= eta).  EXACT = false: FP64, double-double where
// FP64 is unclear, and *amb set where double-double is unclear too (the pair
// is then left to k_exact); EXACT = true: exact arithmetic there (slab ws;
// *limit set if the expansions outgrow it).
struct PairDec {
  bool nc, filt, core, active, infeas;
  int code;
  double D;
};
// NW_FP64: FP64 alone, *amb set where a value lies in the relative band of
// 1e-9 around its threshold (the narrow phase's first pass, k_narrow);
// NW_DD: FP64, then the exact-in-FP64 check and double-double in the band,
// *amb set within 1e-20 of the threshold (k_band); NW_EXACT: the whole
// ladder, exact arithmetic last (k_exact).
constexpr int NW_FP64 = 0, NW_DD = 1, NW_EXACT = 2;
template <int MODE>
__device__ __forceinline__ PairDec narrow_pair(const SceneDev& S, const double* x, int type, int i, int j, bool* amb,
                                               double* ws, bool* limit) {
  constexpr bool EXACT = MODE == NW_EXACT;
  PairDec r{false, false, false, false, false, 0, 0.0};
  int v[4];
  pair_verts(S, type, i, j, v);
  d3 P[4] = {load3(x, v[0]), load3(x, v[1]), load3(x, v[2]), load3(x, v[3])};
  const Near nr = type == BF_PT ? classify_pt(P) : classify_ee(P);
  r.code = nr.code;
  r.D = nr.D;
  auto dec = [&](dd T, bool lt) {
    if constexpr (EXACT) return decide_sq_exact(r.code, P, r.D, T, lt, ws, limit);
    else if constexpr (MODE == NW_DD) return decide_sq(r.code, P, r.D, T, lt, amb);
    else return decide_fp64(r.D, T.hi, lt, amb);
  };
  r.nc = !is_culled(S, type, i, j) && dec(dd_sq(S.h), true);  // d < h (culled pairs: not in contact)
  if (r.nc) {
    if constexpr (EXACT) r.filt = is_filtered_exact(S, type, v, ws, limit);
    else if constexpr (MODE == NW_DD) r.filt = is_filtered(S, type, v, amb);
    else r.filt = is_filtered_fp64(S, type, v, amb);
    r.core = !r.filt && in_core(S, type, i, j);
    dd T;
    double eta;
    if (r.filt) {  // Eq. 4 second case: (d_min, 0)
      const int c = S.comp[v[0]];
      T = dd{S.thr2[2 * c], S.thr2[2 * c + 1]};
      eta = 0.0;
    } else {       // Eq. 4 first case: (h, eta); (h, 0) while in the core set (Sec. 3.4)
      T = dd_sq(S.h);
      eta = r.core ? 0.0 : S.eta;
    }
    // Eq. 2: d < a.  Unfiltered, a = h: the decision d < h already taken
    // (r.nc), which the exact path would otherwise repeat
    r.active = r.filt ? dec(T, true) : true;
    if (r.active) r.infeas = eta > 0.0 ? dec(dd_sq(eta), false) : !(r.D > 0.0);
  }
  return r;
}

// Pass 1 of the narrow phase: tile b = candidates [b*NW_TILE, (b+1)*NW_TILE).
// Active pairs are compacted inside the tile by kind, in candidate order,
// into the staging arrays; a candidate whose decision double-double cannot
// settle is staged as a fourth kind (its candidate index), for k_exact.
// Per-kind counts go to kcnt[K*G + b] and the tile's N_c / N_filt /
// N_infeasible (without the deferred ones) to ccnt[3b..3b+2].  No global
// atomics.
__global__ __launch_bounds__(256) void k_narrow(SceneDev S, const double* x, const int* ci, const int* cj,
                                                const unsigned char* ct, const long long* cand_count, long long ccap,
                                                StageWs W) {
  long long n = *cand_count;
  if (n > ccap) n = ccap;
  const int G = gridDim.x;
  const long long base = (long long)blockIdx.x * NW_TILE;
  const int lane = lane_id(), w = threadIdx.x >> 6;
  __shared__ int wc[NW_ITEMS][4][NW_KINDS];
  __shared__ int cc[4][3];
  int ri[NW_ITEMS], rj[NW_ITEMS], rk[NW_ITEMS], lr[NW_ITEMS];
  unsigned rm[NW_ITEMS];
  double rd[NW_ITEMS];
  int c_nc = 0, c_f = 0, c_inf = 0;
#pragma unroll
  for (int it = 0; it < NW_ITEMS; ++it) {
    long long k = base + it * 256 + threadIdx.x;
    PairDec pd{false, false, false, false, false, 0, 0.0};
    int type = 0, i = 0, j = 0;
    bool amb = false;
    if (k < n) {
      type = ct[k]; i = ci[k]; j = cj[k];
      pd = narrow_pair<NW_FP64>(S, x, type, i, j, &amb, nullptr, nullptr);
    }
    if (amb) pd.nc = pd.filt = pd.core = pd.active = pd.infeas = false;  // k_exact decides
    c_nc += pd.nc; c_f += pd.nc && pd.filt; c_inf += pd.infeas;
    rk[it] = amb ? NW_DEFER : (pd.active ? kind_rank(pd.code) : NW_KINDS);
    ri[it] = amb ? (int)k : i;
    rj[it] = j;
    rm[it] = (unsigned)type | ((unsigned)pd.code << 8) |
             ((unsigned)((pd.filt ? BF_F_FILTERED : 0) | (pd.infeas ? BF_F_INFEASIBLE : 0) |
                         (pd.core ? BF_F_CORE : 0)) << 16);
    rd[it] = sqrt(pd.D);
#pragma unroll
    for (int K = 0; K < NW_KINDS; ++K) {
      unsigned long long m = __ballot(rk[it] == K);
      if (lane == 0) wc[it][w][K] = __popcll(m);
      if (rk[it] == K) lr[it] = lanes_below(m);
    }
  }
  c_nc = wave_sum(c_nc); c_f = wave_sum(c_f); c_inf = wave_sum(c_inf);
  if (lane == 0) { cc[w][0] = c_nc; cc[w][1] = c_f; cc[w][2] = c_inf; }
  __syncthreads();
  int tot[NW_KINDS] = {0, 0, 0, 0};
#pragma unroll
  for (int it = 0; it < NW_ITEMS; ++it)
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int K = 0; K < NW_KINDS; ++K) tot[K] += wc[it][q][K];
  const int koff[NW_KINDS] = {0, tot[0], tot[0] + tot[1], tot[0] + tot[1] + tot[2]};
#pragma unroll
  for (int it = 0; it < NW_ITEMS; ++it) {
    if (rk[it] >= NW_KINDS) continue;
    int K = rk[it];
    int off = koff[K] + lr[it];
    for (int i2 = 0; i2 < NW_ITEMS; ++i2)
      for (int q = 0; q < 4; ++q)
        if (i2 < it || (i2 == it && q < w)) off += wc[i2][q][K];
    long long p = base + off;
    W.si[p] = ri[it];
    W.sj[p] = rj[it];
    W.sm[p] = rm[it];
    W.sd[p] = rd[it];
  }
  if (threadIdx.x == 0) {
    for (int K = 0; K < NW_KINDS; ++K) W.kcnt[K * G + blockIdx.x] = tot[K];
    if (blockIdx.x == 0) W.kcnt[NW_KINDS * G] = 0;
    int a = 0, b = 0, c = 0;
    for (int q = 0; q < 4; ++q) { a += cc[q][0]; b += cc[q][1]; c += cc[q][2]; }
    W.ccnt[3 * blockIdx.x] = a;
    W.ccnt[3 * blockIdx.x + 1] = b;
    W.ccnt[3 * blockIdx.x + 2] = c;
  }
}

// Pass 2: copy each tile's staged pairs to their kind-major position
// kofs[K*G + b] + r of the active list, and the deferred candidates to the
// deferred list (in tile order: candidate order); block 0 also writes the
// counters (k_exact then adds the deferred pairs' share).
__global__ __launch_bounds__(256) void k_compact(StageWs W, int G, int* ai, int* aj, unsigned char* at,
                                                 unsigned char* acode, unsigned char* aflags, double* adist,
                                                 long long acap, long long* act_count, long long* counters,
                                                 unsigned* status) {
  const int b = blockIdx.x;
  const long long base = (long long)b * NW_TILE;
  int koff = 0;
  for (int K = 0; K < NW_KINDS - 1; ++K) {
    int cnt = W.kcnt[K * G + b];
    long long dst = W.kofs[K * G + b];
    for (int r = threadIdx.x; r < cnt; r += blockDim.x) {
      long long src = base + koff + r, d = dst + r;
      if (d < acap) {
        unsigned m = W.sm[src];
        ai[d] = W.si[src];
        aj[d] = W.sj[src];
        at[d] = (unsigned char)(m & 0xff);
        acode[d] = (unsigned char)((m >> 8) & 0xff);
        aflags[d] = (unsigned char)((m >> 16) & 0xff);
        adist[d] = W.sd[src];
      }
    }
    koff += cnt;
  }
  {  // deferred candidates (their indices)
    const int cnt = W.kcnt[NW_DEFER * G + b];
    const long long dst = W.kofs[NW_DEFER * G + b] - W.kofs[NW_DEFER * G];
    for (int r = threadIdx.x; r < cnt; r += blockDim.x) W.dfr[dst + r] = W.si[base + koff + r];
  }
  if (b == 0) {
    if (threadIdx.x == 0) *W.n2 = 0;  // k_band appends to the second list afresh
    __shared__ long long red[3][256];
    long long a = 0, f = 0, c = 0;
    for (int q = threadIdx.x; q < G; q += blockDim.x) {
      a += W.ccnt[3 * q]; f += W.ccnt[3 * q + 1]; c += W.ccnt[3 * q + 2];
    }
    red[0][threadIdx.x] = a; red[1][threadIdx.x] = f; red[2][threadIdx.x] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
      long long A = 0, F = 0, C = 0;
      for (int q = 0; q < (int)blockDim.x; ++q) { A += red[0][q]; F += red[1][q]; C += red[2][q]; }
      long long nact = W.kofs[NW_DEFER * G];
      counters[0] = A; counters[1] = F; counters[2] = nact; counters[3] = C;
      *act_count = nact;
    }
  }
}

// The result record of a decided deferred candidate, at its deferred index
// q in the staging arrays (free again after k_compact): ids, type, code,
// flags, the decisions (bits 24..27: active, d < h, filtered and d < h,
// expansion room exceeded) and d.
__device__ __forceinline__ void put_deferred(const StageWs& W, long long q, int type, int i, int j, const PairDec& pd,
                                             bool limit) {
  W.si[q] = i;
  W.sj[q] = j;
  W.sm[q] = (unsigned)type | ((unsigned)pd.code << 8) |
            ((unsigned)((pd.filt ? BF_F_FILTERED : 0) | (pd.infeas ? BF_F_INFEASIBLE : 0) |
                        (pd.core ? BF_F_CORE : 0)) << 16) |
            (pd.active ? 1u << 24 : 0u) | (pd.nc ? 1u << 25 : 0u) | (pd.nc && pd.filt ? 1u << 26 : 0u) |
            (limit ? 1u << 27 : 0u);
  W.sd[q] = sqrt(pd.D);
}

// Pass 3: the deferred candidates (a value in FP64's band around its
// threshold), one per thread: the exact-in-FP64 check and double-double
// settle most (lattice geometry); the rest, within 1e-20 of a threshold,
// go to the second list (any order: each result goes to its own index).
__global__ __launch_bounds__(256) void k_band(SceneDev S, const double* x, const int* ci, const int* cj,
                                              const unsigned char* ct, StageWs W, int G) {
  const long long ndef = W.kofs[NW_KINDS * G] - W.kofs[NW_DEFER * G];
  for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < ndef; q += grid_stride()) {
    const long long k = W.dfr[q];
    const int type = ct[k], i = ci[k], j = cj[k];
    bool amb = false;
    const PairDec pd = narrow_pair<NW_DD>(S, x, type, i, j, &amb, nullptr, nullptr);
    if (amb) W.dfr2[atomicAdd(W.n2, 1)] = (int)q;
    else put_deferred(W, q, type, i, j, pd, false);
  }
}

// Pass 4: the second list in exact arithmetic.  XP_TPB threads per
// work-group, each with an expansion slab in LDS, over contiguous ranges of
// the list.
__global__ __launch_bounds__(XP_TPB) void k_exact(SceneDev S, const double* x, const int* ci, const int* cj,
                                                  const unsigned char* ct, StageWs W) {
  __shared__ double slab[XP_TPB * XP_WS];
  const long long n2 = *W.n2;
  const long long R = (n2 + gridDim.x - 1) / gridDim.x, r0 = blockIdx.x * R, r1 = min(n2, r0 + R);
  double* ws = slab + threadIdx.x * XP_WS;
  for (long long r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
    const long long q = W.dfr2[r], k = W.dfr[q];
    const int type = ct[k], i = ci[k], j = cj[k];
    bool limit = false;
    const PairDec pd = narrow_pair<NW_EXACT>(S, x, type, i, j, nullptr, ws, &limit);
    put_deferred(W, q, type, i, j, pd, limit);
  }
}

// Pass 5: counts of the deferred results per contiguous range of the
// deferred list (range b of XP_BLOCKS into W.xcnt[5b..5b+4]: active, N_c,
// N_filt, N_infeasible, exceeded).
__global__ __launch_bounds__(256) void k_dfr_count(StageWs W, int G) {
  const long long ndef = W.kofs[NW_KINDS * G] - W.kofs[NW_DEFER * G];
  const long long R = (ndef + gridDim.x - 1) / gridDim.x, q0 = blockIdx.x * R, q1 = min(ndef, q0 + R);
  int c[5] = {0, 0, 0, 0, 0};
  for (long long q = q0 + threadIdx.x; q < q1; q += blockDim.x) {
    const unsigned m = W.sm[q];
    c[0] += (m >> 24) & 1u;
    c[1] += (m >> 25) & 1u;
    c[2] += (m >> 26) & 1u;
    c[3] += ((m >> 24) & 1u) && (((m >> 16) & 0xffu) & BF_F_INFEASIBLE);
    c[4] += (m >> 27) & 1u;
  }
#pragma unroll
  for (int t = 0; t < 5; ++t) c[t] = block_sum256(c[t]);
  if (threadIdx.x < 5) W.xcnt[5 * blockIdx.x + threadIdx.x] = c[threadIdx.x];
}

// Pass 6: the deferred pairs that are active are appended after the
// compacted ones, in candidate order: work-group b copies its range's, after
// the active pairs of all earlier ranges.  Work-group 0 adds the counts and
// raises the step's overflow and infeasible bits.
__global__ __launch_bounds__(256) void k_exact_emit(StageWs W, int G, int* ai, int* aj, unsigned char* at,
                                                    unsigned char* acode, unsigned char* aflags, double* adist,
                                                    long long acap, long long* act_count, long long* counters,
                                                    unsigned* status) {
  const long long ndef = W.kofs[NW_KINDS * G] - W.kofs[NW_DEFER * G];
  const long long nact0 = W.kofs[NW_DEFER * G];  // the compacted pairs (k_compact's count)
  const long long R = (ndef + gridDim.x - 1) / gridDim.x, q0 = blockIdx.x * R, q1 = min(ndef, q0 + R);
  long long before = 0;
  for (int b = threadIdx.x; b < (int)blockIdx.x; b += blockDim.x) before += W.xcnt[5 * b];
  before = block_sum256(before);
  long long run = nact0 + before;
  for (long long c0 = q0; c0 < q1; c0 += blockDim.x) {
    const long long q = c0 + threadIdx.x;
    const unsigned m = q < q1 ? W.sm[q] : 0u;
    const bool active = (m >> 24) & 1u;
    int tot;
    const int ex = block_excl_scan256(active ? 1 : 0, &tot);
    if (active) {
      const long long d = run + ex;
      if (d < acap) {
        ai[d] = W.si[q];
        aj[d] = W.sj[q];
        at[d] = (unsigned char)(m & 0xffu);
        acode[d] = (unsigned char)((m >> 8) & 0xffu);
        aflags[d] = (unsigned char)((m >> 16) & 0xffu);
        adist[d] = W.sd[q];
      }
    }
    run += tot;
  }
  if (blockIdx.x == 0) {
    long long s[5] = {0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < (int)gridDim.x; b += blockDim.x)
      for (int t = 0; t < 5; ++t) s[t] += W.xcnt[5 * b + t];
    for (int t = 0; t < 5; ++t) s[t] = block_sum256(s[t]);
    if (threadIdx.x == 0) {
      const long long nact = nact0 + s[0];
      counters[0] += s[1];
      counters[1] += s[2];
      counters[2] = nact;
      counters[3] += s[3];
      *act_count = nact;
      status[1] = (unsigned)min(ndef, 0xffffffffll);  // deferred candidates of this step (diagnostics)
      status[2] = (unsigned)*W.n2;                      // of which decided in exact arithmetic
      unsigned bits = 0;
      if (nact > acap) bits |= BF_S_ACT_OVERFLOW;
      if (counters[3] > 0) bits |= BF_S_INFEASIBLE;
      if (s[4] > 0) bits |= BF_S_EXACT_LIMIT;
      if (bits) atomicOr(status, bits);
    }
  }
}

// ---------------------------------------------------------------------------
// Packed pair Hessian: the upper triangle of the symmetric 12 x 12 matrix by
// 3 x 3 blocks, 78 doubles.  Block-row s (the rows of stencil vertex s)
// holds block (s, s) as its upper triangle (xx, xy, xz, yy, yz, zz), then
// blocks (s, t), t > s, row-major; block-rows 0..3 follow one another
// (offsets 0, 33, 57, 72).
// ---------------------------------------------------------------------------
constexpr int PK_N = 78;
__host__ __device__ constexpr int pk_off(int s) { return s == 0 ? 0 : s == 1 ? 33 : s == 2 ? 57 : 72; }
__host__ __device__ constexpr int pk_len(int s) { return 6 + 9 * (3 - s); }
// packed index of entry (I, J) of the 12 x 12 matrix, I <= J or not
__host__ __device__ constexpr int pk_index(int I, int J) {
  const int a = I < J ? I : J, b = I < J ? J : I;
  const int s = a / 3, i = a % 3, t = b / 3, j = b % 3;
  if (s == t) return pk_off(s) + (i == 0 ? j : i == 1 ? 2 + j : 5);
  return pk_off(s) + 6 + 9 * (t - s - 1) + 3 * i + j;
}
// tables: the (row, column) of each packed entry, and for each stencil slot
// s the packed source of each entry of its band (rows 3s..3s+2, 36 doubles)
struct PkTables {
  unsigned char row[PK_N], col[PK_N];
  unsigned char band[4][36];
  constexpr PkTables() : row(), col(), band() {
    for (int I = 0; I < 12; ++I)
      for (int J = I; J < 12; ++J) {
        row[pk_index(I, J)] = (unsigned char)I;
        col[pk_index(I, J)] = (unsigned char)J;
      }
    for (int sl = 0; sl < 4; ++sl)
      for (int o = 0; o < 36; ++o) band[sl][o] = (unsigned char)pk_index(3 * sl + o / 12, o % 12);
  }
};
__constant__ PkTables kPk = PkTables();

// ---------------------------------------------------------------------------
// Barrier evaluation (Eq. 2, Eq. 3) and PSD projection
// ---------------------------------------------------------------------------
// One wave per work-group, one pair per lane.  Each lane keeps its pair's
// projected Hessian in reduced form (registers); its packed upper triangle
// then goes out one block-row at a time: the lanes write the block-row's
// entries of their rows into a small LDS tile (one row at a time, from the
// reduced form), and the wave stores the 64 pairs' segments (33, 24, 15 and 6
// contiguous entries) as runs (stores straight from each lane's registers
// would scatter every instruction over 64 records).  The records are FP64,
// or FP32 in the mixed mode (HT), whose projection is FP32 already.  The
// energies of each 64-pair tile are summed in a fixed order into epart
// (partials of the total).
constexpr int PK_STRIDE = 33;  // LDS doubles per pair in the staging tile (the longest block-row)
template <int I, class HT>
__device__ __forceinline__ void flush_row(const PairOut& h, double* buf, HT* H, long long k0, int rows) {
  constexpr int s = I / 3, i = I % 3;
  const int lane = threadIdx.x;
  double r[12];
  hess_row<I>(h, r);
  double* my = buf + PK_STRIDE * lane;
#pragma unroll
  for (int j = i; j < 3; ++j) my[pk_index(I, 3 * s + j) - pk_off(s)] = r[3 * s + j];
#pragma unroll
  for (int c = 3 * s + 3; c < 12; ++c) my[pk_index(I, c) - pk_off(s)] = r[c];
  if constexpr (i == 2) {  // the block-row is complete: store the tile's segments
    __syncthreads();
    constexpr int len = pk_len(s);
    for (int idx = lane; idx < rows * len; idx += 64) {
      const int p = idx / len, e = idx - p * len;
      H[PK_N * (k0 + p) + pk_off(s) + e] = (HT)buf[PK_STRIDE * p + e];
    }
    __syncthreads();
  }
}
template <int I, class HT>
__device__ __forceinline__ void flush_rows(const PairOut& h, double* buf, HT* H, long long k0, int rows) {
  flush_row<I>(h, buf, H, k0, rows);
  if constexpr (I + 1 < 12) flush_rows<I + 1>(h, buf, H, k0, rows);
}

template <bool MIXED>
__global__ __launch_bounds__(64) void k_eval(SceneDev S, const double* x, const int* ai, const int* aj,
                                             const unsigned char* at, const unsigned char* acode,
                                             const unsigned char* aflags, const unsigned long long* act_count,
                                             long long acap, double* E, double* G, void* Hv, double* epart) {
  using HT = typename std::conditional<MIXED, float, double>::type;
  HT* H = (HT*)Hv;
  __shared__ double buf[64 * PK_STRIDE];
  long long n = (long long)*act_count;
  if (n > acap) n = acap;
  const int lane = threadIdx.x;
  for (long long k0 = (long long)blockIdx.x * 64; k0 < n; k0 += (long long)gridDim.x * 64) {
    const long long k = k0 + lane;
    PairOut h;
    h.E = 0.0;
    h.kind = H_ZERO;
    h.eig_ok = 1;
    if (k < n) {
      int type = at[k], code = acode[k], fl = aflags[k];
      int v[4];
      pair_verts(S, type, ai[k], aj[k], v);
      if (fl & BF_F_INFEASIBLE) {
        h.E = INFINITY;
        zero_grad(G + 12 * k);
      } else {
        d3 P[4] = {load3(x, v[0]), load3(x, v[1]), load3(x, v[2]), load3(x, v[3])};
        double a, eta;
        if (fl & BF_F_FILTERED) { a = S.dmin[S.comp[v[0]]]; eta = 0.0; }
        else { a = S.h; eta = (fl & BF_F_CORE) ? 0.0 : S.eta; }
        eval_pair<MIXED>(P, code, a, eta, S.kappa, G + 12 * k, h);
      }
      E[k] = h.E;
    }
    if (__ballot(!h.eig_ok) != 0ull && lane == 0 && S.status) atomicOr(S.status, (unsigned)BF_S_EIG_NOCONV);
    double e = h.E, y = 0.0, z = 0.0;
    wave_ordered_sum3(e, y, z);
    if (lane == 0 && epart) epart[k0 / 64] = e;
    flush_rows<0>(h, buf, H, k0, (int)min((long long)64, n - k0));
  }
}

// ---------------------------------------------------------------------------
// Assembly (owner computes): every stencil vertex of every feasible active
// pair gets an incidence entry 4k + s (pair k, slot s).  A counting sort
// groups the entries by vertex; one thread per vertex then sums its gradient
// and assembles its BSR row.  No floating-point atomics, and every sum is
// taken in increasing entry order, so the result does not depend on thread
// timing.
// ---------------------------------------------------------------------------
// Incidence counts of the feasible active pairs' stencil vertices.
// Runs of equal values in consecutive lanes of a wave (the active list is in
// query order, so a primitive's pairs share stencil vertices lane after
// lane): this lane's run starts at lane `start` and the run has `len` lanes
// (valid at the run's first lane).  Every lane of the wave must call it.
__device__ __forceinline__ void lane_runs(int key, int& start, int& len, bool& head) {
  const int lane = lane_id();
  const int prev = __shfl_up(key, 1, 64);
  head = lane == 0 || key != prev;
  const unsigned long long heads = __ballot(head);
  const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
  start = 63 - __clzll(heads & upto);
  const unsigned long long after = heads & ~upto;
  len = (after ? __ffsll((long long)after) - 1 : 64) - lane;
}

// Incidence counts of the feasible active pairs' stencil vertices; one
// atomic per run of equal vertices in consecutive lanes (whole waves step
// through the list together).
__global__ __launch_bounds__(256) void k_inc_count(SceneDev S, const int* ai, const int* aj, const unsigned char* at,
                                                   const unsigned char* aflags, const unsigned long long* act_count,
                                                   long long acap, int* inc_cnt, int* mid_count,
                                                   int* big_count) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *mid_count = *big_count = 0;  // pass A appends to the lists afresh
  long long n = (long long)*act_count;
  if (n > acap) n = acap;
  const int lane = lane_id();
  for (long long w0 = blockIdx.x * (long long)blockDim.x + (threadIdx.x & ~63); w0 < n; w0 += grid_stride()) {
    const long long k = w0 + lane;
    int v[4] = {-1, -1, -1, -1};
    if (k < n && !(aflags[k] & BF_F_INFEASIBLE)) pair_verts(S, at[k], ai[k], aj[k], v);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      int start, len;
      bool head;
      lane_runs(v[s], start, len, head);
      if (head && v[s] >= 0) atomicAdd(&inc_cnt[v[s]], len);
    }
  }
}

// Total energy from the per-tile partials, in a fixed order (one wave).
__device__ __forceinline__ void energy_total(const double* epart, long long ntiles, double* E_out) {
  const int lane = lane_id();
  const long long per = (ntiles + 63) / 64;
  double e = 0.0;
  for (long long q = lane * per; q < ntiles && q < (lane + 1) * per; ++q) e += epart[q];
  double y = 0.0, z = 0.0;
  wave_ordered_sum3(e, y, z);
  if (lane == 0) *E_out = e;
}

// scatter the entries into their vertex segments; returns the counts to zero
// (one atomic per run of equal vertices in consecutive lanes, as counted)
__global__ __launch_bounds__(256) void k_inc_fill(SceneDev S, const int* ai, const int* aj, const unsigned char* at,
                                                  const unsigned char* aflags, const unsigned long long* act_count,
                                                  long long acap, int* inc_cnt, const int* inc_off, int* inc) {
  long long n = (long long)*act_count;
  if (n > acap) n = acap;
  const int lane = lane_id();
  for (long long w0 = blockIdx.x * (long long)blockDim.x + (threadIdx.x & ~63); w0 < n; w0 += grid_stride()) {
    const long long k = w0 + lane;
    int v[4] = {-1, -1, -1, -1};
    if (k < n && !(aflags[k] & BF_F_INFEASIBLE)) pair_verts(S, at[k], ai[k], aj[k], v);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      int start, len;
      bool head;
      lane_runs(v[s], start, len, head);
      int top = 0;
      if (head && v[s] >= 0) top = atomicSub(&inc_cnt[v[s]], len);
      top = __shfl(top, start, 64);
      if (v[s] >= 0) inc[inc_off[v[s]] + top - 1 - (lane - start)] = (int)(4 * k + s);
    }
  }
}

// ---- per-row assembly ------------------------------------------------------
// A row with m incidence entries takes one of four paths: m <= ROW_S in the
// registers of a 16-lane team (four rows a wave), m <= ROW_L in the
// registers of one wave, m <= ROW_M in one wave's LDS, m <= ROW_H by a
// 256-thread block in LDS; beyond ROW_H one lane works in global memory
// (correct, slow).  Cloth rows reach a few hundred entries, rod rows a
// dozen or two.
constexpr int ROW_S = 16;  // rows with m <= ROW_S: one 16-lane team each, four rows a wave
constexpr int ROW_L = 32;
constexpr int ROW_M = 256;
constexpr int ROW_M_TAB = 4 * ROW_M;  // hash slots: at least the row's 4m candidate columns (tables
                                      // take pow2(4m + 1) slots up to this: always room for every key)
constexpr int ROW_H = 1024;            // 20 KiB of LDS: eight blocks a CU, so a few thousand such rows run at once
constexpr int ROW_H_TAB = 4 * ROW_H;
constexpr int EMPTY = -1;
constexpr int PAD = 0x7fffffff;

__device__ __forceinline__ int pow2_at_least(int n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
}

// Bitonic sort of a[0..P) (P a power of two) by the NT threads of the block.
template <int NT> __device__ __forceinline__ void team_bitonic(int* a, int P) {
  for (int k = 2; k <= P; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < P; i += NT) {
        int l = i ^ j;
        if (l > i) {
          int x = a[i], y = a[l];
          bool up = (i & k) == 0;
          if ((x > y) == up) { a[i] = y; a[l] = x; }
        }
      }
      __syncthreads();
    }
}

// Bitonic sorts across the lanes of a wave: 64 values (one per lane) and
// 128 values (element i in lane i & 63, register i >> 6).
__device__ __forceinline__ int wave_sort64(int x) {
  const int lane = lane_id();
#pragma unroll
  for (int k = 2; k <= 64; k <<= 1)
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      int y = __shfl_xor(x, j, 64);
      bool keep_min = ((lane & j) == 0) == ((lane & k) == 0);
      x = keep_min ? min(x, y) : max(x, y);
    }
  return x;
}
__device__ __forceinline__ void wave_sort128(int& a0, int& a1) {
  const int lane = lane_id();
#pragma unroll
  for (int k = 2; k <= 128; k <<= 1)
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j == 64) {
        int lo = min(a0, a1), hi = max(a0, a1);
        a0 = lo; a1 = hi;
        continue;
      }
      int b0 = __shfl_xor(a0, j, 64), b1 = __shfl_xor(a1, j, 64);
      bool lower = (lane & j) == 0;
      bool min0 = lower == ((lane & k) == 0), min1 = lower == (((lane + 64) & k) == 0);
      a0 = min0 ? min(a0, b0) : max(a0, b0);
      a1 = min1 ? min(a1, b1) : max(a1, b1);
    }
}

// Sorts inside the 16-lane teams of a wave (team t = lanes 16t..16t+15):
// 16 values (one per lane) and 64 values (element i in lane i & 15,
// register i >> 4).
// Value of lane (this lane xor j) within the lane's row of 16, j = 1, 2, 4
// or 8, by DPP moves instead of an LDS permute: quad permutations give xor 1,
// 2 and 3, the row's half mirror xor 7 and its mirror xor 15, so xor 4 =
// 7 ^ 3 and xor 8 = 15 ^ 7 take two moves.  j must fold to a constant.
__device__ __forceinline__ int team_xor(int x, int j) {
  if (j == 1) return __builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
  if (j == 2) return __builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
  if (j == 4)  // row_half_mirror, then quad_perm [3,2,1,0]
    return __builtin_amdgcn_mov_dpp(__builtin_amdgcn_mov_dpp(x, 0x141, 0xF, 0xF, false), 0x1B, 0xF, 0xF, false);
  // row_mirror, then row_half_mirror
  return __builtin_amdgcn_mov_dpp(__builtin_amdgcn_mov_dpp(x, 0x140, 0xF, 0xF, false), 0x141, 0xF, 0xF, false);
}

__device__ __forceinline__ int team_sort16(int x) {
  const int tl = lane_id() & 15;
#pragma unroll
  for (int k = 2; k <= 16; k <<= 1)
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      int y = team_xor(x, j);
      bool keep_min = ((tl & j) == 0) == ((tl & k) == 0);
      x = keep_min ? min(x, y) : max(x, y);
    }
  return x;
}
__device__ __forceinline__ void team_sort64(int (&a)[4]) {
  const int tl = lane_id() & 15;
#pragma unroll
  for (int k = 2; k <= 64; k <<= 1)
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j >= 16) {  // partner in another register of the same lane
        const int rj = j >> 4;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (r & rj) continue;
          const bool up = ((16 * r + tl) & k) == 0;
          const int lo = min(a[r], a[r | rj]), hi = max(a[r], a[r | rj]);
          a[r] = up ? lo : hi;
          a[r | rj] = up ? hi : lo;
        }
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * r + tl;
          const int y = team_xor(a[r], j);
          const bool keep_min = ((i & j) == 0) == ((i & k) == 0);
          a[r] = keep_min ? min(a[r], y) : max(a[r], y);
        }
      }
    }
}
// the 16 bits of a wave ballot that belong to this lane's team
__device__ __forceinline__ unsigned team_bits(unsigned long long m) {
  return (unsigned)((m >> (lane_id() & 48)) & 0xffffull);
}

// Insert key into an LDS open-addressing set of T slots (T a power of two
// larger than or equal to the number of distinct keys ever inserted).
__device__ __forceinline__ void set_insert(int* tab, int T, int key) {
  unsigned h = ((unsigned)key * 0x9E3779B1u) & (unsigned)(T - 1);
  while (true) {
    int old = atomicCAS(&tab[h], EMPTY, key);
    if (old == EMPTY || old == key) return;
    h = (h + 1) & (unsigned)(T - 1);
  }
}

__device__ void isort_global(int* a, int m) {
  for (int i = 1; i < m; ++i) {
    int x = a[i], j = i - 1;
    while (j >= 0 && a[j] > x) { a[j + 1] = a[j]; --j; }
    a[j + 1] = x;
  }
}

// One lane, global memory: sort the entries and store the distinct sorted
// columns; *count = their number.
__device__ void row_a_serial(const SceneDev& S, const int* ai, const int* aj, const unsigned char* at, int b, int m,
                             int* inc, int* cb, int* count, int4* stn) {
  isort_global(inc + b, m);
  for (int q = 0; q < m; ++q) {
    int k = inc[b + q] >> 2;
    int vv[4];
    pair_verts(S, at[k], ai[k], aj[k], vv);
    stn[b + q] = make_int4(vv[0], vv[1], vv[2], vv[3]);
    for (int c = 0; c < 4; ++c) cb[4 * q + c] = vv[c];
  }
  isort_global(cb, 4 * m);
  int u = 0;
  for (int q = 0; q < 4 * m; ++q)
    if (q == 0 || cb[q] != cb[q - 1]) cb[u++] = cb[q];
  *count = u;
}

// Pass A (structure; needs the active list only): sort the row's incidence
// entries (so every sum of pass B runs in a fixed order) and store its
// distinct columns (the stencil vertices of its pairs) sorted at
// colbuf[4 * inc_off[v] ...]; rowcnt[v] = their number.

// Rows with m <= ROW_S, one per 16-lane team: entry q in lane q, candidate
// column 4q + c in lane (4q + c) & 15, register (4q + c) >> 4.  `mine` is
// false on teams without such a row (their lanes take part in the
// shuffles with padding only).
__device__ __forceinline__ void row_a_team(const SceneDev& S, const int* ai, const int* aj, const unsigned char* at,
                                           bool mine, int v, int b, int m, int* inc, int* colbuf, int* rowcnt,
                                           int4* stn) {
  const int tl = lane_id() & 15;
  int e = mine && tl < m ? inc[b + tl] : PAD;
  e = team_sort16(e);
  int vv[4] = {PAD, PAD, PAD, PAD};
  if (mine && tl < m) {
    inc[b + tl] = e;
    const int k = e >> 2;
    pair_verts(S, at[k], ai[k], aj[k], vv);
    stn[b + tl] = make_int4(vv[0], vv[1], vv[2], vv[3]);
  }
  const int t4 = tl & 3;
  int c[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int q = 4 * r + (tl >> 2);
    const int w0 = __shfl(vv[0], q, 16), w1 = __shfl(vv[1], q, 16), w2 = __shfl(vv[2], q, 16),
              w3 = __shfl(vv[3], q, 16);
    c[r] = t4 == 0 ? w0 : t4 == 1 ? w1 : t4 == 2 ? w2 : w3;
  }
  team_sort64(c);
  int* cb = colbuf + 4LL * b;
  int u = 0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    int p = __shfl_up(c[r], 1, 16);
    const int last = r > 0 ? __shfl(c[r - 1], 15, 16) : PAD;
    if (tl == 0) p = last;
    const bool f = c[r] != PAD && ((r == 0 && tl == 0) || c[r] != p);
    const unsigned msk = team_bits(__ballot(f));
    if (f && mine) cb[u + __popc(msk & ((1u << tl) - 1u))] = c[r];
    u += __popc(msk);
  }
  if (mine && tl == 0) rowcnt[v] = u;
}

// One row with ROW_S < m <= ROW_M by the whole wave (a block of one wave).
__device__ void row_a_wave(const SceneDev& S, const int* ai, const int* aj, const unsigned char* at, int v, int b,
                           int m, int* inc, int* colbuf, int* rowcnt, int* ent, int* tab, int4* stn) {
  const int lane = threadIdx.x;
  int* cb = colbuf + 4LL * b;
  if (m <= ROW_L) {
    // registers: entry q in lane q, candidate column 4q + t in lane
    // (4q + t) & 63, register (4q + t) >> 6
    int e = lane < m ? inc[b + lane] : PAD;
    e = wave_sort64(e);
    int vv[4] = {PAD, PAD, PAD, PAD};
    if (lane < m) {
      inc[b + lane] = e;
      const int k = e >> 2;
      pair_verts(S, at[k], ai[k], aj[k], vv);
      stn[b + lane] = make_int4(vv[0], vv[1], vv[2], vv[3]);
    }
    const int t = lane & 3, q0 = lane >> 2, q1 = 16 + (lane >> 2);
    int w0 = __shfl(vv[0], q0, 64), w1 = __shfl(vv[1], q0, 64), w2 = __shfl(vv[2], q0, 64),
        w3 = __shfl(vv[3], q0, 64);
    int c0 = t == 0 ? w0 : t == 1 ? w1 : t == 2 ? w2 : w3;
    w0 = __shfl(vv[0], q1, 64); w1 = __shfl(vv[1], q1, 64); w2 = __shfl(vv[2], q1, 64); w3 = __shfl(vv[3], q1, 64);
    int c1 = t == 0 ? w0 : t == 1 ? w1 : t == 2 ? w2 : w3;
    wave_sort128(c0, c1);
    const int p0 = __shfl_up(c0, 1, 64), last0 = __shfl(c0, 63, 64);
    int p1 = __shfl_up(c1, 1, 64);
    if (lane == 0) p1 = last0;
    const bool f0 = c0 != PAD && (lane == 0 || c0 != p0);
    const bool f1 = c1 != PAD && c1 != p1;
    const unsigned long long m0 = __ballot(f0), m1 = __ballot(f1);
    const int u0 = __popcll(m0);
    if (f0) cb[lanes_below(m0)] = c0;
    if (f1) cb[u0 + lanes_below(m1)] = c1;
    if (lane == 0) rowcnt[v] = u0 + __popcll(m1);
    return;
  }
  // LDS
  const int Pm = pow2_at_least(m);
  for (int q = lane; q < Pm; q += 64) ent[q] = q < m ? inc[b + q] : PAD;
  const int T = min(ROW_M_TAB, pow2_at_least(4 * m + 1));
  for (int q = lane; q < T; q += 64) tab[q] = EMPTY;
  __syncthreads();
  team_bitonic<64>(ent, Pm);
  for (int q = lane; q < m; q += 64) {
    int e = ent[q], k = e >> 2;
    inc[b + q] = e;
    int vv[4];
    pair_verts(S, at[k], ai[k], aj[k], vv);
    stn[b + q] = make_int4(vv[0], vv[1], vv[2], vv[3]);
#pragma unroll
    for (int c = 0; c < 4; ++c) set_insert(tab, T, vv[c]);
  }
  __syncthreads();
  int u = 0;  // compact the set in place (a chunk is read before any of it is written)
  for (int c = 0; c < T; c += 64) {
    int x = tab[c + lane];
    bool ok = x != EMPTY;
    unsigned long long msk = __ballot(ok);
    if (ok) tab[u + lanes_below(msk)] = x;
    u += __popcll(msk);
  }
  const int P = pow2_at_least(u > 0 ? u : 1);
  for (int q = u + lane; q < P; q += 64) tab[q] = PAD;
  __syncthreads();
  team_bitonic<64>(tab, P);
  for (int q = lane; q < u; q += 64) cb[q] = tab[q];
  if (lane == 0) rowcnt[v] = u;
  __syncthreads();
}

// Rows 4j .. 4j + 3 per block of one wave: first the rows with m <= ROW_S
// (a team each), then those with m <= ROW_M one after another.
__global__ __launch_bounds__(64) void k_row_a(SceneDev S, const int* ai, const int* aj, const unsigned char* at,
                                              const int* inc_off, int* inc, int* colbuf, int* rowcnt, int* mid,
                                              int* big, int4* stn) {
  __shared__ int ent[ROW_M];
  __shared__ int tab[ROW_M_TAB];
  const int t = lane_id() >> 4;
  for (long long v0 = 4LL * blockIdx.x; v0 < S.nv; v0 += 4LL * gridDim.x) {
    const int v = (int)v0 + t;
    int b = 0, m = 0;
    if (v < S.nv) {
      b = inc_off[v];
      m = inc_off[v + 1] - b;
    }
    const bool small = v < S.nv && m <= ROW_S;
    if (__all(!small || m == 0)) {  // nothing to sort in this group
      if (small && (lane_id() & 15) == 0) rowcnt[v] = 0;
    } else {
      row_a_team(S, ai, aj, at, small, v, b, m, inc, colbuf, rowcnt, stn);
    }
    // rows for the one-wave path of pass B: appended to mid[0 .. mid[nv]) (any order)
    const unsigned long long lead = __ballot((lane_id() & 15) == 0 && v < S.nv && m > ROW_S && m <= ROW_M);
    if (lead != 0) {
      int base = 0;
      if (lane_id() == 0) base = atomicAdd(&mid[S.nv], __popcll(lead));
      base = __shfl(base, 0, 64);
      if ((lead >> lane_id()) & 1ull) mid[base + lanes_below(lead)] = v;
    }
    // rows for the block-per-row paths: appended to big[0 .. big[nv])
    const unsigned long long blead = __ballot((lane_id() & 15) == 0 && v < S.nv && m > ROW_M);
    if (blead != 0) {
      int base = 0;
      if (lane_id() == 0) base = atomicAdd(&big[S.nv], __popcll(blead));
      base = __shfl(base, 0, 64);
      if ((blead >> lane_id()) & 1ull) big[base + lanes_below(blead)] = v;
    }
#pragma unroll 1
    for (int r = 0; r < 4; ++r) {
      const int vr = __shfl(v, 16 * r, 64), br = __shfl(b, 16 * r, 64), mr = __shfl(m, 16 * r, 64);
      if (vr >= S.nv || mr <= ROW_S || mr > ROW_M) continue;  // uniform over the wave
      row_a_wave(S, ai, aj, at, vr, br, mr, inc, colbuf, rowcnt, ent, tab, stn);
    }
  }
}

// Rows with m > ROW_M (passes A and B): one 256-thread block per row, the
// rows taken from pass A's list strided over the blocks (they cluster in
// space, and so in vertex numbering: a list spreads them evenly).
__global__ __launch_bounds__(256) void k_row_a_big(SceneDev S, const int* ai, const int* aj, const unsigned char* at,
                                                   const int* inc_off, int* inc, int* colbuf, int* rowcnt,
                                                   const int* big, int4* stn) {
  __shared__ int ent[ROW_H];
  __shared__ int tab[ROW_H_TAB];
  const int tid = threadIdx.x;
  const int nbig = big[S.nv];
  for (int r = blockIdx.x; r < nbig; r += gridDim.x) {
    const int v = big[r];
    const int b = inc_off[v], m = inc_off[v + 1] - b;
    int* cb = colbuf + 4LL * b;
    if (m > ROW_H) {
      if (tid == 0) row_a_serial(S, ai, aj, at, b, m, inc, cb, rowcnt + v, stn);
      __syncthreads();
      continue;
    }
    const int Pm = pow2_at_least(m);
    for (int q = tid; q < Pm; q += 256) ent[q] = q < m ? inc[b + q] : PAD;
    const int T = min(ROW_H_TAB, pow2_at_least(4 * m + 1));
    for (int q = tid; q < T; q += 256) tab[q] = EMPTY;
    __syncthreads();
    team_bitonic<256>(ent, Pm);
    for (int q = tid; q < m; q += 256) {
      int e = ent[q], k = e >> 2;
      inc[b + q] = e;
      int vv[4];
      pair_verts(S, at[k], ai[k], aj[k], vv);
      stn[b + q] = make_int4(vv[0], vv[1], vv[2], vv[3]);
#pragma unroll
      for (int c = 0; c < 4; ++c) set_insert(tab, T, vv[c]);
    }
    __syncthreads();
    int u = 0;
    for (int c = 0; c < T; c += 256) {
      int x = tab[c + tid];
      int tot;
      int o = block_excl_scan256(x != EMPTY ? 1 : 0, &tot);  // synchronises: the chunk is read
      if (x != EMPTY) tab[u + o] = x;
      u += tot;
      __syncthreads();
    }
    const int P = pow2_at_least(u > 0 ? u : 1);
    for (int q = u + tid; q < P; q += 256) tab[q] = PAD;
    __syncthreads();
    team_bitonic<256>(tab, P);
    for (int q = tid; q < u; q += 256) cb[q] = tab[q];
    if (tid == 0) rowcnt[v] = u;
    __syncthreads();
  }
}

// Slot (0..3) of vertex c in a pair's stencil, -1 if absent.
__device__ __forceinline__ int slot_of(const int* vv, int c) {
  return vv[0] == c ? 0 : vv[1] == c ? 1 : vv[2] == c ? 2 : vv[3] == c ? 3 : -1;
}

// Pass B of one row by the NT threads of the block.  Every thread owns up to
// two of the row's columns per pass (2 NT columns a pass).  The row's entries
// are taken CH at a time: NT / CH threads per entry load the entry's band
// (rows 3s..3s+2 of its pair's 12 x 12 Hessian: 36 contiguous doubles) into
// LDS beside the pair's stencil vertices; each owner then adds the 3x3 blocks
// of its columns from LDS, entries in sorted order.
template <int NT, int CH, class HT>
__device__ __forceinline__ void row_b(const SceneDev& S, const int* ai, const int* aj, const unsigned char* at,
                                      const int* inc, int b, int m, const int* cb, int r0, int u, const double* G,
                                      const HT* H, double* grow, int* col, double* val, int* vs, HT* band,
                                      double* gw, const int4* stn) {
  constexpr int TPE = NT / CH, PART = 36 / TPE;  // threads per entry, doubles per thread
  static_assert(TPE * PART == 36, "band split");
  const int tid = threadIdx.x, lane = lane_id();
  double gsum[3] = {0.0, 0.0, 0.0};  // the row's gradient (thread 0), chunk by chunk in entry order
  if (m == 0 && tid == 0) grow[0] = grow[1] = grow[2] = 0.0;
  for (int cbase = 0; cbase < u; cbase += 2 * NT) {
    const int ca = cbase + tid < u ? cb[cbase + tid] : EMPTY;
    const int cz = cbase + NT + tid < u ? cb[cbase + NT + tid] : EMPTY;
    double A[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, Z[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int qc = 0; qc < m; qc += CH) {
      const int nq = min(CH, m - qc);
      const int q = tid / TPE, part = tid % TPE;
      double gx = 0.0, gy = 0.0, gz = 0.0;
      if (q < nq) {
        const int e = inc[b + qc + q], k = e >> 2;
        const HT* src = H + (long long)PK_N * k;  // the band of slot e & 3, gathered from the packed record
        const unsigned char* map = kPk.band[e & 3] + PART * part;
        HT* dst = band + 36 * q + PART * part;
#pragma unroll
        for (int o = 0; o < PART; ++o) dst[o] = src[map[o]];
        if (part == 0) {
          const int4 w4 = stn[b + qc + q];
          vs[4 * q] = w4.x;
          vs[4 * q + 1] = w4.y;
          vs[4 * q + 2] = w4.z;
          vs[4 * q + 3] = w4.w;
          if (cbase == 0) {
            const double* gk = G + 12LL * k + 3 * (e & 3);
            gx = gk[0]; gy = gk[1]; gz = gk[2];
          }
        }
      }
      if (cbase == 0) {  // gradient of this chunk: fixed-order sums over the lanes, then the waves
        wave_ordered_sum3(gx, gy, gz);
        if (NT == 64) {
          if (tid == 0) { gsum[0] += gx; gsum[1] += gy; gsum[2] += gz; }
        } else {
          if (lane == 0) { gw[3 * (tid >> 6)] = gx; gw[3 * (tid >> 6) + 1] = gy; gw[3 * (tid >> 6) + 2] = gz; }
        }
      }
      __syncthreads();
      if (NT != 64 && cbase == 0 && tid == 0)
        for (int a = 0; a < 3; ++a) gsum[a] += ((gw[a] + gw[3 + a]) + gw[6 + a]) + gw[9 + a];
      for (int r = 0; r < nq; ++r) {
        const int w[4] = {vs[4 * r], vs[4 * r + 1], vs[4 * r + 2], vs[4 * r + 3]};
        const HT* bq = band + 36 * r;
        const int sa = slot_of(w, ca), sz = slot_of(w, cz);
        if (sa >= 0) {
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) A[3 * i + j] += bq[12 * i + 3 * sa + j];
        }
        if (sz >= 0) {
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) Z[3 * i + j] += bq[12 * i + 3 * sz + j];
        }
      }
      __syncthreads();
    }
    if (cbase == 0 && tid == 0) { grow[0] = gsum[0]; grow[1] = gsum[1]; grow[2] = gsum[2]; }
    if (ca != EMPTY) {
      col[r0 + cbase + tid] = ca;
#pragma unroll
      for (int o = 0; o < 9; ++o) val[9LL * (r0 + cbase + tid) + o] = A[o];
    }
    if (cz != EMPTY) {
      col[r0 + cbase + NT + tid] = cz;
#pragma unroll
      for (int o = 0; o < 9; ++o) val[9LL * (r0 + cbase + NT + tid) + o] = Z[o];
    }
  }
}

// Pass B of rows with m <= ROW_S, one per 16-lane team.  Lane q < m holds
// entry q: its pair's stencil vertices go to the team's slice of vs, its
// gradient part into a fixed-order tree over the team's lanes.  Lane tl owns
// column tl of each group of 16.  The entries are taken
// four at a time: four lanes per entry copy its band (36 contiguous
// doubles) into the team's slice of `band`, then each owner adds the 3x3
// blocks of its columns, entries in sorted order.  Teams with m = 0 and
// u = 0 only take part in the shuffles and barriers (a block is one wave).
constexpr int TEAM_CH = 4;  // entries per chunk and team
template <class HT>
__device__ __forceinline__ void row_b_team(const SceneDev& S, const int* ai, const int* aj, const unsigned char* at,
                                           bool mine, const int* inc, int b, int m, const int* cb, int r0, int u,
                                           const double* G, const HT* H, double* grow, int* col, double* val,
                                           int* vs, HT* band, const int4* stn) {
  const int lane = lane_id(), tl = lane & 15;
  int* vst = vs + 4 * ROW_S * (lane >> 4);
  HT* bt = band + 36 * TEAM_CH * (lane >> 4);
  int e = 0;
  int vv[4] = {EMPTY, EMPTY, EMPTY, EMPTY};
  double gx = 0.0, gy = 0.0, gz = 0.0;
  if (tl < m) {
    e = inc[b + tl];
    const int k = e >> 2;
    const int4 w4 = stn[b + tl];
    vv[0] = w4.x; vv[1] = w4.y; vv[2] = w4.z; vv[3] = w4.w;
    const double* gk = G + 12LL * k + 3 * (e & 3);
    gx = gk[0]; gy = gk[1]; gz = gk[2];
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) vst[4 * tl + c] = vv[c];
#pragma unroll
  for (int o = 1; o < 16; o <<= 1) {
    const double tx = __shfl_down(gx, o, 16), ty = __shfl_down(gy, o, 16), tz = __shfl_down(gz, o, 16);
    if ((tl & (2 * o - 1)) == 0) { gx += tx; gy += ty; gz += tz; }
  }
  if (mine && tl == 0) { grow[0] = gx; grow[1] = gy; grow[2] = gz; }
  const int r = tl >> 2, part = tl & 3;  // chunk entry and quarter of its band copied by this lane
  for (int cbase = 0; !__all(cbase >= u); cbase += 16) {
    const int ca = cbase + tl < u ? cb[cbase + tl] : EMPTY;
    double A[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int qc = 0; !__all(qc >= m); qc += TEAM_CH) {
      const int eq = __shfl(e, qc + r, 16);
      __syncthreads();  // the stencils are written, the previous chunk is read
      if (qc + r < m) {
        const HT* src = H + (long long)PK_N * (eq >> 2);  // the band of slot eq & 3, from the packed record
        const unsigned char* map = kPk.band[eq & 3] + 9 * part;
        HT* dst = bt + 36 * r + 9 * part;
#pragma unroll
        for (int o = 0; o < 9; ++o) dst[o] = src[map[o]];
      }
      __syncthreads();
      const int nq = min(TEAM_CH, m - qc);
#pragma unroll 1
      for (int q = 0; q < nq; ++q) {
        const int w[4] = {vst[4 * (qc + q)], vst[4 * (qc + q) + 1], vst[4 * (qc + q) + 2], vst[4 * (qc + q) + 3]};
        const HT* bq = bt + 36 * q;
        const int sa = slot_of(w, ca);
        if (sa >= 0) {
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) A[3 * i + j] += bq[12 * i + 3 * sa + j];
        }
      }
    }
    if (ca != EMPTY) {
      col[r0 + cbase + tl] = ca;
#pragma unroll
      for (int o = 0; o < 9; ++o) val[9LL * (r0 + cbase + tl) + o] = A[o];
    }
  }
}

// Pass B for rows with m <= ROW_M, blocks of one wave.  The first
// nmid_blocks blocks take the rows that pass A listed (ROW_S < m <= ROW_M)
// one at a time (strided over the list); every other block takes four
// consecutive rows and works on those with m <= ROW_S, a team each.  Block
// 0 also stores the block count and the total energy.
template <class HT>
__global__ __launch_bounds__(64) void k_row_b(SceneDev S, const int* ai, const int* aj, const unsigned char* at,
                                              const int* inc_off, const int* inc, const int* colbuf, const double* G,
                                              const HT* H, double* g, const int* row_ptr, int* col, double* val,
                                              long long cap, long long* nnzb, unsigned* status,
                                              const unsigned long long* act_count, long long acap,
                                              const double* epart, double* E_out, const int* mid, int nmid_blocks,
                                              const int4* stn) {
  // shared by both paths: 4 teams x ROW_S stencils / 32 entries' stencils,
  // 4 teams x TEAM_CH bands / 32 bands (a listed row's entries 32 at a time:
  // fewer dependent rounds of band loads than 16, and 64 take too much LDS)
  __shared__ int vs[4 * 4 * ROW_S];
  __shared__ HT band[32 * 36];  // the bands in the records' precision (summed in FP64)
  static_assert(4 * TEAM_CH <= 32, "team bands fit the shared band buffer");
  if (blockIdx.x == 0) {
    if (threadIdx.x == 0) {
      const long long t = row_ptr[S.nv];
      *nnzb = t;
      if (t > cap) atomicOr(status, (unsigned)BF_S_BSR_OVERFLOW);
    }
    // energy: the per-tile sums of the evaluation kernel, in tile order
    long long n = (long long)*act_count;
    if (n > acap) n = acap;
    energy_total(epart, (n + 63) / 64, E_out);
  }
  if ((int)blockIdx.x < nmid_blocks) {  // the listed rows, one at a time by the whole wave
    const int n = mid[S.nv];
    for (int q = blockIdx.x; q < n; q += nmid_blocks) {
      const int v = mid[q];
      const int b = inc_off[v], m = inc_off[v + 1] - b;
      const int r0 = row_ptr[v], r1 = row_ptr[v + 1];
      if (r1 > cap) continue;  // overflow: reported by block 0
      row_b<64, 32>(S, ai, aj, at, inc, b, m, colbuf + 4LL * b, r0, r1 - r0, G, H, g + 3LL * v, col, val, vs, band,
                    nullptr, stn);
    }
    return;
  }
  const int t = lane_id() >> 4;
  const int nteam_blocks = (int)gridDim.x - nmid_blocks;
  for (long long v0 = 4LL * ((int)blockIdx.x - nmid_blocks); v0 < S.nv; v0 += 4LL * nteam_blocks) {
    const int v = (int)v0 + t;
    int b = 0, m = 0, r0 = 0, r1 = 0;
    if (v < S.nv) {
      b = inc_off[v];
      m = inc_off[v + 1] - b;
      r0 = row_ptr[v];
      r1 = row_ptr[v + 1];
    }
    const bool small = v < S.nv && m <= ROW_S;
    // columns are stored only when the row fits the output (overflow is reported above)
    const int u = small && r1 <= cap ? r1 - r0 : 0;
    row_b_team(S, ai, aj, at, small, inc, b, small ? m : 0, colbuf + 4LL * b, r0, u, G, H, g + 3LL * v, col, val, vs,
               band, stn);
  }
}

template <class HT>
__global__ __launch_bounds__(256) void k_row_b_big(SceneDev S, const int* ai, const int* aj, const unsigned char* at,
                                                   const int* inc_off, const int* inc, const int* colbuf,
                                                   const double* G, const HT* H, double* g, const int* row_ptr,
                                                   int* col, double* val, long long cap, const int* big,
                                                   const int4* stn) {
  __shared__ int vs[4 * 64];
  __shared__ HT band[64 * 36];
  __shared__ double gw[12];
  const int nbig = big[S.nv];
  for (int r = blockIdx.x; r < nbig; r += gridDim.x) {
    const int v = big[r];
    const int b = inc_off[v], m = inc_off[v + 1] - b;
    const int r0 = row_ptr[v], r1 = row_ptr[v + 1];
    if (r1 > cap) continue;  // uniform across the block
    row_b<256, 64>(S, ai, aj, at, inc, b, m, colbuf + 4LL * b, r0, r1 - r0, G, H, g + 3LL * v, col, val, vs, band,
                    gw, stn);
  }
}

// ---------------------------------------------------------------------------
// Line search (Sec. 3.3, last paragraph; App. A): additive CCD with the
// filtered offsets, and the energy alone at a trial point.
// ---------------------------------------------------------------------------

// Additive CCD (Li, Kaufman and Jiang 2021, C-IPC) of one stencil with offset
// xi along the displacements P: the distance between the primitives closes
// at most at rate lp (largest displacement on one side plus the largest on
// the other, after the stencil's mean displacement is removed), so steps of
// (1 - s) of the gap, then 0.9 of the current gap, never reach the offset.
// The search stops before the step after which the gap is below s of the
// initial gap, or at the full step 1, or after max_iter steps.  Positions
// advance by additions of products (no fused multiply-add).
// The search as a state that advances one step at a time (a lane whose pair
// finishes can take the next pair while the others keep stepping).
struct Accd {
  d3 X[4], P[4];
  double lp, xi, xi2, g, t, tl;
  int type, it;
};

// Set-up of one stencil: returns true when steps are needed, else the step
// in t (1 without relative motion, 0 at or inside the offset).
__device__ __forceinline__ bool accd_setup(Accd& A, int type, const d3* X0, const d3* P0, double xi, double s,
                                           double& t) {
  d3 pm;
  pm.x = (((P0[0].x + P0[1].x) + P0[2].x) + P0[3].x) / 4.0;
  pm.y = (((P0[0].y + P0[1].y) + P0[2].y) + P0[3].y) / 4.0;
  pm.z = (((P0[0].z + P0[1].z) + P0[2].z) + P0[3].z) / 4.0;
  double nr[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    A.X[k] = X0[k];
    A.P[k] = P0[k] - pm;
    nr[k] = sqrt(dot(A.P[k], A.P[k]));
  }
  A.type = type;
  A.it = 0;
  A.lp = type == BF_PT ? nr[0] + fmax(nr[1], fmax(nr[2], nr[3])) : fmax(nr[0], nr[1]) + fmax(nr[2], nr[3]);
  if (A.lp == 0.0) { t = 1.0; return false; }
  A.xi = xi;
  A.xi2 = xi * xi;
  const double D = type == BF_PT ? classify_pt(A.X).D : classify_ee(A.X).D;
  const double gap0 = (D - A.xi2) / (sqrt(D) + xi);
  if (!(gap0 > 0.0)) { t = 0.0; return false; }  // at or inside the offset already
  A.g = s * gap0;
  A.t = 0.0;
  A.tl = (1.0 - s) * gap0 / A.lp;
  return true;
}

// One step: returns false once the search has ended, with the step in t.
__device__ __forceinline__ bool accd_step(Accd& A, int max_iter, double& t) {
  A.it += 1;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    A.X[k].x = __dadd_rn(A.X[k].x, __dmul_rn(A.tl, A.P[k].x));
    A.X[k].y = __dadd_rn(A.X[k].y, __dmul_rn(A.tl, A.P[k].y));
    A.X[k].z = __dadd_rn(A.X[k].z, __dmul_rn(A.tl, A.P[k].z));
  }
  const double D = A.type == BF_PT ? classify_pt(A.X).D : classify_ee(A.X).D;
  const double gap = (D - A.xi2) / (sqrt(D) + A.xi);
  if (A.t > 0.0 && gap < A.g) { t = A.t; return false; }
  A.t += A.tl;
  if (A.t > 1.0) { t = 1.0; return false; }
  A.tl = 0.9 * gap / A.lp;
  if (A.it >= max_iter) { t = A.t; return false; }
  return true;
}

// Exact swept-box test of a candidate (the definition of the CCD pair set):
// the boxes of each primitive's vertices at x and x + p, gap below h on
// every axis, in double.
__device__ __forceinline__ bool swept_within(int type, const d3* X, const d3* P, double h) {
  const int na = type == BF_PT ? 1 : 2;
  double lo[2][3], hi[2][3];
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int c = 0; c < 3; ++c) { lo[q][c] = INFINITY; hi[q][c] = -INFINITY; }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int q = k < na ? 0 : 1;
    const double a[3] = {X[k].x, X[k].y, X[k].z}, b[3] = {X[k].x + P[k].x, X[k].y + P[k].y, X[k].z + P[k].z};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      lo[q][c] = fmin(lo[q][c], fmin(a[c], b[c]));
      hi[q][c] = fmax(hi[q][c], fmax(a[c], b[c]));
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c)
    if (!(fmax(lo[1][c] - hi[0][c], lo[0][c] - hi[1][c]) < h)) return false;
  return true;
}

// Per candidate: ACCD if its swept boxes are within h (offset 0 for filtered
// stencils, eta otherwise; Eq. 4), t = -1 otherwise (and its step count);
// the minimum per block.
// Lists of capacity up to ACCD_REFILL_MAX (a few candidates per lane of the
// chip) are launched on at most ACCD_REFILL_BLOCKS blocks, which split the
// list into contiguous shares, one per wave.  Once half a wave's lanes have no search in progress, those
// lanes set up the next candidates of the share, and every round each lane
// with a search in progress takes one step, so lanes whose searches end early
// are refilled instead of idling until the longest search of their wave ends
// (a refill waits on the candidates' loads, so it is done for many lanes at
// once).  Longer lists: one candidate per lane at a time over the whole grid,
// where other waves hide each wave's loads.  The step of each pair does not
// depend on which lane computes it.
constexpr long long ACCD_REFILL_MAX = 1 << 21;
constexpr int ACCD_REFILL_BLOCKS = 512;
__global__ __launch_bounds__(256) void k_accd(SceneDev S, const double* x, const double* pdisp, const int* ci,
                                              const int* cj, const unsigned char* ct, const long long* cand_count,
                                              long long ccap, double s, int max_iter, double* tpair, int* iters,
                                              double* bmin) {
  long long n = *cand_count;
  if (n > ccap) n = ccap;
  const int lane = lane_id();
  double tmin = 1.0;
  if ((int)gridDim.x <= ACCD_REFILL_BLOCKS) {  // the launch's choice (by capacity)
    const int blocks = (int)gridDim.x;
    {
      const long long nwaves = (long long)blocks * (blockDim.x >> 6);
      const long long wv = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
      const long long share = (n + nwaves - 1) / nwaves;
      long long next = wv * share;  // next candidate of the share (same on every lane)
      const long long end = next + share < n ? next + share : n;
      Accd A;
      long long k = -1;             // this lane's candidate in progress
      while (true) {
        if (__popcll(__ballot(k < 0)) >= 32) while (true) {
          const bool need = k < 0;
          const unsigned long long needy = __ballot(need);
          if (needy == 0 || next >= end) break;
          if (need) {
            const long long kk = next + lanes_below(needy);
            if (kk < end) {
              const int type = ct[kk];
              int v[4];
              pair_verts(S, type, ci[kk], cj[kk], v);
              d3 X[4], P[4];
#pragma unroll
              for (int q = 0; q < 4; ++q) { X[q] = load3(x, v[q]); P[q] = load3(pdisp, v[q]); }
              double t = -1.0;
              bool go = false;
              if (!is_culled(S, type, ci[kk], cj[kk]) && swept_within(type, X, P, S.h)) {
                const double xi = is_filtered(S, type, v, nullptr) || in_core(S, type, ci[kk], cj[kk]) ? 0.0 : S.eta;
                go = accd_setup(A, type, X, P, xi, s, t);
              }
              if (go) {
                k = kk;
              } else {  // decided at set-up
                if (t >= 0.0) tmin = fmin(tmin, t);
                if (tpair) tpair[kk] = t;
                if (iters) iters[kk] = 0;
              }
            }
          }
          next += __popcll(needy);
        }
        if (__ballot(k >= 0) == 0) break;  // the share is done
        if (k >= 0) {
          double t;
          if (!accd_step(A, max_iter, t)) {
            tmin = fmin(tmin, t);
            if (tpair) tpair[k] = t;
            if (iters) iters[k] = A.it;
            k = -1;
          }
        }
      }
    }
  } else {
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n; k += grid_stride()) {
      const int type = ct[k];
      int v[4];
      pair_verts(S, type, ci[k], cj[k], v);
      d3 X[4], P[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) { X[q] = load3(x, v[q]); P[q] = load3(pdisp, v[q]); }
      double t = -1.0;
      int it = 0;
      if (!is_culled(S, type, ci[k], cj[k]) && swept_within(type, X, P, S.h)) {
        const double xi = is_filtered(S, type, v, nullptr) || in_core(S, type, ci[k], cj[k]) ? 0.0 : S.eta;
        Accd A;
        if (accd_setup(A, type, X, P, xi, s, t)) {
          while (accd_step(A, max_iter, t)) {
          }
          it = A.it;
        }
        tmin = fmin(tmin, t);
      }
      if (tpair) tpair[k] = t;
      if (iters) iters[k] = it;
    }
  }
  for (int o = 32; o > 0; o >>= 1) tmin = fmin(tmin, __shfl_xor(tmin, o, 64));
  __shared__ double wm[4];
  if (lane == 0) wm[threadIdx.x >> 6] = tmin;
  __syncthreads();
  if (threadIdx.x == 0) bmin[blockIdx.x] = fmin(fmin(wm[0], wm[1]), fmin(wm[2], wm[3]));
}

__global__ __launch_bounds__(256) void k_min_final(const double* bmin, int nb, double* out) {
  double m = 1.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) m = fmin(m, bmin[b]);
  for (int o = 32; o > 0; o >>= 1) m = fmin(m, __shfl_xor(m, o, 64));
  __shared__ double wm[4];
  if (lane_id() == 0) wm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) *out = fmin(fmin(wm[0], wm[1]), fmin(wm[2], wm[3]));
}

// Energy alone (Eq. 2 with the parameters of Eq. 4) of every candidate at x
// (or at x + alpha p when pdisp is given, alpha read from device memory):
// the same decisions as the narrow phase (d < h, the filter, d < a, d <= eta
// gives +inf); per block a fixed-order sum (each thread's candidates in
// order, then the lanes, then the four waves).
__global__ __launch_bounds__(256) void k_energy(SceneDev S, const double* x, const double* pdisp, const double* alpha,
                                                const int* ci, const int* cj, const unsigned char* ct,
                                                const long long* cand_count, long long ccap, double* bsum) {
  long long n = *cand_count;
  if (n > ccap) n = ccap;
  const dd h2 = dd_sq(S.h), e2 = dd_sq(S.eta);
  const double al = pdisp ? *alpha : 0.0;
  double e = 0.0;
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n; k += grid_stride()) {
    const int type = ct[k];
    int v[4];
    pair_verts(S, type, ci[k], cj[k], v);
    d3 P[4] = {load3(x, v[0]), load3(x, v[1]), load3(x, v[2]), load3(x, v[3])};
    if (pdisp) {  // trial point x + alpha p (a product, then a sum: no fused multiply-add)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const d3 d = load3(pdisp, v[q]);
        P[q].x = __dadd_rn(P[q].x, __dmul_rn(al, d.x));
        P[q].y = __dadd_rn(P[q].y, __dmul_rn(al, d.y));
        P[q].z = __dadd_rn(P[q].z, __dmul_rn(al, d.z));
      }
    }
    if (is_culled(S, type, ci[k], cj[k])) continue;
    const Near nr = type == BF_PT ? classify_pt(P) : classify_ee(P);
    if (!decide_sq(nr.code, P, nr.D, h2, true, nullptr)) continue;  // d >= h
    dd T;
    double a, eta;
    if (is_filtered(S, type, v, nullptr)) {
      const int c = S.comp[v[0]];
      T = dd{S.thr2[2 * c], S.thr2[2 * c + 1]};
      a = S.dmin[c];
      eta = 0.0;
    } else {
      T = h2;
      a = S.h;
      eta = in_core(S, type, ci[k], cj[k]) ? 0.0 : S.eta;
    }
    if (!decide_sq(nr.code, P, nr.D, T, true, nullptr)) continue;  // inactive: d >= a
    const bool infeas = eta > 0.0 ? decide_sq(nr.code, P, nr.D, e2, false, nullptr) : !(nr.D > 0.0);
    if (infeas) {
      e += INFINITY;
      continue;
    }
    double b, b1, b2;
    barrier3<double>(sqrt(nr.D), a, eta, b, b1, b2);
    e += S.kappa * b;
  }
  double y = 0.0, z = 0.0;
  wave_ordered_sum3(e, y, z);
  __shared__ double ws[4];
  if (lane_id() == 0) ws[threadIdx.x >> 6] = e;
  __syncthreads();
  if (threadIdx.x == 0) bsum[blockIdx.x] = ((ws[0] + ws[1]) + ws[2]) + ws[3];
}

// Fixed-order total of the per-block sums (one wave).
__global__ __launch_bounds__(64) void k_sum_final(const double* bsum, int nb, double* out) {
  energy_total(bsum, nb, out);
}

// ---------------------------------------------------------------------------
// Lagged friction (App. A: IPC's contact and friction energies; the lagged
// model of Li et al. 2020)
// ---------------------------------------------------------------------------

// Closest-point weights of sub-case `code` at X: the relative displacement of
// the pair's two closest points is sum_q w[q] dX_q.
__device__ __forceinline__ void friction_weights(int code, const d3* X, double* w) {
  const int kind = case_kind(code);
  if (kind == K_PT) {  // point 0 against the projection onto triangle (1, 2, 3)
    const d3 u = X[2] - X[1], v = X[3] - X[1], r = X[0] - X[1];
    const double uu = dot(u, u), uv = dot(u, v), vv = dot(v, v), ru = dot(r, u), rv = dot(r, v);
    const double det = uu * vv - uv * uv;
    const double b1 = (vv * ru - uv * rv) / det, b2 = (uu * rv - uv * ru) / det;
    w[0] = 1.0; w[1] = -(1.0 - b1 - b2); w[2] = -b1; w[3] = -b2;
    return;
  }
  if (kind == K_EE) {  // the two line points at parameters (alpha, beta)
    // in double-double: for nearly parallel edges the 2 x 2 system loses
    // about log10(1 / sin^2) digits, which FP64 cannot spare
    const q3 Q[4] = {q3_of(X[0]), q3_of(X[1]), q3_of(X[2]), q3_of(X[3])};
    const q3 ea = Q[1] - Q[0], eb = Q[3] - Q[2], r = Q[0] - Q[2];
    const dd A = dot(ea, ea), B = dot(ea, eb), C = dot(eb, eb), D = dot(ea, r), E = dot(eb, r);
    const dd den = A * C - B * B;
    const dd al = (B * E - C * D) / den, be = (A * E - B * D) / den;
    const dd one = dd_of(1.0);
    w[0] = (one - al).hi; w[1] = al.hi; w[2] = -(one - be).hi; w[3] = -be.hi;
    return;
  }
  int s0, s1, s2;
  case_slots(code, s0, s1, s2);
  double w0 = 1.0, w1 = -1.0, w2 = 0.0;  // point-point
  if (kind == K_PE) {                    // point s0 against edge (s1, s2) at parameter beta
    const d3 p = pick4(X, s0), e0 = pick4(X, s1), e1 = pick4(X, s2);
    const d3 e = e1 - e0;
    const double beta = dot(p - e0, e) / dot(e, e);
    w1 = -(1.0 - beta);
    w2 = -beta;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) w[q] = (q == s0 ? w0 : 0.0) + (q == s1 ? w1 : 0.0) + (q == s2 ? w2 : 0.0);
}

// Per active pair at the lagged positions: lambda = kappa |b'(d)| (0 when the
// pair is infeasible or not inside (eta, a)), weights w[4], contact normal n.
__global__ __launch_bounds__(256) void k_friction_lag(SceneDev S, const double* xl, const int* ai, const int* aj,
                                                      const unsigned char* at, const unsigned char* acode,
                                                      const unsigned char* aflags,
                                                      const unsigned long long* act_count, long long acap,
                                                      double* lam, double* wout, double* nout) {
  long long n = (long long)*act_count;
  if (n > acap) n = acap;
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n; k += grid_stride()) {
    const int type = at[k], code = acode[k], fl = aflags[k];
    int v[4];
    pair_verts(S, type, ai[k], aj[k], v);
    const d3 X[4] = {load3(xl, v[0]), load3(xl, v[1]), load3(xl, v[2]), load3(xl, v[3])};
    double w[4];
    friction_weights(code, X, w);
    d3 c = w[0] * X[0];
#pragma unroll
    for (int q = 1; q < 4; ++q) c = c + w[q] * X[q];
    const double cn = sqrt(dot(c, c));
    double l = 0.0;
    if (!(fl & BF_F_INFEASIBLE)) {
      double a, eta;
      if (fl & BF_F_FILTERED) { a = S.dmin[S.comp[v[0]]]; eta = 0.0; }
      else { a = S.h; eta = (fl & BF_F_CORE) ? 0.0 : S.eta; }
      const double d = sqrt(sqd_case<double>(code, X));
      if (d < a && d > eta) {
        double b, b1, b2;
        barrier3<double>(d, a, eta, b, b1, b2);
        l = S.kappa * fabs(b1);
      }
    }
    lam[k] = l;
#pragma unroll
    for (int q = 0; q < 4; ++q) wout[4 * k + q] = w[q];
    nout[3 * k] = c.x / cn;
    nout[3 * k + 1] = c.y / cn;
    nout[3 * k + 2] = c.z / cn;
  }
}

// Friction of every active pair at x against the lagged xl: with dt the part
// of sum_q w_q (x_q - xl_q) orthogonal to n and y = |dt|, energy
// mu lambda f0(y) (f0 = y at y >= eh, the smoothing cubic below), gradient
// w_q mu lambda f1(y)/y dt and Hessian blocks w_q w_r M with
// M = mu lambda ((f1' y - f1)/y^3 dt dt^T + f1/y (I - n n^T)), positive
// semidefinite as it stands.  Written into, or added to, the pair's E, G and
// H; one wave per 64 pairs also stores the tile's energy sum.
//
// Four waves per 64 pairs.  Each lane of the first wave computes its pair's
// w[4], force f[3] and M[9] and leaves them in LDS; the four waves then
// write the tile's 64 x 12 gradient and 64 x 78 packed Hessian entries as one
// contiguous run each (thread t takes entries t, t + 256, ...), rebuilding
// every entry from LDS as w_q f_i or w_q w_r M_ij.  Stores straight from each
// lane's registers would scatter every instruction over 64 records 624 bytes
// apart; the extra waves shorten the store loop of a tile.
constexpr int FR_ST = 17;  // LDS doubles per pair: w[4], f[3], M[9], pad (odd stride)
// Hessian records in the scene's precision (HT: FP32 in the mixed mode), the
// accumulation rounded once in that precision.
__device__ __forceinline__ double add_rn(double a, double b) { return __dadd_rn(a, b); }
__device__ __forceinline__ float add_rn(float a, float b) { return __fadd_rn(a, b); }
template <class HT>
__global__ __launch_bounds__(256) void k_friction_eval(SceneDev S, const double* x, const double* xl, const int* ai,
                                                      const int* aj, const unsigned char* at,
                                                      const unsigned long long* act_count, long long acap,
                                                      const double* lam, const double* win, const double* nin,
                                                      double mu, double eh, int accumulate, double* E, double* G,
                                                      HT* H, double* epart) {
  __shared__ double sm[64 * FR_ST];
  long long n = (long long)*act_count;
  if (n > acap) n = acap;
  const int tid = threadIdx.x, lane = tid & 63;
  const long long k0 = (long long)blockIdx.x * 64, k = k0 + lane;
  double e = 0.0;
  if (k0 < n) {
    double* my = sm + FR_ST * lane;
    if (tid < 64 && k < n) {
      int v[4];
      pair_verts(S, at[k], ai[k], aj[k], v);
      double w[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) w[q] = win[4 * k + q];
      const d3 nn = {nin[3 * k], nin[3 * k + 1], nin[3 * k + 2]};
      d3 dl = {0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < 4; ++q) dl = dl + w[q] * (load3(x, v[q]) - load3(xl, v[q]));
      const double dn = dot(dl, nn);
      const d3 dt = dl - dn * nn;
      const double y = sqrt(dot(dt, dt));
      double f0, g1, c1;  // f0, f1/y, (f1' y - f1)/y^3
      if (y >= eh) {
        f0 = y;
        g1 = 1.0 / y;
        c1 = -1.0 / (y * y * y);
      } else {
        f0 = -y * y * y / (3.0 * eh * eh) + y * y / eh + eh / 3.0;
        g1 = -y / (eh * eh) + 2.0 / eh;
        c1 = y > 0.0 ? -1.0 / (eh * eh * y) : 0.0;
      }
      const double ml = mu * lam[k];
      const double Ek = ml * f0;
      const d3 gv = (ml * g1) * dt;
      const double t[3] = {dt.x, dt.y, dt.z}, nv[3] = {nn.x, nn.y, nn.z};
#pragma unroll
      for (int q = 0; q < 4; ++q) my[q] = w[q];
      my[4] = gv.x;
      my[5] = gv.y;
      my[6] = gv.z;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
          my[7 + 3 * i + j] = ml * (c1 * t[i] * t[j] + g1 * ((i == j ? 1.0 : 0.0) - nv[i] * nv[j]));
      // accumulate: one rounded addition onto what is there (no contraction
      // with the product), so the sum equals contact + friction exactly
      E[k] = accumulate ? __dadd_rn(E[k], Ek) : Ek;
      e = E[k];
    }
    __syncthreads();
    const int rows = (int)(n - k0 < 64 ? n - k0 : 64);
    double* Gt = G + 12 * k0;
#pragma unroll
    for (int it = 0; it < 3; ++it) {
      const int idx = it * 256 + tid, pp = idx / 12, c = idx - 12 * pp;
      if (pp < rows) {
        const double* ps = sm + FR_ST * pp;
        const double val = __dmul_rn(ps[c / 3], ps[4 + c % 3]);
        Gt[idx] = accumulate ? __dadd_rn(Gt[idx], val) : val;
      }
    }
    HT* Ht = H + PK_N * k0;
    for (int it = 0; it < (64 * PK_N + 255) / 256; ++it) {  // the packed upper triangles, as one run
      const int idx = it * 256 + tid, pp = idx / PK_N, rem = idx - PK_N * pp;
      if (pp < rows) {
        const int rw = kPk.row[rem], cl = kPk.col[rem];
        const double* ps = sm + FR_ST * pp;
        const HT val = (HT)__dmul_rn(ps[rw / 3] * ps[cl / 3], ps[7 + 3 * (rw % 3) + cl % 3]);
        Ht[idx] = accumulate ? add_rn(Ht[idx], val) : val;
      }
    }
  }
  if (tid < 64) {  // the first wave holds the tile's energies
    double y2 = 0.0, z2 = 0.0;
    wave_ordered_sum3(e, y2, z2);
    if (tid == 0 && epart && k0 < acap) epart[blockIdx.x] = e;
  }
}

// ---------------------------------------------------------------------------
// Temporary zero offset (Sec. 3.4): marking, release, count
// ---------------------------------------------------------------------------

// Insert every candidate with d < h and d <= eta that is not a filtered
// stencil (exact decisions, as in the narrow phase).
__global__ __launch_bounds__(256) void k_core_mark(SceneDev S, const double* x, const int* ci, const int* cj,
                                                   const unsigned char* ct, const long long* cand_count,
                                                   long long ccap, unsigned long long* keys, unsigned char* live,
                                                   unsigned mask, long long cap, unsigned long long* count,
                                                   unsigned* status) {
  long long n = *cand_count;
  if (n > ccap) n = ccap;
  const dd h2 = dd_sq(S.h), e2 = dd_sq(S.eta);
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n; k += grid_stride()) {
    const int type = ct[k], i = ci[k], j = cj[k];
    int v[4];
    pair_verts(S, type, i, j, v);
    d3 P[4] = {load3(x, v[0]), load3(x, v[1]), load3(x, v[2]), load3(x, v[3])};
    if (is_culled(S, type, i, j)) continue;
    const Near nr = type == BF_PT ? classify_pt(P) : classify_ee(P);
    if (!decide_sq(nr.code, P, nr.D, h2, true, nullptr)) continue;    // d >= h
    if (is_filtered(S, type, v, nullptr)) continue;                  // stencils have no offset anyway
    if (!decide_sq(nr.code, P, nr.D, e2, false, nullptr)) continue;  // d > eta
    const unsigned long long key = core_key_of(type, i, j);
    unsigned h = core_hash(key) & mask;
    bool placed = false;
    for (unsigned p = 0; p <= mask; ++p) {
      const unsigned long long old = atomicCAS(&keys[h], CORE_EMPTY, key);
      if (old == CORE_EMPTY || old == key) {
        live[h] = 1;
        placed = old == CORE_EMPTY;
        break;
      }
      h = (h + 1) & mask;
    }
    if (!placed || (long long)atomicAdd(count, 1ull) >= cap) atomicOr(status, (unsigned)BF_S_CORE_OVERFLOW);
  }
}

// Release, for good, every live pair now at d > eta.
__global__ __launch_bounds__(256) void k_core_release(SceneDev S, const double* x, const unsigned long long* keys,
                                                      unsigned char* live, unsigned slots) {
  const dd e2 = dd_sq(S.eta);
  for (unsigned q = blockIdx.x * blockDim.x + threadIdx.x; q < slots; q += grid_stride()) {
    if (!live[q]) continue;
    const unsigned long long key = keys[q];
    const int type = (int)(key >> 62), i = (int)((key >> 31) & 0x7fffffffull), j = (int)(key & 0x7fffffffull);
    int v[4];
    pair_verts(S, type, i, j, v);
    d3 P[4] = {load3(x, v[0]), load3(x, v[1]), load3(x, v[2]), load3(x, v[3])};
    const Near nr = type == BF_PT ? classify_pt(P) : classify_ee(P);
    if (!decide_sq(nr.code, P, nr.D, e2, false, nullptr)) live[q] = 0;
  }
}

// Number of live pairs (one block).
__global__ __launch_bounds__(256) void k_core_count(const unsigned char* live, unsigned slots, long long* out) {
  long long c = 0;
  for (unsigned q = threadIdx.x; q < slots; q += blockDim.x) c += live[q];
  c = block_sum256(c);
  if (threadIdx.x == 0) *out = c;
}

__global__ void k_fill_u8(unsigned char* a, long long n, unsigned char v) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += grid_stride()) a[i] = v;
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
// Under the Euclidean reading (candidates found on the rest pose): dbar^2 of
// the rest-pose distance in double-double, rounded; a pair whose decision
// dbar < h double-double leaves open goes to the tie list (k_refmin_tie
// decides it exactly), and a pair of one component whose primitives touch
// at rest (dbar^2 <= 1e-12 h^2) sets bit 0 of flags[1].
__device__ __forceinline__ void refmin_put(unsigned long long* best, int c, unsigned long long key) {
  // one atomic per wave when every contributing lane has the same component
  const int first = __ffsll((long long)__ballot(c >= 0)) - 1;
  const int c0 = __shfl(c, first < 0 ? 0 : first, 64);
  const bool uniform = __ballot(c >= 0 && c != c0) == 0ull;
  if (uniform) {
    unsigned long long mk = key;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      unsigned long long y = __shfl_xor(mk, o, 64);
      mk = y < mk ? y : mk;
    }
    if (lane_id() == 0 && c0 >= 0) atomicMin(&best[c0], mk);
  } else if (c >= 0) {
    atomicMin(&best[c], key);
  }
}
__device__ __forceinline__ double rest_sq_dd(const d3* P, int code) {
  q3 Q[4] = {q3_of(P[0]), q3_of(P[1]), q3_of(P[2]), q3_of(P[3])};
  const dd q = sqd_case<dd>(code, Q);
  return q.hi + q.lo;  // round to nearest double
}
__global__ __launch_bounds__(256) void k_refmin(SceneDev S, const int* ci, const int* cj, const unsigned char* ct,
                                                const long long* count, long long cap, unsigned long long* best,
                                                long long* ties, long long tie_cap, unsigned long long* flags) {
  long long n = *count;
  if (n > cap) n = cap;
  const long long n_up = (n + 63) / 64 * 64;  // whole waves iterate together
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n_up; k += grid_stride()) {
    int c = -1;
    unsigned long long key = ~0ull;
    if (k < n) {
      int v[4];
      pair_verts(S, ct[k], ci[k], cj[k], v);
      if (S.comp[v[0]] == S.comp[v[2]]) {
        double val = -1.0;
        if (S.refdist == BF_REFDIST_EUCLID_REST) {
          d3 P[4];
          const Near nr = rest_near(S, ct[k], v, P);
          if (!(nr.D > 1e-12 * S.h * S.h)) {
            atomicOr(&flags[1], 1ull);
          } else {
            bool amb = false;
            const bool below = decide_sq(nr.code, P, nr.D, dd_sq(S.h), true, &amb);
            if (amb) {
              const unsigned long long t = atomicAdd(&flags[0], 1ull);
              if ((long long)t < tie_cap) ties[t] = k;
            } else if (below) {
              val = rest_sq_dd(P, nr.code);
            }
          }
        } else if (S.kind == 0) {
          double sa0 = S.ref[v[0]], sa1 = S.ref[v[1]], sb0 = S.ref[v[2]], sb1 = S.ref[v[3]];
          double gap = fmax(fmin(sb0, sb1) - fmax(sa0, sa1), fmin(sa0, sa1) - fmax(sb0, sb1));
          if (gap > 0.0 && gap < S.h) val = gap;
        } else {
          dd q = ref_sqdist_q(S, ct[k], v);
          if (dd_lt(dd_of(0.0), q) && dd_lt(q, dd_sq(S.h))) val = q.hi + q.lo;  // round to nearest double
        }
        if (val >= 0.0) {
          c = S.comp[v[0]];
          key = (unsigned long long)__double_as_longlong(val);
        }
      }
    }
    refmin_put(best, c, key);
  }
}

// The tie list of k_refmin (rest-pose distances within 1e-20 of h): dbar < h
// decided in exact arithmetic (expansions in an LDS slab per thread, as in
// k_exact); the pairs below h join the minimum.  Bit 1 of flags[1]: an
// expansion outgrew its slab.
__global__ __launch_bounds__(XP_TPB) void k_refmin_tie(SceneDev S, const int* ci, const int* cj,
                                                       const unsigned char* ct, const long long* ties,
                                                       long long tie_cap, unsigned long long* flags,
                                                       unsigned long long* best) {
  __shared__ double slab[XP_TPB * XP_WS];
  double* ws = slab + threadIdx.x * XP_WS;
  long long nt = (long long)flags[0];
  if (nt > tie_cap) nt = tie_cap;
  for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < nt; q += (long long)gridDim.x * blockDim.x) {
    const long long k = ties[q];
    int v[4];
    pair_verts(S, ct[k], ci[k], cj[k], v);
    d3 P[4];
    const Near nr = rest_near(S, ct[k], v, P);
    bool limit = false;
    const bool below = decide_sq_exact(nr.code, P, nr.D, dd_sq(S.h), true, ws, &limit);
    if (limit) atomicOr(&flags[1], 2ull);
    else if (below)
      atomicMin(&best[S.comp[v[0]]], (unsigned long long)__double_as_longlong(rest_sq_dd(P, nr.code)));
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

__global__ void k_status_take(unsigned* status, unsigned* dst) {
  if (threadIdx.x == 0) {
    dst[0] = status[0];
    status[0] = 0u;
  }
}
void run_status_take(unsigned* status, unsigned* dst, hipStream_t st) {
  hipLaunchKernelGGL(k_status_take, dim3(1), dim3(64), 0, st, status, dst);
}

void run_zero_i64(long long* a, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_ll, dim3(1), dim3(64), 0, st, a, n, nullptr, 0);
}

void run_lift_ref(const SceneDev& S, double* xref, hipStream_t st) {
  hipLaunchKernelGGL(k_lift_ref, dim3(nblocks(S.nv)), dim3(256), 0, st, S, xref);
}

template <int PQ>
static void launch_pairs(const SceneDev& S, int nquery, const BroadWs& W, bool l2, int* oi, int* oj,
                         unsigned char* ot, long long cap, long long* count, unsigned* status, int* seg_r,
                         unsigned* seg_t, long long seg_cap, hipStream_t st) {
  static_assert(PQ <= PQ_MAX, "pair_cnt, pair_bsum and pair_bseg hold PQ_MAX threads per query");
  int nb = (nquery * PQ + 255) / 256;
  hipLaunchKernelGGL(k_pair_count<PQ>, dim3(nb), dim3(256), 0, st, S, nquery, W.box, W.grid, W.cell_start,
                     W.sorted_id, W.sorted_box, W.sorted_vid, S.h, l2, W.pair_cnt, W.pair_bsum, W.pair_bseg, W.seg_count,
                     seg_r, seg_t,
                     seg_cap);
  scan_excl(W.pair_bsum, W.pair_bofs, nullptr, nb + 1, W.scan_tmp, status, st);
  hipLaunchKernelGGL(k_pair_emit<PQ>, dim3(nb), dim3(256), 0, st, S, nquery, W.box, W.grid, W.cell_start,
                     W.sorted_id, W.sorted_box, W.sorted_vid, S.h, l2, W.pair_cnt, W.pair_bofs, W.pair_bseg, seg_r, seg_t,
                     oi, oj, ot,
                     cap, count, status);
}

void run_broad(const SceneDev& S, const double* x, const double* pdisp, const BroadWs& W, int* oi, int* oj,
               unsigned char* ot, long long cap, long long* count, unsigned* status, int* seg_r, unsigned* seg_t,
               long long seg_cap, hipStream_t st) {
  int np = S.ne + S.nt + (S.kind == 1 ? S.nv : 0);
  int nstored = S.ne + S.nt;
  int nquery = S.kind == 1 ? S.nv + S.ne : S.ne;
  int nscan_max = 2 * W.max_cells + 1;
  const int* nscan_dev = &W.grid->nscan;
  hipLaunchKernelGGL(k_bounds, dim3(nblocks(np, 256, BOUNDS_BLOCKS)), dim3(256), 0, st, S, x, pdisp, np, W.box,
                     W.part, W.done, S.h, W.max_cells, W.grid, count);
  // cell counts are zero on entry: the scatter below returns them to zero
  hipLaunchKernelGGL(k_count, dim3(nblocks(nstored)), dim3(256), 0, st, nstored, S.ne, W.box, W.grid, W.cell_cnt,
                     W.cell_of, W.seg_count);
  scan_excl(W.cell_cnt, W.cell_start, nscan_dev, nscan_max, W.scan_tmp, status, st);
  hipLaunchKernelGGL(k_scatter, dim3(nblocks(nstored)), dim3(256), 0, st, nstored, W.box, W.cell_of, W.cell_cnt,
                     W.cell_start, W.placed_id, W.placed_box);
  hipLaunchKernelGGL(k_cell_order, dim3(nblocks(nstored)), dim3(256), 0, st, S, nstored, W.cell_of, W.cell_start,
                     W.placed_id, W.placed_box, W.sorted_id, W.sorted_box, W.sorted_vid);
  // boxes swept along a displacement (the line search): the per-axis test
  // alone, so that the candidates are the pairs whose swept boxes are within h
  const bool l2 = pdisp == nullptr;
  // one thread per (query, share of its cells): no grid-stride here
  switch (S.pq) {
    case 2: launch_pairs<2>(S, nquery, W, l2, oi, oj, ot, cap, count, status, seg_r, seg_t, seg_cap, st); break;
    case 8: launch_pairs<8>(S, nquery, W, l2, oi, oj, ot, cap, count, status, seg_r, seg_t, seg_cap, st); break;
    case 16: launch_pairs<16>(S, nquery, W, l2, oi, oj, ot, cap, count, status, seg_r, seg_t, seg_cap, st); break;
    default: launch_pairs<4>(S, nquery, W, l2, oi, oj, ot, cap, count, status, seg_r, seg_t, seg_cap, st); break;
  }
}

void run_accd(const SceneDev& S, const double* x, const double* pdisp, const int* ci, const int* cj,
              const unsigned char* ct, const long long* ccount, long long ccap, double s, int max_iter, double* tpair,
              int* iters, double* bred, double* t_out, hipStream_t st) {
  const int nb = ccap <= ACCD_REFILL_MAX ? nblocks(ccap, 256, ACCD_REFILL_BLOCKS)
                                        : std::max(ACCD_REFILL_BLOCKS + 1, nblocks(ccap, 256, LINE_BLOCKS));
  hipLaunchKernelGGL(k_accd, dim3(nb), dim3(256), 0, st, S, x, pdisp, ci, cj, ct, ccount, ccap, s, max_iter, tpair,
                     iters, bred);
  hipLaunchKernelGGL(k_min_final, dim3(1), dim3(256), 0, st, bred, nb, t_out);
}

void run_core_mark(const SceneDev& S, const double* x, const int* ci, const int* cj, const unsigned char* ct,
                   const long long* ccount, long long ccap, unsigned long long* keys, unsigned char* live,
                   unsigned slots, long long cap, long long* count, unsigned* status, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_u64, dim3(nblocks(slots)), dim3(256), 0, st, keys, (long long)slots, CORE_EMPTY);
  hipLaunchKernelGGL(k_fill_u8, dim3(nblocks(slots)), dim3(256), 0, st, live, (long long)slots, (unsigned char)0);
  hipLaunchKernelGGL(k_zero_ll, dim3(1), dim3(64), 0, st, count, 1, nullptr, 0);
  hipLaunchKernelGGL(k_core_mark, dim3(nblocks(ccap)), dim3(256), 0, st, S, x, ci, cj, ct, ccount, ccap, keys, live,
                     slots - 1, cap, (unsigned long long*)count, status);
}

void run_core_release(const SceneDev& S, const double* x, hipStream_t st) {
  const unsigned slots = S.core_mask + 1;
  hipLaunchKernelGGL(k_core_release, dim3(nblocks(slots)), dim3(256), 0, st, S, x, S.core_key,
                     const_cast<unsigned char*>(S.core_live), slots);
}

void run_core_count(const SceneDev& S, long long* out, hipStream_t st) {
  hipLaunchKernelGGL(k_core_count, dim3(1), dim3(256), 0, st, S.core_live, S.core_mask + 1, out);
}

void run_friction_lag(const SceneDev& S, const double* xl, const int* ai, const int* aj, const unsigned char* at,
                      const unsigned char* acode, const unsigned char* aflags, const long long* act_count,
                      long long acap, double* lam, double* w, double* n, hipStream_t st) {
  hipLaunchKernelGGL(k_friction_lag, dim3(nblocks(acap)), dim3(256), 0, st, S, xl, ai, aj, at, acode, aflags,
                     (const unsigned long long*)act_count, acap, lam, w, n);
}

void run_friction_eval(const SceneDev& S, const double* x, const double* xl, const int* ai, const int* aj,
                       const unsigned char* at, const long long* act_count, long long acap, const double* lam,
                       const double* w, const double* n, double mu, double eh, int accumulate, double* E, double* G,
                       void* H, double* epart, hipStream_t st) {
  if (S.mixed)
    hipLaunchKernelGGL(k_friction_eval<float>, dim3(nblocks(acap, 64, 1 << 30)), dim3(256), 0, st, S, x, xl, ai, aj,
                       at, (const unsigned long long*)act_count, acap, lam, w, n, mu, eh, accumulate, E, G, (float*)H,
                       epart);
  else
    hipLaunchKernelGGL(k_friction_eval<double>, dim3(nblocks(acap, 64, 1 << 30)), dim3(256), 0, st, S, x, xl, ai, aj,
                       at, (const unsigned long long*)act_count, acap, lam, w, n, mu, eh, accumulate, E, G,
                       (double*)H, epart);
}

void run_energy(const SceneDev& S, const double* x, const double* pdisp, const double* alpha, const int* ci,
                const int* cj, const unsigned char* ct, const long long* ccount, long long ccap, double* bred,
                double* E_out, hipStream_t st) {
  const int nb = nblocks(ccap, 256, LINE_BLOCKS);
  hipLaunchKernelGGL(k_energy, dim3(nb), dim3(256), 0, st, S, x, pdisp, alpha, ci, cj, ct, ccount, ccap, bred);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(64), 0, st, bred, nb, E_out);
}

void run_narrow(const SceneDev& S, const double* x, const int* ci, const int* cj, const unsigned char* ct,
                const long long* ccount, long long ccap, const StageWs& W, hipStream_t st) {
  int G = (int)((ccap + NW_TILE - 1) / NW_TILE);
  hipLaunchKernelGGL(k_narrow, dim3(G), dim3(256), 0, st, S, x, ci, cj, ct, ccount, ccap, W);
}

void run_compact(const SceneDev& S, const double* x, const int* ci, const int* cj, const unsigned char* ct,
                 long long ccap, const StageWs& W, int* ai, int* aj, unsigned char* at, unsigned char* acode,
                 unsigned char* aflags, double* adist, long long acap, long long* act_count, long long* counters,
                 unsigned* status, hipStream_t st) {
  int G = (int)((ccap + NW_TILE - 1) / NW_TILE);
  scan_excl(W.kcnt, W.kofs, nullptr, NW_KINDS * G + 1, W.scan_tmp, status, st);
  hipLaunchKernelGGL(k_compact, dim3(G), dim3(256), 0, st, W, G, ai, aj, at, acode, aflags, adist, acap, act_count,
                     counters, status);
  hipLaunchKernelGGL(k_band, dim3(BAND_BLOCKS), dim3(256), 0, st, S, x, ci, cj, ct, W, G);
  hipLaunchKernelGGL(k_exact, dim3(XP_BLOCKS), dim3(XP_TPB), 0, st, S, x, ci, cj, ct, W);
  hipLaunchKernelGGL(k_dfr_count, dim3(XP_BLOCKS), dim3(256), 0, st, W, G);
  hipLaunchKernelGGL(k_exact_emit, dim3(XP_BLOCKS), dim3(256), 0, st, W, G, ai, aj, at, acode, aflags, adist, acap,
                     act_count, counters, status);
}

void run_eval(const SceneDev& S, const double* x, const int* ai, const int* aj, const unsigned char* at,
              const unsigned char* acode, const unsigned char* aflags, const long long* act_count, long long acap,
              double* E, double* G, void* H, double* epart, hipStream_t st) {
  if (S.mixed)
    hipLaunchKernelGGL(k_eval<true>, dim3(nblocks(acap, 64, 65535)), dim3(64), 0, st, S, x, ai, aj, at, acode,
                       aflags, (const unsigned long long*)act_count, acap, E, G, H, epart);
  else
    hipLaunchKernelGGL(k_eval<false>, dim3(nblocks(acap, 64, 65535)), dim3(64), 0, st, S, x, ai, aj, at, acode,
                       aflags, (const unsigned long long*)act_count, acap, E, G, H, epart);
}

// the big rows' lists are strided over these blocks: enough for a block per
// row on the workloads (a few thousand big rows), the rest exit at once
static inline int big_grid_of(int nv) { return std::max(1, std::min(nv, 4096)); }

void run_asm_structure(const SceneDev& S, const int* ai, const int* aj, const unsigned char* at,
                       const unsigned char* aflags, const long long* act_count, long long acap, const AsmWs& A,
                       hipStream_t st) {
  const unsigned long long* nact = (const unsigned long long*)act_count;
  // incidence counts are zero on entry: k_inc_fill returns them to zero
  hipLaunchKernelGGL(k_inc_count, dim3(nblocks(acap)), dim3(256), 0, st, S, ai, aj, at, aflags, nact, acap,
                     A.inc_cnt, A.mid + S.nv, A.big + S.nv);
  scan_excl(A.inc_cnt, A.inc_off, nullptr, S.nv + 1, A.scan_tmp, S.status, st);
  hipLaunchKernelGGL(k_inc_fill, dim3(nblocks(acap)), dim3(256), 0, st, S, ai, aj, at, aflags, nact, acap, A.inc_cnt,
                     A.inc_off, A.inc);
  const int rows_grid = std::max(1, std::min((S.nv + 3) / 4, 1 << 20));  // four rows a block
  hipLaunchKernelGGL(k_row_a, dim3(rows_grid), dim3(64), 0, st, S, ai, aj, at, A.inc_off, A.inc, A.colbuf, A.rowcnt,
                     A.mid, A.big, A.stn);
  hipLaunchKernelGGL(k_row_a_big, dim3(big_grid_of(S.nv)), dim3(256), 0, st, S, ai, aj, at, A.inc_off, A.inc,
                     A.colbuf, A.rowcnt, A.big, A.stn);
}

template <class HT>
static void launch_rows_b(const SceneDev& S, const int* ai, const int* aj, const unsigned char* at,
                          const unsigned long long* nact, long long acap, const double* G, const HT* H, double* E_out,
                          double* g, int* row_ptr, int* col, double* val, long long bsr_cap, long long* nnzb,
                          const AsmWs& A, unsigned* status, hipStream_t st) {
  const int rows_grid = std::max(1, std::min((S.nv + 3) / 4, 1 << 20));  // four rows a block
  const int mid_grid = std::max(1, std::min(S.nv, 1 << 20));  // listed rows: a block each (the rest exit)
  hipLaunchKernelGGL(k_row_b<HT>, dim3(mid_grid + rows_grid), dim3(64), 0, st, S, ai, aj, at, A.inc_off, A.inc,
                     A.colbuf, G, H, g, row_ptr, col, val, bsr_cap, nnzb, status, nact, acap, A.epart, E_out, A.mid,
                     mid_grid, A.stn);
  hipLaunchKernelGGL(k_row_b_big<HT>, dim3(big_grid_of(S.nv)), dim3(256), 0, st, S, ai, aj, at, A.inc_off, A.inc,
                     A.colbuf, G, H, g, row_ptr, col, val, bsr_cap, A.big, A.stn);
}

void run_asm_values(const SceneDev& S, const int* ai, const int* aj, const unsigned char* at,
                    const long long* act_count, long long acap, const double* G, const void* H, double* E_out,
                    double* g, int* row_ptr, int* col, double* val, long long bsr_cap, long long* nnzb,
                    const AsmWs& A, unsigned* status, hipStream_t st) {
  const unsigned long long* nact = (const unsigned long long*)act_count;
  scan_excl(A.rowcnt, row_ptr, nullptr, S.nv + 1, A.scan_tmp, status, st);
  if (S.mixed)
    launch_rows_b(S, ai, aj, at, nact, acap, G, (const float*)H, E_out, g, row_ptr, col, val, bsr_cap, nnzb, A,
                  status, st);
  else
    launch_rows_b(S, ai, aj, at, nact, acap, G, (const double*)H, E_out, g, row_ptr, col, val, bsr_cap, nnzb, A,
                  status, st);
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
  scan_excl(flag, scan, nullptr, S.nv, scan_tmp, S.status, st);
  hipLaunchKernelGGL(k_cc_label, dim3(nblocks(S.nv)), dim3(256), 0, st, lab, scan, S.nv, comp);
  int last_scan = 0, last_flag = 0;
  if (hipMemcpyAsync(&last_scan, scan + S.nv - 1, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess) return -1;
  if (hipMemcpyAsync(&last_flag, flag + S.nv - 1, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess) return -1;
  if (hipStreamSynchronize(st) != hipSuccess) return -1;
  return last_scan + last_flag;
}

void run_refmin(const SceneDev& S, const int* ci, const int* cj, const unsigned char* ct, const long long* count,
                long long cap, unsigned long long* best, long long* ties, long long tie_cap,
                unsigned long long* flags, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_ll, dim3(1), dim3(64), 0, st, (long long*)flags, 2, nullptr, 0);
  hipLaunchKernelGGL(k_refmin, dim3(nblocks(cap)), dim3(256), 0, st, S, ci, cj, ct, count, cap, best, ties, tie_cap,
                     flags);
  if (S.refdist == BF_REFDIST_EUCLID_REST)
    hipLaunchKernelGGL(k_refmin_tie, dim3(XP_BLOCKS), dim3(XP_TPB), 0, st, S, ci, cj, ct, ties, tie_cap, flags, best);
}

}  // namespace bfc
