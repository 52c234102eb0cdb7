// C ABI of libbfc: scene lifecycle, argument checks, workspace, and the four
// per-step calls of the contact path (build_candidates, filter_pairs,
// eval_barrier, assemble_grad_hess).  See include/bfc.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "bfc_kernels.h"

using namespace bfc;

struct bf_scene {
  bf_params prm;
  int kind = 0, nv = 0, ne = 0, nt = 0, nc = 0;
  int* d_edges = nullptr;
  int* d_tris = nullptr;
  double* d_ref = nullptr;
  double* d_xrest = nullptr;  // [V,3] rest pose under BF_REFDIST_EUCLID_REST
  int* d_comp = nullptr;
  double* d_dmin = nullptr;
  double* d_thr2 = nullptr;
  unsigned* d_status = nullptr;
  double* d_line = nullptr;  // [LINE_BLOCKS] per-block minima / sums of the line-search calls
  int* d_eidx = nullptr;     // culling mode: [E] element index along the polyline
  int* d_eloop = nullptr;    // culling mode: [E] edge count of the edge's polyline if closed, else 0
  // temporary zero offset (Sec. 3.4): pair keys and live flags, core_slots a power of two (0: no set)
  unsigned long long* core_key = nullptr;
  unsigned char* core_live = nullptr;
  unsigned core_slots = 0;
  std::vector<void*> core_allocs;
  std::vector<int> comp_h;
  std::vector<double> dmin2_h, dmin_h;
  BroadWs bw{};
  StageWs sw{};
  AsmWs aw{};
  long long act_cap = 0;
  // lagged friction: the assembly structure of the lagged list, built once by
  // friction_lag and read by every friction_assemble until the next one
  AsmWs faw{};
  long long fasm_cap = 0;
  std::vector<void*> fasm_allocs;
  const void* fric_list = nullptr;  // the lagged list (its pair ids) the structure belongs to
  std::vector<void*> allocs;        // scene-lifetime allocations
  std::vector<void*> asm_allocs;    // assembly scratch (regrown by reserve)
  std::vector<void*> stage_allocs;  // narrow-phase staging (regrown by reserve)
  int pq = 4;                       // threads per broad-phase query (tunable)
  bool in_ws = false;                // scene memory carved from the caller's workspace (bf_scene_create_ws)
  bool shared_step = false;          // no step workspaces of its own: bound per request (serving loop)
  hipStream_t last = nullptr;
  // eval_barrier runs the structural part of the assembly on `side`, beside
  // the evaluation kernel; assemble_grad_hess then only adds the values
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bool prepared = false;             // structure built for the active list at prepared_for
  const void* prepared_for = nullptr;
  // per-stage timing (bf_scene_set_timing): an event pair around each stage's
  // kernels, recorded on the stream they run on, outside graph capture
  bool timing = false;
  hipEvent_t tev[BF_T_COUNT][2] = {};
  bool tev_set[BF_T_COUNT] = {};
};

namespace {

thread_local std::string g_err;

bf_status fail(bf_status s, const char* msg) {
  g_err = msg;
  return s;
}
bf_status fail_hip(hipError_t e, const char* where) {
  g_err = std::string(where) + ": " + hipGetErrorString(e);
  return BF_E_DEVICE;
}

// Scene memory is stream-ordered (hipMallocAsync / hipFreeAsync on the
// stream of the call that creates, regrows or destroys it), so destroying a
// scene never waits for work of other scenes on other streams.
thread_local hipStream_t g_alloc_stream = nullptr;

// A caller's workspace (bf_scene_create_ws): while g_arena is set, dalloc
// carves 256-byte aligned pieces from it instead of allocating, and records
// nothing to free; with a null base it only adds up the bytes
// (bf_workspace_bytes).
struct Arena {
  char* base = nullptr;
  size_t cap = 0, off = 0;
};
thread_local Arena* g_arena = nullptr;
inline bool sizing_only() { return g_arena && !g_arena->base; }

template <class T> T* dalloc(std::vector<void*>& list, size_t n, hipError_t* err) {
  void* p = nullptr;
  size_t bytes = n * sizeof(T);
  if (bytes == 0) bytes = sizeof(T);
  if (g_arena) {
    const size_t o = (g_arena->off + 255) & ~(size_t)255;
    g_arena->off = o + bytes;
    if (!g_arena->base || *err != hipSuccess) return nullptr;
    if (g_arena->off > g_arena->cap) {
      *err = hipErrorOutOfMemory;
      return nullptr;
    }
    return (T*)(g_arena->base + o);
  }
  hipError_t e = hipMallocAsync(&p, bytes, g_alloc_stream);
  if (e != hipSuccess) {
    *err = e;
    return nullptr;
  }
  list.push_back(p);
  return (T*)p;
}

long long next_pow2(long long v) {
  long long p = 1;
  while (p < v) p <<= 1;
  return p;
}

SceneDev dev_view(const bf_scene* s) {
  SceneDev S;
  S.kind = s->kind;
  S.nv = s->nv;
  S.ne = s->ne;
  S.nt = s->nt;
  S.edges = s->d_edges;
  S.tris = s->d_tris;
  S.ref = s->d_ref;
  S.xrest = s->d_xrest;
  S.refdist = s->prm.refdist;
  S.comp = s->d_comp;
  S.dmin = s->d_dmin;
  S.thr2 = s->d_thr2;
  S.h = s->prm.h;
  S.eta = s->prm.eta;
  S.kappa = s->prm.kappa;
  S.filter = s->prm.filter;
  S.eidx = s->d_eidx;
  S.eloop = s->d_eloop;
  S.cull_r = s->prm.cull_radius;
  S.core_key = s->core_slots ? s->core_key : nullptr;
  S.core_live = s->core_live;
  S.core_mask = s->core_slots ? s->core_slots - 1 : 0;
  S.mixed = s->prm.prec == BF_MIXED;
  S.pq = s->pq;
  S.status = s->d_status;
  return S;
}

void free_list(std::vector<void*>& l, hipStream_t st = g_alloc_stream) {
  for (void* p : l) (void)hipFreeAsync(p, st);
  l.clear();
}

// One assembly workspace for lists of up to act_cap pairs (incidence counts
// cleared, as the structure pass expects them).
bf_status alloc_asm_ws(const bf_scene* s, long long act_cap, std::vector<void*>& allocs, AsmWs* out,
                       const char* who) {
  if (act_cap > (1LL << 28)) return fail(BF_E_ARG, "active capacity above 2^28 pairs");  // assembly item field
  free_list(allocs);
  hipError_t e = hipSuccess;
  AsmWs A{};
  A.inc_cnt = dalloc<int>(allocs, s->nv + 1, &e);
  A.inc_off = dalloc<int>(allocs, s->nv + 1, &e);
  A.inc = dalloc<int>(allocs, 4 * act_cap, &e);
  A.colbuf = dalloc<int>(allocs, 16 * act_cap, &e);
  A.stn = dalloc<int4>(allocs, 4 * act_cap, &e);
  A.rowcnt = dalloc<int>(allocs, s->nv + 1, &e);
  A.mid = dalloc<int>(allocs, s->nv + 1, &e);
  A.big = dalloc<int>(allocs, s->nv + 1, &e);
  A.epart = dalloc<double>(allocs, (act_cap + 63) / 64 + 1, &e);
  A.scan_tmp = dalloc<int>(allocs, scan_tmp_ints(s->nv + 1), &e);
  if (e != hipSuccess)
    return g_arena ? fail(BF_E_CAPACITY, "bf_scene_create_ws: workspace smaller than bf_workspace_bytes")
                   : fail(BF_E_NOMEM, who);
  if (sizing_only()) return BF_OK;
  if (hipMemsetAsync(A.inc_cnt, 0, sizeof(int) * (s->nv + 1), g_alloc_stream) != hipSuccess ||
      hipMemsetAsync(A.scan_tmp, 0, sizeof(int) * SCAN_LB_STATE, g_alloc_stream) != hipSuccess ||
      hipMemsetAsync(A.rowcnt, 0, sizeof(int) * (s->nv + 1), g_alloc_stream) != hipSuccess ||
      (!g_arena && hipStreamSynchronize(g_alloc_stream) != hipSuccess))  // a workspace: stream order suffices
    return fail(BF_E_DEVICE, who);
  *out = A;
  return BF_OK;
}

bf_status alloc_asm(bf_scene* s, long long act_cap) {
  bf_status r = alloc_asm_ws(s, act_cap, s->asm_allocs, &s->aw, "bf_scene_reserve: assembly workspace");
  if (r == BF_OK) s->act_cap = act_cap;
  return r;
}

// Culling mode: order every polyline of a rod mesh.  eidx[e] = position of
// edge e along its polyline (walked from an end, or from its smallest vertex
// when closed); eloop[e] = the polyline's edge count when it is closed, 0
// when open.  False if a vertex lies on more than two edges.
bool polyline_order(int nv, int ne, const int32_t* edges, std::vector<int>& eidx, std::vector<int>& eloop) {
  std::vector<int> deg(nv, 0), adj(2LL * nv, -1);  // incident edges per vertex
  for (int e = 0; e < ne; ++e)
    for (int k = 0; k < 2; ++k) {
      const int v = edges[2 * e + k];
      if (deg[v] == 2) return false;
      adj[2 * v + deg[v]++] = e;
    }
  eidx.assign(ne, -1);
  eloop.assign(ne, 0);
  auto walk = [&](int v0) {  // from v0 along unvisited edges; returns the edges in order
    std::vector<int> order;
    int v = v0, prev = -1;
    while (true) {
      int next = -1;
      for (int k = 0; k < deg[v]; ++k)
        if (adj[2 * v + k] != prev && eidx[adj[2 * v + k]] < 0) { next = adj[2 * v + k]; break; }
      if (next < 0) break;
      eidx[next] = (int)order.size();
      order.push_back(next);
      v = edges[2 * next] == v ? edges[2 * next + 1] : edges[2 * next];
      prev = next;
    }
    return order;
  };
  for (int v = 0; v < nv; ++v)
    if (deg[v] == 1 && eidx[adj[2 * v]] < 0) walk(v);           // open polylines, from an end
  for (int v = 0; v < nv; ++v)
    if (deg[v] == 2 && eidx[adj[2 * v]] < 0) {                  // closed loops
      const std::vector<int> order = walk(v);
      for (int e : order) eloop[e] = (int)order.size();
    }
  return true;
}

bf_status alloc_stage(bf_scene* s, long long cand_cap) {
  free_list(s->stage_allocs);
  hipError_t e = hipSuccess;
  StageWs W{};
  long long G = (cand_cap + NW_TILE - 1) / NW_TILE;
  W.si = dalloc<int>(s->stage_allocs, G * NW_TILE, &e);
  W.sj = dalloc<int>(s->stage_allocs, G * NW_TILE, &e);
  W.sm = dalloc<unsigned>(s->stage_allocs, G * NW_TILE, &e);
  W.sd = dalloc<double>(s->stage_allocs, G * NW_TILE, &e);
  W.kcnt = dalloc<int>(s->stage_allocs, NW_KINDS * G + 1, &e);
  W.kofs = dalloc<int>(s->stage_allocs, NW_KINDS * G + 1, &e);
  W.ccnt = dalloc<int>(s->stage_allocs, 3 * G, &e);
  W.dfr = dalloc<long long>(s->stage_allocs, G * NW_TILE, &e);
  W.dfr2 = dalloc<int>(s->stage_allocs, G * NW_TILE, &e);
  W.n2 = dalloc<int>(s->stage_allocs, 1, &e);
  W.xcnt = dalloc<int>(s->stage_allocs, 5LL * XP_BLOCKS, &e);
  W.scan_tmp = dalloc<int>(s->stage_allocs, scan_tmp_ints(NW_KINDS * G + 1), &e);
  if (e != hipSuccess)
    return g_arena ? fail(BF_E_CAPACITY, "bf_scene_create_ws: workspace smaller than bf_workspace_bytes")
                   : fail(BF_E_NOMEM, "bf_scene_reserve: device allocation failed");
  W.cap = G * NW_TILE;
  if (sizing_only()) return BF_OK;
  if (hipMemsetAsync(W.scan_tmp, 0, sizeof(int) * SCAN_LB_STATE, g_alloc_stream) != hipSuccess ||
      (!g_arena && hipStreamSynchronize(g_alloc_stream) != hipSuccess))
    return fail(BF_E_DEVICE, "bf_scene_reserve: clearing the scan state failed");
  W.cap = G * NW_TILE;
  s->sw = W;
  return BF_OK;
}

// Stencil primitives must not be degenerate in rest space (the reference
// distances of Sec. 3.2 divide by rest edge lengths): an edge whose two rest
// parameters are equal, or a triangle whose rest edge vectors have a zero
// cross product (evaluated in double; exactly zero for coincident or
// collinear rest vertices on a lattice).  Returns the message, or null.
const char* degenerate_rest(const bf_mesh_desc& m, int nv, int ne, int nt) {
  const double* u = m.ref_h;
  for (int e = 0; e < ne; ++e) {
    const int a = m.edges_h[2 * e], b = m.edges_h[2 * e + 1];
    const bool same = m.kind == BF_ROD ? u[a] == u[b] : (u[2 * a] == u[2 * b] && u[2 * a + 1] == u[2 * b + 1]);
    if (same) return "bf_scene_create: an edge has zero rest length";
  }
  for (int t = 0; t < nt; ++t) {
    const int a = m.tris_h[3 * t], b = m.tris_h[3 * t + 1], c = m.tris_h[3 * t + 2];
    const double ux = u[2 * b] - u[2 * a], uy = u[2 * b + 1] - u[2 * a + 1];
    const double vx = u[2 * c] - u[2 * a], vy = u[2 * c + 1] - u[2 * a + 1];
    if (ux * vy - uy * vx == 0.0) return "bf_scene_create: a triangle has zero rest area";
  }
  (void)nv;
  return nullptr;
}

// Per-stage timing: record the start / stop event of a stage on st (no-op
// unless timing is on and st is not being captured).
struct StageTimer {
  bf_scene* s;
  int stage;
  hipStream_t st;
  bool on;
  StageTimer(bf_scene* s_, int stage_, hipStream_t st_) : s(s_), stage(stage_), st(st_), on(false) {
    if (!s->timing) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    on = hipEventRecord(s->tev[stage][0], st) == hipSuccess;
  }
  ~StageTimer() {
    if (on && hipEventRecord(s->tev[stage][1], st) == hipSuccess) s->tev_set[stage] = true;
  }
};

}  // namespace

// A scene that failed during creation: its memory back, in stream order.
void discard_scene(bf_scene* s) {
  free_list(s->asm_allocs);
  free_list(s->stage_allocs);
  free_list(s->allocs);
  delete s;
}

// Every buffer the scene keeps: topology, rest data, broad-phase and
// narrow-phase workspaces, assembly workspace, per-component thresholds
// (sized by the vertex count, a bound on the components) and the culling
// tables.  With g_arena set, carved from the caller's workspace (or only
// counted, bf_workspace_bytes).
bf_status alloc_broad(bf_scene* s, std::vector<void*>& allocs);
bf_status alloc_persistent(bf_scene* s, long long cand_cap, long long act_cap) {
  const int nv = s->nv, ne = s->ne, nt = s->nt;
  hipError_t e = hipSuccess;
  const int nref = s->kind == BF_ROD ? nv : 2 * nv;
  s->d_edges = dalloc<int>(s->allocs, 2LL * ne, &e);
  s->d_tris = dalloc<int>(s->allocs, std::max(3LL * nt, 3LL), &e);
  s->d_ref = dalloc<double>(s->allocs, nref, &e);
  if (s->prm.refdist == BF_REFDIST_EUCLID_REST) s->d_xrest = dalloc<double>(s->allocs, 3LL * nv, &e);
  s->d_comp = dalloc<int>(s->allocs, nv, &e);
  s->d_status = dalloc<unsigned>(s->allocs, 4, &e);
  s->d_line = dalloc<double>(s->allocs, LINE_BLOCKS, &e);
  s->d_dmin = dalloc<double>(s->allocs, nv, &e);
  s->d_thr2 = dalloc<double>(s->allocs, 2LL * nv, &e);
  if (s->prm.filter == BF_FILTER_CULL) {
    s->d_eidx = dalloc<int>(s->allocs, ne, &e);
    s->d_eloop = dalloc<int>(s->allocs, ne, &e);
  }
  if (e != hipSuccess)
    return fail(g_arena ? BF_E_CAPACITY : BF_E_NOMEM,
                g_arena ? "bf_scene_create_ws: workspace smaller than bf_workspace_bytes"
                        : "bf_scene_create: device allocation failed");
  if (s->shared_step) return BF_OK;  // the broad phase's and the step's workspaces come with each request
  bf_status r = alloc_broad(s, s->allocs);
  if (r == BF_OK) r = alloc_asm(s, act_cap);
  if (r == BF_OK) r = alloc_stage(s, cand_cap);
  return r;
}

// The broad phase's workspace (grid, boxes, cell-sorted primitives, pair
// counts), with what its kernels expect at zero cleared on g_alloc_stream
// (cell counts, the single-pass scans' state, the bounds reduction's counter).
bf_status alloc_broad(bf_scene* s, std::vector<void*>& allocs) {
  const int nv = s->nv, ne = s->ne, nt = s->nt;
  hipError_t e = hipSuccess;
  const int np = ne + nt + (s->kind == BF_SHELL ? nv : 0);
  BroadWs& W = s->bw;
  W.max_cells = (int)std::min<long long>(std::max<long long>(4096, 2LL * np), 1LL << 26);
  const long long nscan = 2LL * W.max_cells + 1;
  const long long nq = (long long)(s->kind == BF_SHELL ? nv + ne : ne) * PQ_MAX + 1;
  W.box = dalloc<Box>(allocs, np, &e);
  W.cell_of = dalloc<int>(allocs, ne + nt, &e);
  W.part = dalloc<float>(allocs, 8LL * BOUNDS_BLOCKS, &e);
  W.done = dalloc<unsigned>(allocs, 1, &e);
  W.grid = dalloc<Grid>(allocs, 1, &e);
  W.cell_cnt = dalloc<int>(allocs, nscan, &e);
  W.cell_start = dalloc<int>(allocs, nscan, &e);
  W.sorted_id = dalloc<int>(allocs, ne + nt, &e);
  W.sorted_box = dalloc<Box>(allocs, ne + nt, &e);
  W.sorted_vid = dalloc<int4>(allocs, ne + nt, &e);
  W.placed_id = dalloc<int>(allocs, ne + nt, &e);
  W.placed_box = dalloc<Box>(allocs, ne + nt, &e);
  W.pair_cnt = dalloc<int>(allocs, nq, &e);
  W.pair_bsum = dalloc<int>(allocs, nq / 256 + 2, &e);
  W.pair_bofs = dalloc<int>(allocs, nq / 256 + 2, &e);
  W.pair_bseg = dalloc<long long>(allocs, nq / 256 + 2, &e);
  W.seg_count = dalloc<unsigned long long>(allocs, 1, &e);
  W.scan_tmp = dalloc<int>(allocs, std::max(std::max(scan_tmp_ints(nscan), scan_tmp_ints(nv + 1)), scan_tmp_ints(nq)),
                           &e);
  if (e != hipSuccess)
    return fail(g_arena ? BF_E_CAPACITY : BF_E_NOMEM,
                g_arena ? "bf_scene_create_ws: workspace smaller than bf_workspace_bytes"
                        : "bf_scene_create: device allocation failed");
  if (sizing_only()) return BF_OK;
  if (hipMemsetAsync(W.cell_cnt, 0, sizeof(int) * nscan, g_alloc_stream) != hipSuccess ||
      hipMemsetAsync(W.scan_tmp, 0, sizeof(int) * SCAN_LB_STATE, g_alloc_stream) != hipSuccess ||
      hipMemsetAsync(W.done, 0, sizeof(unsigned), g_alloc_stream) != hipSuccess)
    return fail(BF_E_DEVICE, "broad-phase workspace");
  return BF_OK;
}

extern "C" {

const char* bf_last_error(void) { return g_err.c_str(); }

bf_status bf_set_scan_poll_limit(int32_t polls) {
  if (polls < 0) return fail(BF_E_ARG, "bf_set_scan_poll_limit: polls must be >= 0");
  g_scan_polls = polls;
  return BF_OK;
}

static bf_status check_scene_args(const bf_mesh_desc* mesh, const bf_params* params, int64_t cand_cap,
                                  int64_t act_cap) {
  if (!mesh || !params) return fail(BF_E_ARG, "bf_scene_create: null argument");
  if (mesh->kind != BF_ROD && mesh->kind != BF_SHELL) return fail(BF_E_ARG, "bf_scene_create: bad kind");
  if (mesh->n_verts < 2 || mesh->n_edges < 1 || !mesh->edges_h || !mesh->ref_h)
    return fail(BF_E_ARG, "bf_scene_create: need >= 2 vertices, >= 1 edge, edges and rest parameters");
  if (mesh->kind == BF_SHELL && (mesh->n_tris < 1 || !mesh->tris_h))
    return fail(BF_E_ARG, "bf_scene_create: shells need triangles");
  if (mesh->n_verts > (1LL << 30) || mesh->n_edges > (1LL << 30) || mesh->n_tris > (1LL << 30))
    return fail(BF_E_ARG, "bf_scene_create: mesh too large (> 2^30 primitives)");
  if (!(params->h > 0.0) || !(params->eta >= 0.0) || !(params->eta < params->h) || !(params->kappa > 0.0) ||
      !std::isfinite(params->h))
    return fail(BF_E_ARG, "bf_scene_create: need h > 0, 0 <= eta < h, kappa > 0");
  if (params->prec != BF_FP64 && params->prec != BF_MIXED) return fail(BF_E_ARG, "bf_scene_create: bad prec");
  if (params->filter != BF_FILTER_PAPER && params->filter != BF_FILTER_NONE && params->filter != BF_FILTER_CULL)
    return fail(BF_E_ARG, "bf_scene_create: bad filter mode");
  if (params->filter == BF_FILTER_CULL && (mesh->kind != BF_ROD || params->cull_radius < 1))
    return fail(BF_E_ARG, "bf_scene_create: culling is defined for rods, with a radius of at least one element");
  if (params->refdist != BF_REFDIST_PARAM && params->refdist != BF_REFDIST_EUCLID_REST)
    return fail(BF_E_ARG, "bf_scene_create: bad reference-distance mode");
  if (params->refdist == BF_REFDIST_EUCLID_REST) {
    if (!mesh->ref_pos_h) return fail(BF_E_ARG, "bf_scene_create: BF_REFDIST_EUCLID_REST needs the rest pose");
    for (long long k = 0; k < 3LL * mesh->n_verts; ++k)
      if (!std::isfinite(mesh->ref_pos_h[k])) return fail(BF_E_ARG, "bf_scene_create: rest pose not finite");
  }
  if (cand_cap < 1 || act_cap < 1) return fail(BF_E_ARG, "bf_scene_create: capacities must be >= 1");
  int nv = (int)mesh->n_verts, ne = (int)mesh->n_edges, nt = mesh->kind == BF_SHELL ? (int)mesh->n_tris : 0;
  for (long long k = 0; k < 2LL * ne; ++k)
    if (mesh->edges_h[k] < 0 || mesh->edges_h[k] >= nv) return fail(BF_E_ARG, "bf_scene_create: edge vertex out of range");
  for (long long k = 0; k < 3LL * nt; ++k)
    if (mesh->tris_h[k] < 0 || mesh->tris_h[k] >= nv) return fail(BF_E_ARG, "bf_scene_create: triangle vertex out of range");
  for (int e = 0; e < ne; ++e)
    if (mesh->edges_h[2 * e] == mesh->edges_h[2 * e + 1]) return fail(BF_E_ARG, "bf_scene_create: degenerate edge");
  if (const char* why = degenerate_rest(*mesh, nv, ne, nt)) return fail(BF_E_DEGENERATE, why);
  return BF_OK;
}

static bf_status create_scene(const bf_mesh_desc* mesh, const bf_params* params, int64_t cand_cap,
                              int64_t act_cap, void* stream, Arena* arena, bf_scene** out,
                              bool shared_step = false) {
  if (!out) return fail(BF_E_ARG, "bf_scene_create: null argument");
  *out = nullptr;
  if (bf_status r = check_scene_args(mesh, params, cand_cap, act_cap); r != BF_OK) return r;
  const int nv = (int)mesh->n_verts, ne = (int)mesh->n_edges, nt = mesh->kind == BF_SHELL ? (int)mesh->n_tris : 0;

  hipStream_t st = (hipStream_t)stream;
  g_alloc_stream = st;
  bf_scene* s = new bf_scene;
  s->prm = *params;
  s->kind = mesh->kind;
  s->nv = nv;
  s->ne = ne;
  s->nt = nt;
  s->last = st;
  const bool euclid = params->refdist == BF_REFDIST_EUCLID_REST;
  const int nref = s->kind == BF_ROD ? nv : 2 * nv;
  s->in_ws = arena != nullptr;
  s->shared_step = shared_step;
  g_arena = arena;
  const bf_status ra = alloc_persistent(s, cand_cap, act_cap);
  g_arena = nullptr;
  if (bf_status r = ra; r != BF_OK) {
    discard_scene(s);
    return r;
  }
  hipError_t e = hipSuccess;
  hipError_t he;
  if ((he = hipMemcpyAsync(s->d_edges, mesh->edges_h, sizeof(int) * 2LL * ne, hipMemcpyHostToDevice, st)) ||
      (nt && (he = hipMemcpyAsync(s->d_tris, mesh->tris_h, sizeof(int) * 3LL * nt, hipMemcpyHostToDevice, st))) ||
      (he = hipMemcpyAsync(s->d_ref, mesh->ref_h, sizeof(double) * nref, hipMemcpyHostToDevice, st)) ||
      (euclid &&
       (he = hipMemcpyAsync(s->d_xrest, mesh->ref_pos_h, sizeof(double) * 3LL * nv, hipMemcpyHostToDevice, st))) ||
      (he = hipMemsetAsync(s->d_status, 0, 4 * sizeof(unsigned), st))) {
    discard_scene(s);
    return fail_hip(he, "bf_scene_create: upload");
  }

  // --- precompute (Sec. 3.2): components ------------------------------------
  std::vector<void*> tmp;
  int* lab = dalloc<int>(tmp, nv, &e);
  int* flag = dalloc<int>(tmp, nv, &e);
  int* scan = dalloc<int>(tmp, nv, &e);
  int* changed = dalloc<int>(tmp, 1, &e);
  int* sct = dalloc<int>(tmp, scan_tmp_ints(nv + 1), &e);  // the scans' scratch (its state words at zero)
  if (e != hipSuccess || hipMemsetAsync(sct, 0, sizeof(int) * SCAN_LB_STATE, st) != hipSuccess) {
    free_list(tmp);
    discard_scene(s);
    return fail(BF_E_NOMEM, "bf_scene_create: device allocation failed");
  }
  SceneDev S = dev_view(s);
  int nc = run_components(S, lab, flag, scan, s->d_comp, sct, changed, st);
  free_list(tmp);
  if (nc <= 0) {
    discard_scene(s);
    return fail(BF_E_DEVICE, "bf_scene_create: component labelling failed");
  }
  s->nc = nc;
  s->comp_h.resize(nv);
  if (params->filter == BF_FILTER_CULL) {
    std::vector<int> eidx, eloop;
    if (!polyline_order(nv, ne, mesh->edges_h, eidx, eloop)) {
      discard_scene(s);
      return fail(BF_E_ARG, "bf_scene_create: culling needs polylines (no vertex on more than two edges)");
    }
    if (hipMemcpyAsync(s->d_eidx, eidx.data(), sizeof(int) * ne, hipMemcpyHostToDevice, st) ||
        hipMemcpyAsync(s->d_eloop, eloop.data(), sizeof(int) * ne, hipMemcpyHostToDevice, st) ||
        hipStreamSynchronize(st)) {
      discard_scene(s);
      return fail(BF_E_NOMEM, "bf_scene_create: culling tables");
    }
  }

  // --- precompute: d_min per component over stencil pairs with 0 < dbar < h,
  // found by the same broad phase run on the rest parameters lifted to 3D
  // (or on the rest pose, under the Euclidean reading)
  std::vector<unsigned long long> best(nc, 0x7ff0000000000000ull);  // +inf
  long long cap = std::max<long long>(cand_cap, 1024);
  // a scene without a broad-phase workspace of its own (its steps bring one)
  // borrows one for the precompute, freed below or with the scene on failure
  if (s->shared_step && alloc_broad(s, s->stage_allocs) != BF_OK) {
    discard_scene(s);
    return fail(BF_E_NOMEM, "bf_scene_create: device allocation failed");
  }
  const BroadWs& W = s->bw;
  const long long tie_cap = std::max<long long>(4096, cap / 16);
  for (int attempt = 0; attempt < 4; ++attempt) {
    std::vector<void*> t2;
    double* xref = euclid ? nullptr : dalloc<double>(t2, 3LL * nv, &e);
    int* ci = dalloc<int>(t2, cap, &e);
    int* cj = dalloc<int>(t2, cap, &e);
    unsigned char* ct = dalloc<unsigned char>(t2, cap, &e);
    long long* cnt = dalloc<long long>(t2, 1, &e);
    unsigned long long* dbest = dalloc<unsigned long long>(t2, nc, &e);
    long long* ties = dalloc<long long>(t2, tie_cap, &e);
    unsigned long long* flags = dalloc<unsigned long long>(t2, 2, &e);  // tie count, degenerate / limit bits
    if (e != hipSuccess) {
      free_list(t2);
      discard_scene(s);
      return fail(BF_E_NOMEM, "bf_scene_create: device allocation failed");
    }
    S = dev_view(s);
    if (!euclid) run_lift_ref(S, xref, st);
    run_broad(S, euclid ? s->d_xrest : xref, nullptr, W, ci, cj, ct, cap, cnt, s->d_status, nullptr, nullptr, 0,
              st);  // no staging yet
    (void)hipMemcpyAsync(dbest, best.data(), sizeof(unsigned long long) * nc, hipMemcpyHostToDevice, st);
    run_refmin(S, ci, cj, ct, cnt, cap, dbest, ties, tie_cap, flags, st);
    long long hcnt = 0;
    unsigned long long hflags[2] = {0, 0};
    (void)hipMemcpyAsync(&hcnt, cnt, sizeof(long long), hipMemcpyDeviceToHost, st);
    (void)hipMemcpyAsync(hflags, flags, sizeof(hflags), hipMemcpyDeviceToHost, st);
    std::vector<unsigned long long> got(nc);
    (void)hipMemcpyAsync(got.data(), dbest, sizeof(unsigned long long) * nc, hipMemcpyDeviceToHost, st);
    (void)hipMemcpyAsync(s->comp_h.data(), s->d_comp, sizeof(int) * nv, hipMemcpyDeviceToHost, st);
    he = hipStreamSynchronize(st);
    free_list(t2);
    if (he != hipSuccess) {
      discard_scene(s);
      return fail_hip(he, "bf_scene_create: precompute");
    }
    if (hcnt <= cap && (long long)hflags[0] <= tie_cap) {
      const char* why = (hflags[1] & 1ull) ? "bf_scene_create: two primitives of the rest pose touch"
                        : (hflags[1] & 2ull) ? "bf_scene_create: a rest-pose distance needs more exact "
                                               "arithmetic than the expansions hold"
                                             : nullptr;
      if (why) {
        discard_scene(s);
        return fail(BF_E_DEGENERATE, why);
      }
      best = got;
      break;
    }
    cap = std::max(cap, hcnt + hcnt / 8 + 1024);
    if (attempt == 3 || (long long)hflags[0] > tie_cap) {
      discard_scene(s);
      return fail(BF_E_CAPACITY, (long long)hflags[0] > tie_cap
                                     ? "bf_scene_create: too many rest-pose distances tie with h"
                                     : "bf_scene_create: rest-space candidate list kept overflowing");
    }
  }
  if (s->shared_step) {
    free_list(s->stage_allocs, st);
    s->bw = BroadWs{};
  }
  s->dmin2_h.assign(nc, INFINITY);
  s->dmin_h.assign(nc, INFINITY);
  std::vector<double> thr2(2LL * nc, INFINITY);
  for (int c = 0; c < nc; ++c) {
    double v;
    std::memcpy(&v, &best[c], sizeof(double));
    if (!(v < INFINITY)) {
      thr2[2 * c + 1] = 0.0;
      continue;
    }
    if (s->kind == BF_ROD && !euclid) {  // the minimum gap; threshold its exact square
      s->dmin_h[c] = v;
      s->dmin2_h[c] = v * v;
      thr2[2 * c] = v * v;
      thr2[2 * c + 1] = std::fma(v, v, -(v * v));
    } else {                  // canonical d_min^2 (rounded once); d_min its IEEE sqrt
      s->dmin2_h[c] = v;
      s->dmin_h[c] = std::sqrt(v);
      thr2[2 * c] = v;
      thr2[2 * c + 1] = 0.0;
    }
  }
  if ((he = hipMemcpyAsync(s->d_dmin, s->dmin_h.data(), sizeof(double) * nc, hipMemcpyHostToDevice, st)) ||
      (he = hipMemcpyAsync(s->d_thr2, thr2.data(), sizeof(double) * 2 * nc, hipMemcpyHostToDevice, st)) ||
      (he = hipMemsetAsync(s->d_status, 0, 4 * sizeof(unsigned), st)) || (he = hipStreamSynchronize(st))) {
    discard_scene(s);
    return fail_hip(he, "bf_scene_create: upload d_min");
  }
  bf_status r = BF_OK;
  if (((he = hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking)) != hipSuccess ||
                     (he = hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming)) != hipSuccess ||
                     (he = hipEventCreateWithFlags(&s->ev_join, hipEventDisableTiming)) != hipSuccess))
    r = fail_hip(he, "bf_scene_create: side stream");
  if (r != BF_OK) {
    if (s->ev_join) (void)hipEventDestroy(s->ev_join);
    if (s->ev_fork) (void)hipEventDestroy(s->ev_fork);
    if (s->side) (void)hipStreamDestroy(s->side);
    discard_scene(s);
    return r;
  }
  *out = s;
  return BF_OK;
}

bf_status bf_scene_create(const bf_mesh_desc* mesh, const bf_params* params, int64_t cand_cap, int64_t act_cap,
                          void* stream, bf_scene** out) {
  return create_scene(mesh, params, cand_cap, act_cap, stream, nullptr, out);
}

bf_status bf_workspace_bytes(const bf_mesh_desc* mesh, const bf_params* params, int64_t cand_cap, int64_t act_cap,
                             int64_t* bytes_h) {
  if (!bytes_h) return fail(BF_E_ARG, "bf_workspace_bytes: null argument");
  if (bf_status r = check_scene_args(mesh, params, cand_cap, act_cap); r != BF_OK) return r;
  bf_scene probe;  // host fields only: the allocation sequence is counted, nothing is allocated
  probe.prm = *params;
  probe.kind = mesh->kind;
  probe.nv = (int)mesh->n_verts;
  probe.ne = (int)mesh->n_edges;
  probe.nt = mesh->kind == BF_SHELL ? (int)mesh->n_tris : 0;
  Arena a;
  g_arena = &a;
  const bf_status r = alloc_persistent(&probe, cand_cap, act_cap);
  g_arena = nullptr;
  if (r != BF_OK) return r;
  *bytes_h = (int64_t)a.off + 255;  // room to align an unaligned base
  return BF_OK;
}

bf_status bf_scene_create_ws(const bf_mesh_desc* mesh, const bf_params* params, int64_t cand_cap, int64_t act_cap,
                             void* ws_d, int64_t ws_bytes, void* stream, bf_scene** out) {
  if (!ws_d || ws_bytes < 1) return fail(BF_E_ARG, "bf_scene_create_ws: null or empty workspace");
  const uintptr_t b0 = (uintptr_t)ws_d, b1 = (b0 + 255) & ~(uintptr_t)255;
  if ((int64_t)(b1 - b0) >= ws_bytes) return fail(BF_E_CAPACITY, "bf_scene_create_ws: workspace too small");
  Arena a;
  a.base = (char*)b1;
  a.cap = (size_t)(ws_bytes - (int64_t)(b1 - b0));
  return create_scene(mesh, params, cand_cap, act_cap, stream, &a, out);
}

bf_status bf_scene_reserve(bf_scene* s, int64_t cand_cap, int64_t act_cap) {
  if (!s || act_cap < 1 || cand_cap < 1) return fail(BF_E_ARG, "bf_scene_reserve: bad argument");
  if (s->in_ws && (act_cap > s->act_cap || cand_cap > s->sw.cap))
    return fail(BF_E_STATE, "bf_scene_reserve: a scene in a caller's workspace cannot grow");
  if (act_cap <= s->act_cap && cand_cap <= s->sw.cap) return BF_OK;
  hipError_t he = hipDeviceSynchronize();
  if (he != hipSuccess) return fail_hip(he, "bf_scene_reserve");
  g_alloc_stream = nullptr;
  bf_status r = BF_OK;
  if (act_cap > s->act_cap) r = alloc_asm(s, act_cap);
  if (r == BF_OK && cand_cap > s->sw.cap) r = alloc_stage(s, cand_cap);
  if (r == BF_OK && (he = hipDeviceSynchronize()) != hipSuccess) return fail_hip(he, "bf_scene_reserve");
  return r;
}

bf_status bf_scene_destroy(bf_scene* s) {
  if (!s) return BF_OK;
  // freed in stream order after the work last enqueued for the scene (work
  // on the side stream always joins back into that stream)
  free_list(s->asm_allocs, s->last);
  free_list(s->stage_allocs, s->last);
  free_list(s->core_allocs, s->last);
  free_list(s->fasm_allocs, s->last);
  free_list(s->allocs, s->last);
  if (s->ev_join) (void)hipEventDestroy(s->ev_join);
  if (s->ev_fork) (void)hipEventDestroy(s->ev_fork);
  if (s->side) (void)hipStreamDestroy(s->side);
  for (int k = 0; k < BF_T_COUNT; ++k)
    for (int e = 0; e < 2; ++e)
      if (s->tev[k][e]) (void)hipEventDestroy(s->tev[k][e]);
  delete s;
  return BF_OK;
}

bf_status bf_scene_info(bf_scene* s, int32_t* comp_h, int32_t* n_comp, double* dmin2_h, double* dmin_h,
                        int32_t cap_c) {
  if (!s) return fail(BF_E_ARG, "bf_scene_info: null scene");
  if (comp_h) std::memcpy(comp_h, s->comp_h.data(), sizeof(int) * s->nv);
  if (n_comp) *n_comp = s->nc;
  for (int c = 0; c < s->nc && c < cap_c; ++c) {
    if (dmin2_h) dmin2_h[c] = s->dmin2_h[c];
    if (dmin_h) dmin_h[c] = s->dmin_h[c];
  }
  return BF_OK;
}

bf_status build_candidates(bf_scene* s, const double* x_d, bf_pairs* cand, void* stream) {
  if (!s || !x_d || !cand || !cand->i_d || !cand->j_d || !cand->type_d || !cand->count_d || cand->cap < 1)
    return fail(BF_E_ARG, "build_candidates: null argument or capacity < 1");
  hipStream_t st = (hipStream_t)stream;
  s->last = st;
  StageTimer tm(s, BF_T_BROAD, st);
  // the narrow phase's staging buffers hold the count pass's segments (they
  // are free until filter_pairs, which runs after this call on the stream)
  run_broad(dev_view(s), x_d, nullptr, s->bw, cand->i_d, cand->j_d, cand->type_d, cand->cap,
            (long long*)cand->count_d, s->d_status, s->sw.si, s->sw.sm, s->sw.cap, st);
  hipError_t he = hipGetLastError();
  return he == hipSuccess ? BF_OK : fail_hip(he, "build_candidates");
}

bf_status build_candidates_swept(bf_scene* s, const double* x_d, const double* p_d, bf_pairs* cand, void* stream) {
  if (!s || !x_d || !p_d || !cand || !cand->i_d || !cand->j_d || !cand->type_d || !cand->count_d || cand->cap < 1)
    return fail(BF_E_ARG, "build_candidates_swept: null argument or capacity < 1");
  hipStream_t st = (hipStream_t)stream;
  s->last = st;
  run_broad(dev_view(s), x_d, p_d, s->bw, cand->i_d, cand->j_d, cand->type_d, cand->cap, (long long*)cand->count_d,
            s->d_status, s->sw.si, s->sw.sm, s->sw.cap, st);
  hipError_t he = hipGetLastError();
  return he == hipSuccess ? BF_OK : fail_hip(he, "build_candidates_swept");
}

bf_status max_step_accd(bf_scene* s, const double* x_d, const double* p_d, const bf_pairs* cand, double accd_s,
                        int32_t max_iter, double* t_d, double* tpair_d, int32_t* iters_d, void* stream) {
  if (!s || !x_d || !p_d || !cand || !cand->i_d || !cand->j_d || !cand->type_d || !cand->count_d || !t_d ||
      cand->cap < 1)
    return fail(BF_E_ARG, "max_step_accd: null argument or capacity < 1");
  if (!(accd_s > 0.0 && accd_s < 1.0) || max_iter < 1)
    return fail(BF_E_ARG, "max_step_accd: accd_s must lie in (0, 1) and max_iter be at least 1");
  hipStream_t st = (hipStream_t)stream;
  s->last = st;
  run_accd(dev_view(s), x_d, p_d, cand->i_d, cand->j_d, cand->type_d, (const long long*)cand->count_d, cand->cap,
           accd_s, max_iter, tpair_d, iters_d, s->d_line, t_d, st);
  hipError_t he = hipGetLastError();
  return he == hipSuccess ? BF_OK : fail_hip(he, "max_step_accd");
}

bf_status bf_core_mark(bf_scene* s, const double* x_d, const bf_pairs* cand, int64_t cap, int64_t* count_d,
                       void* stream) {
  if (!s || !x_d || !cand || !cand->i_d || !cand->j_d || !cand->type_d || !cand->count_d || !count_d || cap < 1 ||
      cand->cap < 1)
    return fail(BF_E_ARG, "bf_core_mark: null argument or capacity < 1");
  if (cap > (1LL << 29)) return fail(BF_E_ARG, "bf_core_mark: capacity above 2^29 pairs");
  hipStream_t st = (hipStream_t)stream;
  s->last = st;
  unsigned slots = 64;
  while ((long long)slots < 2 * cap) slots <<= 1;
  if (slots > s->core_slots) {  // grow: as bf_scene_reserve, between device synchronisations
    hipError_t he = hipDeviceSynchronize();
    if (he != hipSuccess) return fail_hip(he, "bf_core_mark");
    g_alloc_stream = nullptr;
    free_list(s->core_allocs, nullptr);
    s->core_slots = 0;
    hipError_t e = hipSuccess;
    s->core_key = dalloc<unsigned long long>(s->core_allocs, slots, &e);
    s->core_live = dalloc<unsigned char>(s->core_allocs, slots, &e);
    if (e != hipSuccess) {
      free_list(s->core_allocs, nullptr);
      return fail(BF_E_NOMEM, "bf_core_mark: device allocation failed");
    }
    if ((he = hipDeviceSynchronize()) != hipSuccess) return fail_hip(he, "bf_core_mark");
    s->core_slots = slots;
  }
  SceneDev S = dev_view(s);
  S.core_key = nullptr;  // marking uses the plain offsets
  run_core_mark(S, x_d, cand->i_d, cand->j_d, cand->type_d, (const long long*)cand->count_d, cand->cap, s->core_key,
                s->core_live, s->core_slots, cap, (long long*)count_d, s->d_status, st);
  hipError_t he = hipGetLastError();
  return he == hipSuccess ? BF_OK : fail_hip(he, "bf_core_mark");
}

bf_status friction_lag(bf_scene* s, const double* xlag_d, const bf_active* act, bf_friction* fr, void* stream) {
  if (!s || !xlag_d || !act || !fr || !fr->lam_d || !fr->w_d || !fr->n_d || !act->p.count_d || !act->p.i_d ||
      !act->p.j_d || !act->p.type_d || !act->code_d || !act->flags_d)
    return fail(BF_E_ARG, "friction_lag: null argument");
  if (fr->cap < act->p.cap) return fail(BF_E_CAPACITY, "friction_lag: friction capacity below active capacity");
  hipStream_t st = (hipStream_t)stream;
  s->last = st;
  if (act->p.cap > s->fasm_cap) {  // (re)size the friction assembly's workspace
    hipError_t he = hipDeviceSynchronize();
    if (he != hipSuccess) return fail_hip(he, "friction_lag");
    g_alloc_stream = nullptr;
    s->fasm_cap = 0;
    s->fric_list = nullptr;
    bf_status r = alloc_asm_ws(s, act->p.cap, s->fasm_allocs, &s->faw, "friction_lag: assembly workspace");
    if (r != BF_OK) return r;
    s->fasm_cap = act->p.cap;
  }
  const SceneDev S = dev_view(s);
  run_friction_lag(S, xlag_d, act->p.i_d, act->p.j_d, act->p.type_d, act->code_d, act->flags_d,
                   (const long long*)act->p.count_d, act->p.cap, fr->lam_d, fr->w_d, fr->n_d, st);
  run_asm_structure(S, act->p.i_d, act->p.j_d, act->p.type_d, act->flags_d, (const long long*)act->p.count_d,
                    act->p.cap, s->faw, st);
  s->fric_list = act->p.i_d;
  hipError_t he = hipGetLastError();
  return he == hipSuccess ? BF_OK : fail_hip(he, "friction_lag");
}

bf_status friction_assemble(bf_scene* s, const bf_active* act, const bf_local* loc, double* E_d, double* g_d,
                            bf_bsr* H, void* stream) {
  if (!s || !act || !loc || !E_d || !g_d || !H || !H->row_ptr_d || !H->col_d || !H->val_d || !H->nnzb_d ||
      H->cap < 1 || !act->p.count_d || !loc->G_d || !loc->H_d)
    return fail(BF_E_ARG, "friction_assemble: null argument or capacity < 1");
  if (!s->fric_list || act->p.i_d != s->fric_list)
    return fail(BF_E_STATE, "friction_assemble: not the list of the last friction_lag");
  if (act->p.cap > s->act_cap || act->p.cap > s->fasm_cap)
    return fail(BF_E_CAPACITY, "friction_assemble: lagged capacity exceeds the scene reserve (bf_scene_reserve)");
  hipStream_t st = (hipStream_t)stream;
  s->last = st;
  AsmWs F = s->faw;
  F.epart = s->aw.epart;  // friction_eval's per-tile energy sums
  run_asm_values(dev_view(s), act->p.i_d, act->p.j_d, act->p.type_d, (const long long*)act->p.count_d, act->p.cap,
                 loc->G_d, loc->H_d, E_d, g_d, H->row_ptr_d, H->col_d, H->val_d, H->cap, (long long*)H->nnzb_d, F,
                 s->d_status, st);
  hipError_t he = hipGetLastError();
  return he == hipSuccess ? BF_OK : fail_hip(he, "friction_assemble");
}

bf_status friction_eval(bf_scene* s, const double* x_d, const double* xlag_d, const bf_active* act,
                        const bf_friction* fr, double mu, double eps_vh, int32_t accumulate, bf_local* out,
                        void* stream) {
  if (!s || !x_d || !xlag_d || !act || !fr || !fr->lam_d || !fr->w_d || !fr->n_d || !out || !out->E_d ||
      !out->G_d || !out->H_d || !act->p.count_d || !act->p.i_d || !act->p.j_d || !act->p.type_d)
    return fail(BF_E_ARG, "friction_eval: null argument");
  if (!(mu >= 0.0) || !(eps_vh > 0.0)) return fail(BF_E_ARG, "friction_eval: need mu >= 0 and eps_vh > 0");
  if (fr->cap < act->p.cap || out->cap < act->p.cap)
    return fail(BF_E_CAPACITY, "friction_eval: friction or local capacity below active capacity");
  hipStream_t st = (hipStream_t)stream;
  s->last = st;
  const bool fits = act->p.cap <= s->act_cap;
  run_friction_eval(dev_view(s), x_d, xlag_d, act->p.i_d, act->p.j_d, act->p.type_d,
                    (const long long*)act->p.count_d, act->p.cap, fr->lam_d, fr->w_d, fr->n_d, mu, eps_vh,
                    accumulate ? 1 : 0, out->E_d, out->G_d, out->H_d, fits ? s->aw.epart : nullptr, st);
  hipError_t he = hipGetLastError();
  return he == hipSuccess ? BF_OK : fail_hip(he, "friction_eval");
}

bf_status bf_core_live(bf_scene* s, int64_t* count_d, void* stream) {
  if (!s || !count_d) return fail(BF_E_ARG, "bf_core_live: null argument");
  hipStream_t st = (hipStream_t)stream;
  s->last = st;
  if (!s->core_slots) run_zero_i64((long long*)count_d, 1, st);  // a kernel, not a memset: capturable
  else run_core_count(dev_view(s), (long long*)count_d, st);
  hipError_t he = hipGetLastError();
  return he == hipSuccess ? BF_OK : fail_hip(he, "bf_core_live");
}

bf_status bf_core_clear(bf_scene* s) {
  if (!s) return fail(BF_E_ARG, "bf_core_clear: null scene");
  free_list(s->core_allocs, s->last);
  s->core_key = nullptr;
  s->core_live = nullptr;
  s->core_slots = 0;
  return BF_OK;
}

bf_status eval_energy(bf_scene* s, const double* x_d, const double* p_d, const double* alpha_d, const bf_pairs* cand,
                      double* E_d, void* stream) {
  if (!s || !x_d || !cand || !cand->i_d || !cand->j_d || !cand->type_d || !cand->count_d || !E_d || cand->cap < 1)
    return fail(BF_E_ARG, "eval_energy: null argument or capacity < 1");
  if ((p_d == nullptr) != (alpha_d == nullptr))
    return fail(BF_E_ARG, "eval_energy: p_d and alpha_d are given together or not at all");
  hipStream_t st = (hipStream_t)stream;
  s->last = st;
  run_energy(dev_view(s), x_d, p_d, alpha_d, cand->i_d, cand->j_d, cand->type_d, (const long long*)cand->count_d,
             cand->cap, s->d_line, E_d, st);
  hipError_t he = hipGetLastError();
  return he == hipSuccess ? BF_OK : fail_hip(he, "eval_energy");
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free energy evaluation: the per-block partial sums of
// eval_energy live in this file-scope device array instead of the scene's
// scratch.  Its address is taken once per device with hipGetSymbolAddress
// (with that device current) and kept; host code never passes the array's
// name itself to a kernel.  Every call on one device shares the array, which
// keeps the last call's partials (each call overwrites every partial it
// reads): calls that overlap on one device race.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[LINE_BLOCKS];
namespace {
constexpr int MAX_DEVICES = 64;
double* g_scratch_ptr[MAX_DEVICES] = {};
std::mutex g_scratch_mu;

bf_status scratch_of_device(double** out) {
  int dev = -1;
  hipError_t he = hipGetDevice(&dev);
  if (he != hipSuccess) return fail_hip(he, "eval_energy_noalloc: hipGetDevice");
  if (dev < 0 || dev >= MAX_DEVICES) return fail(BF_E_DEVICE, "eval_energy_noalloc: device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    he = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (he != hipSuccess || !p) return fail_hip(he, "eval_energy_noalloc: hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = (double*)p;
  }
  *out = g_scratch_ptr[dev];
  return BF_OK;
}
}  // namespace

extern "C" {

bf_status eval_energy_noalloc(bf_scene* s, const double* x_d, const double* p_d, const double* alpha_d,
                              const bf_pairs* cand, double* E_d, void* stream) {
  if (!s || !x_d || !cand || !cand->i_d || !cand->j_d || !cand->type_d || !cand->count_d || !E_d || cand->cap < 1)
    return fail(BF_E_ARG, "eval_energy_noalloc: null argument or capacity < 1");
  if ((p_d == nullptr) != (alpha_d == nullptr))
    return fail(BF_E_ARG, "eval_energy_noalloc: p_d and alpha_d are given together or not at all");
  // one partial per work-group of the energy kernel (it strides over the list
  // with at most LINE_BLOCKS work-groups), and the array holds LINE_BLOCKS
  const long long parts = std::min<long long>((cand->cap + 255) / 256, LINE_BLOCKS);
  if (parts > (long long)(sizeof(scratch) / sizeof(double)))
    return fail(BF_E_CAPACITY, "eval_energy_noalloc: more partial sums than the static scratch holds");
  double* part = nullptr;
  bf_status r = scratch_of_device(&part);
  if (r != BF_OK) return r;
  hipStream_t st = (hipStream_t)stream;
  s->last = st;
  run_energy(dev_view(s), x_d, p_d, alpha_d, cand->i_d, cand->j_d, cand->type_d, (const long long*)cand->count_d,
             cand->cap, part, E_d, st);
  hipError_t he = hipGetLastError();
  return he == hipSuccess ? BF_OK : fail_hip(he, "eval_energy_noalloc");
}

bf_status filter_pairs(bf_scene* s, const double* x_d, const bf_pairs* cand, bf_active* act, void* stream) {
  if (!s || !x_d || !cand || !act || !cand->count_d || !act->p.i_d || !act->p.j_d || !act->p.type_d ||
      !act->p.count_d || !act->code_d || !act->flags_d || !act->dist_d || !act->counters_d || act->p.cap < 1)
    return fail(BF_E_ARG, "filter_pairs: null argument or capacity < 1");
  if (cand->cap > s->sw.cap)
    return fail(BF_E_CAPACITY, "filter_pairs: candidate capacity exceeds the scene reserve (bf_scene_reserve)");
  hipStream_t st = (hipStream_t)stream;
  s->last = st;
  s->prepared = false;
  if (s->core_slots) run_core_release(dev_view(s), x_d, st);  // Sec. 3.4: pairs now beyond eta leave the set
  {
    StageTimer tm(s, BF_T_NARROW, st);
    run_narrow(dev_view(s), x_d, cand->i_d, cand->j_d, cand->type_d, (const long long*)cand->count_d, cand->cap,
               s->sw, st);
  }
  {
    StageTimer tm(s, BF_T_COMPACT, st);
    run_compact(dev_view(s), x_d, cand->i_d, cand->j_d, cand->type_d, cand->cap, s->sw, act->p.i_d, act->p.j_d,
                act->p.type_d, act->code_d, act->flags_d, act->dist_d, act->p.cap, (long long*)act->p.count_d,
                (long long*)act->counters_d, s->d_status, st);
  }
  hipError_t he = hipGetLastError();
  return he == hipSuccess ? BF_OK : fail_hip(he, "filter_pairs");
}

bf_status eval_barrier(bf_scene* s, const double* x_d, const bf_active* act, bf_local* out, void* stream) {
  if (!s || !x_d || !act || !out || !out->E_d || !out->G_d || !out->H_d || !act->p.count_d)
    return fail(BF_E_ARG, "eval_barrier: null argument");
  if (out->cap < act->p.cap) return fail(BF_E_CAPACITY, "eval_barrier: local capacity below active capacity");
  hipStream_t st = (hipStream_t)stream;
  s->last = st;
  const SceneDev S = dev_view(s);
  hipError_t he = hipSuccess;
  // the assembly's structure needs the active list only: build it on the
  // side stream while the evaluation kernel runs, join before returning.
  // Not while the stream is being captured into a graph: a batch capture that
  // forked the side stream from inside a lane crashed in the runtime, so
  // captured steps build the structure in assemble_grad_hess instead.
  hipStreamCaptureStatus cap_status = hipStreamCaptureStatusNone;
  if ((he = hipStreamIsCapturing(st, &cap_status)) != hipSuccess) return fail_hip(he, "eval_barrier");
  const bool fits = act->p.cap <= s->act_cap;
  const bool fork = fits && cap_status == hipStreamCaptureStatusNone && act->flags_d && act->p.i_d &&
                    act->p.j_d && act->p.type_d;
  if (fork) {
    if ((he = hipEventRecord(s->ev_fork, st)) != hipSuccess || (he = hipStreamWaitEvent(s->side, s->ev_fork, 0)))
      return fail_hip(he, "eval_barrier: fork");
    StageTimer tm(s, BF_T_ASM_STRUCT, s->side);
    run_asm_structure(S, act->p.i_d, act->p.j_d, act->p.type_d, act->flags_d, (const long long*)act->p.count_d,
                      act->p.cap, s->aw, s->side);
  }
  {
    StageTimer tm(s, BF_T_EVAL, st);
    run_eval(S, x_d, act->p.i_d, act->p.j_d, act->p.type_d, act->code_d, act->flags_d,
             (const long long*)act->p.count_d, act->p.cap, out->E_d, out->G_d, out->H_d,
             fits ? s->aw.epart : nullptr, st);
  }
  if (fork) {
    if ((he = hipEventRecord(s->ev_join, s->side)) != hipSuccess || (he = hipStreamWaitEvent(st, s->ev_join, 0)))
      return fail_hip(he, "eval_barrier: join");
    s->prepared = true;
    s->prepared_for = act->p.i_d;
  }
  he = hipGetLastError();
  return he == hipSuccess ? BF_OK : fail_hip(he, "eval_barrier");
}

bf_status assemble_grad_hess(bf_scene* s, const bf_active* act, const bf_local* loc, double* E_d, double* g_d,
                             bf_bsr* H, void* stream) {
  if (!s || !act || !loc || !E_d || !g_d || !H || !H->row_ptr_d || !H->col_d || !H->val_d || !H->nnzb_d ||
      H->cap < 1 || !act->p.count_d)
    return fail(BF_E_ARG, "assemble_grad_hess: null argument or capacity < 1");
  if (act->p.cap > s->act_cap)
    return fail(BF_E_CAPACITY, "assemble_grad_hess: active capacity exceeds the scene reserve (bf_scene_reserve)");
  hipStream_t st = (hipStream_t)stream;
  s->last = st;
  const SceneDev S = dev_view(s);
  if (!(s->prepared && s->prepared_for == act->p.i_d)) {
    StageTimer tm(s, BF_T_ASM_STRUCT, st);
    run_asm_structure(S, act->p.i_d, act->p.j_d, act->p.type_d, act->flags_d, (const long long*)act->p.count_d,
                      act->p.cap, s->aw, st);
  }
  s->prepared = false;
  StageTimer tm(s, BF_T_ASM_VALUES, st);
  run_asm_values(S, act->p.i_d, act->p.j_d, act->p.type_d, (const long long*)act->p.count_d, act->p.cap, loc->G_d,
                 loc->H_d, E_d, g_d, H->row_ptr_d, H->col_d, H->val_d, H->cap, (long long*)H->nnzb_d, s->aw,
                 s->d_status, st);
  hipError_t he = hipGetLastError();
  return he == hipSuccess ? BF_OK : fail_hip(he, "assemble_grad_hess");
}

bf_status bf_scene_deferred(bf_scene* s, int64_t* n_band_h, int64_t* n_exact_h) {
  if (!s) return fail(BF_E_ARG, "bf_scene_deferred: null scene");
  hipError_t he = hipStreamSynchronize(s->last);
  unsigned v[2] = {0, 0};
  if (he == hipSuccess) he = hipMemcpy(v, s->d_status + 1, sizeof(v), hipMemcpyDeviceToHost);
  if (he != hipSuccess) return fail_hip(he, "bf_scene_deferred");
  if (n_band_h) *n_band_h = v[0];
  if (n_exact_h) *n_exact_h = v[1];
  return BF_OK;
}

bf_status bf_scene_set_timing(bf_scene* s, int32_t on) {
  if (!s) return fail(BF_E_ARG, "bf_scene_set_timing: null scene");
  if (on && !s->tev[0][0]) {
    for (int k = 0; k < BF_T_COUNT; ++k)
      for (int e = 0; e < 2; ++e) {
        hipError_t he = hipEventCreate(&s->tev[k][e]);
        if (he != hipSuccess) return fail_hip(he, "bf_scene_set_timing");
      }
  }
  s->timing = on != 0;
  for (int k = 0; k < BF_T_COUNT; ++k) s->tev_set[k] = false;
  return BF_OK;
}

bf_status bf_scene_stage_ms(bf_scene* s, float* ms_h) {
  if (!s || !ms_h) return fail(BF_E_ARG, "bf_scene_stage_ms: null argument");
  for (int k = 0; k < BF_T_COUNT; ++k) {
    ms_h[k] = -1.0f;
    if (!s->tev_set[k]) continue;
    hipError_t he = hipEventSynchronize(s->tev[k][1]);
    if (he == hipSuccess) he = hipEventElapsedTime(&ms_h[k], s->tev[k][0], s->tev[k][1]);
    if (he != hipSuccess) return fail_hip(he, "bf_scene_stage_ms");
  }
  return BF_OK;
}

}  // extern "C"

// For the serving loop (bfc_serve.hip): the status word into device memory
// and cleared, in stream order; and the library's error message.
bf_status bfc_status_take(bf_scene* s, uint32_t* dst_d, void* stream) {
  if (!s || !dst_d) return fail(BF_E_ARG, "bf_serve: null argument");
  hipStream_t st = (hipStream_t)stream;
  s->last = st;
  run_status_take(s->d_status, dst_d, st);
  const hipError_t he = hipGetLastError();
  return he == hipSuccess ? BF_OK : fail_hip(he, "bf_serve: status");
}
bf_status bfc_fail(bf_status code, const char* msg) { return fail(code, msg); }

// Scenes whose step workspaces (broad phase, narrow-phase staging, assembly)
// are lent per request from a pool, so that only their persistent part
// stays resident.  bfc_scene_bytes_shared: the persistent bytes (as
// bf_workspace_bytes); bfc_step_bytes: the bytes of the step workspaces for
// the mesh and the given capacities; bfc_scene_create_shared:
// bf_scene_create_ws without step workspaces; bfc_scene_bind_step: carve
// them for this scene from ws_d (clearing, on the stream, what the step
// expects at zero).
bf_status bfc_scene_bytes_shared(const bf_mesh_desc* mesh, const bf_params* params, int64_t* bytes_h) {
  if (!bytes_h) return fail(BF_E_ARG, "bf_serve: null argument");
  if (bf_status r = check_scene_args(mesh, params, 1, 1); r != BF_OK) return r;
  bf_scene probe;
  probe.prm = *params;
  probe.kind = mesh->kind;
  probe.nv = (int)mesh->n_verts;
  probe.ne = (int)mesh->n_edges;
  probe.nt = mesh->kind == BF_SHELL ? (int)mesh->n_tris : 0;
  probe.shared_step = true;
  Arena a;
  g_arena = &a;
  const bf_status r = alloc_persistent(&probe, 1, 1);
  g_arena = nullptr;
  if (r != BF_OK) return r;
  *bytes_h = (int64_t)a.off + 255;
  return BF_OK;
}

bf_status bfc_step_bytes(const bf_mesh_desc* mesh, int64_t cand_cap, int64_t act_cap, int64_t* bytes_h) {
  if (!bytes_h || !mesh || mesh->n_verts < 1 || cand_cap < 1 || act_cap < 1)
    return fail(BF_E_ARG, "bf_serve: bad argument");
  bf_scene probe;
  probe.kind = mesh->kind;
  probe.nv = (int)mesh->n_verts;
  probe.ne = (int)mesh->n_edges;
  probe.nt = mesh->kind == BF_SHELL ? (int)mesh->n_tris : 0;
  Arena a;
  g_arena = &a;
  bf_status r = alloc_asm(&probe, act_cap);
  if (r == BF_OK) r = alloc_stage(&probe, cand_cap);
  if (r == BF_OK) r = alloc_broad(&probe, probe.allocs);
  g_arena = nullptr;
  if (r != BF_OK) return r;
  *bytes_h = (int64_t)a.off + 255;
  return BF_OK;
}

bf_status bfc_scene_create_shared(const bf_mesh_desc* mesh, const bf_params* params, int64_t cand_cap,
                                  void* ws_d, int64_t ws_bytes, void* stream, bf_scene** out) {
  if (!ws_d || ws_bytes < 1) return fail(BF_E_ARG, "bf_serve: null or empty workspace");
  const uintptr_t b0 = (uintptr_t)ws_d, b1 = (b0 + 255) & ~(uintptr_t)255;
  if ((int64_t)(b1 - b0) >= ws_bytes) return fail(BF_E_CAPACITY, "bf_serve: workspace too small");
  Arena a;
  a.base = (char*)b1;
  a.cap = (size_t)(ws_bytes - (int64_t)(b1 - b0));
  return create_scene(mesh, params, std::max<int64_t>(cand_cap, 1), 1, stream, &a, out, true);
}

bf_status bfc_scene_bind_step(bf_scene* s, void* ws_d, int64_t ws_bytes, int64_t cand_cap, int64_t act_cap,
                              void* stream) {
  if (!s || !s->shared_step || !ws_d) return fail(BF_E_ARG, "bf_serve: bad step binding");
  const uintptr_t b0 = (uintptr_t)ws_d, b1 = (b0 + 255) & ~(uintptr_t)255;
  Arena a;
  a.base = (char*)b1;
  a.cap = (size_t)(ws_bytes - (int64_t)(b1 - b0));
  g_arena = &a;
  g_alloc_stream = (hipStream_t)stream;
  AsmWs A{};
  bf_status r = alloc_asm_ws(s, act_cap, s->asm_allocs, &A, "bf_serve: step workspace");
  if (r == BF_OK) {
    s->aw = A;
    s->act_cap = act_cap;
    r = alloc_stage(s, cand_cap);
  }
  if (r == BF_OK) r = alloc_broad(s, s->allocs);  // carved from the block: nothing is recorded to free
  g_arena = nullptr;
  s->prepared = false;
  return r;
}

extern "C" {

bf_status bf_status_word(bf_scene* s, uint32_t* bits_h, int32_t clear) {
  if (!s || !bits_h) return fail(BF_E_ARG, "bf_status_word: null argument");
  hipError_t he = hipStreamSynchronize(s->last);
  if (he != hipSuccess) return fail_hip(he, "bf_status_word");
  unsigned v = 0;
  he = hipMemcpy(&v, s->d_status, sizeof(unsigned), hipMemcpyDeviceToHost);
  if (he != hipSuccess) return fail_hip(he, "bf_status_word");
  *bits_h = v;
  if (clear) {
    he = hipMemset(s->d_status, 0, sizeof(unsigned));
    if (he != hipSuccess) return fail_hip(he, "bf_status_word");
  }
  return BF_OK;
}

}  // extern "C"

// ===========================================================================
// Tuning and batches
// ===========================================================================
struct bf_batch {
  std::vector<bf_batch_item> items;
  std::vector<int> lane_of;
  int lanes = 1;
  hipStream_t origin = nullptr;      // capture stream
  std::vector<hipStream_t> lane_st;  // default priority
  std::vector<hipEvent_t> events;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;         // recorded after every launch
};

namespace {

bf_status run_item(const bf_batch_item& it, hipStream_t st) {
  bf_status r = build_candidates(it.scene, it.x_d, const_cast<bf_pairs*>(&it.cand), st);
  if (r == BF_OK) r = filter_pairs(it.scene, it.x_d, &it.cand, const_cast<bf_active*>(&it.act), st);
  if (r == BF_OK) r = eval_barrier(it.scene, it.x_d, &it.act, const_cast<bf_local*>(&it.loc), st);
  if (r == BF_OK) r = assemble_grad_hess(it.scene, &it.act, &it.loc, it.E_d, it.g_d, const_cast<bf_bsr*>(&it.H), st);
  return r;
}

void batch_release_graph(bf_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  for (hipEvent_t e : b->events) (void)hipEventDestroy(e);
  b->events.clear();
  for (hipStream_t s : b->lane_st) (void)hipStreamDestroy(s);
  b->lane_st.clear();
}

// Assign items to lanes (largest first, least loaded lane), then capture one
// step of every item: fork from the origin stream, each lane runs its items in
// order, join back.
bf_status batch_capture(bf_batch* b, int lanes) {
  batch_release_graph(b);
  const int n = (int)b->items.size();
  lanes = std::max(1, std::min(lanes, n));
  b->lanes = lanes;
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  auto cost = [&](int i) {
    const bf_scene* s = b->items[i].scene;
    return (long long)s->ne + s->nt + (s->kind == BF_SHELL ? s->nv : 0);
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return cost(a) > cost(c); });
  std::vector<long long> load(lanes, 0);
  b->lane_of.assign(n, 0);
  for (int i : order) {
    int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    b->lane_of[i] = l;
    load[l] += cost(i);
  }
  hipError_t he;
  for (int l = 0; l < lanes; ++l) {
    hipStream_t st;
    if ((he = hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) != hipSuccess) return fail_hip(he, "bf_batch");
    b->lane_st.push_back(st);
  }
  for (int k = 0; k < 1 + lanes; ++k) {
    hipEvent_t e;
    if ((he = hipEventCreateWithFlags(&e, hipEventDisableTiming)) != hipSuccess) return fail_hip(he, "bf_batch");
    b->events.push_back(e);
  }
  // the four calls record their stream in the scene (the stream bf_scene_destroy
  // and bf_status_word order against); under capture that would be a lane stream
  // of this batch, destroyed with it, so each scene's stream is put back after
  std::vector<hipStream_t> last(n);
  for (int i = 0; i < n; ++i) last[i] = b->items[i].scene->last;
  struct Restore {
    bf_batch* b;
    std::vector<hipStream_t>& last;
    ~Restore() {
      for (size_t i = 0; i < last.size(); ++i) b->items[i].scene->last = last[i];
    }
  } restore{b, last};
  if ((he = hipStreamBeginCapture(b->origin, hipStreamCaptureModeThreadLocal)) != hipSuccess)
    return fail_hip(he, "bf_batch: begin capture");
  bf_status r = BF_OK;
  if ((he = hipEventRecord(b->events[0], b->origin)) != hipSuccess) r = fail_hip(he, "bf_batch: fork");
  for (int l = 0; l < lanes && r == BF_OK; ++l)
    if ((he = hipStreamWaitEvent(b->lane_st[l], b->events[0], 0)) != hipSuccess) r = fail_hip(he, "bf_batch: fork");
  for (int l = 0; l < lanes && r == BF_OK; ++l)
    for (int i = 0; i < n && r == BF_OK; ++i)
      if (b->lane_of[i] == l) r = run_item(b->items[i], b->lane_st[l]);
  for (int l = 0; l < lanes && r == BF_OK; ++l) {
    if ((he = hipEventRecord(b->events[1 + l], b->lane_st[l])) != hipSuccess ||
        (he = hipStreamWaitEvent(b->origin, b->events[1 + l], 0)) != hipSuccess)
      r = fail_hip(he, "bf_batch: join");
  }
  hipGraph_t g = nullptr;
  he = hipStreamEndCapture(b->origin, &g);
  if (r != BF_OK) {
    if (g) (void)hipGraphDestroy(g);
    return r;
  }
  if (he != hipSuccess) return fail_hip(he, "bf_batch: end capture");
  b->graph = g;
  if ((he = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0)) != hipSuccess)
    return fail_hip(he, "bf_batch: instantiate");
  return BF_OK;
}

}  // namespace

extern "C" {

bf_status bf_scene_set_pq(bf_scene* s, int32_t pq) {
  static_assert(PQ_MAX >= 16, "the per-thread broad-phase buffers are sized for PQ_MAX threads per query");
  if (!s || (pq != 2 && pq != 4 && pq != 8 && pq != 16))
    return fail(BF_E_ARG, "bf_scene_set_pq: pq must be 2, 4, 8 or 16");
  s->pq = pq;
  return BF_OK;
}

bf_status bf_scene_tune(bf_scene* s, const double* x_d, bf_pairs* cand, int32_t reps, void* stream,
                        int32_t* pq_out) {
  if (!s || !x_d || !cand || reps < 1) return fail(BF_E_ARG, "bf_scene_tune: bad argument");
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0, e1;
  hipError_t he;
  if ((he = hipEventCreate(&e0)) != hipSuccess) return fail_hip(he, "bf_scene_tune");
  if ((he = hipEventCreate(&e1)) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail_hip(he, "bf_scene_tune");
  }
  const int choices[4] = {2, 4, 8, 16};
  int best = s->pq;
  float best_ms = INFINITY;
  bf_status r = BF_OK;
  for (int c = 0; c < 4 && r == BF_OK; ++c) {
    s->pq = choices[c];
    r = build_candidates(s, x_d, cand, stream);  // warm
    std::vector<float> t;
    for (int k = 0; k < reps && r == BF_OK; ++k) {
      float ms = 0.0f;
      if ((he = hipEventRecord(e0, st)) != hipSuccess) { r = fail_hip(he, "bf_scene_tune"); break; }
      r = build_candidates(s, x_d, cand, stream);
      if (r != BF_OK) break;
      if ((he = hipEventRecord(e1, st)) != hipSuccess || (he = hipEventSynchronize(e1)) != hipSuccess ||
          (he = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) {
        r = fail_hip(he, "bf_scene_tune");
        break;
      }
      t.push_back(ms);
    }
    if (r != BF_OK) break;
    std::nth_element(t.begin(), t.begin() + t.size() / 2, t.end());
    if (t[t.size() / 2] < best_ms) {
      best_ms = t[t.size() / 2];
      best = choices[c];
    }
  }
  s->pq = best;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (r == BF_OK && pq_out) *pq_out = best;
  return r;
}

bf_status bf_batch_create(const bf_batch_item* items, int32_t n, int32_t lanes, void* stream, bf_batch** out) {
  if (!items || n < 1 || !out || lanes < 0) return fail(BF_E_ARG, "bf_batch_create: bad argument");
  for (int i = 0; i < n; ++i)
    if (!items[i].scene || !items[i].x_d) return fail(BF_E_ARG, "bf_batch_create: item without scene or positions");
  hipStream_t st = (hipStream_t)stream;
  hipError_t he = hipStreamSynchronize(st);
  if (he != hipSuccess) return fail_hip(he, "bf_batch_create");
  bf_batch* b = new bf_batch();
  b->items.assign(items, items + n);
  if ((he = hipStreamCreateWithFlags(&b->origin, hipStreamNonBlocking)) != hipSuccess ||
      (he = hipEventCreateWithFlags(&b->done, hipEventDisableTiming)) != hipSuccess) {
    if (b->origin) (void)hipStreamDestroy(b->origin);
    delete b;
    return fail_hip(he, "bf_batch_create");
  }
  // lanes = 0: as many as the device has hardware queues for one process
  // (4).  The batch is captured once: tuning the lane count by capturing,
  // timing and destroying several graphs in a row was followed by a crash in
  // the runtime at the next launch (host segmentation fault, cause not
  // known), so that path is gone.
  bf_status r = batch_capture(b, lanes > 0 ? lanes : 4);
  if (r == BF_OK && (he = hipStreamSynchronize(b->origin)) != hipSuccess) r = fail_hip(he, "bf_batch_create");
  if (r != BF_OK) {
    bf_batch_destroy(b);
    return r;
  }
  *out = b;
  return BF_OK;
}

bf_status bf_batch_step(bf_batch* b, void* stream) {
  if (!b || !b->exec) return fail(BF_E_STATE, "bf_batch_step: batch not captured");
  hipStream_t st = (hipStream_t)stream;
  hipError_t he = hipGraphLaunch(b->exec, st);
  if (he == hipSuccess) he = hipEventRecord(b->done, st);
  if (he != hipSuccess) return fail_hip(he, "bf_batch_step");
  for (auto& it : b->items) it.scene->last = st;
  return BF_OK;
}

bf_status bf_batch_info(const bf_batch* b, int32_t* lanes, int32_t* lane_of_h) {
  if (!b) return fail(BF_E_ARG, "bf_batch_info: null batch");
  if (lanes) *lanes = b->lanes;
  if (lane_of_h)
    for (size_t i = 0; i < b->lane_of.size(); ++i) lane_of_h[i] = b->lane_of[i];
  return BF_OK;
}

bf_status bf_batch_destroy(bf_batch* b) {
  if (!b) return BF_OK;
  if (b->done) (void)hipEventSynchronize(b->done);  // the last launch only
  if (b->origin) (void)hipStreamSynchronize(b->origin);
  batch_release_graph(b);
  if (b->done) (void)hipEventDestroy(b->done);
  if (b->origin) (void)hipStreamDestroy(b->origin);
  delete b;
  return BF_OK;
}

}  // extern "C"
