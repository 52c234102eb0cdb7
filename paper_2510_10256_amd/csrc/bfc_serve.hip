// Serving loop in the library (bf_serve_*): contact-evaluation requests for
// many registered scenes, each a whole step (the four calls of the path) at
// positions the host sends.
//
// A worker thread owns the device side, and a builder thread creates the
// scenes that admission makes resident (the request waits on its slot while
// the worker runs the others).  All device memory of the server is
// one block of the budget's size, divided by the admission policy (a heap
// over the block, bfc_admit.h): a resident scene holds only what persists
// between its steps (topology, rest data and filter precompute, broad-phase
// workspace), and a request on the device holds, for its duration, a step
// block with everything else (narrow-phase staging, assembly workspace,
// candidate and active lists, per-pair results, BSR, positions, gradient),
// bound to its scene for the request.  Admitted requests run on `slots`
// streams at once; a request completes when its energy, counters, status
// word and (if asked for) gradient are back in host memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "bfc.h"
#include "bfc_admit.h"

// from bfc_api.hip: copy the scene's status word to dst (device) and clear
// it, in stream order; scenes whose step workspaces are lent per request
bf_status bfc_status_take(bf_scene* s, uint32_t* dst_d, void* stream);
bf_status bfc_fail(bf_status code, const char* msg);
bf_status bfc_scene_bytes_shared(const bf_mesh_desc* mesh, const bf_params* params, int64_t* bytes_h);
bf_status bfc_step_bytes(const bf_mesh_desc* mesh, int64_t cand_cap, int64_t act_cap, int64_t* bytes_h);
bf_status bfc_scene_create_shared(const bf_mesh_desc* mesh, const bf_params* params, int64_t cand_cap,
                                  void* ws_d, int64_t ws_bytes, void* stream, bf_scene** out);
bf_status bfc_scene_bind_step(bf_scene* s, void* ws_d, int64_t ws_bytes, int64_t cand_cap, int64_t act_cap,
                              void* stream);

namespace {

using Clock = std::chrono::steady_clock;

size_t up256(size_t v) { return (v + 255) & ~(size_t)255; }

struct ScenePin {  // results of one request, copied back in one piece
  double E;
  int64_t counters[4];
  int64_t nnzb;
  int64_t n_bp;
  uint32_t status;
};

struct Reg {  // a registered scene (its residency is the admission policy's)
  std::vector<int32_t> edges, tris;
  std::vector<double> ref, ref_pos;
  bf_mesh_desc mesh{};
  bf_params prm{};
  int64_t cand_cap = 0, act_cap = 0, bsr_cap = 0;
  int64_t ws_bytes = 0;                  // resident (persistent) part
  int64_t step_bytes = 0, io_bytes = 0;  // a step's workspaces, then its buffers
  bf_scene* scene = nullptr;
  bool building = false;  // its creation is queued or running on the builder thread
};

// The step buffers of one request, carved from its step block.
struct StepIO {
  bf_pairs cand{};
  bf_active act{};
  bf_local loc{};
  bf_bsr bsr{};
  double *x_d = nullptr, *E_d = nullptr, *g_d = nullptr;
  uint32_t* st_d = nullptr;
};

struct Req {
  int64_t ticket = 0;
  int32_t scene = 0;
  std::vector<double> x;
  double* g_h = nullptr;
  int bypassed = 0;
  int retries = 0;
  Clock::time_point t0;
  bf_serve_result res{};
};

struct Slot {
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;
  StepIO io{};
  double* x_pin = nullptr;
  double* g_pin = nullptr;
  ScenePin* r_pin = nullptr;
  Req* req = nullptr;
  int creating = 0;  // the request waits for its scene: 1 being built, 2 built, 3 the build failed
};

struct Build {  // a scene creation for the builder thread
  int scene;
  int64_t off;
};

struct Dev;

}  // namespace

struct bf_server {
  int device = 0;
  char* base = nullptr;  // the budget's device block
  std::vector<Reg> regs;
  std::vector<Slot> slots;
  bfc::Admission<Req, Dev> adm;
  std::deque<Req*> queue;
  std::unordered_map<int64_t, Req*> tickets;
  int64_t next_ticket = 1;
  int64_t retried = 0;  // overflow re-runs so far
  bool stopping = false;
  std::mutex mu;
  std::condition_variable cv_work, cv_done, cv_build;
  std::thread worker, builder;
  std::deque<Build> builds;
  bool stop_builder = false;
  hipStream_t create_st = nullptr;
};

namespace {

// The buffers of one scene's step, carved from its step block after the step
// workspaces.
// Bytes of one pair's Hessian record: 78 doubles, or 78 floats in the mixed mode.
int64_t h_bytes_of(const Reg& r) { return r.prm.prec == BF_MIXED ? 312 : 624; }

int64_t io_bytes_of(const Reg& r) {
  const int64_t V = r.mesh.n_verts, C = r.cand_cap, A = r.act_cap, B = r.bsr_cap, HB = h_bytes_of(r);
  size_t n = 0;
  for (size_t b : {(size_t)(4 * C), (size_t)(4 * C), (size_t)C, (size_t)8,                            // candidates
                   (size_t)(4 * A), (size_t)(4 * A), (size_t)A, (size_t)8, (size_t)A, (size_t)A,  // active
                   (size_t)(8 * A), (size_t)32,                                                   // dist, counters
                   (size_t)(8 * A), (size_t)(96 * A), (size_t)(HB * A),                           // E, G, H
                   (size_t)(4 * (V + 1)), (size_t)(4 * B), (size_t)(72 * B), (size_t)8,           // BSR
                   (size_t)(24 * V), (size_t)8, (size_t)(24 * V), (size_t)4})                     // x, E, g, status
    n = up256(n) + b;
  return (int64_t)up256(n);
}

void carve_io(const Reg& reg, char* base, StepIO& r) {
  const int64_t V = reg.mesh.n_verts, C = reg.cand_cap, A = reg.act_cap, B = reg.bsr_cap;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = up256(off);
    char* p = base + off;
    off += bytes;
    return (void*)p;
  };
  r.cand.i_d = (int32_t*)take(4 * C);
  r.cand.j_d = (int32_t*)take(4 * C);
  r.cand.type_d = (uint8_t*)take(C);
  r.cand.count_d = (int64_t*)take(8);
  r.cand.cap = C;
  r.act.p.i_d = (int32_t*)take(4 * A);
  r.act.p.j_d = (int32_t*)take(4 * A);
  r.act.p.type_d = (uint8_t*)take(A);
  r.act.p.count_d = (int64_t*)take(8);
  r.act.p.cap = A;
  r.act.code_d = (uint8_t*)take(A);
  r.act.flags_d = (uint8_t*)take(A);
  r.act.dist_d = (double*)take(8 * A);
  r.act.counters_d = (int64_t*)take(32);
  r.loc.E_d = (double*)take(8 * A);
  r.loc.G_d = (double*)take(96 * A);
  r.loc.H_d = take(h_bytes_of(reg) * A);
  r.loc.cap = A;
  r.bsr.row_ptr_d = (int32_t*)take(4 * (V + 1));
  r.bsr.col_d = (int32_t*)take(4 * B);
  r.bsr.val_d = (double*)take(72 * B);
  r.bsr.nnzb_d = (int64_t*)take(8);
  r.bsr.cap = B;
  r.x_d = (double*)take(24 * V);
  r.E_d = (double*)take(8);
  r.g_d = (double*)take(24 * V);
  r.st_d = (uint32_t*)take(4);
}

void launch(bf_server* sv, int k, Req* q);

// The device side of the admission policy.  A scene's creation (uploads
// and the filter precompute, synchronising its own stream) goes to the
// builder thread, so that the worker keeps launching and completing other
// requests meanwhile; the request waits on its slot until the scene is
// built.
struct Dev {
  bf_server* sv;
  bool create(int k, int64_t off) {
    sv->regs[k].building = true;
    sv->builds.push_back({k, off});
    sv->cv_build.notify_one();
    return true;
  }
  void destroy(int k) {  // the scene is idle: its last request has completed
    Reg& r = sv->regs[k];
    (void)bf_scene_destroy(r.scene);
    r.scene = nullptr;
  }
  void start(Req* q, int k) {
    Slot& sl = sv->slots[k];
    if (sv->regs[q->scene].building) {
      sl.req = q;
      sl.creating = 1;
      return;
    }
    launch(sv, k, q);
  }
  void reject(Req* q, bool too_big) {
    q->res.error = too_big ? bfc_fail(BF_E_CAPACITY, "bf_serve: the scene and its step are above the budget")
                           : bfc_fail(BF_E_NOMEM, "bf_serve: scene creation failed");
    q->res.retries = q->retries;
    q->res.ms = std::chrono::duration<double, std::milli>(Clock::now() - q->t0).count();
    q->res.done = 1;
    sv->cv_done.notify_all();
  }
};

// The builder thread: creates the scenes admission placed, one at a time,
// in its block of the budget, on a stream of its own.
void build_scenes(bf_server* sv) {
  (void)hipSetDevice(sv->device);
  std::unique_lock<std::mutex> lk(sv->mu);
  while (true) {
    sv->cv_build.wait(lk, [&] { return sv->stop_builder || !sv->builds.empty(); });
    if (sv->builds.empty()) break;  // stopping, nothing left
    const Build b = sv->builds.front();
    sv->builds.pop_front();
    Reg& r = sv->regs[b.scene];
    lk.unlock();  // the scene is busy (its request waits for it): nobody else touches it
    bf_scene* scene = nullptr;
    const bf_status st = bfc_scene_create_shared(&r.mesh, &r.prm, r.cand_cap, sv->base + b.off, r.ws_bytes,
                                                 sv->create_st, &scene);
    lk.lock();
    r.scene = st == BF_OK ? scene : nullptr;
    r.building = false;
    for (Slot& sl : sv->slots)
      if (sl.req && sl.creating == 1 && sl.req->scene == b.scene) sl.creating = st == BF_OK ? 2 : 3;
    sv->cv_work.notify_one();
  }
}

void launch(bf_server* sv, int k, Req* q) {
  Slot& sl = sv->slots[k];
  Reg& reg = sv->regs[q->scene];
  char* blk = sv->base + sv->adm.slots[k].off;  // step workspaces, then the step's buffers
  const int64_t V = reg.mesh.n_verts;
  std::memcpy(sl.x_pin, q->x.data(), sizeof(double) * 3 * V);
  hipError_t he = hipSuccess;
  StepIO& r = sl.io;
  carve_io(reg, blk + reg.step_bytes, r);
  bf_status st = bfc_scene_bind_step(reg.scene, blk, reg.step_bytes, reg.cand_cap, reg.act_cap, sl.st);
  if (st == BF_OK && (he = hipMemcpyAsync(r.x_d, sl.x_pin, sizeof(double) * 3 * V, hipMemcpyHostToDevice, sl.st)) !=
                         hipSuccess)
    st = bfc_fail(BF_E_DEVICE, "bf_serve: upload");
  if (st == BF_OK) st = build_candidates(reg.scene, r.x_d, &r.cand, sl.st);
  if (st == BF_OK) st = filter_pairs(reg.scene, r.x_d, &r.cand, &r.act, sl.st);
  if (st == BF_OK) st = eval_barrier(reg.scene, r.x_d, &r.act, &r.loc, sl.st);
  if (st == BF_OK) st = assemble_grad_hess(reg.scene, &r.act, &r.loc, r.E_d, r.g_d, &r.bsr, sl.st);
  if (st == BF_OK) st = bfc_status_take(reg.scene, r.st_d, sl.st);
  ScenePin* rp = sl.r_pin;
  if (st == BF_OK &&
      ((he = hipMemcpyAsync(&rp->E, r.E_d, 8, hipMemcpyDeviceToHost, sl.st)) != hipSuccess ||
       (he = hipMemcpyAsync(rp->counters, r.act.counters_d, 32, hipMemcpyDeviceToHost, sl.st)) != hipSuccess ||
       (he = hipMemcpyAsync(&rp->nnzb, r.bsr.nnzb_d, 8, hipMemcpyDeviceToHost, sl.st)) != hipSuccess ||
       (he = hipMemcpyAsync(&rp->n_bp, r.cand.count_d, 8, hipMemcpyDeviceToHost, sl.st)) != hipSuccess ||
       (he = hipMemcpyAsync(&rp->status, r.st_d, 4, hipMemcpyDeviceToHost, sl.st)) != hipSuccess ||
       (q->g_h && (he = hipMemcpyAsync(sl.g_pin, r.g_d, sizeof(double) * 3 * V, hipMemcpyDeviceToHost, sl.st)) !=
                      hipSuccess)))
    st = bfc_fail(BF_E_DEVICE, "bf_serve: result copy");
  // the event marks the end of everything enqueued, also after a failed call,
  // so that the step block is released only once the stream is past it
  if (hipEventRecord(sl.ev, sl.st) != hipSuccess) {
    if (st == BF_OK) st = bfc_fail(BF_E_DEVICE, "bf_serve: event");
    (void)hipStreamSynchronize(sl.st);
  }
  q->res.error = st;
  sl.req = q;
}

// Capacities that fit the sizes a step reported (its counters hold the
// sizes required), with an eighth to spare.  After an active-list overflow
// the block count is that of the pairs kept, a lower bound: the BSR grows
// by it now and by the full count if the next run overflows it.
bool grow_caps(Reg& r, const ScenePin& rp) {
  const uint32_t over = rp.status & (BF_S_CAND_OVERFLOW | BF_S_ACT_OVERFLOW | BF_S_BSR_OVERFLOW);
  if (!over) return false;
  // a count that does not show the overflow (not expected) doubles the capacity
  auto grow = [](int64_t& cap, int64_t n, bool flagged) {
    if (n > cap) cap = n + n / 8 + 1024;
    else if (flagged) cap *= 2;
  };
  grow(r.cand_cap, rp.n_bp, over & BF_S_CAND_OVERFLOW);
  grow(r.act_cap, rp.counters[2], over & BF_S_ACT_OVERFLOW);
  grow(r.bsr_cap, rp.nnzb, over & BF_S_BSR_OVERFLOW);
  int64_t sb = 0;
  if (bfc_step_bytes(&r.mesh, r.cand_cap, r.act_cap, &sb) != BF_OK) return false;
  r.step_bytes = (int64_t)up256((size_t)sb);
  r.io_bytes = io_bytes_of(r);
  return true;
}

// A request leaves its slot: its step block is released, results go into
// its record (the caller's gradient too), the scene becomes idle.  A step
// whose buffers overflowed runs again (at the head of the queue) with the
// capacities it reported, up to four times, while the scene and the larger
// step still fit the budget.
void finish(bf_server* sv, int k) {
  Slot& sl = sv->slots[k];
  Req* q = sl.req;
  Reg& r = sv->regs[q->scene];
  sv->adm.done(k, q->scene);
  sl.req = nullptr;
  if (q->res.error == BF_OK) {
    const ScenePin* rp = sl.r_pin;
    if (q->retries < 4 && grow_caps(r, *rp)) {
      bfc::AdmitScene& a = sv->adm.sc[q->scene];
      a.need = r.step_bytes + r.io_bytes;
      sv->adm.update_limit();
      if (bfc::Heap::round(a.fp) + bfc::Heap::round(a.need) <= sv->adm.heap.size()) {
        ++q->retries;
        ++sv->retried;
        sv->queue.push_front(q);
        return;
      }
    }
    q->res.E = rp->E;
    for (int c = 0; c < 4; ++c) q->res.counts[c] = rp->counters[c];
    q->res.counts[4] = rp->nnzb;
    q->res.n_bp = rp->n_bp;
    q->res.status = rp->status;
    if (q->g_h) std::memcpy(q->g_h, sl.g_pin, sizeof(double) * 3 * r.mesh.n_verts);
  }
  q->res.retries = q->retries;
  q->res.ms = std::chrono::duration<double, std::milli>(Clock::now() - q->t0).count();
  q->res.done = 1;
}

void work(bf_server* sv) {
  (void)hipSetDevice(sv->device);
  std::unique_lock<std::mutex> lk(sv->mu);
  while (true) {
    bool any_done = false;
    for (Slot& sl : sv->slots) {
      if (!sl.req) continue;
      const int k = (int)(&sl - sv->slots.data());
      if (sl.creating == 1) continue;  // its scene is being built
      if (sl.creating == 2) {          // built: the request runs now
        sl.creating = 0;
        launch(sv, k, sl.req);
        continue;
      }
      if (sl.creating == 3) {  // the build failed: the request completes unserved
        Req* q = sl.req;
        sl.req = nullptr;
        sl.creating = 0;
        sv->adm.abort_fresh(k, q->scene);
        q->res.error = bfc_fail(BF_E_NOMEM, "bf_serve: scene creation failed");
        q->res.retries = q->retries;
        q->res.ms = std::chrono::duration<double, std::milli>(Clock::now() - q->t0).count();
        q->res.done = 1;
        any_done = true;
        continue;
      }
      const hipError_t e = hipEventQuery(sl.ev);
      if (e == hipErrorNotReady) continue;
      if (e != hipSuccess && sl.req->res.error == BF_OK) sl.req->res.error = BF_E_DEVICE;
      finish(sv, k);
      any_done = true;
    }
    if (any_done) sv->cv_done.notify_all();
    if (!sv->queue.empty()) {
      Dev dev{sv};
      sv->adm.pass(dev, sv->queue);
    }
    bool active = false;
    for (Slot& sl : sv->slots) active = active || sl.req;
    if (sv->stopping && sv->queue.empty() && !active) break;
    // requests on the device: poll again shortly; otherwise sleep until a submit
    if (active) sv->cv_work.wait_for(lk, std::chrono::microseconds(20));
    else sv->cv_work.wait_for(lk, std::chrono::milliseconds(5));
  }
}

}  // namespace

extern "C" {

bf_status bf_serve_start(const bf_serve_config* cfg, bf_server** out) {
  if (!cfg || !out || cfg->n_scenes < 1 || !cfg->meshes || !cfg->params || !cfg->cand_cap || !cfg->act_cap ||
      !cfg->bsr_cap || cfg->slots < 1 || cfg->slots > 64 || cfg->budget_bytes < 1 || cfg->max_bypass < 0)
    return bfc_fail(BF_E_ARG, "bf_serve_start: bad configuration");
  *out = nullptr;
  if (hipSetDevice(cfg->device) != hipSuccess) return bfc_fail(BF_E_DEVICE, "bf_serve_start: device");
  bf_server* sv = new bf_server;
  sv->device = cfg->device;
  sv->adm.heap.reset(cfg->budget_bytes);
  sv->adm.max_bypass = cfg->max_bypass;
  sv->regs.resize(cfg->n_scenes);
  sv->adm.sc.resize(cfg->n_scenes);
  int64_t vmax = 0;
  for (int k = 0; k < cfg->n_scenes; ++k) {
    const bf_mesh_desc& m = cfg->meshes[k];
    Reg& r = sv->regs[k];
    if (!m.edges_h || !m.ref_h || m.n_verts < 2 || m.n_edges < 1 || (m.kind == BF_SHELL && !m.tris_h)) {
      delete sv;
      return bfc_fail(BF_E_ARG, "bf_serve_start: bad scene");
    }
    r.edges.assign(m.edges_h, m.edges_h + 2 * m.n_edges);
    if (m.kind == BF_SHELL) r.tris.assign(m.tris_h, m.tris_h + 3 * m.n_tris);
    r.ref.assign(m.ref_h, m.ref_h + (m.kind == BF_ROD ? m.n_verts : 2 * m.n_verts));
    if (m.ref_pos_h) r.ref_pos.assign(m.ref_pos_h, m.ref_pos_h + 3 * m.n_verts);
    r.mesh = m;
    r.mesh.edges_h = r.edges.data();
    r.mesh.tris_h = m.kind == BF_SHELL ? r.tris.data() : nullptr;
    r.mesh.ref_h = r.ref.data();
    r.mesh.ref_pos_h = m.ref_pos_h ? r.ref_pos.data() : nullptr;
    r.prm = cfg->params[k];
    r.cand_cap = cfg->cand_cap[k];
    r.act_cap = cfg->act_cap[k];
    r.bsr_cap = cfg->bsr_cap[k];
    if (r.bsr_cap < 1) {
      delete sv;
      return bfc_fail(BF_E_ARG, "bf_serve_start: BSR capacity must be >= 1");
    }
    bf_status st = bfc_scene_bytes_shared(&r.mesh, &r.prm, &r.ws_bytes);
    if (st == BF_OK) st = bfc_step_bytes(&m, r.cand_cap, r.act_cap, &r.step_bytes);
    if (st != BF_OK) {
      delete sv;
      return st;
    }
    r.ws_bytes = (int64_t)up256((size_t)r.ws_bytes);
    r.step_bytes = (int64_t)up256((size_t)r.step_bytes);
    r.io_bytes = io_bytes_of(r);
    bfc::AdmitScene& a = sv->adm.sc[k];
    a.fp = r.ws_bytes;
    a.need = r.step_bytes + r.io_bytes;
    if (bfc::Heap::round(a.fp) + bfc::Heap::round(a.need) > sv->adm.heap.size()) {
      delete sv;
      return bfc_fail(BF_E_CAPACITY, "bf_serve_start: a scene and its step are above the budget");
    }
    vmax = std::max<int64_t>(vmax, m.n_verts);
  }
  sv->slots.resize(cfg->slots);
  sv->adm.slots.resize(cfg->slots);
  sv->adm.update_limit();
  if (hipMalloc((void**)&sv->base, (size_t)sv->adm.heap.size()) != hipSuccess) {
    sv->base = nullptr;
    delete sv;
    return bfc_fail(BF_E_NOMEM, "bf_serve_start: the budget's device block");
  }
  bool ok = hipStreamCreateWithFlags(&sv->create_st, hipStreamNonBlocking) == hipSuccess;
  for (Slot& sl : sv->slots) {
    ok = ok && hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&sl.x_pin, sizeof(double) * 3 * vmax, hipHostMallocDefault) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&sl.g_pin, sizeof(double) * 3 * vmax, hipHostMallocDefault) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&sl.r_pin, sizeof(ScenePin), hipHostMallocDefault) == hipSuccess;
  }
  if (!ok) {
    sv->stopping = true;
    (void)bf_serve_stop(sv);
    return bfc_fail(BF_E_DEVICE, "bf_serve_start: streams or pinned buffers");
  }
  sv->builder = std::thread(build_scenes, sv);
  sv->worker = std::thread(work, sv);
  *out = sv;
  return BF_OK;
}

bf_status bf_serve_submit(bf_server* sv, int32_t scene, const double* x_h, double* g_h, int64_t* ticket_h) {
  if (!sv || !x_h || !ticket_h || scene < 0 || scene >= (int32_t)sv->regs.size())
    return bfc_fail(BF_E_ARG, "bf_serve_submit: bad argument");
  Req* q = new Req;
  q->scene = scene;
  q->x.assign(x_h, x_h + 3 * sv->regs[scene].mesh.n_verts);
  q->g_h = g_h;
  q->t0 = Clock::now();
  q->res.scene = scene;
  {
    std::lock_guard<std::mutex> g(sv->mu);
    if (sv->stopping) {
      delete q;
      return bfc_fail(BF_E_STATE, "bf_serve_submit: the server is stopping");
    }
    q->ticket = sv->next_ticket++;
    sv->tickets[q->ticket] = q;
    sv->queue.push_back(q);
    *ticket_h = q->ticket;
  }
  sv->cv_work.notify_one();
  return BF_OK;
}

bf_status bf_serve_poll(bf_server* sv, int64_t ticket, int32_t wait, bf_serve_result* out) {
  if (!sv || !out) return bfc_fail(BF_E_ARG, "bf_serve_poll: null argument");
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->tickets.find(ticket);
  if (it == sv->tickets.end()) return bfc_fail(BF_E_ARG, "bf_serve_poll: unknown ticket");
  Req* q = it->second;
  if (wait) sv->cv_done.wait(lk, [&] { return q->res.done != 0; });
  *out = q->res;
  if (q->res.done) {
    sv->tickets.erase(it);
    delete q;
  }
  return BF_OK;
}

bf_status bf_serve_stop(bf_server* sv) {
  if (!sv) return BF_OK;
  {
    std::lock_guard<std::mutex> g(sv->mu);
    sv->stopping = true;
  }
  sv->cv_work.notify_one();
  if (sv->worker.joinable()) sv->worker.join();  // every request completed, so no build is left
  {
    std::lock_guard<std::mutex> g(sv->mu);
    sv->stop_builder = true;
  }
  sv->cv_build.notify_one();
  if (sv->builder.joinable()) sv->builder.join();
  (void)hipSetDevice(sv->device);
  for (Reg& r : sv->regs)
    if (r.scene) (void)bf_scene_destroy(r.scene);  // idle: the worker has drained every request
  for (Slot& sl : sv->slots) {
    if (sl.ev) (void)hipEventDestroy(sl.ev);
    if (sl.st) (void)hipStreamDestroy(sl.st);
    if (sl.x_pin) (void)hipHostFree(sl.x_pin);
    if (sl.g_pin) (void)hipHostFree(sl.g_pin);
    if (sl.r_pin) (void)hipHostFree(sl.r_pin);
  }
  if (sv->base) (void)hipFree(sv->base);
  if (sv->create_st) (void)hipStreamDestroy(sv->create_st);
  for (auto& kv : sv->tickets) delete kv.second;
  delete sv;
  return BF_OK;
}

bf_status bf_serve_info(bf_server* sv, int32_t* resident_h, int64_t* used_bytes_h, int64_t* sizes_h,
                        int64_t* events_h) {
  if (!sv) return bfc_fail(BF_E_ARG, "bf_serve_info: null server");
  std::lock_guard<std::mutex> g(sv->mu);
  int n = 0;
  for (size_t k = 0; k < sv->regs.size(); ++k) {
    n += sv->adm.sc[k].off >= 0;
    if (sizes_h) {
      sizes_h[2 * k] = sv->adm.sc[k].fp;
      sizes_h[2 * k + 1] = sv->adm.sc[k].need;
    }
  }
  if (resident_h) *resident_h = n;
  if (used_bytes_h) *used_bytes_h = sv->adm.heap.used();
  if (events_h) {
    events_h[0] = sv->adm.created;
    events_h[1] = sv->adm.evicted;
    events_h[2] = sv->retried;
    events_h[3] = sv->adm.heap.peak();
  }
  return BF_OK;
}

}  // extern "C"
