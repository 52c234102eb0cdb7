// Serving loop in the library (bf_serve_*): contact-evaluation requests for
// many registered scenes, each a whole step (the four calls of the path) at
// positions the host sends.
//
// A worker thread owns the device side.  Admission takes queued requests in
// arrival order; a request whose scene is busy, or whose scene does not fit
// the device-memory budget yet, may be passed by later ones, at most
// max_bypass times (then it blocks the requests behind it).  A scene that is
// not resident is created in one device block of its own (the scene
// workspace of bf_workspace_bytes plus the buffers of its step) after idle
// resident scenes are evicted, least recently used first.  Admitted requests
// run on `slots` streams at once; a request completes when its energy,
// counters, status word and (if asked for) gradient are back in host memory.
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

// from bfc_api.hip: copy the scene's status word to dst (device) and clear
// it, in stream order
bf_status bfc_status_take(bf_scene* s, uint32_t* dst_d, void* stream);
bf_status bfc_fail(bf_status code, const char* msg);

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

struct Reg {  // a registered scene
  std::vector<int32_t> edges, tris;
  std::vector<double> ref, ref_pos;
  bf_mesh_desc mesh{};
  bf_params prm{};
  int64_t cand_cap = 0, act_cap = 0, bsr_cap = 0;
  int64_t ws_bytes = 0, io_bytes = 0;
  // resident state
  bf_scene* scene = nullptr;
  char* mem = nullptr;
  bf_pairs cand{};
  bf_active act{};
  bf_local loc{};
  bf_bsr bsr{};
  double *x_d = nullptr, *E_d = nullptr, *g_d = nullptr;
  uint32_t* st_d = nullptr;
  bool busy = false;
  uint64_t last_use = 0;
  int64_t footprint() const { return ws_bytes + io_bytes; }
};

struct Req {
  int64_t ticket = 0;
  int32_t scene = 0;
  std::vector<double> x;
  double* g_h = nullptr;
  int bypassed = 0;
  Clock::time_point t0;
  bf_serve_result res{};
};

struct Slot {
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;
  double* x_pin = nullptr;
  double* g_pin = nullptr;
  ScenePin* r_pin = nullptr;
  Req* req = nullptr;
};

}  // namespace

struct bf_server {
  int device = 0;
  int64_t budget = 0, used = 0;
  int max_bypass = 8;
  std::vector<Reg> regs;
  std::vector<Slot> slots;
  std::deque<Req*> queue;
  std::unordered_map<int64_t, Req*> tickets;
  int64_t next_ticket = 1;
  uint64_t clock = 0;
  bool stopping = false;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::thread worker;
  hipStream_t create_st = nullptr;
};

namespace {

// The buffers of one scene's step, carved after its workspace.
int64_t io_bytes_of(const Reg& r) {
  const int64_t V = r.mesh.n_verts, C = r.cand_cap, A = r.act_cap, B = r.bsr_cap;
  size_t n = 0;
  for (size_t b : {(size_t)(4 * C), (size_t)(4 * C), (size_t)C, (size_t)8,                            // candidates
                   (size_t)(4 * A), (size_t)(4 * A), (size_t)A, (size_t)8, (size_t)A, (size_t)A,  // active
                   (size_t)(8 * A), (size_t)32,                                                   // dist, counters
                   (size_t)(8 * A), (size_t)(96 * A), (size_t)(624 * A),                          // E, G, H
                   (size_t)(4 * (V + 1)), (size_t)(4 * B), (size_t)(72 * B), (size_t)8,           // BSR
                   (size_t)(24 * V), (size_t)8, (size_t)(24 * V), (size_t)4})                     // x, E, g, status
    n = up256(n) + b;
  return (int64_t)up256(n);
}

void carve_io(Reg& r) {
  const int64_t V = r.mesh.n_verts, C = r.cand_cap, A = r.act_cap, B = r.bsr_cap;
  size_t off = (size_t)r.ws_bytes;
  auto take = [&](size_t bytes) {
    off = up256(off);
    char* p = r.mem + off;
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
  r.loc.H_d = (double*)take(624 * A);
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

void evict(bf_server* sv, Reg& r) {
  if (r.scene) (void)bf_scene_destroy(r.scene);
  if (r.mem) (void)hipFree(r.mem);  // the scene is idle: its last request has completed
  r.scene = nullptr;
  r.mem = nullptr;
  sv->used -= r.footprint();
}

bf_status make_resident(bf_server* sv, Reg& r) {
  hipError_t he = hipMalloc((void**)&r.mem, (size_t)r.footprint());
  if (he != hipSuccess) {
    r.mem = nullptr;
    return bfc_fail(BF_E_NOMEM, "bf_serve: scene allocation failed");
  }
  bf_status st = bf_scene_create_ws(&r.mesh, &r.prm, r.cand_cap, r.act_cap, r.mem, r.ws_bytes, sv->create_st,
                                    &r.scene);
  if (st != BF_OK) {
    (void)hipFree(r.mem);
    r.mem = nullptr;
    r.scene = nullptr;
    return st;
  }
  carve_io(r);
  sv->used += r.footprint();
  return BF_OK;
}

void launch(bf_server* sv, Slot& sl, Req* q) {
  Reg& r = sv->regs[q->scene];
  const int64_t V = r.mesh.n_verts;
  std::memcpy(sl.x_pin, q->x.data(), sizeof(double) * 3 * V);
  bf_status st = BF_OK;
  hipError_t he = hipMemcpyAsync(r.x_d, sl.x_pin, sizeof(double) * 3 * V, hipMemcpyHostToDevice, sl.st);
  if (he != hipSuccess) st = bfc_fail(BF_E_DEVICE, "bf_serve: upload");
  if (st == BF_OK) st = build_candidates(r.scene, r.x_d, &r.cand, sl.st);
  if (st == BF_OK) st = filter_pairs(r.scene, r.x_d, &r.cand, &r.act, sl.st);
  if (st == BF_OK) st = eval_barrier(r.scene, r.x_d, &r.act, &r.loc, sl.st);
  if (st == BF_OK) st = assemble_grad_hess(r.scene, &r.act, &r.loc, r.E_d, r.g_d, &r.bsr, sl.st);
  if (st == BF_OK) st = bfc_status_take(r.scene, r.st_d, sl.st);
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
  if (st == BF_OK && hipEventRecord(sl.ev, sl.st) != hipSuccess) st = bfc_fail(BF_E_DEVICE, "bf_serve: event");
  q->res.error = st;
  r.busy = true;
  r.last_use = ++sv->clock;
  sl.req = q;
}

// A request leaves its slot: results into its record (caller's gradient
// too), the scene becomes idle.
void finish(bf_server* sv, Slot& sl) {
  Req* q = sl.req;
  Reg& r = sv->regs[q->scene];
  if (q->res.error == BF_OK) {
    const ScenePin* rp = sl.r_pin;
    q->res.E = rp->E;
    for (int k = 0; k < 4; ++k) q->res.counts[k] = rp->counters[k];
    q->res.counts[4] = rp->nnzb;
    q->res.n_bp = rp->n_bp;
    q->res.status = rp->status;
    if (q->g_h) std::memcpy(q->g_h, sl.g_pin, sizeof(double) * 3 * r.mesh.n_verts);
  }
  q->res.ms = std::chrono::duration<double, std::milli>(Clock::now() - q->t0).count();
  q->res.done = 1;
  r.busy = false;
  sl.req = nullptr;
}

// Start what can start now (arrival order, bypass bound, budget).
void admit(bf_server* sv, std::unique_lock<std::mutex>& lk) {
  std::deque<Req*> kept;
  bool blocked = false;
  while (!sv->queue.empty()) {
    Req* q = sv->queue.front();
    sv->queue.pop_front();
    int free_slot = -1;
    for (size_t k = 0; k < sv->slots.size(); ++k)
      if (!sv->slots[k].req) { free_slot = (int)k; break; }
    Reg& r = sv->regs[q->scene];
    if (blocked || free_slot < 0 || r.busy) {
      if (!blocked && free_slot >= 0) ++q->bypassed;
      blocked = blocked || q->bypassed > sv->max_bypass;
      kept.push_back(q);
      continue;
    }
    if (!r.scene) {
      // room: evict idle scenes, least recently used first
      while (sv->used + r.footprint() > sv->budget) {
        Reg* lru = nullptr;
        for (Reg& o : sv->regs)
          if (o.scene && !o.busy && (!lru || o.last_use < lru->last_use)) lru = &o;
        if (!lru) break;
        evict(sv, *lru);
      }
      if (sv->used + r.footprint() > sv->budget) {  // the busy scenes hold the memory: wait
        ++q->bypassed;
        blocked = blocked || q->bypassed > sv->max_bypass;
        kept.push_back(q);
        continue;
      }
      lk.unlock();  // creation synchronises its own stream; submitters may go on meanwhile
      const bf_status st = make_resident(sv, r);
      lk.lock();
      if (st != BF_OK) {
        q->res.error = st;
        q->res.ms = std::chrono::duration<double, std::milli>(Clock::now() - q->t0).count();
        q->res.done = 1;
        sv->cv_done.notify_all();
        continue;
      }
    }
    launch(sv, sv->slots[free_slot], q);
  }
  sv->queue = std::move(kept);
}

void work(bf_server* sv) {
  (void)hipSetDevice(sv->device);
  std::unique_lock<std::mutex> lk(sv->mu);
  while (true) {
    bool any_done = false;
    for (Slot& sl : sv->slots) {
      if (!sl.req) continue;
      const hipError_t e = hipEventQuery(sl.ev);
      if (e == hipErrorNotReady) continue;
      if (e != hipSuccess && sl.req->res.error == BF_OK) sl.req->res.error = BF_E_DEVICE;
      finish(sv, sl);
      any_done = true;
    }
    if (any_done) sv->cv_done.notify_all();
    if (!sv->queue.empty()) admit(sv, lk);
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
  sv->budget = cfg->budget_bytes;
  sv->max_bypass = cfg->max_bypass;
  sv->regs.resize(cfg->n_scenes);
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
    const bf_status st = bf_workspace_bytes(&r.mesh, &r.prm, r.cand_cap, r.act_cap, &r.ws_bytes);
    if (st != BF_OK) {
      delete sv;
      return st;
    }
    r.ws_bytes = (int64_t)up256((size_t)r.ws_bytes);
    r.io_bytes = io_bytes_of(r);
    if (r.footprint() > sv->budget) {
      delete sv;
      return bfc_fail(BF_E_CAPACITY, "bf_serve_start: a scene alone is above the budget");
    }
    vmax = std::max<int64_t>(vmax, m.n_verts);
  }
  sv->slots.resize(cfg->slots);
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
  if (sv->worker.joinable()) sv->worker.join();
  (void)hipSetDevice(sv->device);
  for (Reg& r : sv->regs)
    if (r.scene) evict(sv, r);
  for (Slot& sl : sv->slots) {
    if (sl.ev) (void)hipEventDestroy(sl.ev);
    if (sl.st) (void)hipStreamDestroy(sl.st);
    if (sl.x_pin) (void)hipHostFree(sl.x_pin);
    if (sl.g_pin) (void)hipHostFree(sl.g_pin);
    if (sl.r_pin) (void)hipHostFree(sl.r_pin);
  }
  if (sv->create_st) (void)hipStreamDestroy(sv->create_st);
  for (auto& kv : sv->tickets) delete kv.second;
  delete sv;
  return BF_OK;
}

bf_status bf_serve_info(bf_server* sv, int32_t* resident_h, int64_t* used_bytes_h, int64_t* footprint_h) {
  if (!sv) return bfc_fail(BF_E_ARG, "bf_serve_info: null server");
  std::lock_guard<std::mutex> g(sv->mu);
  int n = 0;
  for (size_t k = 0; k < sv->regs.size(); ++k) {
    n += sv->regs[k].scene != nullptr;
    if (footprint_h) footprint_h[k] = sv->regs[k].footprint();
  }
  if (resident_h) *resident_h = n;
  if (used_bytes_h) *used_bytes_h = sv->used;
  return BF_OK;
}

}  // extern "C"
