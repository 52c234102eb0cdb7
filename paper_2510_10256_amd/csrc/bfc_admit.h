// Admission of the serving loop, as host logic over a device-memory budget
// (no device calls: the device side is the Dev argument, so that the policy
// runs the same against the GPU and against a fake device in CPU tests).
//
// Everything the server holds on the device lives in one block of the
// budget's size (a Heap over it): each resident scene's persistent state,
// and for each request on the device the step's workspaces and buffers.
// Scenes are placed from the low end and below a limit that keeps, at the
// high end, room for the largest step of any registered scene; steps go
// where they fit, the high end first.  So a step never needs a scene
// evicted while other steps run: it waits for them instead (steps last
// milliseconds; a scene evicted must be built again).  A pass walks the
// queue in arrival order.  A request starts when a slot is free, its scene
// is not busy, and its scene (if not resident) and its step fit; room for a
// scene is made by evicting the idle resident scenes of the range that
// frees a long enough block at the least cost (bytes to build again, then
// the least recently used).  A request that cannot start while a slot is
// free lets later ones pass in at most max_bypass passes; after that it
// blocks the queue behind it.  A request that could not fit even in an
// empty budget is rejected.
#pragma once
#include <stdint.h>

#include <algorithm>
#include <deque>
#include <vector>

#include "bfc_heap.h"

namespace bfc {

struct AdmitScene {  // what admission knows of a registered scene
  int64_t fp = 0;      // bytes it holds while resident
  int64_t need = 0;    // bytes of one step (workspaces and buffers)
  int64_t off = -1;    // its resident block, -1: not resident
  bool busy = false;   // a request of it is on the device
  uint64_t last_use = 0;
};

struct AdmitSlot {
  bool busy = false;
  int64_t off = -1, bytes = 0;  // the step block of its request
};

// Dev:
//   bool create(int scene, int64_t off)  build the scene in its block at off, now or later (false: failed now;
//                                        a build that fails later is undone with abort_fresh)
//   void destroy(int scene)              tear down an idle resident scene
//   void start(Req* q, int slot)         run q on the slot (its step block is set)
//   void reject(Req* q, bool too_big)    complete q unserved (too_big: above the whole budget)
// Req: fields `scene` and `bypassed`.
template <class Req, class Dev>
struct Admission {
  Heap heap;
  std::vector<AdmitScene> sc;
  std::vector<AdmitSlot> slots;
  int max_bypass = 8;
  uint64_t clock = 0;
  int64_t created = 0, evicted = 0;
  int64_t limit = 0;  // scene blocks end at or below this offset

  // The scenes' limit: the budget less the largest step (at the scenes'
  // current capacities), but never below the largest scene; scenes that
  // cannot run within the budget at all do not count.  Call after a change
  // of sizes.
  void update_limit() {
    int64_t step = 0, fp = 0;
    for (const AdmitScene& a : sc) {
      if (Heap::round(a.fp) + Heap::round(a.need) > heap.size()) continue;
      step = std::max(step, Heap::round(a.need));
      fp = std::max(fp, Heap::round(a.fp));
    }
    limit = std::max(std::min(heap.size(), fp), heap.size() - step);
  }

  void evict(Dev& dev, int s) {
    dev.destroy(s);
    heap.release(sc[s].off, sc[s].fp);
    sc[s].off = -1;
    ++evicted;
  }

  // Room for a block of `bytes` below `end`: among the ranges of that length
  // that hold no step and no busy (or kept) scene, the one whose idle scenes
  // are the fewest bytes to build again (then the least recently used);
  // those scenes are evicted.  Ranges start at 0 or at an edge of a block: any
  // other range can slide left to one without covering more.  False if
  // every range holds a step or a busy scene.
  bool make_room(Dev& dev, int64_t bytes, int keep, int64_t end) {
    const int64_t n = Heap::round(bytes < 1 ? 1 : bytes);
    struct B {
      int64_t lo, hi;
      int scene;  // -1: fixed (a step, or a busy or kept scene)
    };
    std::vector<B> bl;
    for (int k = 0; k < (int)sc.size(); ++k)
      if (sc[k].off >= 0)
        bl.push_back({sc[k].off, sc[k].off + Heap::round(sc[k].fp), (sc[k].busy || k == keep) ? -1 : k});
    for (const AdmitSlot& sl : slots)
      if (sl.busy) bl.push_back({sl.off, sl.off + Heap::round(sl.bytes), -1});
    std::sort(bl.begin(), bl.end(), [](const B& a, const B& b) { return a.lo < b.lo; });
    std::vector<int64_t> starts{0};
    for (const B& b : bl) {
      starts.push_back(b.lo);
      starts.push_back(b.hi);
    }
    int64_t best_cost = -1, best_lo = -1;
    uint64_t best_age = 0;
    size_t first = 0;  // first block that ends after the range start (starts ascend)
    std::sort(starts.begin(), starts.end());
    for (int64_t lo : starts) {
      const int64_t hi = lo + n;
      if (hi > end) break;
      while (first < bl.size() && bl[first].hi <= lo) ++first;
      int64_t cost = 0;
      uint64_t age = 0;
      bool ok = true;
      for (size_t i = first; i < bl.size() && bl[i].lo < hi; ++i) {
        if (bl[i].scene < 0) { ok = false; break; }
        cost += bl[i].hi - bl[i].lo;
        age = std::max<uint64_t>(age, sc[bl[i].scene].last_use);
      }
      if (ok && (best_lo < 0 || cost < best_cost || (cost == best_cost && age < best_age))) {
        best_cost = cost;
        best_lo = lo;
        best_age = age;
      }
    }
    if (best_lo < 0) return false;
    for (const B& b : bl)
      if (b.scene >= 0 && b.lo < best_lo + n && b.hi > best_lo) evict(dev, b.scene);
    return true;
  }

  bool any_busy() const {
    for (const AdmitSlot& s : slots)
      if (s.busy) return true;
    return false;
  }

  // 1: started, 0: must wait, -1: rejected.
  int place(Dev& dev, Req* q, int slot) {
    const int s = q->scene;
    AdmitScene& a = sc[s];
    if (Heap::round(a.fp) + Heap::round(a.need) > heap.size()) {
      dev.reject(q, true);
      return -1;
    }
    bool fresh = a.off < 0;
    if (fresh) {
      a.off = heap.alloc(a.fp, true, limit);
      if (a.off < 0 && make_room(dev, a.fp, s, limit)) a.off = heap.alloc(a.fp, true, limit);
      if (a.off < 0) {
        if (any_busy()) return 0;  // steps and busy scenes are in the way: wait for them
        dev.reject(q, false);      // not reached: with nothing on the device the range below the limit is free
        return -1;
      }
    }
    int64_t step = heap.alloc(a.need, false);
    if (step < 0) {
      if (any_busy()) {  // wait for the steps on the device rather than evict
        if (fresh) {
          heap.release(a.off, a.fp);
          a.off = -1;
        }
        return 0;
      }
      // nothing runs, and the step is above the room kept for steps (its
      // scene's capacities grew): evict what is in the way, at worst every
      // idle scene and this scene's own block
      if (make_room(dev, a.need, s, heap.size())) step = heap.alloc(a.need, false);
      if (step < 0) {
        if (fresh) heap.release(a.off, a.fp);
        else evict(dev, s);
        a.off = -1;
        for (int k = 0; k < (int)sc.size(); ++k)
          if (sc[k].off >= 0) evict(dev, k);
        fresh = true;
        step = heap.alloc(a.need, false);
        a.off = step < 0 ? -1 : heap.alloc(a.fp, true);
        if (a.off < 0) {  // not reached: an empty budget holds both blocks
          if (step >= 0) heap.release(step, a.need);
          dev.reject(q, false);
          return -1;
        }
      }
    }
    if (fresh) {
      if (!dev.create(s, a.off)) {
        heap.release(step, a.need);
        heap.release(a.off, a.fp);
        a.off = -1;
        dev.reject(q, false);
        return -1;
      }
      ++created;
    }
    slots[slot].busy = true;
    slots[slot].off = step;
    slots[slot].bytes = a.need;
    a.busy = true;
    a.last_use = ++clock;
    dev.start(q, slot);
    return 1;
  }

  // One pass over the queue; requests that stay are kept in order.
  void pass(Dev& dev, std::deque<Req*>& queue) {
    std::deque<Req*> kept;
    bool blocked = false;
    while (!queue.empty()) {
      Req* q = queue.front();
      queue.pop_front();
      int free_slot = -1;
      for (int k = 0; k < (int)slots.size(); ++k)
        if (!slots[k].busy) { free_slot = k; break; }
      if (!blocked && free_slot >= 0 && !sc[q->scene].busy) {
        const int r = place(dev, q, free_slot);
        if (r != 0) continue;  // started or rejected
      }
      if (!blocked && free_slot >= 0) ++q->bypassed;
      blocked = blocked || q->bypassed > max_bypass;
      kept.push_back(q);
    }
    queue.swap(kept);
  }

  // The request on `slot` has completed: its step block is free, its scene idle.
  void done(int slot, int scene) {
    heap.release(slots[slot].off, slots[slot].bytes);
    slots[slot] = AdmitSlot{};
    sc[scene].busy = false;
  }

  // The scene of the request on `slot` was accepted for creation (create
  // returned true) but could not be built: both blocks are free again and
  // the scene is not resident.
  void abort_fresh(int slot, int scene) {
    done(slot, scene);
    heap.release(sc[scene].off, sc[scene].fp);
    sc[scene].off = -1;
    --created;
  }
};

}  // namespace bfc
