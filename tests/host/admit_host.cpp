// Host build of the serving loop's heap and admission policy (bfc_heap.h,
// bfc_admit.h) against a fake device: random arrivals and completions on a
// virtual clock, every block checked against every other live block.
// Usage: admit_host <seed> <mode>; mode 0: heap against a byte map, mode 1:
// admission.  Prints one line of counts; exit 1 with a message on a failed
// check.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <set>
#include <vector>

#include "bfc_admit.h"

#define CHECK(c, ...)                                                     \
  do {                                                                    \
    if (!(c)) {                                                           \
      std::fprintf(stderr, "check failed at line %d: %s: ", __LINE__, #c); \
      std::fprintf(stderr, __VA_ARGS__);                                  \
      std::fprintf(stderr, "\n");                                         \
      std::exit(1);                                                       \
    }                                                                     \
  } while (0)

// Heap against a map of 256-byte units: a block never overlaps another or
// leaves the heap, alloc fails only when no run of free units is long
// enough, and low / high placement take the lowest / highest fitting run.
static void heap_test(unsigned seed) {
  std::mt19937_64 rng(seed);
  const int units = 512;
  bfc::Heap h((int64_t)units * 256);
  std::vector<int> owner(units, -1);
  std::map<int, std::pair<int64_t, int64_t>> live;  // id -> (off, bytes)
  int next = 0, fails = 0, allocs = 0;
  for (int it = 0; it < 20000; ++it) {
    if (live.empty() || rng() % 100 < 55) {
      const int64_t bytes = 1 + (int64_t)(rng() % (40 * 256));
      const bool low = rng() % 2;
      const int n = (int)((bytes + 255) / 256);
      const int lim = rng() % 3 ? units : (int)(rng() % (units + 1));  // low blocks end at or below
      // expected: the first (low, ending within the limit) or last (high)
      // maximal free run of length >= n
      int want = -1;
      for (int u = 0; u < units;) {
        if (owner[u] >= 0) { ++u; continue; }
        int e = u;
        while (e < units && owner[e] < 0) ++e;
        if (e - u >= n) {
          if (low) { if (want < 0 && u + n <= lim) want = u; }
          else want = e - n;
        }
        u = e;
      }
      const int64_t off = h.alloc(bytes, low, low ? (int64_t)lim * 256 : -1);
      if (want < 0) {
        CHECK(off == -1, "alloc of %lld units should fail", (long long)n);
        ++fails;
        continue;
      }
      CHECK(off == (int64_t)want * 256, "alloc at %lld, expected unit %d", (long long)off, want);
      for (int u = want; u < want + n; ++u) owner[u] = next;
      live[next++] = {off, bytes};
      ++allocs;
    } else {
      auto itl = live.begin();
      std::advance(itl, rng() % live.size());
      const int u0 = (int)(itl->second.first / 256), n = (int)((itl->second.second + 255) / 256);
      for (int u = u0; u < u0 + n; ++u) {
        CHECK(owner[u] == itl->first, "unit %d owned by %d", u, owner[u]);
        owner[u] = -1;
      }
      h.release(itl->second.first, itl->second.second);
      live.erase(itl);
    }
    int used = 0, runs = 0;
    for (int u = 0; u < units; ++u) {
      used += owner[u] >= 0;
      runs += owner[u] < 0 && (u == 0 || owner[u - 1] >= 0);
    }
    CHECK(h.used() == (int64_t)used * 256, "used %lld, map %d units", (long long)h.used(), used);
    CHECK(h.ranges() == runs, "free ranges %d, map %d (merging)", h.ranges(), runs);
  }
  std::printf("heap ok allocs=%d fails=%d\n", allocs, fails);
}

struct Req {
  int scene = 0;
  int bypassed = 0;
  int id = 0;
};

struct Fake;
using Adm = bfc::Admission<Req, Fake>;

struct Fake {
  Adm* adm = nullptr;
  std::mt19937_64* rng = nullptr;
  std::map<int64_t, int64_t> blocks;  // live device blocks: off -> end
  std::vector<int> running;           // request id per slot, -1 free
  std::vector<Req*> on_slot;
  int rejected = 0, too_big = 0, started = 0, create_fail = 0;
  int failed_scene = -1;    // the scene whose creation just failed
  std::set<int> fail_later;  // scenes whose accepted creation will fail
  std::set<int> waiting;    // ids of queued requests
  std::vector<int> passed;  // per request: later requests started while it waited

  void add(int64_t off, int64_t bytes) {
    const int64_t end = off + bfc::Heap::round(bytes);
    CHECK(off >= 0 && end <= adm->heap.size(), "block [%lld,%lld) outside the heap", (long long)off, (long long)end);
    auto it = blocks.lower_bound(off);
    CHECK(it == blocks.end() || it->first >= end, "block at %lld overlaps the next", (long long)off);
    CHECK(it == blocks.begin() || std::prev(it)->second <= off, "block at %lld overlaps the previous", (long long)off);
    blocks[off] = end;
  }
  void remove(int64_t off) {
    CHECK(blocks.erase(off) == 1, "no block at %lld", (long long)off);
  }
  bool create(int s, int64_t off) {
    CHECK(!adm->sc[s].busy, "creating a busy scene %d", s);
    if ((*rng)() % 50 == 0) {  // a failed creation leaves nothing behind
      ++create_fail;
      failed_scene = s;
      return false;
    }
    add(off, adm->sc[s].fp);
    if ((*rng)() % 50 == 0) fail_later.insert(s);  // accepted, fails before its request runs
    return true;
  }
  void destroy(int s) {
    CHECK(!adm->sc[s].busy, "evicting busy scene %d", s);
    remove(adm->sc[s].off);
  }
  void start(Req* q, int slot) {
    CHECK(running[slot] < 0, "slot %d taken", slot);
    CHECK(adm->sc[q->scene].off >= 0, "scene %d not resident", q->scene);
    add(adm->slots[slot].off, adm->slots[slot].bytes);
    running[slot] = q->id;
    on_slot[slot] = q;
    ++started;
    waiting.erase(q->id);
    for (int w : waiting) {
      if (w > q->id) break;
      ++passed[w];
    }
  }
  void reject(Req* q, bool big) {
    const bfc::AdmitScene& a = adm->sc[q->scene];
    const bool above = bfc::Heap::round(a.fp) + bfc::Heap::round(a.need) > adm->heap.size();
    CHECK(big == above, "rejected scene %d: too_big %d, above %d", q->scene, (int)big, (int)above);
    CHECK(big || failed_scene == q->scene, "scene %d rejected though it fits and its creation did not fail",
          q->scene);
    failed_scene = -1;
    ++rejected;
    too_big += big;
    waiting.erase(q->id);
    delete q;
  }
};

static void admission_test(unsigned seed) {
  std::mt19937_64 rng(seed);
  const int n_scenes = 40 + (int)(rng() % 40), n_slots = 1 + (int)(rng() % 6), max_bypass = (int)(rng() % 6);
  Adm adm;
  adm.max_bypass = max_bypass;
  adm.sc.resize(n_scenes);
  adm.slots.resize(n_slots);
  std::lognormal_distribution<double> ln(std::log(60e3), 1.0);
  double total = 0.0;
  for (auto& a : adm.sc) {
    a.fp = 1 + (int64_t)ln(rng);
    a.need = 1 + (int64_t)(3.0 * ln(rng));
    total += (double)a.fp;
  }
  // a budget well below the scenes' total, so that eviction binds
  const int64_t size = std::max<int64_t>(2 << 20, (int64_t)((0.2 + 0.2 * (double)(rng() % 1000) / 1000.0) * total));
  adm.heap.reset(size);
  adm.sc[0].fp = size;  // one scene that can never fit
  adm.update_limit();
  Fake dev;
  dev.adm = &adm;
  dev.rng = &rng;
  dev.running.assign(n_slots, -1);
  dev.on_slot.assign(n_slots, nullptr);
  std::deque<Req*> queue;
  int next_id = 0, completed = 0;
  const int n_req = 4000;
  dev.passed.assign(n_req, 0);
  for (int t = 0; next_id < n_req || !queue.empty() || adm.any_busy(); ++t) {
    CHECK(t < 10 * n_req, "no progress: %zu queued", queue.size());
    // arrivals
    const int arrive = next_id < n_req ? (int)(rng() % 4) : 0;
    for (int a = 0; a < arrive && next_id < n_req; ++a) {
      Req* q = new Req;
      q->scene = (int)(rng() % n_scenes);
      q->id = next_id++;
      dev.waiting.insert(q->id);
      queue.push_back(q);
    }
    // creations that fail after they were accepted: the request never ran
    for (int k = 0; k < n_slots; ++k) {
      if (dev.running[k] < 0 || !dev.fail_later.count(dev.on_slot[k]->scene)) continue;
      Req* q = dev.on_slot[k];
      dev.fail_later.erase(q->scene);
      dev.remove(adm.slots[k].off);
      dev.remove(adm.sc[q->scene].off);
      adm.abort_fresh(k, q->scene);
      CHECK(adm.sc[q->scene].off < 0 && !adm.sc[q->scene].busy, "scene %d left resident", q->scene);
      dev.running[k] = -1;
      dev.on_slot[k] = nullptr;
      ++dev.rejected;
      delete q;
    }
    // completions
    for (int k = 0; k < n_slots; ++k) {
      if (dev.running[k] < 0 || rng() % 3) continue;
      Req* q = dev.on_slot[k];
      dev.remove(adm.slots[k].off);
      adm.done(k, q->scene);
      dev.running[k] = -1;
      dev.on_slot[k] = nullptr;
      ++completed;
      if (rng() % 20 == 0 && !adm.sc[q->scene].busy) {  // capacities grown
        adm.sc[q->scene].need += 1 + (int64_t)(rng() % 200000);
        adm.update_limit();
      }
      delete q;
    }
    adm.pass(dev, queue);
    // invariants
    int64_t held = 0;
    for (auto& kv : dev.blocks) held += kv.second - kv.first;
    CHECK(held == adm.heap.used(), "blocks hold %lld, heap says %lld", (long long)held, (long long)adm.heap.used());
    CHECK(adm.heap.used() <= size, "over budget");
    std::set<int> busy;
    for (int k = 0; k < n_slots; ++k)
      if (dev.running[k] >= 0) CHECK(busy.insert(dev.on_slot[k]->scene).second, "two requests of one scene");
  }
  CHECK(completed + dev.rejected == n_req, "completed %d + rejected %d != %d", completed, dev.rejected, n_req);
  // a request that cannot start is passed over in at most max_bypass + 1
  // admission passes (then it blocks the queue), each starting at most one
  // later request per slot
  int most = 0;
  for (int p : dev.passed) most = p > most ? p : most;
  CHECK(most <= (max_bypass + 1) * n_slots, "passed by %d later requests (bound %d)", most,
        (max_bypass + 1) * n_slots);
  std::printf("admission ok scenes=%d slots=%d started=%d rejected=%d too_big=%d created=%lld evicted=%lld "
              "create_fail=%d peak=%lld size=%lld most_passed=%d limit=%lld\n",
              n_scenes, n_slots, dev.started, dev.rejected, dev.too_big, (long long)adm.created,
              (long long)adm.evicted, dev.create_fail, (long long)adm.heap.peak(), (long long)size, most, (long long)adm.limit);
}

int main(int argc, char** argv) {
  if (argc != 3) return 2;
  const unsigned seed = (unsigned)std::atoi(argv[1]);
  if (std::atoi(argv[2]) == 0) heap_test(seed);
  else admission_test(seed);
  return 0;
}
