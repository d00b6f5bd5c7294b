// serve.hip -- served subtree solves with continuous batching: every request
// is one DEOCT run (Algorithm 4) on its own dataset (the problem of
// eq. opt_all), and all resident requests advance together, one generation
// per scheduling round.
//
// Device memory: one pool of hbm_budget bytes allocated at creation and
// carved by a host-side first-fit allocator; a request holds its tile
// layout, population, counters and result staging there from admission
// until its result has been packed.  Admission is FIFO: the head of the
// queue waits for a slot and for pool room.
//
// A round queues, on the context's stream:
//  - for each newly admitted request: rank encoding (asynchronous NaN check),
//    tile layout, initial population and its decode;
//  - per depth present: one fitness launch covering every resident request
//    of that depth (blocks split over the requests in proportion to their
//    tiles; each request keeps its own trees and counters), then one DE
//    launch with a block per request (epilogue, selection, best, next trial),
//    each request at its own generation;
//  - for each request past its last generation: decode and evaluate the best
//    individual and pack the result into pinned host memory, followed by an
//    event.
// Each request's draws are keyed by its own seed and problem id 0, so its
// result is the result of subtree_solve on the same data, whatever else is
// in flight.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <vector>

#include "de_body.h"
#include "internal.h"

namespace mh {
namespace {

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// First-fit allocator over [0, size) with coalescing of neighbouring free
// blocks.  Offsets and sizes are multiples of 256.
class Pool {
 public:
  void init(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
  }
  bool alloc(size_t bytes, size_t *off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes, o = it->first + bytes;
        free_.erase(it);
        if (rest) free_[o] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && off + bytes == nx->first) {
      bytes += nx->second;
      nx = free_.erase(nx);
    }
    if (nx != free_.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == off) {
        pv->second += bytes;
        return;
      }
    }
    free_[off] = bytes;
  }

 private:
  std::map<size_t, size_t> free_;
};

// Where a request's state sits inside its pool block.
struct Carve {
  size_t tiles, tile_bytes, nu, pop, trial, cost, tcost, feat, tau, best, cnt, f1, t1, lab1,
      corr1, cost1, nan, err, total;
  uint32_t max_tiles;
};

Carve carve(uint32_t n, uint32_t F, uint32_t K, uint32_t D, uint32_t P) {
  const uint32_t SB = (1u << D) - 1u, SL = 1u << D, m = 2 * SB;
  Carve c{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align256(bytes ? bytes : 1);
    return at;
  };
  const TileHdr h = tile_layout(n, F, K, 1);
  c.tile_bytes = h.total_bytes;
  c.max_tiles = h.max_tiles;
  c.tiles = take(h.total_bytes);
  c.nu = take((size_t)F * 4);
  c.pop = take((size_t)P * m * 8);
  c.trial = take((size_t)P * m * 8);
  c.cost = take((size_t)P * 8);
  c.tcost = take((size_t)P * 8);
  c.feat = take((size_t)P * SB);
  c.tau = take((size_t)P * SB * 4);
  c.best = take(4);
  c.cnt = take(cnt_bytes(1, D, K, P));
  c.f1 = take(SB);
  c.t1 = take((size_t)SB * 4);
  c.lab1 = take(SL);
  c.corr1 = take(4);
  c.cost1 = take(8);
  c.nan = take(4);
  c.err = take(4);
  c.total = o;
  return c;
}

struct Req {
  uint64_t id = 0;
  const float *X = nullptr;
  const uint8_t *y = nullptr;
  uint32_t n = 0, F = 0, K = 0, D = 0;
  mh_de_params prm{};
  uint64_t t_submit = 0, t_admit = 0;
  size_t off = 0;
  Carve cv{};
  uint8_t *base = nullptr;
  uint32_t g = 0;  // next generation index to queue (0..G; G + 1 = done)
  int slot = -1;
  bool solo = false;  // solved whole by one cooperative launch at admission
  bool cancelled = false;  // by mh_server_cancel or the time limit

  template <typename T>
  T *at(size_t o) const {
    return reinterpret_cast<T *>(base + o);
  }
  const uint32_t *ctot() const {
    const TileHdr h = tile_layout(n, F, K, 1);
    return reinterpret_cast<const uint32_t *>(base + cv.tiles + h.off_ctot);
  }
  DeDev de() const {
    return DeDev{prm.P, D, F, prm.G, prm.M, prm.CR, prm.seed, at<uint32_t>(cv.nu), true};
  }
};

constexpr int RING = 4;           // rounds whose descriptors may be in flight
constexpr uint32_t MAX_SLOTS = 256;

uint32_t waves_for(uint32_t P) {
  uint32_t w = pad64(P) / 64;
  return w > 4 ? 8 : (w > 2 ? 4 : w);
}

}  // namespace
}  // namespace mh

struct mh_server {
  mh_ctx *ctx = nullptr;
  mh::Ctx *c = nullptr;
  uint8_t *pool_base = nullptr;
  size_t pool_bytes = 0;
  mh::Pool pool;
  uint32_t max_slots = 0;
  std::vector<int> free_slots;
  mh::ResultOut *pinned = nullptr;
  std::vector<hipEvent_t> slot_ev;
  std::deque<mh::Req> queue;
  std::vector<mh::Req> active;    // generating
  std::vector<mh::Req> retiring;  // result packed, waiting for its event
  std::deque<mh_result> done;
  // per-round job descriptors: pinned staging ring and one device buffer
  uint8_t *ring[mh::RING] = {};
  hipEvent_t ring_ev[mh::RING] = {};
  bool ring_used[mh::RING] = {};
  size_t desc_bytes = 0;
  uint8_t *desc_dev = nullptr;
  uint64_t rounds = 0;
  mh_status sticky = MH_OK;
  // requests with at least this many tiles run whole as one cooperative
  // launch (0: never); MHDEOCT_SERVE_SOLO_TILES, default two per CU
  uint32_t solo_tiles = 0;
  // mh_server_set_limits: queued requests at most (0: no limit) and the
  // time from submission after which a request is cancelled (0: none)
  uint32_t max_queued = 0;
  uint64_t timeout_ns = 0;
};

namespace mh {
namespace {

size_t desc_capacity(uint32_t max_slots, uint32_t num_cu) {
  // per depth group: jobs and their block map, each 256-byte aligned
  const size_t max_blocks = (size_t)num_cu * 16 + max_slots;
  const size_t per = align256((size_t)max_slots * sizeof(FitJob)) +
                     align256((size_t)max_slots * sizeof(GenJob)) + align256(max_blocks * 2);
  return 5 * per;
}

mh_status admit(mh_server *s, Req &q) {
  Ctx *c = s->c;
  hipStream_t st = c->stream;
  const uint32_t ld = std::max(256u, (q.n + 255u) & ~255u);
  uint32_t *ranks = (uint32_t *)arena_get(c, "srv_ranks", (size_t)q.F * ld * 4);
  if (!ranks) return MH_ENOMEM;
  uint32_t *nu = q.at<uint32_t>(q.cv.nu);
  mh_status r = launch_rank_encode(c, q.X, q.n, q.F, ld, ranks, nu, q.at<uint32_t>(q.cv.nan));
  if (r) return r;
  mh_dataset ds{q.n, q.F, q.K, ld, ranks, q.y, nu};
  r = launch_tile_build(c, &ds, nullptr, nullptr, q.n, 1, q.base + q.cv.tiles, q.cv.tile_bytes);
  if (r) return r;
  MH_HIP(c, hipMemsetAsync(q.at<uint32_t>(q.cv.cnt), 0, cnt_bytes(1, q.D, q.K, q.prm.P), st));
  r = launch_de_init(c, q.prm.P, q.D, q.F, q.prm.seed, nullptr, 0, 1, nullptr, 0,
                     q.at<double>(q.cv.pop), true);
  if (r) return r;
  if (c->persist && s->solo_tiles && q.cv.max_tiles >= s->solo_tiles) {
    // a request that fills the device by itself: its whole run as one
    // cooperative launch (the plain form's kernel), finished at admission
    const PersistFinal fin{q.at<uint8_t>(q.cv.f1), q.at<uint32_t>(q.cv.t1),
                           q.at<uint8_t>(q.cv.lab1), q.at<uint32_t>(q.cv.corr1),
                           q.at<double>(q.cv.cost1)};
    bool used = false;
    r = launch_deoct_persist(c, q.base + q.cv.tiles, q.F, q.K, q.n, q.D, &q.prm, 0, nu,
                             q.at<double>(q.cv.pop), q.at<double>(q.cv.cost),
                             q.at<uint32_t>(q.cv.best), q.at<uint32_t>(q.cv.err), &fin, &used);
    if (r) return r;
    if (used) {
      q.solo = true;
      q.g = q.prm.G + 1;
      return MH_OK;
    }
  }
  return launch_decode(c, q.at<double>(q.cv.pop), q.prm.P, q.D, q.F, nu, q.at<uint8_t>(q.cv.feat),
                       q.at<uint32_t>(q.cv.tau), 1, nullptr, true);
}

// The best individual of a finished request: decode, evaluate (labels,
// correct, cost) and pack into the slot's pinned record.
mh_status retire(mh_server *s, Req &q) {
  Ctx *c = s->c;
  const uint32_t SB = (1u << q.D) - 1u, SL = 1u << q.D;
  uint32_t *nu = q.at<uint32_t>(q.cv.nu);
  if (q.solo) {
    // the cooperative launch wrote the best tree; its barrier flag goes along
    mh_status r = launch_pack_result(c, q.D, q.at<uint8_t>(q.cv.f1), q.at<uint32_t>(q.cv.t1),
                                     q.at<uint8_t>(q.cv.lab1), q.at<uint32_t>(q.cv.corr1),
                                     q.at<double>(q.cv.cost1), q.at<uint32_t>(q.cv.err),
                                     q.at<uint32_t>(q.cv.nan), s->pinned + q.slot);
    if (r) return r;
    MH_HIP(c, hipEventRecord(s->slot_ev[q.slot], c->stream));
    return MH_OK;
  }
  mh_status r = launch_decode(c, q.at<double>(q.cv.pop), q.prm.P, q.D, q.F, nu,
                              q.at<uint8_t>(q.cv.f1), q.at<uint32_t>(q.cv.t1), 1,
                              q.at<uint32_t>(q.cv.best), true);
  if (r) return r;
  FitnessOut fb;
  fb.label = q.at<uint8_t>(q.cv.lab1);
  fb.correct = q.at<uint32_t>(q.cv.corr1);
  fb.cost = q.at<double>(q.cv.cost1);
  r = launch_fitness_tiles(c, q.base + q.cv.tiles, q.F, q.K, q.n, 1, q.cv.max_tiles,
                           q.at<uint8_t>(q.cv.f1), q.at<uint32_t>(q.cv.t1), 1, q.D,
                           q.prm.n_min, q.prm.alpha, q.at<uint32_t>(q.cv.cnt), fb);
  if (r) return r;
  mh_status st = launch_pack_result(c, q.D, q.at<uint8_t>(q.cv.f1), q.at<uint32_t>(q.cv.t1),
                                    q.at<uint8_t>(q.cv.lab1), q.at<uint32_t>(q.cv.corr1),
                                    q.at<double>(q.cv.cost1), nullptr,
                                    q.at<uint32_t>(q.cv.nan), s->pinned + q.slot);
  if (st) return st;
  MH_HIP(c, hipEventRecord(s->slot_ev[q.slot], c->stream));
  return MH_OK;
}

// Moves requests whose packed result has landed to the done list.  With
// `wait`, blocks on the oldest one first.
mh_status collect(mh_server *s, bool wait) {
  Ctx *c = s->c;
  if (wait && !s->retiring.empty())
    MH_HIP(c, hipEventSynchronize(s->slot_ev[s->retiring.front().slot]));
  size_t kept = 0;
  for (size_t i = 0; i < s->retiring.size(); ++i) {
    Req &q = s->retiring[i];
    const hipError_t e = hipEventQuery(s->slot_ev[q.slot]);
    if (e == hipErrorNotReady) {
      if (kept != i) s->retiring[kept] = q;
      ++kept;
      continue;
    }
    if (e != hipSuccess) return hip_fail(c, e, "hipEventQuery");
    const ResultOut &o = s->pinned[q.slot];
    mh_result res;
    std::memset(&res, 0, sizeof(res));
    res.req_id = q.id;
    res.status = (o.flag & 2u) ? MH_EINVAL : o.flag ? MH_EDEVICE : MH_OK;
    if (q.cancelled) res.status = MH_ECANCELED;
    res.n = q.n;
    res.F = q.F;
    res.K = q.K;
    res.tree.D = q.D;
    const uint32_t SB = (1u << q.D) - 1u, SL = 1u << q.D;
    std::memcpy(res.tree.feat, o.tree.feat, SB);
    std::memcpy(res.tree.tau, o.tree.tau, (size_t)SB * 4);
    std::memcpy(res.tree.label, o.tree.label, SL);
    res.tree.correct = o.tree.correct;
    res.tree.cost = o.tree.cost;
    res.t_submit_ns = q.t_submit;
    res.t_admit_ns = q.t_admit;
    res.t_done_ns = now_ns();
    s->done.push_back(res);
    s->free_slots.push_back(q.slot);
  }
  s->retiring.resize(kept);
  return MH_OK;
}

// One generation of every active request: per depth, a fitness launch over
// all of them and a DE launch with a block per request.
mh_status generation(mh_server *s) {
  Ctx *c = s->c;
  hipStream_t st = c->stream;
  const int k = (int)(s->rounds % RING);
  if (s->ring_used[k]) MH_HIP(c, hipEventSynchronize(s->ring_ev[k]));
  uint8_t *host = s->ring[k];
  size_t used = 0;
  struct Launch {
    uint32_t D, waves, F_max, n_blocks, n_jobs, P_max;
    size_t fit, gen, map;
  };
  std::vector<Launch> launches;
  for (uint32_t D = 1; D <= 5; ++D) {
    std::vector<Req *> js;
    for (Req &q : s->active)
      if (q.D == D && q.g <= q.prm.G) js.push_back(&q);
    if (js.empty()) continue;
    Launch L{D, 0, 0, 0, (uint32_t)js.size(), 0, 0, 0, 0};
    uint64_t tiles = 0;
    for (Req *q : js) {
      L.P_max = std::max(L.P_max, q->prm.P);
      L.F_max = std::max(L.F_max, q->F);
      tiles += q->cv.max_tiles;
    }
    L.waves = waves_for(L.P_max);
    const uint32_t want =
        (uint32_t)c->num_cu * c->fit_blocks_per_cu * std::max(1u, 4u / L.waves);
    L.fit = used;
    used += align256((size_t)L.n_jobs * sizeof(FitJob));
    L.gen = used;
    used += align256((size_t)L.n_jobs * sizeof(GenJob));
    L.map = used;
    FitJob *fj = reinterpret_cast<FitJob *>(host + L.fit);
    GenJob *gj = reinterpret_cast<GenJob *>(host + L.gen);
    std::vector<uint16_t> job_of;
    for (uint32_t j = 0; j < L.n_jobs; ++j) {
      Req &q = *js[j];
      uint64_t nb = tiles ? (uint64_t)want * q.cv.max_tiles / tiles : 1;
      nb = std::max<uint64_t>(1, std::min<uint64_t>(nb, q.cv.max_tiles));
      FitJob f;
      f.hdr = reinterpret_cast<const TileHdr *>(q.base + q.cv.tiles);
      f.feat = q.at<uint8_t>(q.cv.feat);
      f.tau = q.at<uint32_t>(q.cv.tau);
      f.cnt = q.at<uint32_t>(q.cv.cnt);
      f.P = q.prm.P;
      f.blk0 = (uint32_t)job_of.size();
      f.nblk = (uint32_t)nb;
      f.pad = 0;
      fj[j] = f;
      job_of.insert(job_of.end(), (size_t)nb, (uint16_t)j);
      const uint32_t g = q.g;
      gj[j] = make_gen_job(q.de(), 0, g + 1, g == 0, q.at<double>(q.cv.pop),
                           q.at<double>(q.cv.cost), q.at<double>(q.cv.trial),
                           q.at<uint32_t>(q.cv.best), g < q.prm.G ? q.at<double>(q.cv.trial) : nullptr,
                           q.at<uint8_t>(q.cv.feat), q.at<uint32_t>(q.cv.tau),
                           q.at<uint32_t>(q.cv.cnt), q.ctot(), q.K, q.prm.n_min, q.prm.alpha,
                           L.P_max);
    }
    L.n_blocks = (uint32_t)job_of.size();
    if (used + align256((size_t)L.n_blocks * 2) > s->desc_bytes)
      return fail(c, MH_EINVAL, "server descriptor space exhausted");
    std::memcpy(host + L.map, job_of.data(), job_of.size() * 2);
    used += align256((size_t)L.n_blocks * 2);
    launches.push_back(L);
  }
  if (launches.empty()) return MH_OK;
  MH_HIP(c, hipMemcpyAsync(s->desc_dev, host, used, hipMemcpyHostToDevice, st));
  MH_HIP(c, hipEventRecord(s->ring_ev[k], st));
  s->ring_used[k] = true;
  s->rounds += 1;
  for (const Launch &L : launches) {
    mh_status r = launch_fitness_jobs(c, L.D, L.waves, L.F_max,
                                      reinterpret_cast<const FitJob *>(s->desc_dev + L.fit),
                                      reinterpret_cast<const uint16_t *>(s->desc_dev + L.map),
                                      L.n_blocks);
    if (r) return r;
    r = launch_de_jobs(c, L.D, reinterpret_cast<const GenJob *>(s->desc_dev + L.gen), L.n_jobs,
                       L.P_max);
    if (r) return r;
  }
  for (Req &q : s->active)
    if (q.g <= q.prm.G) q.g += 1;
  return MH_OK;
}

// The result record of a request that ends cancelled: no tree.
void push_cancelled(mh_server *s, const Req &q) {
  mh_result res;
  std::memset(&res, 0, sizeof(res));
  res.req_id = q.id;
  res.status = MH_ECANCELED;
  res.n = q.n;
  res.F = q.F;
  res.K = q.K;
  res.tree.D = q.D;
  res.t_submit_ns = q.t_submit;
  res.t_admit_ns = q.t_admit;
  res.t_done_ns = now_ns();
  s->done.push_back(res);
}

// Cancelled requests leave: queued ones at once; resident ones that are
// still stepped generation by generation give their slot and pool block
// back (work already queued on the stream that uses the block runs before
// any later use of it); a whole-request run, or a result already being
// packed, finishes on the device and is reported cancelled when it lands.
void drop_cancelled(mh_server *s) {
  if (s->timeout_ns) {
    const uint64_t t = now_ns();
    for (Req &q : s->queue)
      if (t - q.t_submit > s->timeout_ns) q.cancelled = true;
    for (Req &q : s->active)
      if (t - q.t_submit > s->timeout_ns) q.cancelled = true;
  }
  for (auto it = s->queue.begin(); it != s->queue.end();) {
    if (it->cancelled) {
      push_cancelled(s, *it);
      it = s->queue.erase(it);
    } else {
      ++it;
    }
  }
  size_t kept = 0;
  for (size_t i = 0; i < s->active.size(); ++i) {
    Req &q = s->active[i];
    if (q.cancelled && !q.solo) {
      s->pool.release(q.off, q.cv.total);
      s->free_slots.push_back(q.slot);
      push_cancelled(s, q);
      continue;
    }
    if (kept != i) s->active[kept] = q;
    ++kept;
  }
  s->active.resize(kept);
}

// Whether a queued request will run whole at admission.
bool c_solo(const mh_server *s, const Req &q) {
  return s->c->persist && s->solo_tiles && q.cv.max_tiles >= s->solo_tiles;
}

mh_status round_once(mh_server *s) {
  drop_cancelled(s);
  mh_status r = collect(s, s->active.empty() && s->queue.empty());
  if (r) return r;
  // admission, in submission order; at most one whole-request run per round,
  // so that the resident requests get a generation between two of them
  bool solo_run = false;
  while (!s->queue.empty() && !s->free_slots.empty()) {
    Req &q = s->queue.front();
    const bool solo = c_solo(s, q);
    if (solo && solo_run) break;
    solo_run = solo_run || solo;
    size_t off = 0;
    if (!s->pool.alloc(q.cv.total, &off)) break;
    q.off = off;
    q.base = s->pool_base + off;
    q.slot = s->free_slots.back();
    s->free_slots.pop_back();
    q.t_admit = now_ns();
    q.g = 0;
    r = admit(s, q);
    if (r) return r;
    s->active.push_back(q);
    s->queue.pop_front();
  }
  r = generation(s);
  if (r) return r;
  // requests past their last generation: pack the result, free the pool block
  // (later work on the stream may reuse it; the result copy is queued first)
  size_t kept = 0;
  for (size_t i = 0; i < s->active.size(); ++i) {
    Req &q = s->active[i];
    if (q.g <= q.prm.G) {
      if (kept != i) s->active[kept] = q;
      ++kept;
      continue;
    }
    r = retire(s, q);
    if (r) return r;
    s->pool.release(q.off, q.cv.total);
    s->retiring.push_back(q);
  }
  s->active.resize(kept);
  return MH_OK;
}

}  // namespace
}  // namespace mh

using namespace mh;

#define SRV_OR_FAIL(s)                                                      \
  do {                                                                      \
    if (!(s)) return fail(nullptr, MH_EINVAL, "server is null");            \
    if ((s)->sticky) return (s)->sticky;                                    \
    hipError_t e_ = hipSetDevice((s)->c->device);                           \
    if (e_ != hipSuccess) return hip_fail((s)->c, e_, "hipSetDevice");      \
  } while (0)

extern "C" {

mh_status mh_server_footprint(uint32_t n, uint32_t F, uint32_t K, uint32_t D, uint32_t P,
                              uint64_t *bytes) {
  if (!bytes || F == 0 || F > 80 || K == 0 || K > MH_MAX_CLASSES || D < 1 || D > 5 || P < 3 ||
      P > 512)
    return MH_EINVAL;
  *bytes = carve(n, F, K, D, P).total;
  return MH_OK;
}

mh_status mh_server_create(mh_ctx *ctx, uint64_t hbm_budget, uint32_t max_slots,
                           mh_server **out) {
  if (!ctx || !out) return fail(nullptr, MH_EINVAL, "null context or output");
  Ctx *c = &ctx->c;
  if (max_slots == 0 || max_slots > MAX_SLOTS)
    return fail(c, MH_EINVAL, "max_slots must be in 1..256");
  if (hbm_budget < 4096) return fail(c, MH_EINVAL, "hbm_budget too small");
  MH_HIP(c, hipSetDevice(c->device));
  mh_server *s = new mh_server();
  s->ctx = ctx;
  s->c = c;
  s->max_slots = max_slots;
  s->solo_tiles = 2u * (uint32_t)c->num_cu;
  if (const char *v = std::getenv("MHDEOCT_SERVE_SOLO_TILES")) s->solo_tiles = (uint32_t)std::max(0, atoi(v));
  s->pool_bytes = (size_t)hbm_budget & ~(size_t)255;
  s->desc_bytes = desc_capacity(max_slots, (uint32_t)c->num_cu);
  hipError_t e = hipMalloc((void **)&s->pool_base, s->pool_bytes);
  if (e == hipSuccess) e = hipMalloc((void **)&s->desc_dev, s->desc_bytes);
  if (e == hipSuccess) e = hipHostMalloc((void **)&s->pinned, sizeof(ResultOut) * max_slots);
  for (int k = 0; k < RING && e == hipSuccess; ++k) {
    e = hipHostMalloc((void **)&s->ring[k], s->desc_bytes);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ring_ev[k], hipEventDisableTiming);
  }
  s->slot_ev.assign(max_slots, nullptr);
  for (uint32_t i = 0; i < max_slots && e == hipSuccess; ++i)
    e = hipEventCreateWithFlags(&s->slot_ev[i], hipEventDisableTiming);
  if (e != hipSuccess) {
    mh_server_destroy(s);
    return hip_fail(c, e, "server allocation");
  }
  s->pool.init(s->pool_bytes);
  for (int i = (int)max_slots - 1; i >= 0; --i) s->free_slots.push_back(i);
  *out = s;
  return MH_OK;
}

void mh_server_destroy(mh_server *s) {
  if (!s) return;
  (void)hipSetDevice(s->c->device);
  (void)hipStreamSynchronize(s->c->stream);
  if (s->pool_base) (void)hipFree(s->pool_base);
  if (s->desc_dev) (void)hipFree(s->desc_dev);
  if (s->pinned) (void)hipHostFree(s->pinned);
  for (int k = 0; k < RING; ++k) {
    if (s->ring[k]) (void)hipHostFree(s->ring[k]);
    if (s->ring_ev[k]) (void)hipEventDestroy(s->ring_ev[k]);
  }
  for (hipEvent_t ev : s->slot_ev)
    if (ev) (void)hipEventDestroy(ev);
  delete s;
}

mh_status mh_server_submit(mh_server *s, uint64_t req_id, const float *X, const uint8_t *labels,
                           uint32_t n, uint32_t F, uint32_t K, uint32_t D,
                           const mh_de_params *prm) {
  SRV_OR_FAIL(s);
  Ctx *c = s->c;
  if (F == 0 || F > 80) return fail(c, MH_EINVAL, "served requests need 1 <= F <= 80");
  if (K == 0 || K > MH_MAX_CLASSES) return fail(c, MH_EINVAL, "K must be in 1..255");
  if (D < 1 || D > 5) return fail(c, MH_EINVAL, "served requests need depth 1..5");
  if (n > 0 && (!X || !labels)) return fail(c, MH_EINVAL, "null X or labels");
  if ((uint64_t)n * F >= 0xFFFFFFFFull) return fail(c, MH_EINVAL, "n * F too large");
  if (mh_status r = check_de(c, prm, D)) return r;
  if (prm->P > 512) return fail(c, MH_EINVAL, "served requests need P <= 512");
  Req q;
  q.id = req_id;
  q.X = X;
  q.y = labels;
  q.n = n;
  q.F = F;
  q.K = K;
  q.D = D;
  q.prm = *prm;
  q.cv = carve(n, F, K, D, prm->P);
  if (q.cv.total > s->pool_bytes)
    return fail(c, MH_ENOMEM, "request footprint exceeds the server's HBM budget");
  if (s->max_queued && s->queue.size() >= s->max_queued)
    return fail(c, MH_EBUSY, "the server's queue is full");
  q.t_submit = now_ns();
  s->queue.push_back(q);
  return MH_OK;
}

mh_status mh_server_set_limits(mh_server *s, uint32_t max_queued, uint64_t timeout_ns) {
  SRV_OR_FAIL(s);
  s->max_queued = max_queued;
  s->timeout_ns = timeout_ns;
  return MH_OK;
}

mh_status mh_server_cancel(mh_server *s, uint64_t req_id) {
  SRV_OR_FAIL(s);
  for (Req &q : s->queue)
    if (q.id == req_id && !q.cancelled) {
      q.cancelled = true;
      return MH_OK;
    }
  for (Req &q : s->active)
    if (q.id == req_id && !q.cancelled) {
      q.cancelled = true;
      return MH_OK;
    }
  for (Req &q : s->retiring)
    if (q.id == req_id && !q.cancelled) {
      q.cancelled = true;
      return MH_OK;
    }
  return fail(s->c, MH_EINVAL, "no queued or running request has this id");
}

mh_status mh_server_pump(mh_server *s, uint32_t ticks, uint32_t *n_active, uint32_t *n_queued) {
  SRV_OR_FAIL(s);
  for (uint32_t t = 0; t < ticks; ++t) {
    if (s->active.empty() && s->queue.empty() && s->retiring.empty()) break;
    mh_status r = round_once(s);
    if (r) {
      s->sticky = r;
      return r;
    }
  }
  drop_cancelled(s);
  if (mh_status r = collect(s, false)) {
    s->sticky = r;
    return r;
  }
  if (n_active) *n_active = (uint32_t)(s->active.size() + s->retiring.size());
  if (n_queued) *n_queued = (uint32_t)s->queue.size();
  return MH_OK;
}

mh_status mh_server_poll(mh_server *s, mh_result *out, uint32_t max, uint32_t *n_done) {
  SRV_OR_FAIL(s);
  if (!n_done || (max && !out)) return fail(s->c, MH_EINVAL, "null output");
  if (mh_status r = collect(s, false)) {
    s->sticky = r;
    return r;
  }
  uint32_t k = 0;
  while (k < max && !s->done.empty()) {
    out[k++] = s->done.front();
    s->done.pop_front();
  }
  *n_done = k;
  return MH_OK;
}

}  // extern "C"
