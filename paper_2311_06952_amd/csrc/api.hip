// api.hip -- the C ABI (include/mhdeoct.h): context, arena, argument checks
// and the host-side orchestration of the device kernels.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "de_body.h"
#include "device_common.h"
#include "internal.h"


namespace mh {

static thread_local std::string g_create_err;

// Device scratch of fitness_eval_static, the entry point that allocates
// nothing: the tile layout and counters of one call.  Each GPU the library
// runs on holds its own copy from the library's load until the process ends.
// In host code the array's name is not a device address: its per-device
// address comes from hipGetSymbolAddress, looked up once per device when the
// first context on that device is created, and only that address is used.
constexpr size_t STATIC_SCRATCH_BYTES = size_t(64) << 20;
static __device__ __align__(256) uint8_t scratch[STATIC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static std::map<int, uint8_t *> g_scratch_addr;

// The current device's copy of `scratch` (the device must be current).
static hipError_t static_scratch_of(int device, uint8_t **out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(device);
  if (it == g_scratch_addr.end()) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
      *out = nullptr;
      return e;
    }
    it = g_scratch_addr.emplace(device, static_cast<uint8_t *>(p)).first;
  }
  *out = it->second;
  return hipSuccess;
}

mh_status fail(Ctx *ctx, mh_status code, const std::string &msg) {
  if (ctx) ctx->err = msg;
  else g_create_err = msg;
  return code;
}

mh_status hip_fail(Ctx *ctx, hipError_t e, const char *what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return fail(ctx, e == hipErrorOutOfMemory ? MH_ENOMEM : MH_EDEVICE, m);
}

uint32_t tiles_bucket(uint32_t max_tiles, uint32_t num_cu) {
  uint32_t per_cu = num_cu ? max_tiles / num_cu : max_tiles, b = 0;
  while (per_cu) {
    ++b;
    per_cu >>= 1;
  }
  return b;
}

constexpr size_t PROF_MAX_PAIRS = 4096;

int occupancy(Ctx *ctx, const void *kern, int threads, size_t lds) {
  for (const Ctx::Occ &o : ctx->occ)
    if (o.kern == kern && o.threads == threads && o.lds == lds) return o.per_cu;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, lds) != hipSuccess) {
    (void)hipGetLastError();
    per_cu = 0;
  }
  if (ctx->occ.size() < 256) ctx->occ.push_back({kern, threads, lds, per_cu});
  return per_cu;
}

int coop_per_cu(Ctx *ctx, const void *kern, int threads, size_t lds) {
  int r = occupancy(ctx, kern, threads, lds);
  if (lds > 0) r = (int)std::min<size_t>((size_t)r, ((size_t)ctx->max_lds - 2048) / lds);
  if (r >= 3) r -= 1;
  return std::min(r, 4);
}

hipError_t launch_grid_sync(Ctx *ctx, const void *kern, dim3 grid, dim3 block, void **args,
                            size_t lds) {
  return hipLaunchKernel(kern, grid, block, args, lds, ctx->stream);
}

bool coop_is_bad(const Ctx *ctx, const void *kern, uint32_t grid) {
  for (const auto &p : ctx->coop_bad)
    if (p.first == kern && p.second == grid) return true;
  return false;
}

void coop_note_failure(Ctx *ctx) {
  if (ctx->last_coop_kern && !coop_is_bad(ctx, ctx->last_coop_kern, ctx->last_coop_grid))
    ctx->coop_bad.push_back({ctx->last_coop_kern, ctx->last_coop_grid});
}

mh_status wait_stream(Ctx *ctx) {
  if (!ctx->done_ev) MH_HIP(ctx, hipEventCreateWithFlags(&ctx->done_ev, hipEventDisableTiming));
  MH_HIP(ctx, hipEventRecord(ctx->done_ev, ctx->stream));
  const auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    const hipError_t e = hipEventQuery(ctx->done_ev);
    if (e == hipSuccess) return MH_OK;
    if (e != hipErrorNotReady) return hip_fail(ctx, e, "hipEventQuery");
    if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(50)) break;
  }
  MH_HIP(ctx, hipEventSynchronize(ctx->done_ev));
  return MH_OK;
}

uint32_t *host_words(Ctx *ctx) {
  if (!ctx->hwords) {
    const hipError_t e = hipHostMalloc((void **)&ctx->hwords, 64 * sizeof(uint32_t));
    if (e != hipSuccess) {
      ctx->hwords = nullptr;
      hip_fail(ctx, e, "hipHostMalloc");
      return nullptr;
    }
  }
  return ctx->hwords;
}

mh_status prof_collect(Ctx *ctx) {
  MH_HIP(ctx, hipStreamSynchronize(ctx->stream));
  for (size_t i = 0; i + 1 < ctx->prof_used; i += 2) {
    float ms = 0.f;
    MH_HIP(ctx, hipEventElapsedTime(&ms, ctx->prof_ev[i], ctx->prof_ev[i + 1]));
    ctx->prof_ms += ms;
  }
  ctx->prof_used = 0;
  return MH_OK;
}

bool prof_pair(Ctx *ctx, hipEvent_t *e0, hipEvent_t *e1) {
  *e0 = *e1 = nullptr;
  if (!ctx->profile) return false;
  if (ctx->prof_used + 2 > ctx->prof_ev.size()) {
    if (ctx->prof_ev.size() >= 2 * PROF_MAX_PAIRS) {
      if (prof_collect(ctx) != MH_OK) return false;
    } else {
      hipEvent_t a = nullptr, b = nullptr;
      if (hipEventCreate(&a) != hipSuccess) return false;
      if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return false;
      }
      ctx->prof_ev.push_back(a);
      ctx->prof_ev.push_back(b);
    }
  }
  *e0 = ctx->prof_ev[ctx->prof_used];
  *e1 = ctx->prof_ev[ctx->prof_used + 1];
  ctx->prof_used += 2;
  return true;
}

void *arena_get(Ctx *ctx, const char *name, size_t bytes) {
  if (bytes == 0) bytes = 256;
  bytes = align256(bytes);
  for (auto &b : ctx->arena.bufs) {
    if (b.name == name) {
      if (b.bytes >= bytes) return b.ptr;
      // the stream may still use the old buffer
      if (hipStreamSynchronize(ctx->stream) != hipSuccess) return nullptr;
      (void)hipFree(b.ptr);
      b.ptr = nullptr;
      b.bytes = 0;
      if (hipMalloc(&b.ptr, bytes) != hipSuccess) {
        ctx->err = std::string("device allocation failed for ") + name;
        b.ptr = nullptr;
        return nullptr;
      }
      b.bytes = bytes;
      return b.ptr;
    }
  }
  Arena::Buf nb;
  nb.name = name;
  if (hipMalloc(&nb.ptr, bytes) != hipSuccess) {
    ctx->err = std::string("device allocation failed for ") + name;
    return nullptr;
  }
  nb.bytes = bytes;
  ctx->arena.bufs.push_back(nb);
  return nb.ptr;
}

// Tile path limits: depth templates 1..5, one LDS tile <= 64 KiB, ranks and
// thresholds below 2^31 (the search step's sign test).
static bool tile_path_ok(uint32_t D, uint32_t F, uint32_t n) {
  return D >= 1 && D <= 5 && F <= 80 && n < (1u << 31);
}
// Fewer trees than this leave most lanes of the tile kernel idle (lane =
// tree) while it still stages every tile: the walk kernel (lane = sample)
// evaluates them instead.
constexpr uint32_t TILE_MIN_TREES = 4;

static mh_status check_dataset(Ctx *ctx, const mh_dataset *ds) {
  if (!ds) return fail(ctx, MH_EINVAL, "dataset is null");
  if (ds->F == 0 || ds->F > MH_MAX_FEATURES) return fail(ctx, MH_EINVAL, "F must be in 1..255");
  if (ds->K == 0 || ds->K > MH_MAX_CLASSES) return fail(ctx, MH_EINVAL, "K must be in 1..255");
  if (ds->ld < ds->n) return fail(ctx, MH_EINVAL, "ld must be >= n");
  if (ds->n > 0 && (!ds->ranks || !ds->labels)) return fail(ctx, MH_EINVAL, "null ranks or labels");
  if (!ds->n_unique) return fail(ctx, MH_EINVAL, "null n_unique");
  return MH_OK;
}

// Reads the dataset's status word, if it has one (synchronises).
static mh_status check_ds_status(Ctx *ctx, const mh_dataset *ds) {
  if (!ds->status) return MH_OK;
  uint32_t *h = host_words(ctx);
  if (!h) return MH_ENOMEM;
  MH_HIP(ctx, hipMemcpyAsync(h, ds->status, 4, hipMemcpyDeviceToHost, ctx->stream));
  MH_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (h[0] & 1u) return fail(ctx, MH_EINVAL, "X holds a NaN");
  if (h[0]) return fail(ctx, MH_EDEVICE, "rank encoding failed on the device");
  return MH_OK;
}

mh_status check_de(Ctx *ctx, const mh_de_params *p, uint32_t D) {
  if (!p) return fail(ctx, MH_EINVAL, "DE params are null");
  if (p->P < 3 || p->P > MH_MAX_POP) return fail(ctx, MH_EINVAL, "P must be in 3..1024");
  if (D < 1 || D > MH_MAX_DEPTH) return fail(ctx, MH_EINVAL, "D must be in 1..10");
  if (p->G >= (1u << 24)) return fail(ctx, MH_EINVAL, "G must be < 2^24");
  if (!(p->CR >= 0.0 && p->CR <= 1.0)) return fail(ctx, MH_EINVAL, "CR must be in [0, 1]");
  if (!(p->alpha >= 0.0)) return fail(ctx, MH_EINVAL, "alpha must be >= 0");
  if (p->M != p->M) return fail(ctx, MH_EINVAL, "M is NaN");
  if (p->n_min < 1) return fail(ctx, MH_EINVAL, "n_min must be >= 1");
  if ((1u << D) * 2u + 4u >= (1u << 20)) return fail(ctx, MH_EINVAL, "too many genes");
  return MH_OK;
}

// Evaluate P trees (feat/tau, device) over a subset: tile path when a tile
// set is given, else the walk path.
struct EvalSet {
  const mh_dataset *ds;
  const uint32_t *idx;
  uint32_t n_sub;
  const void *tiles;  // nullptr: walk path
  uint32_t max_tiles;
  uint32_t *cnt;
  uint32_t *leafcnt;  // walk path: caller scratch for the leaf counts (null: the arena's)
};

static mh_status eval_trees(Ctx *ctx, const EvalSet &es, const uint8_t *feat, const uint32_t *tau,
                            uint32_t P, uint32_t D, uint32_t n_min, double alpha,
                            const FitnessOut &out) {
  if (es.tiles && P >= TILE_MIN_TREES)
    return launch_fitness_tiles(ctx, es.tiles, es.ds->F, es.ds->K, es.n_sub, 1, es.max_tiles, feat,
                                tau, P, D, n_min, alpha, es.cnt, out);
  return launch_fitness_walk(ctx, es.ds, es.idx, es.n_sub, feat, tau, P, D, n_min, alpha, out,
                             es.leafcnt);
}

// Device bytes of the tile layout and counters (tile path) or the leaf
// counts (walk path) that one fitness evaluation of P depth-D trees over
// n_sub samples of ds uses, each part 256-byte aligned.
static size_t eval_scratch_bytes(const mh_dataset *ds, uint32_t n_sub, uint32_t D, uint32_t P) {
  if (tile_path_ok(D, ds->F, ds->n) && P >= TILE_MIN_TREES)
    return align256(tile_layout(n_sub, ds->F, ds->K, 1).total_bytes) +
           align256(cnt_bytes(1, D, ds->K, P));
  return align256(walk_scratch_bytes(P, D, ds->K));
}

// static_base: caller-provided scratch of eval_scratch_bytes (null: the
// context arena's buffers tile_name and cnt_name).  min_trees: the tile
// layout is built only for at least this many trees (DEOCT builds it for its
// population whatever the size: its kernels all read it).
static mh_status prepare_eval(Ctx *ctx, const mh_dataset *ds, const uint32_t *idx, uint32_t n_sub,
                              uint32_t D, uint32_t P, const char *tile_name, const char *cnt_name,
                              EvalSet &es, uint8_t *static_base = nullptr,
                              uint32_t min_trees = 0) {
  es.ds = ds;
  es.idx = idx;
  es.n_sub = n_sub;
  es.tiles = nullptr;
  es.cnt = nullptr;
  es.max_tiles = 0;
  const bool use_tiles = tile_path_ok(D, ds->F, ds->n) && P >= min_trees;
  es.leafcnt = use_tiles ? nullptr : reinterpret_cast<uint32_t *>(static_base);
  if (!use_tiles) return MH_OK;
  TileHdr h = tile_layout(n_sub, ds->F, ds->K, 1);
  void *tiles = static_base ? static_base : arena_get(ctx, tile_name, h.total_bytes);
  uint32_t *cnt = static_base
                      ? reinterpret_cast<uint32_t *>(static_base + align256(h.total_bytes))
                      : (uint32_t *)arena_get(ctx, cnt_name, cnt_bytes(1, D, ds->K, P));
  if (!tiles || !cnt) return MH_ENOMEM;
  mh_status s = launch_tile_build(ctx, ds, idx, nullptr, n_sub, 1, tiles, h.total_bytes);
  if (s) return s;
  es.tiles = tiles;
  es.cnt = cnt;
  es.max_tiles = h.max_tiles;
  return MH_OK;
}

// DEOCT (Algorithm 4) fully on the device; the best tree goes to *out.
static mh_status deoct(Ctx *ctx, const mh_dataset *ds, const uint32_t *idx, uint32_t n_sub,
                       uint32_t D, const mh_de_params *prm, const double *warm_host, uint32_t W,
                       uint64_t prob, mh_tree *out, int depth = 0) {
  const uint32_t P = prm->P, SB = (1u << D) - 1u, SL = 1u << D, m = 2 * SB, K = ds->K;
  hipStream_t st = ctx->stream;
  EvalSet es;
  mh_status s = prepare_eval(ctx, ds, idx, n_sub, D, P, "ss_tiles", "ss_cnt", es);
  if (s) return s;
  double *pop = (double *)arena_get(ctx, "ss_pop", (size_t)P * m * 8);
  double *trial = (double *)arena_get(ctx, "ss_trial", (size_t)P * m * 8);
  double *cost = (double *)arena_get(ctx, "ss_cost", (size_t)P * 8);
  double *tcost = (double *)arena_get(ctx, "ss_tcost", (size_t)P * 8);
  uint8_t *feat = (uint8_t *)arena_get(ctx, "ss_feat", (size_t)P * SB);
  uint32_t *tau = (uint32_t *)arena_get(ctx, "ss_tau", (size_t)P * SB * 4);
  uint32_t *best = (uint32_t *)arena_get(ctx, "ss_best", 256);
  uint8_t *f1 = (uint8_t *)arena_get(ctx, "ss_f1", SB);
  uint32_t *t1 = (uint32_t *)arena_get(ctx, "ss_t1", (size_t)SB * 4);
  uint8_t *lab1 = (uint8_t *)arena_get(ctx, "ss_lab1", SL);
  uint32_t *corr1 = (uint32_t *)arena_get(ctx, "ss_corr1", 256);
  double *cost1 = (double *)arena_get(ctx, "ss_cost1", 256);
  double *warm = nullptr;
  if (W > 0) {
    warm = (double *)arena_get(ctx, "ss_warm", (size_t)W * m * 8);
    if (!warm) return MH_ENOMEM;
    // host genes from the C ABI; device genes from the moving horizon
    MH_HIP(ctx, hipMemcpyAsync(warm, warm_host, (size_t)W * m * 8, hipMemcpyDefault, st));
  }
  if (!pop || !trial || !cost || !tcost || !feat || !tau || !best || !f1 || !t1 || !lab1 ||
      !corr1 || !cost1)
    return MH_ENOMEM;
  DeDev de{P, D, ds->F, prm->G, prm->M, prm->CR, prm->seed, ds->n_unique, true};
  uint32_t *err = (uint32_t *)arena_get(ctx, "ss_err", 256);
  if (!err) return MH_ENOMEM;
  // g = 0: initialise, decode, evaluate
  s = launch_de_init(ctx, P, D, ds->F, prm->seed, nullptr, prob, 1, warm, W, pop, true);
  if (s) return s;
  bool persisted = false;
  if (es.tiles && ctx->persist) {
    const PersistFinal fin{f1, t1, lab1, corr1, cost1};
    s = launch_deoct_persist(ctx, es.tiles, ds->F, K, n_sub, D, prm, prob, ds->n_unique, pop, cost,
                             best, err, &fin, &persisted);
    if (s) return s;
  }
  if (!persisted) {
    // (the cooperative launch clears its own flag and counters)
    s = launch_zero(ctx, {{es.cnt, es.cnt ? cnt_bytes(1, D, K, P) : 0}, {err, 4}});
    if (s) return s;
    s = launch_decode(ctx, pop, P, D, ds->F, ds->n_unique, feat, tau, 1, nullptr, true);
    if (s) return s;
  }
  if (persisted) {
    // the whole run happened in the cooperative launch
  } else if (es.tiles) {
    // tile path: per generation the counting kernel, then the epilogue fused
    // with selection, best and the next trial
    const TileHdr h = tile_layout(n_sub, ds->F, K, 1);
    const uint32_t *ctot =
        reinterpret_cast<const uint32_t *>(reinterpret_cast<const uint8_t *>(es.tiles) + h.off_ctot);
    // (a problem without samples has no block to finish it: separate step)
    const bool fuse = ctx->fuse_de && fusable(P, D, ds->F) && n_sub > 0;
    uint32_t *done = (uint32_t *)arena_get(ctx, "ss_done", 256);
    if (!done) return MH_ENOMEM;
    MH_HIP(ctx, hipMemsetAsync(done, 0, 4, st));
    const uint32_t *segoff =
        reinterpret_cast<const uint32_t *>(reinterpret_cast<const uint8_t *>(es.tiles) + h.off_segoff);
    for (uint32_t g = 0; g <= prm->G; ++g) {
      if (fuse) {
        // one launch per generation: counting, then the DE step in the block
        // that finishes last
        FuseArgs fa = make_fuse(de, nullptr, prob, 1, g + 1, g == 0, pop, cost, trial, best,
                                g < prm->G ? trial : nullptr, feat, tau, es.cnt, ctot, K,
                                prm->n_min, prm->alpha, done, segoff);
        s = launch_fitness_count(ctx, es.tiles, ds->F, K, n_sub, 1, es.max_tiles, feat, tau, P, D,
                                 es.cnt, &fa);
        if (s) return s;
        continue;
      }
      s = launch_fitness_count(ctx, es.tiles, ds->F, K, n_sub, 1, es.max_tiles, feat, tau, P, D,
                               es.cnt, nullptr);
      if (s) return s;
      s = launch_de_gen(ctx, de, nullptr, prob, 1, g + 1, g == 0, pop, cost, trial, best,
                        g < prm->G ? trial : nullptr, feat, tau, es.cnt, ctot, K, prm->n_min,
                        prm->alpha);
      if (s) return s;
    }
  } else {
    // walk path (depth above 5, wide data): per generation the walk kernel
    // and the leaf epilogue give the trial costs, then one launch makes the
    // selection, best and the next trial (a thread per node and individual);
    // the trial population alternates between two buffers
    double *trial2 = (double *)arena_get(ctx, "ss_trial2", (size_t)P * m * 8);
    if (!trial2) return MH_ENOMEM;
    FitnessOut fo;
    fo.cost = cost;
    s = eval_trees(ctx, es, feat, tau, P, D, prm->n_min, prm->alpha, fo);
    if (s) return s;
    // best of generation 0, and the trial population of generation 1
    s = launch_de_select_mutate(ctx, de, prob, 1, pop, cost, nullptr, nullptr, best,
                                prm->G >= 1 ? trial : nullptr, feat, tau);
    if (s) return s;
    FitnessOut ft;
    ft.cost = tcost;
    double *cur = trial, *nxt = trial2;
    for (uint32_t g = 1; g <= prm->G; ++g) {
      s = eval_trees(ctx, es, feat, tau, P, D, prm->n_min, prm->alpha, ft);
      if (s) return s;
      s = launch_de_select_mutate(ctx, de, prob, g + 1, pop, cost, cur, tcost, best,
                                  g < prm->G ? nxt : nullptr, feat, tau);
      if (s) return s;
      std::swap(cur, nxt);
    }
  }
  if (!persisted) {
    // the best individual: decode and evaluate for its labels (the
    // cooperative launch counted it in a last pass of its own)
    s = launch_decode(ctx, pop, P, D, ds->F, ds->n_unique, f1, t1, 1, best, true);
    if (s) return s;
    FitnessOut fb;
    fb.label = lab1;
    fb.correct = corr1;
    fb.cost = cost1;
    // a single-tree evaluation: left out of the population-kernel timing
    const bool prof = ctx->profile;
    ctx->profile = false;
    s = eval_trees(ctx, es, f1, t1, 1, D, prm->n_min, prm->alpha, fb);
    ctx->profile = prof;
    if (s) return s;
  }
  if (!ctx->result) {
    MH_HIP(ctx, hipHostMalloc((void **)&ctx->result, sizeof(ResultOut)));
    std::memset(ctx->result, 0, sizeof(ResultOut));
  }
  s = launch_pack_result(ctx, D, f1, t1, lab1, corr1, cost1, err, ds->status, ctx->result);
  if (s) return s;
  s = wait_stream(ctx);
  if (s) return s;
  std::memset(out, 0, sizeof(*out));
  out->D = D;
  std::memcpy(out->feat, ctx->result->tree.feat, SB);
  std::memcpy(out->tau, ctx->result->tree.tau, (size_t)SB * 4);
  std::memcpy(out->label, ctx->result->tree.label, SL);
  out->correct = ctx->result->tree.correct;
  out->cost = ctx->result->tree.cost;
  const uint32_t flag = ctx->result->flag;
  if ((flag & 1u) && persisted && depth < 4) {
    // the cooperative grid did not run all at once: not again, and the run
    // is redone (results do not depend on the launch form)
    coop_note_failure(ctx);
    return deoct(ctx, ds, idx, n_sub, D, prm, warm_host, W, prob, out, depth + 1);
  }
  if (flag & 1u) return fail(ctx, MH_EDEVICE, "DEOCT grid barrier: a wait gave up");
  if (flag & 2u) return fail(ctx, MH_EINVAL, "X holds a NaN");
  if (flag) return fail(ctx, MH_EDEVICE, "rank encoding failed on the device");
  (void)K;
  return MH_OK;
}

// Sequential moving-horizon step: DEOCT on the samples at node t, problem id
// t; returns the root of the best subtree.
static mh_status solve_node(Ctx *ctx, const mh_dataset *ds, const uint32_t *node_of, uint32_t t,
                            uint32_t De, const mh_de_params *prm, const double *warm, uint32_t W,
                            uint8_t *feat, uint32_t *tau) {
  uint32_t *idx = (uint32_t *)arena_get(ctx, "mh_idx", (size_t)(ds->n ? ds->n : 1) * 4);
  uint32_t *cursor = nullptr;
  if (!idx) return MH_ENOMEM;
  mh_status s = launch_compact(ctx, node_of, ds->n, t, idx);
  if (s) return s;
  cursor = (uint32_t *)arena_get(ctx, "mh_cursor", 256);
  uint32_t n_t = 0;
  MH_HIP(ctx, hipMemcpyAsync(&n_t, cursor, 4, hipMemcpyDeviceToHost, ctx->stream));
  MH_HIP(ctx, hipStreamSynchronize(ctx->stream));
  mh_tree tr;
  s = deoct(ctx, ds, idx, n_t, De, prm, warm, W, t, &tr);
  if (s) return s;
  *feat = tr.feat[0];
  *tau = tr.tau[0];
  return MH_OK;
}

static mh_status solve_all(Ctx *ctx, const mh_dataset *ds, uint32_t D, const mh_de_params *prm,
                           const double *warm, uint32_t W, mh_tree *out) {
  return deoct(ctx, ds, nullptr, ds->n, D, prm, warm, W, 0, out);
}

}  // namespace mh

using namespace mh;

#define CTX_OR_FAIL(ctx)                                              \
  do {                                                                \
    if (!(ctx)) return fail(nullptr, MH_EINVAL, "context is null");   \
    hipError_t e_ = hipSetDevice((ctx)->c.device);                    \
    if (e_ != hipSuccess) return hip_fail(&(ctx)->c, e_, "hipSetDevice"); \
  } while (0)

extern "C" {

const char *mh_version(void) { return "mhdeoct-gfx950 0.1"; }

mh_status mh_ctx_create(int device, void *hip_stream, mh_ctx **out) {
  if (!out) return fail(nullptr, MH_EINVAL, "out is null");
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDeviceCount");
  if (device < 0 || device >= ndev) return fail(nullptr, MH_EINVAL, "no such device");
  e = hipSetDevice(device);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipSetDevice");
  mh_ctx *c = new mh_ctx();
  c->c.device = device;
  c->c.stream = reinterpret_cast<hipStream_t>(hip_stream);
  // (a failed lookup leaves only fitness_eval_static unusable: it reports it)
  if (static_scratch_of(device, &c->c.static_scratch) != hipSuccess) {
    (void)hipGetLastError();
    c->c.static_scratch = nullptr;
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
      cus > 0)
    c->c.num_cu = cus;
  // launch-shape overrides for tuning sweeps
  if (const char *v = std::getenv("MHDEOCT_FIT_BLOCKS_PER_CU")) c->c.fit_blocks_per_cu = (uint32_t)std::max(1, atoi(v));
  if (const char *v = std::getenv("MHDEOCT_FIT_MIN_TILES")) c->c.fit_min_tiles = (uint32_t)std::max(1, atoi(v));
  if (const char *v = std::getenv("MHDEOCT_FUSE_DE")) c->c.fuse_de = atoi(v) != 0;
  if (const char *v = std::getenv("MHDEOCT_PERSIST")) c->c.persist = atoi(v) != 0;
  if (const char *v = std::getenv("MHDEOCT_PERSIST_RESIDENT"))
    c->c.persist_resident = atoi(v) != 0;
  if (const char *v = std::getenv("MHDEOCT_PERSIST_HALVES"))
    c->c.persist_halves = atoi(v) >= 4 ? 4u : (atoi(v) == 1 ? 1u : 2u);
  if (const char *v = std::getenv("MHDEOCT_PERSIST_BLOCKS_PER_CU"))
    c->c.persist_blocks_per_cu = (uint32_t)std::max(1, atoi(v));
  if (const char *v = std::getenv("MHDEOCT_RANK_COOP")) c->c.rank_coop = atoi(v) != 0;
  if (const char *v = std::getenv("MHDEOCT_DEBUG")) c->c.debug = atoi(v) != 0;
  if (const char *v = std::getenv("MHDEOCT_WALK_IT")) c->c.walk_it = (uint32_t)std::max(0, atoi(v));
  if (const char *v = std::getenv("MHDEOCT_WALK_LDS"))
    c->c.walk_lds = atoi(v) > 0 ? (size_t)std::min(std::max(atoi(v), 8192), 150 * 1024) : 0;
  if (const char *v = std::getenv("MHDEOCT_SELECT_TPI")) {
    const int t = atoi(v);
    c->c.de_select_tpi = (t == 1 || t == 2 || t == 4 || t == 8) ? (uint32_t)t : 0u;
  }
  if (const char *v = std::getenv("MHDEOCT_WAIT_TICKS"))
    c->c.wait_ticks = std::min<uint64_t>(strtoull(v, nullptr, 10), 200000000ull);
  if (const char *v = std::getenv("MHDEOCT_RANK_R")) {
    const int r = atoi(v);
    c->c.rank_coop_R = (r >= 256 && r <= 8192 && (r & (r - 1)) == 0) ? (uint32_t)r : 0u;
  }
  int coop = 0;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, device) == hipSuccess)
    c->c.coop = coop != 0;
  int lds_max = 0;
  if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, device) ==
          hipSuccess &&
      lds_max >= 64 * 1024)
    c->c.max_lds = (uint32_t)std::min(lds_max, 160 * 1024);
  *out = c;
  return MH_OK;
}

void mh_ctx_destroy(mh_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->c.device);
  (void)hipStreamSynchronize(ctx->c.stream);
  for (auto &b : ctx->c.arena.bufs) (void)hipFree(b.ptr);
  for (hipEvent_t e : ctx->c.prof_ev) (void)hipEventDestroy(e);
  if (ctx->c.result) (void)hipHostFree(ctx->c.result);
  if (ctx->c.hwords) (void)hipHostFree(ctx->c.hwords);
  if (ctx->c.done_ev) (void)hipEventDestroy(ctx->c.done_ev);
  delete ctx;
}

const char *mh_last_error(const mh_ctx *ctx) {
  return ctx ? ctx->c.err.c_str() : g_create_err.c_str();
}

mh_status mh_ctx_profile(mh_ctx *ctx, int enable) {
  CTX_OR_FAIL(ctx);
  ctx->c.profile = enable != 0;
  return MH_OK;
}

mh_status mh_ctx_stats(mh_ctx *ctx, uint64_t *launches, double *ms, uint64_t *evals,
                       uint64_t *tiles, int reset) {
  CTX_OR_FAIL(ctx);
  if (mh_status s = prof_collect(&ctx->c)) return s;
  if (launches) *launches = ctx->c.prof_launches;
  if (ms) *ms = ctx->c.prof_ms;
  if (evals) *evals = ctx->c.prof_evals;
  if (tiles) *tiles = ctx->c.prof_tiles;
  if (reset) {
    ctx->c.prof_launches = ctx->c.prof_evals = ctx->c.prof_tiles = 0;
    ctx->c.prof_ms = 0.0;
  }
  return MH_OK;
}

mh_status mh_rank_encode(mh_ctx *ctx, const float *X, uint32_t n, uint32_t F, uint32_t ld,
                         uint32_t *ranks, uint32_t *n_unique, uint32_t *status) {
  CTX_OR_FAIL(ctx);
  Ctx *c = &ctx->c;
  if (F == 0 || F > MH_MAX_FEATURES) return fail(c, MH_EINVAL, "F must be in 1..255");
  if (ld < n) return fail(c, MH_EINVAL, "ld must be >= n");
  if ((n > 0 && (!X || !ranks)) || !n_unique) return fail(c, MH_EINVAL, "null pointer");
  return launch_rank_encode(c, X, n, F, ld, ranks, n_unique, status);
}

mh_status tree_decode(mh_ctx *ctx, const double *genes, uint32_t P, uint32_t D, uint32_t F,
                      const uint32_t *n_unique, uint8_t *feat, uint32_t *tau) {
  CTX_OR_FAIL(ctx);
  Ctx *c = &ctx->c;
  if (D < 1 || D > MH_MAX_DEPTH) return fail(c, MH_EINVAL, "D must be in 1..10");
  if (F == 0 || F > MH_MAX_FEATURES) return fail(c, MH_EINVAL, "F must be in 1..255");
  if (P > 0 && (!genes || !n_unique || !feat || !tau)) return fail(c, MH_EINVAL, "null pointer");
  return launch_decode(c, genes, P, D, F, n_unique, feat, tau, 1, nullptr, false);
}

mh_status mh_tileset_bytes(uint32_t n_sub, uint32_t F, uint32_t K, size_t *bytes) {
  if (!bytes || F == 0 || F > MH_MAX_FEATURES || K == 0 || K > MH_MAX_CLASSES)
    return fail(nullptr, MH_EINVAL, "bad tileset size arguments");
  *bytes = tile_layout(n_sub, F, K, 1).total_bytes;
  return MH_OK;
}

mh_status mh_tileset_build(mh_ctx *ctx, const mh_dataset *ds, const uint32_t *idx, uint32_t n_sub,
                           void *tiles, size_t bytes) {
  CTX_OR_FAIL(ctx);
  Ctx *c = &ctx->c;
  mh_status s = check_dataset(c, ds);
  if (s) return s;
  if (!idx && n_sub > ds->n) return fail(c, MH_EINVAL, "n_sub > n without idx");
  if (!tiles) return fail(c, MH_EINVAL, "tiles is null");
  return launch_tile_build(c, ds, idx, nullptr, n_sub, 1, tiles, bytes);
}

static mh_status check_fit_args(Ctx *c, uint32_t P, uint32_t D, const uint8_t *feat,
                                const uint32_t *tau, uint32_t n_min, double alpha,
                                const double *cost) {
  if (D < 1 || D > MH_MAX_DEPTH) return fail(c, MH_EINVAL, "D must be in 1..10");
  if (P < 1 || P > MH_MAX_POP) return fail(c, MH_EINVAL, "P must be in 1..1024");
  if (!feat || !tau || !cost) return fail(c, MH_EINVAL, "null feat, tau or cost");
  if (n_min < 1) return fail(c, MH_EINVAL, "n_min must be >= 1");
  if (!(alpha >= 0.0)) return fail(c, MH_EINVAL, "alpha must be >= 0");
  return MH_OK;
}

static mh_status fitness_eval_core(Ctx *c, const mh_dataset *ds, const uint32_t *idx,
                                   uint32_t n_sub, const uint8_t *feat, const uint32_t *tau,
                                   uint32_t P, uint32_t D, uint32_t n_min, double alpha,
                                   uint32_t *counts, uint32_t *correct, uint8_t *label,
                                   double *cost, uint8_t *static_base) {
  mh_status s = check_dataset(c, ds);
  if (s) return s;
  s = check_fit_args(c, P, D, feat, tau, n_min, alpha, cost);
  if (s) return s;
  if (!idx && n_sub > ds->n) return fail(c, MH_EINVAL, "n_sub > n without idx");
  if (static_base) {
    const size_t need = eval_scratch_bytes(ds, n_sub, D, P);
    if (need > STATIC_SCRATCH_BYTES)
      return fail(c, MH_EINVAL,
                  "fitness_eval_static: this evaluation needs " + std::to_string(need) +
                      " bytes of scratch, more than its static limit of " +
                      std::to_string(STATIC_SCRATCH_BYTES) + " (use fitness_eval)");
  }
  EvalSet es;
  s = prepare_eval(c, ds, idx, n_sub, D, P, "fe_tiles", "fe_cnt", es, static_base,
                   TILE_MIN_TREES);
  if (s) return s;
  s = launch_zero(c, {{es.cnt, es.cnt ? cnt_bytes(1, D, ds->K, P) : 0}});
  if (s) return s;
  FitnessOut out;
  out.counts = counts;
  out.correct = correct;
  out.label = label;
  out.cost = cost;
  return eval_trees(c, es, feat, tau, P, D, n_min, alpha, out);
}

mh_status fitness_eval(mh_ctx *ctx, const mh_dataset *ds, const uint32_t *idx, uint32_t n_sub,
                       const uint8_t *feat, const uint32_t *tau, uint32_t P, uint32_t D,
                       uint32_t n_min, double alpha, uint32_t *counts, uint32_t *correct,
                       uint8_t *label, double *cost) {
  CTX_OR_FAIL(ctx);
  return fitness_eval_core(&ctx->c, ds, idx, n_sub, feat, tau, P, D, n_min, alpha, counts, correct,
                           label, cost, nullptr);
}

mh_status fitness_eval_static(mh_ctx *ctx, const mh_dataset *ds, const uint32_t *idx,
                              uint32_t n_sub, const uint8_t *feat, const uint32_t *tau, uint32_t P,
                              uint32_t D, uint32_t n_min, double alpha, uint32_t *counts,
                              uint32_t *correct, uint8_t *label, double *cost) {
  CTX_OR_FAIL(ctx);
  Ctx *c = &ctx->c;
  if (!c->static_scratch)
    return fail(c, MH_EDEVICE, "fitness_eval_static: no address for the static scratch");
  // no timing events either: the call only queues kernels
  const bool prof = c->profile;
  c->profile = false;
  const mh_status s = fitness_eval_core(c, ds, idx, n_sub, feat, tau, P, D, n_min, alpha, counts,
                                        correct, label, cost, c->static_scratch);
  c->profile = prof;
  return s;
}

mh_status fitness_eval_tiles(mh_ctx *ctx, const void *tiles, const uint32_t *n_unique,
                             const uint8_t *feat, const uint32_t *tau, uint32_t P, uint32_t D,
                             uint32_t n_min, double alpha, uint32_t *counts, uint32_t *correct,
                             uint8_t *label, double *cost) {
  CTX_OR_FAIL(ctx);
  Ctx *c = &ctx->c;
  mh_status s = check_fit_args(c, P, D, feat, tau, n_min, alpha, cost);
  if (s) return s;
  if (!tiles) return fail(c, MH_EINVAL, "tiles is null");
  (void)n_unique;
  TileHdr h;
  MH_HIP(c, hipMemcpyAsync(&h, tiles, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  MH_HIP(c, hipStreamSynchronize(c->stream));
  if (h.magic != TILE_MAGIC || h.n_problems != 1) return fail(c, MH_EINVAL, "not a tile set");
  if (!tile_path_ok(D, h.F, 0)) return fail(c, MH_EINVAL, "tile path needs D <= 5 and F <= 80");
  uint32_t *cnt = (uint32_t *)arena_get(c, "fe_cnt", cnt_bytes(1, D, h.K, P));
  if (!cnt) return MH_ENOMEM;
  MH_HIP(c, hipMemsetAsync(cnt, 0, cnt_bytes(1, D, h.K, P), c->stream));
  FitnessOut out;
  out.counts = counts;
  out.correct = correct;
  out.label = label;
  out.cost = cost;
  return launch_fitness_tiles(c, tiles, h.F, h.K, h.n_sub, 1, h.max_tiles, feat, tau, P, D, n_min,
                              alpha, cnt, out);
}

mh_status de_init(mh_ctx *ctx, uint32_t P, uint32_t D, uint32_t F, uint64_t seed,
                  uint64_t problem_id, const double *warm, uint32_t W, double *pop) {
  CTX_OR_FAIL(ctx);
  Ctx *c = &ctx->c;
  if (D < 1 || D > MH_MAX_DEPTH) return fail(c, MH_EINVAL, "D must be in 1..10");
  if (P > MH_MAX_POP || W > P) return fail(c, MH_EINVAL, "bad P or W");
  if (!pop || (W > 0 && !warm)) return fail(c, MH_EINVAL, "null pointer");
  return launch_de_init(c, P, D, F, seed, nullptr, problem_id, 1, warm, W, pop, false);
}

mh_status de_step(mh_ctx *ctx, const mh_de_params *prm, uint32_t D, uint32_t F,
                  uint64_t problem_id, uint32_t g, double *pop, double *cost,
                  const double *trial, const double *trial_cost, uint32_t *best,
                  double *next_trial) {
  CTX_OR_FAIL(ctx);
  Ctx *c = &ctx->c;
  mh_status s = check_de(c, prm, D);
  if (s) return s;
  if (!pop || !cost || !best) return fail(c, MH_EINVAL, "null pop, cost or best");
  if (trial && !trial_cost) return fail(c, MH_EINVAL, "trial without trial_cost");
  if (g >= (1u << 24)) return fail(c, MH_EINVAL, "g must be < 2^24");
  DeDev de{prm->P, D, F, prm->G, prm->M, prm->CR, prm->seed, nullptr, false};
  return launch_de_step(c, de, nullptr, problem_id, 1, g, pop, cost, trial, trial_cost, best,
                        next_trial, nullptr, nullptr);
}

// Runs deoct with the launch configuration mh_autotune chose for this shape,
// if any (the configuration changes timing only, never results).
static mh_status deoct_tuned(Ctx *c, const mh_dataset *ds, const uint32_t *idx, uint32_t n_sub,
                             uint32_t D, const mh_de_params *prm, const double *warm, uint32_t W,
                             uint64_t prob, mh_tree *out) {
  const uint32_t tb = tiles_bucket(tile_layout(n_sub, ds->F, ds->K, 1).max_tiles, (uint32_t)c->num_cu);
  for (const Ctx::Tuned &t : c->tuned) {
    if (t.D == D && t.P == prm->P && t.F == ds->F && t.K == ds->K && t.tiles_bucket == tb) {
      const bool p0 = c->persist;
      const uint32_t h0 = c->persist_halves, b0 = c->persist_blocks_per_cu,
                     f0 = c->fit_blocks_per_cu;
      c->persist = t.persist != 0;
      c->persist_halves = t.halves;
      c->persist_blocks_per_cu = t.persist_bpc;
      c->fit_blocks_per_cu = t.fit_bpc;
      const mh_status s = deoct(c, ds, idx, n_sub, D, prm, warm, W, prob, out);
      c->persist = p0;
      c->persist_halves = h0;
      c->persist_blocks_per_cu = b0;
      c->fit_blocks_per_cu = f0;
      return s;
    }
  }
  return deoct(c, ds, idx, n_sub, D, prm, warm, W, prob, out);
}

mh_status subtree_solve(mh_ctx *ctx, const mh_dataset *ds, const uint32_t *idx, uint32_t n_sub,
                        uint32_t D, const mh_de_params *prm, const double *warm, uint32_t W,
                        uint64_t problem_id, mh_tree *out) {
  CTX_OR_FAIL(ctx);
  Ctx *c = &ctx->c;
  mh_status s = check_dataset(c, ds);
  if (s) return s;
  s = check_de(c, prm, D);
  if (s) return s;
  if (!out) return fail(c, MH_EINVAL, "out is null");
  if (W > prm->P || (W > 0 && !warm)) return fail(c, MH_EINVAL, "bad warm starts");
  if (!idx && n_sub > ds->n) return fail(c, MH_EINVAL, "n_sub > n without idx");
  return deoct_tuned(c, ds, idx, n_sub, D, prm, warm, W, problem_id, out);
}

mh_status subtree_solve_pop(mh_ctx *ctx, const mh_dataset *ds, const uint32_t *idx,
                            uint32_t n_sub, uint32_t D, const mh_de_params *prm,
                            const double *warm, uint32_t W, uint64_t problem_id, mh_tree *out,
                            double *pop_out, double *cost_out) {
  mh_status s = subtree_solve(ctx, ds, idx, n_sub, D, prm, warm, W, problem_id, out);
  if (s) return s;
  Ctx *c = &ctx->c;
  const uint32_t P = prm->P, m = 2u * ((1u << D) - 1u);
  // the run left its final population (gene-major) and costs in the arena
  if (pop_out) {
    const double *pop = (const double *)arena_get(c, "ss_pop", (size_t)P * m * 8);
    if (!pop) return MH_ENOMEM;
    s = launch_pop_rows(c, pop, P, m, pop_out);
    if (s) return s;
  }
  if (cost_out) {
    const double *cost = (const double *)arena_get(c, "ss_cost", (size_t)P * 8);
    if (!cost) return MH_ENOMEM;
    MH_HIP(c, hipMemcpyAsync(cost_out, cost, (size_t)P * 8, hipMemcpyDeviceToDevice, c->stream));
  }
  return wait_stream(c);
}

mh_status mh_autotune(mh_ctx *ctx, const mh_dataset *ds, uint32_t D, const mh_de_params *prm,
                      uint32_t generations, mh_tune_result *out) {
  CTX_OR_FAIL(ctx);
  Ctx *c = &ctx->c;
  mh_status s = check_dataset(c, ds);
  if (s) return s;
  s = check_de(c, prm, D);
  if (s) return s;
  if (!out) return fail(c, MH_EINVAL, "out is null");
  if (generations == 0) return fail(c, MH_EINVAL, "generations must be >= 1");
  s = check_ds_status(c, ds);
  if (s) return s;
  // candidates: the whole-run kernel with one or two tile streams per block
  // and 1, 2 or 4 blocks per CU, and the per-generation kernels with 1, 2 or
  // 4 fitness blocks per CU
  struct Cand {
    uint32_t persist, halves, persist_bpc, fit_bpc;
  };
  std::vector<Cand> cands;
  for (uint32_t hv : {4u, 2u, 1u})
    for (uint32_t b : {1u, 2u, 4u}) cands.push_back({1u, hv, b, c->fit_blocks_per_cu});
  for (uint32_t b : {1u, 2u, 4u}) cands.push_back({0u, 2u, 0u, b});
  mh_de_params p = *prm;
  p.G = generations;
  const bool p0 = c->persist;
  const uint32_t h0 = c->persist_halves, b0 = c->persist_blocks_per_cu, f0 = c->fit_blocks_per_cu;
  std::memset(out, 0, sizeof(*out));
  out->n_candidates = (uint32_t)std::min<size_t>(cands.size(), 16);
  double best_ms = 1e300;
  Cand best = cands.back();
  mh_tree tr;
  for (size_t i = 0; i < cands.size(); ++i) {
    const Cand &cd = cands[i];
    c->persist = cd.persist != 0;
    c->persist_halves = cd.halves;
    c->persist_blocks_per_cu = cd.persist_bpc;
    c->fit_blocks_per_cu = cd.fit_bpc;
    // one untimed run, then the median of three timed ones (each run
    // synchronises when it fills the host result)
    s = deoct(c, ds, nullptr, ds->n, D, &p, nullptr, 0, 0, &tr);
    double t[3];
    for (int k = 0; s == MH_OK && k < 3; ++k) {
      const auto t0 = std::chrono::steady_clock::now();
      s = deoct(c, ds, nullptr, ds->n, D, &p, nullptr, 0, 0, &tr);
      t[k] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    if (s) break;
    std::sort(t, t + 3);
    if (i < 16) out->ms[i] = t[1];
    if (t[1] < best_ms) {
      best_ms = t[1];
      best = cd;
    }
  }
  c->persist = p0;
  c->persist_halves = h0;
  c->persist_blocks_per_cu = b0;
  c->fit_blocks_per_cu = f0;
  if (s) return s;
  const uint32_t tb = tiles_bucket(tile_layout(ds->n, ds->F, ds->K, 1).max_tiles, (uint32_t)c->num_cu);
  Ctx::Tuned e{D, prm->P, ds->F, ds->K, tb, best.persist, best.halves, best.persist_bpc,
               best.fit_bpc};
  bool replaced = false;
  for (Ctx::Tuned &t : c->tuned)
    if (t.D == e.D && t.P == e.P && t.F == e.F && t.K == e.K && t.tiles_bucket == e.tiles_bucket) {
      t = e;
      replaced = true;
    }
  if (!replaced) c->tuned.push_back(e);
  out->persist = best.persist;
  out->halves = best.halves;
  out->persist_blocks_per_cu = best.persist_bpc;
  out->fit_blocks_per_cu = best.fit_bpc;
  out->ms_per_generation = best_ms / (generations + 1);
  return MH_OK;
}

mh_status mh_train(mh_ctx *ctx, const mh_dataset *ds, uint32_t D, uint32_t D_MH,
                   const mh_de_params *prm, uint32_t flags, mh_tree *out) {
  CTX_OR_FAIL(ctx);
  Ctx *c = &ctx->c;
  mh_status s = check_dataset(c, ds);
  if (s) return s;
  s = check_de(c, prm, D);
  if (s) return s;
  if (!out) return fail(c, MH_EINVAL, "out is null");
  if (D_MH < 1) return fail(c, MH_EINVAL, "D_MH must be >= 1");
  if (flags & ~(MH_BATCHED | MH_WS_CART | MH_WS_DEOCT | MH_WS_DEOCT_CART))
    return fail(c, MH_EINVAL, "unknown flags");
  if ((flags & MH_WS_DEOCT_CART) && !(flags & MH_WS_DEOCT))
    return fail(c, MH_EINVAL, "MH_WS_DEOCT_CART needs MH_WS_DEOCT");
  if ((flags & MH_BATCHED) && (std::min(D_MH, D) > 5 || ds->F > 80))
    return fail(c, MH_EINVAL, "the batched form needs subtree depth <= 5 and F <= 80");
  s = check_ds_status(c, ds);
  if (s) return s;
  return mh_train_impl(c, ds, D, D_MH, prm, flags, out, solve_node, solve_all);
}

mh_status split1(mh_ctx *ctx, const mh_dataset *ds, const uint32_t *idx, uint32_t n_sub,
                 uint8_t *feat, uint32_t *tau, uint32_t *correct) {
  CTX_OR_FAIL(ctx);
  Ctx *c = &ctx->c;
  mh_status s = check_dataset(c, ds);
  if (s) return s;
  if (!feat || !tau || !correct) return fail(c, MH_EINVAL, "null output");
  if (!idx && n_sub > ds->n) return fail(c, MH_EINVAL, "n_sub > n without idx");
  return split1_subset(c, ds, idx, n_sub, feat, tau, correct);
}

mh_status cart_tree(mh_ctx *ctx, const mh_dataset *ds, const uint32_t *idx, uint32_t n_sub,
                    uint32_t D, uint8_t *feat, uint32_t *tau) {
  CTX_OR_FAIL(ctx);
  Ctx *c = &ctx->c;
  mh_status s = check_dataset(c, ds);
  if (s) return s;
  if (D < 1 || D > MH_MAX_DEPTH) return fail(c, MH_EINVAL, "D must be in 1..10");
  if (!feat || !tau) return fail(c, MH_EINVAL, "null output");
  if (!idx && n_sub > ds->n) return fail(c, MH_EINVAL, "n_sub > n without idx");
  s = check_ds_status(c, ds);
  if (s) return s;
  return cart_subset(c, ds, idx, n_sub, D, feat, tau);
}

}  // extern "C"
