// internal.h -- host-side internals shared by the library's translation
// units: the context, its device arena, error reporting, the tiled sample
// layout and the kernel launchers each .hip file provides.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <initializer_list>
#include <string>
#include <vector>

#include "../../include/mhdeoct.h"

namespace mh {

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------
struct Arena {
  // Named, growable device buffers owned by the context.  Each name keeps
  // one allocation that is reallocated (without copying) when a larger size
  // is asked for.
  struct Buf {
    std::string name;
    void *ptr = nullptr;
    size_t bytes = 0;
  };
  std::vector<Buf> bufs;
};

struct ResultOut;

struct Ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int num_cu = 256;
  std::string err;
  Arena arena;
  // fitness-kernel timing: each timed launch takes a start/stop event pair
  // that the launch itself records (hipExtLaunchKernelGGL), so the measured
  // interval is the kernel's execution and nothing waits on it; the pairs
  // are read back by mh_ctx_stats (or when the pool is full).
  bool profile = false;
  std::vector<hipEvent_t> prof_ev;
  size_t prof_used = 0;
  uint64_t prof_launches = 0, prof_evals = 0, prof_tiles = 0;
  double prof_ms = 0.0;
  // fitness-kernel launch shape (tunable)
  uint32_t fit_blocks_per_cu = 2;
  uint32_t fit_min_tiles = 1;
  bool fuse_de = false;  // fitness and DE step in one launch per generation (MHDEOCT_FUSE_DE=1)
  bool persist = true;   // whole DEOCT runs as one cooperative launch (MHDEOCT_PERSIST=0 turns off)
  uint32_t persist_blocks_per_cu = 0;  // its blocks per CU; 0 = by size (MHDEOCT_PERSIST_BLOCKS_PER_CU)
  uint32_t persist_halves = 2;         // tile streams per block, 1, 2 or 4 (MHDEOCT_PERSIST_HALVES)
  bool persist_resident = true;        // tiles kept in LDS when they fit (MHDEOCT_PERSIST_RESIDENT)
  bool coop = false;     // the device supports cooperative launches
  uint32_t max_lds = 64u * 1024u;  // dynamic LDS one block may use
  // launch configurations chosen by mh_autotune, by problem shape
  struct Tuned {
    uint32_t D, P, F, K, tiles_bucket;  // shape key
    uint32_t persist, halves, persist_bpc, fit_bpc;
  };
  std::vector<Tuned> tuned;
  // pinned host record for subtree_solve's result (allocated on first use)
  ResultOut *result = nullptr;
  // pinned host words for small status read-backs (allocated on first use)
  uint32_t *hwords = nullptr;
  // event for waits on the stream's completed work (created on first use)
  hipEvent_t done_ev = nullptr;
  // rank encoding in one cooperative launch when it fits (MHDEOCT_RANK_COOP);
  // samples per block forced by MHDEOCT_RANK_R (0 = by size)
  bool rank_coop = true;
  uint32_t rank_coop_R = 0;
  // launch decisions of the cooperative kernels to stderr (MHDEOCT_DEBUG=1)
  bool debug = false;
  // grid-barrier time limit in device wall-clock ticks (MHDEOCT_WAIT_TICKS;
  // tests set a tiny one to exercise the recovery from a barrier that gives up)
  uint64_t wait_ticks = 200000000ull;
  // lanes per individual of the split DE step's selection (MHDEOCT_SELECT_TPI,
  // 1, 2, 4 or 8; 0: one per class up to 4)
  uint32_t de_select_tpi = 0;
  // remembered occupancy queries
  struct Occ {
    const void *kern;
    int threads;
    size_t lds;
    int per_cu;
  };
  std::vector<Occ> occ;
  // cooperative launches (kernel, grid) whose grid barrier gave up: not
  // launched again by this context; and the last one launched
  std::vector<std::pair<const void *, uint32_t>> coop_bad;
  const void *last_coop_kern = nullptr;
  uint32_t last_coop_grid = 0;
  // this device's copy of the allocation-free entry point's static scratch
  // (null when its address could not be looked up)
  uint8_t *static_scratch = nullptr;
  // the walk path's leaf-count buffer (and its bytes) when the last queued
  // epilogue left it all zero (it clears what it reads): the next evaluation
  // into it needs no clearing launch
  const void *walk_zero = nullptr;
  size_t walk_zero_bytes = 0;
  // LDS bytes per block of the walk kernel (MHDEOCT_WALK_LDS; 0 = a third of
  // the CU's LDS, at least 48 KiB)
  size_t walk_lds = 0;
  // samples per thread of the walk kernel (MHDEOCT_WALK_IT: 1, 2 or 4; 0 = by
  // the tile size)
  uint32_t walk_it = 0;
};
// 64 pinned host words of the context, or nullptr (error set).
uint32_t *host_words(Ctx *ctx);
// Waits for the work queued so far on the context's stream: polls an event
// for up to 50 ms (the result of a run is back a few microseconds after the
// device finishes, where a blocking wait takes tens), then blocks.
mh_status wait_stream(Ctx *ctx);
// Blocks of `kern` (threads, dynamic LDS bytes) one CU holds, from the
// occupancy query, remembered per context; 0 when the query fails.
int occupancy(Ctx *ctx, const void *kern, int threads, size_t lds);
// Blocks per CU a cooperative grid of `kern` may use: the occupancy query,
// with a margin (one block less from three blocks up, 2 KiB of LDS per CU
// left over) and at most four.  Grids that the query called co-resident
// were seen not to become resident all at once near those limits (the grid
// barrier then gives up after its time limit).
int coop_per_cu(Ctx *ctx, const void *kern, int threads, size_t lds);
// Launches a kernel whose blocks wait for each other at grid barriers, with
// a grid within coop_per_cu.  By default an ordinary launch: the runtime's
// cooperative launch adds about 17 us of device time per launch (measured
// with an empty kernel: 19.6 against 2.3 us per launch) and, as the failures
// above show, does not make the grid resident either; the barriers' time
// limit and the failure record cover a grid that does not run all at once.
hipError_t launch_grid_sync(Ctx *ctx, const void *kern, dim3 grid, dim3 block, void **args,
                            size_t lds);
// Whether (kern, grid) gave up at a grid barrier before in this context.
bool coop_is_bad(const Ctx *ctx, const void *kern, uint32_t grid);
// Records the last cooperative launch as one whose barrier gave up.
void coop_note_failure(Ctx *ctx);
// Shape key bucket of a tile count: floor(log2(tiles per CU)) + 1 (0 for none).
uint32_t tiles_bucket(uint32_t max_tiles, uint32_t num_cu);

// Checks DE parameters for a depth-D problem (MH_EINVAL with a message).
mh_status check_de(Ctx *ctx, const mh_de_params *p, uint32_t D);

// Returns a device buffer of at least `bytes` for `name`, or nullptr (and
// sets ctx->err) on allocation failure.
void *arena_get(Ctx *ctx, const char *name, size_t bytes);

mh_status fail(Ctx *ctx, mh_status code, const std::string &msg);

// With profiling on, hands out the next event pair for a timed launch (and
// returns true); with it off returns false and leaves *e0 = *e1 = nullptr.
bool prof_pair(Ctx *ctx, hipEvent_t *e0, hipEvent_t *e1);
// Waits for the stream and adds the elapsed time of every used pair to
// prof_ms.
mh_status prof_collect(Ctx *ctx);
mh_status hip_fail(Ctx *ctx, hipError_t e, const char *what);

#define MH_HIP(ctx, call)                                  \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return hip_fail((ctx), e_, #call); \
  } while (0)

#define MH_LAUNCHED(ctx, what)                             \
  do {                                                     \
    hipError_t e_ = hipGetLastError();                     \
    if (e_ != hipSuccess) return hip_fail((ctx), e_, what); \
  } while (0)

// ---------------------------------------------------------------------------
// Tiled sample layout (the fitness kernel's input).
//
// Samples of each (subproblem, class) segment are cut into tiles of at most
// TILE_CAP = 63.  A tile record holds, per feature f, the tile's ranks in
// ascending order (64 u32; unused entries 0x7FFFFFFF) followed, per feature,
// by the 64 prefix masks pm[c] = set of tile positions of the c smallest
// ranks (u64; pm[0] = 0).  "rank < tau" over the tile is then pm[c] with
// c = #{sorted ranks < tau}, found by binary search.
// ---------------------------------------------------------------------------
constexpr uint32_t TILE_CAP = 63;
constexpr uint32_t TILE_W = 64;
constexpr uint32_t TILE_MAGIC = 0x3154484du;  // "MHT1"

struct TileHdr {
  uint32_t magic;
  uint32_t F, K;
  uint32_t n_sub;        // samples in the layout
  uint32_t n_tiles;      // tiles in use (written on the device)
  uint32_t max_tiles;    // capacity
  uint32_t n_problems;   // subproblems
  uint32_t pad0;
  uint64_t off_info;     // u32 [max_tiles]: sub << 16 | class << 8 | count
  uint64_t off_ctot;     // u32 [n_problems][K]: samples per class
  uint64_t off_data;     // [max_tiles][tile_bytes(F)]
  uint64_t off_order;    // u32 [max_tiles][64]: sample ids (build scratch)
  uint64_t off_segoff;   // u32 [n_problems * K + 1]: first tile of a segment
  uint64_t off_cursor;   // u32 [n_problems * K]: fill cursors (build scratch)
  uint64_t total_bytes;
  uint64_t off_perm;     // u8 [max_tiles][F][64]: the tile position of each sorted
                         // rank (past the count, the last one's again); with the
                         // sorted ranks a compact form of the record, the masks
                         // rebuilt from it
  uint32_t pad1[64 - 24];
};
static_assert(sizeof(TileHdr) == 256, "tile header is 256 bytes");

__host__ __device__ inline size_t tile_bytes(uint32_t F) { return (size_t)F * (TILE_W * 4 + TILE_W * 8); }
inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
inline uint32_t max_tiles_for(uint32_t n_sub, uint32_t n_problems, uint32_t K) {
  return (n_sub + TILE_CAP - 1) / TILE_CAP + n_problems * K;
}
// Host-side layout of a tile set (offsets only; no device access).
TileHdr tile_layout(uint32_t n_sub, uint32_t F, uint32_t K, uint32_t n_problems);

// ---------------------------------------------------------------------------
// Kernel launchers (one per .hip file)
// ---------------------------------------------------------------------------
// rank_encode.hip
// With nan_out == nullptr it synchronises and fails with MH_EINVAL if X holds
// a NaN; otherwise it stays asynchronous and sets *nan_out (device u32) to a
// non-zero value when X holds a NaN.
mh_status launch_rank_encode(Ctx *ctx, const float *X, uint32_t n, uint32_t F,
                             uint32_t ld, uint32_t *ranks, uint32_t *n_unique,
                             uint32_t *nan_out = nullptr, bool retry = true);
// Sorts (key, value) pairs by the low `key_bits` of key (stable LSD radix
// sort, 8 bits per pass).  Buffers are ping-ponged; the sorted result ends in
// (*keys, *vals) which may point at the alternate buffers on return.
mh_status radix_sort_pairs(Ctx *ctx, uint64_t **keys, uint32_t **vals, uint64_t *keys_alt,
                           uint32_t *vals_alt, uint32_t count, uint32_t key_bits);

// Exclusive or inclusive scan of n u32 values (in may equal out).
mh_status scan_u32(Ctx *ctx, const uint32_t *in, uint32_t *out, uint32_t n, bool inclusive);

// tiles.hip
// Builds the tiled layout at `base` for samples idx[0..n_sub) (all if
// idx == nullptr); sub_of (device [n_sub], may be null) assigns each sample a
// subproblem < n_problems.
mh_status launch_tile_build(Ctx *ctx, const mh_dataset *ds, const uint32_t *idx,
                            const uint32_t *sub_of, uint32_t n_sub, uint32_t n_problems,
                            void *base, size_t bytes);

// fitness.hip
struct FitnessOut {
  uint32_t *counts = nullptr;   // [sub][P][SL][K]
  uint32_t *correct = nullptr;  // [sub][P]
  uint8_t *label = nullptr;     // [sub][P][SL]
  double *cost = nullptr;       // [sub][P]
};
// Node-count accumulator for a tile set: CNT_REP copies of
// [n_problems][SB][K][Ppad]; fitness blocks add into copy blockIdx % CNT_REP
// so that fewer blocks contend for the same cache lines, and the epilogue sums
// the copies.
constexpr uint32_t CNT_REP = 1;
__host__ __device__ inline size_t cnt_copy_elems(uint32_t n_problems, uint32_t SB, uint32_t K,
                                                 uint32_t P) {
  return (size_t)n_problems * SB * K * ((P + 63u) & ~63u);
}
size_t cnt_bytes(uint32_t n_problems, uint32_t D, uint32_t K, uint32_t P);
__host__ __device__ inline uint32_t pad64(uint32_t P) { return (P + 63u) & ~63u; }
// Evaluate trees feat/tau ([n_problems][P][SB]) over the tile set: accumulates
// into cnt (must be zero), then the epilogue writes `out` and re-zeroes cnt.
mh_status launch_fitness_tiles(Ctx *ctx, const void *tiles, uint32_t F, uint32_t K,
                               uint32_t n_sub, uint32_t n_problems, uint32_t max_tiles,
                               const uint8_t *feat, const uint32_t *tau, uint32_t P,
                               uint32_t D, uint32_t n_min, double alpha, uint32_t *cnt,
                               const FitnessOut &out);
// The two halves of launch_fitness_tiles: the counting kernel (timed when
// profiling) and the epilogue.
struct FuseArgs;
mh_status launch_fitness_count(Ctx *ctx, const void *tiles, uint32_t F, uint32_t K,
                               uint32_t n_sub, uint32_t n_problems, uint32_t max_tiles,
                               const uint8_t *feat, const uint32_t *tau, uint32_t P, uint32_t D,
                               uint32_t *cnt, const FuseArgs *fuse);
uint32_t fitness_block_threads(uint32_t P);
uint32_t fused_threads(uint32_t P);
mh_status launch_fitness_epilogue(Ctx *ctx, const void *tiles, uint32_t F, uint32_t K,
                                  uint32_t n_sub, uint32_t n_problems, const uint8_t *feat,
                                  uint32_t P, uint32_t D, uint32_t n_min, double alpha,
                                  uint32_t *cnt, const FitnessOut &out);
// One population evaluation inside a multi-job launch (k_fitness_jobs):
// trees feat/tau ([P][SB]) over the tile set hdr, counts into cnt ([SB][K]
// [Ppad], zero on entry); the job owns blocks blk0 .. blk0 + nblk - 1.
struct FitJob {
  const TileHdr *hdr;
  const uint8_t *feat;
  const uint32_t *tau;
  uint32_t *cnt;
  uint32_t P, blk0, nblk, pad;
};
// Launches n_blocks blocks of waves * 64 threads; job_of[b] names block b's
// job.  Every job needs P <= waves * 64 and a tile set with F <= F_max.
mh_status launch_fitness_jobs(Ctx *ctx, uint32_t D, uint32_t waves, uint32_t F_max,
                              const FitJob *jobs, const uint16_t *job_of, uint32_t n_blocks);
// Direct per-sample walk for any depth (1..10): one tree at a time, leaf
// counts per (tree, leaf, class), then the same epilogue.
// leafcnt: walk_scratch_bytes(P, D, K) of device scratch the call may use
// (null: the context arena's): the leaf counts.
size_t walk_scratch_bytes(uint32_t P, uint32_t D, uint32_t K);
mh_status launch_fitness_walk(Ctx *ctx, const mh_dataset *ds, const uint32_t *idx,
                              uint32_t n_sub, const uint8_t *feat, const uint32_t *tau,
                              uint32_t P, uint32_t D, uint32_t n_min, double alpha,
                              const FitnessOut &out, uint32_t *leafcnt = nullptr);

// de.hip
// Population layouts: row-major [P][m] (the C ABI) or gene-major [m][P]
// (inside the DE loops, for coalesced access).
struct DeDev {
  uint32_t P, D, F, G;
  double M, CR;
  uint64_t seed;
  const uint32_t *n_unique;
  bool gene_major;
};
mh_status launch_de_init(Ctx *ctx, uint32_t P, uint32_t D, uint32_t F, uint64_t seed,
                         const uint64_t *prob_ids, uint64_t prob_base, uint32_t n_problems,
                         const double *warm, uint32_t W, double *pop, bool gene_major);
// Sets up to MAX_ZERO_RANGES device buffers (byte sizes multiples of 4; null
// or empty entries are skipped) to zero with one launch on the context's
// stream.
constexpr uint32_t MAX_ZERO_RANGES = 8;
struct ZeroRange {
  void *ptr;
  size_t bytes;
};
mh_status launch_zero(Ctx *ctx, std::initializer_list<ZeroRange> ranges);

// A solved tree and a status word, written by the device into pinned host
// memory: bit 0 a device wait gave up, bits 1 and up the rank-encoding status
// of the data (bit 1: X held a NaN).
struct ResultOut {
  mh_tree tree;
  uint32_t flag;
};
// Packs the best tree (f1, t1: its nodes; lab1: leaf labels; corr1, cost1)
// into *out, on the context's stream, with flag = (*flag_a != 0) |
// (*flag_b << 1) (a null pointer reads as 0).
mh_status launch_pack_result(Ctx *ctx, uint32_t D, const uint8_t *f1, const uint32_t *t1,
                             const uint8_t *lab1, const uint32_t *corr1, const double *cost1,
                             const uint32_t *flag_a, const uint32_t *flag_b, ResultOut *out);
// Copies a gene-major population [m][P] (the layout of the DE loops) into
// the row-major [P][m] layout of the C ABI.
mh_status launch_pop_rows(Ctx *ctx, const double *gene_major, uint32_t P, uint32_t m,
                          double *rows);
mh_status launch_decode(Ctx *ctx, const double *genes, uint32_t P, uint32_t D, uint32_t F,
                        const uint32_t *n_unique, uint8_t *feat, uint32_t *tau,
                        uint32_t n_problems, const uint32_t *row_sel, bool gene_major);
// Fitness epilogue fused with the DE step (tile path, depth 1..5): the
// population just evaluated (trial, or pop itself when init) gets its cost
// from the node counts cnt, then selection, best and the next trial.
mh_status launch_de_gen(Ctx *ctx, const DeDev &de, const uint64_t *prob_ids, uint64_t prob_base,
                        uint32_t n_problems, uint32_t g, bool init, double *pop, double *cost,
                        const double *trial, uint32_t *best, double *next_trial, uint8_t *feat,
                        uint32_t *tau, uint32_t *cnt, const uint32_t *ctot, uint32_t K,
                        uint32_t n_min, double alpha);
// Arguments of the fused fitness + DE launch (see fitness.hip), and whether
// a population of P fits one fused block.
FuseArgs make_fuse(const DeDev &de, const uint64_t *prob_ids, uint64_t prob_base,
                   uint32_t n_problems, uint32_t g, bool init, double *pop, double *cost,
                   const double *trial, uint32_t *best, double *next_trial, uint8_t *feat,
                   uint32_t *tau, uint32_t *cnt, const uint32_t *ctot, uint32_t K, uint32_t n_min,
                   double alpha, uint32_t *done, const uint32_t *segoff);
bool fusable(uint32_t P, uint32_t D, uint32_t F);
// A DE generation for one problem inside a multi-job launch: the epilogue of
// cnt (then re-zeroed), selection unless init, best, and the trial of
// generation g into next_trial (decoded into feat/tau) unless it is null.
// P_max is the largest population of the launch.
struct GenJob;
GenJob make_gen_job(const DeDev &de, uint64_t prob, uint32_t g, bool init, double *pop,
                    double *cost,
                    const double *trial, uint32_t *best, double *next_trial, uint8_t *feat,
                    uint32_t *tau, uint32_t *cnt, const uint32_t *ctot, uint32_t K,
                    uint32_t n_min, double alpha, uint32_t P_max);
mh_status launch_de_jobs(Ctx *ctx, uint32_t D, const GenJob *jobs, uint32_t n_jobs,
                         uint32_t P_max);
// One DE step for n_problems problems (block per problem).  When feat/tau are
// given, the new trial population is also decoded into them.
// The DE generation of one problem whose trial costs are in memory (the walk
// path) in one launch spread over the chip: the selection of the trial
// population `trial` (costs trial_cost; null trial: none, generation 1),
// best, and the trial population of generation g into next_trial (a buffer
// other than trial; null: only the selection and best), decoded into
// feat/tau.  pop and cost are updated in place.  Gene-major populations.
mh_status launch_de_select_mutate(Ctx *ctx, const DeDev &de, uint64_t prob, uint32_t g,
                                 double *pop, double *cost, const double *trial,
                                 const double *trial_cost, uint32_t *best, double *next_trial,
                                 uint8_t *feat, uint32_t *tau);
mh_status launch_de_step(Ctx *ctx, const DeDev &de, const uint64_t *prob_ids,
                         uint64_t prob_base, uint32_t n_problems, uint32_t g, double *pop,
                         double *cost, const double *trial, const double *trial_cost,
                         uint32_t *best, double *next_trial, uint8_t *feat, uint32_t *tau);

// persist.hip
// A whole DEOCT run of one problem (tile set `tiles`, n_sub samples) as one
// cooperative launch: pop (gene-major [m][P]) holds the initial population
// on entry and the final one on exit, with cost ([P]) and best ([1]).  err
// (device u32) becomes non-zero if a grid-barrier wait gave up.  Sets *used
// to false, queuing nothing, when the shape does not fit the kernel (depth
// above 5, P above 512, F above 80, LDS, co-residency); the caller then runs
// the per-generation kernels.  With fin, the launch also writes the best
// tree of the last generation (its nodes, leaf classes, correct count and
// cost, all device buffers), counted in one more pass over the tiles.
struct PersistFinal {
  uint8_t *feat;      // [SB]
  uint32_t *tau;      // [SB]
  uint8_t *label;     // [SL]
  uint32_t *correct;  // [1]
  double *cost;       // [1]
};
mh_status launch_deoct_persist(Ctx *ctx, const void *tiles, uint32_t F, uint32_t K,
                               uint32_t n_sub, uint32_t D, const mh_de_params *prm, uint64_t prob,
                               const uint32_t *n_unique, double *pop, double *cost,
                               uint32_t *best, uint32_t *err, const PersistFinal *fin,
                               bool *used);

// The same for the n_problems problems of a multi-problem tile set: each
// problem gets its own group of blocks (in proportion to its tiles), its own
// counters and barrier, and its DE state at problem stride in pop ([m][P]
// per problem), cost ([P] per problem) and best ([n_problems]).
// class_counts: HOST [n_problems][K] samples per class (as in the layout);
// prob_ids: device [n_problems].
mh_status launch_deoct_persist_multi(Ctx *ctx, const void *tiles, uint32_t F, uint32_t K,
                                     uint32_t n_sub, uint32_t n_problems,
                                     const uint32_t *class_counts, uint32_t D,
                                     const mh_de_params *prm, const uint64_t *prob_ids,
                                     const uint32_t *n_unique, double *pop, double *cost,
                                     uint32_t *best, uint32_t *err, bool *used);

// mh.hip
// Exact best depth-1 split (Algorithm 2, horizon-1 branch) of every subset
// {i : sub_of[i] == s}, s < nsub (samples with sub_of >= nsub are ignored;
// sub_of == nullptr puts every sample in subset 0).  tot: device [nsub][K]
// class totals of the subsets.  Writes feat/tau/correct (device, [nsub];
// correct may be null).  gini: CART's Gini split instead (correct gets 0).
mh_status launch_split1(Ctx *ctx, const mh_dataset *ds, const uint32_t *sub_of, uint32_t nsub,
                        const uint32_t *tot, uint8_t *feat, uint32_t *tau, uint32_t *correct,
                        bool gini = false);
// DEOCT for n_problems subproblems at once (problem ids prob_ids, device),
// samples assigned by sub_of (device [n], >= n_problems = not in any).
// Writes the decoded best tree of each problem to feat_out/tau_out (device,
// [n_problems][SB]) and its cost to cost_out (device [n_problems]).
// class_counts (HOST [n_problems][K], may be null) lets the whole run go to
// one cooperative launch.
// warm: device [n_problems][W][2 SB] warm-start genes (W may be 0).
mh_status deoct_batched(Ctx *ctx, const mh_dataset *ds, const uint32_t *sub_of,
                        uint32_t n_problems, const uint64_t *prob_ids, uint32_t D,
                        const mh_de_params *prm, const uint32_t *class_counts,
                        const double *warm, uint32_t W, uint8_t *feat_out, uint32_t *tau_out);
// CART (Gini) of depth D on each subset {i : sub_of[i] == s}, s < nsub:
// feat / tau device [nsub][2^D - 1].  cart_subset: one explicit subset, host
// outputs, synchronises.
mh_status cart_batched(Ctx *ctx, const mh_dataset *ds, const uint32_t *sub_of, uint32_t nsub,
                       uint32_t D, uint8_t *feat, uint32_t *tau);
mh_status cart_subset(Ctx *ctx, const mh_dataset *ds, const uint32_t *idx, uint32_t n_sub,
                      uint32_t D, uint8_t *feat, uint32_t *tau);

// Sequential-form helpers: the samples at node t (device idx, atomics
// order), the exact split of an explicit subset (host outputs), and the
// moving-horizon driver itself.
mh_status launch_compact(Ctx *ctx, const uint32_t *node_of, uint32_t n, uint32_t t, uint32_t *idx);
mh_status split1_subset(Ctx *ctx, const mh_dataset *ds, const uint32_t *idx, uint32_t n_sub,
                        uint8_t *feat, uint32_t *tau, uint32_t *correct);
typedef mh_status (*SolveNodeFn)(Ctx *, const mh_dataset *, const uint32_t *node_of, uint32_t t,
                                 uint32_t De, const mh_de_params *, const double *warm,
                                 uint32_t W, uint8_t *feat, uint32_t *tau);
typedef mh_status (*SolveAllFn)(Ctx *, const mh_dataset *, uint32_t D, const mh_de_params *,
                                const double *warm, uint32_t W, mh_tree *out);
mh_status mh_train_impl(Ctx *ctx, const mh_dataset *ds, uint32_t D, uint32_t D_MH,
                        const mh_de_params *prm, uint32_t flags, mh_tree *out,
                        SolveNodeFn solve_one, SolveAllFn solve_all);
// encode.hip: P trees (device [P][SB]) into genes (device [P][2 SB]).
mh_status launch_tree_encode(Ctx *ctx, const uint8_t *feat, const uint32_t *tau, uint32_t P,
                             uint32_t D, uint32_t F, const uint32_t *n_unique, double *genes);

}  // namespace mh

// The C ABI's context handle.
struct mh_ctx {
  mh::Ctx c;
};
