// persist.hip -- a whole DEOCT run (Algorithm 4) of one problem as a single
// cooperative launch.
//
// Every block evaluates its share of the tiles for all P trees (lane = tree,
// as in the per-generation fitness kernel) and adds its left counts into a
// device counter set.  After a grid barrier, every block reads all counts and
// runs the same epilogue, selection, argmin and mutation for the whole
// population, redundantly: the DE state is a few kilobytes and identical
// arithmetic on identical inputs gives every block the same next population,
// so the counts are the only data that cross blocks.  Thread r keeps
// individual r (parent genes, trial genes, cost) in registers, and the
// post-selection population sits in LDS for the mutation's parent reads.
//
// Counters rotate over three copies: generation g adds into copy g % 3, all
// blocks read it between barriers g and g + 1, and each block zeroes its share
// of copy (g + 1) % 3 during generation g (that copy was last read before
// barrier g - 1 and is next added into after barrier g).  Cross-block data
// (counts, the barrier words) moves only through device-scope atomics and
// agent-scope loads; each wave waits for its own atomics before arriving at a
// barrier.  A barrier wait gives up after a bounded number of polls and
// raises the error flag instead of spinning forever.
//
// The results are those of the per-generation kernels: the same epilogue,
// the same selection and argmin rules, the same random draws and float64
// operations.
#include <hip/hip_runtime.h>

#include <cfloat>

#include "device_common.h"
#include "epilogue.h"
#include "fitness_core.h"
#include "internal.h"

namespace mh {
namespace {

struct PersistArgs {
  const TileHdr *hdr;        // tile set of the problem (one subproblem)
  const uint32_t *n_unique;  // [F]
  double *pop;               // gene-major [m][P]: initial population in, final out
  double *cost;              // [P] out
  uint32_t *best;            // [1] out
  uint32_t *cnt;             // 3 copies of [SB][K][Ppad], zero on entry
  uint32_t *bar;             // barrier arrivals, zero on entry
  uint32_t *err;             // non-zero after a barrier wait gave up
  double M, CR, alpha;
  uint64_t seed, prob;
  uint32_t P, G, n_min, F, K;
};

// A barrier wait gives up after this many ticks of the device wall clock
// (2 s at its usual 100 MHz), or at once when another block already gave up.
constexpr uint64_t WAIT_LIMIT_TICKS = 200000000ull;

// Barrier words, each on its own 256-byte line: [0] arrivals of group
// leaders, [64] release (the number of completed barriers), [128 + 64 g]
// arrivals in group g of BAR_GROUP consecutive blocks.  A block arrives at its
// group; the last arrival of a group arrives at the top; the last top arrival
// publishes the release.  Spreading the arrivals over separate words avoids
// serialising every block on one address.
constexpr uint32_t BAR_GROUP = 16;
__host__ __device__ __forceinline__ uint32_t barrier_words(uint32_t blocks) {
  return 128 + 64 * ((blocks + BAR_GROUP - 1) / BAR_GROUP);
}

// Barrier number k (0-based) of a launch with gridDim.x blocks.
__device__ __forceinline__ void grid_barrier(uint32_t *bar, uint32_t k, uint32_t *err) {
  __builtin_amdgcn_s_waitcnt(0);  // vmcnt(0) expcnt(0) lgkmcnt(0): this wave's atomics are done
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t grp = blockIdx.x / BAR_GROUP;
    const uint32_t gsize = min(BAR_GROUP, gridDim.x - grp * BAR_GROUP);
    const uint32_t ngroups = (gridDim.x + BAR_GROUP - 1) / BAR_GROUP;
    uint32_t *top = bar, *rel = bar + 64;
    const uint32_t old = __hip_atomic_fetch_add(bar + 128 + 64 * grp, 1u, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
    if (old == (k + 1) * gsize - 1) {
      const uint32_t o2 = __hip_atomic_fetch_add(top, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (o2 == (k + 1) * ngroups - 1)
        __hip_atomic_store(rel, k + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const uint64_t t0 = wall_clock64();
    while (__hip_atomic_load(rel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < k + 1) {
      if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
          wall_clock64() - t0 > WAIT_LIMIT_TICKS) {
        __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
  }
  __syncthreads();
}

__host__ __device__ __forceinline__ uint32_t align16u(uint32_t x) { return (x + 15u) & ~15u; }

// LDS: staged tile | rows [m][P] f64 | n_unique [F] | argmin scratch
__host__ __device__ __forceinline__ uint32_t persist_lds_bytes(uint32_t F, uint32_t P, uint32_t m) {
  const uint32_t tile = align16u(mask_region(F) + F * MCOL);
  return tile + align16u(m * P * 8) + align16u(F * 4) + 16 * 8 + 16 * 4;
}

template <int D, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_deoct_persist(PersistArgs pa) {
  constexpr int SB = (1 << D) - 1, SL = 1 << D, m = 2 * SB;
  constexpr uint32_t NT = WAVES * 64;
  extern __shared__ __align__(16) uint8_t lds[];
  const uint32_t P = pa.P, Ppad = pad64(P), K = pa.K, F = pa.F, r = threadIdx.x;
  const bool live = r < P;
  const uint32_t rr = live ? r : 0u;

  const uint8_t *base = reinterpret_cast<const uint8_t *>(pa.hdr);
  const uint32_t n_tiles = pa.hdr->n_tiles;
  const uint32_t *__restrict__ info = reinterpret_cast<const uint32_t *>(base + pa.hdr->off_info);
  const uint8_t *__restrict__ data = base + pa.hdr->off_data;
  const uint32_t *__restrict__ ctot = reinterpret_cast<const uint32_t *>(base + pa.hdr->off_ctot);
  const size_t rec_bytes = tile_bytes(F);
  const uint32_t nchunk = 48u * F;
  const uint32_t t_begin = (uint32_t)((uint64_t)n_tiles * blockIdx.x / gridDim.x);
  const uint32_t t_end = (uint32_t)((uint64_t)n_tiles * (blockIdx.x + 1) / gridDim.x);

  const uint32_t mregion = mask_region(F);
  const uint32_t tile_lds = align16u(mregion + F * MCOL);
  double *rows = reinterpret_cast<double *>(lds + tile_lds);
  uint32_t *s_nu = reinterpret_cast<uint32_t *>(lds + tile_lds + align16u(m * P * 8));
  double *s_cost = reinterpret_cast<double *>(reinterpret_cast<uint8_t *>(s_nu) + align16u(F * 4));
  uint32_t *s_idx = reinterpret_cast<uint32_t *>(s_cost + 16);
  const uint32_t s0 = (uint32_t)(uintptr_t)((__attribute__((address_space(3))) uint8_t *)lds);
  const uint32_t kmask = s0 + mregion - 2u * s0;

  for (uint32_t f = threadIdx.x; f < F; f += NT) s_nu[f] = pa.n_unique[f];
  double gp[m], gt[m];
#pragma unroll
  for (int q = 0; q < m; ++q) gp[q] = pa.pop[(size_t)q * P + rr];
  __syncthreads();

  NodeState<D> ns;
  uint32_t nsplit = 0;
  auto set_tree = [&](const double (&gen)[m]) {
    nsplit = 0;
#pragma unroll
    for (int t = 0; t < SB; ++t) {
      uint32_t f = 0, th = 0;
      if (live) decode_node(gen[t], gen[SB + t], F, s_nu, f, th);
      ns.col[t] = s0 + (f ? f - 1u : 0u) * SCOL;
      ns.thr[t] = f ? th : 0u;
      nsplit += f != 0;
    }
  };
  set_tree(gp);

  const size_t cstride = (size_t)SB * K * Ppad;
  const uint64_t key = de_key(pa.seed, pa.prob);
  double cost_r = 0.0;
  uint4 pf[PF];
  auto prefetch = [&](uint32_t tile) {
    const uint4 *__restrict__ src = reinterpret_cast<const uint4 *>(data + (size_t)tile * rec_bytes);
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      const uint32_t c = threadIdx.x + k * NT;
      if (c < nchunk) pf[k] = src[c];
    }
  };
  if (t_begin < t_end) prefetch(t_begin);

  for (uint32_t g = 0; g <= pa.G; ++g) {
    uint32_t *cnt = pa.cnt + (size_t)(g % 3) * cstride;
    {
      uint32_t *z = pa.cnt + (size_t)((g + 1) % 3) * cstride;
      for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < cstride; i += (size_t)gridDim.x * NT)
        __hip_atomic_store(z + i, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }

    // ---- counts of this block's tiles
#pragma unroll
    for (int t = 0; t < SB; ++t) ns.acc[t] = 0;
    uint32_t cur_cls = 0xFFFFFFFFu;
    auto flush = [&]() {
      if (!live) return;
      uint32_t *c = cnt + (size_t)cur_cls * Ppad + r;
#pragma unroll
      for (int t = 0; t < SB; ++t) {
        if (ns.acc[t]) atomicAdd(c + (size_t)t * K * Ppad, ns.acc[t]);
        ns.acc[t] = 0;
      }
    };
    for (uint32_t tile = t_begin; tile < t_end; ++tile) {
      const uint32_t inf = info[tile];
      const uint32_t cls = (inf >> 8) & 0xFFu, count = inf & 0xFFu;
      if (cls != cur_cls) {
        if (cur_cls != 0xFFFFFFFFu) flush();
        cur_cls = cls;
      }
      __syncthreads();  // the previous tile is no longer read
#pragma unroll
      for (int k = 0; k < PF; ++k) {
        const uint32_t c = threadIdx.x + k * NT;
        if (c < nchunk) stage_chunk(lds, mregion, F, c, pf[k]);
      }
      if (nchunk > PF * NT) {
        const uint4 *__restrict__ src =
            reinterpret_cast<const uint4 *>(data + (size_t)tile * rec_bytes);
        for (uint32_t c = threadIdx.x + PF * NT; c < nchunk; c += NT)
          stage_chunk(lds, mregion, F, c, src[c]);
      }
      __syncthreads();
      // the next tile, or this block's first tile again for the next
      // generation (the layout does not change)
      prefetch(tile + 1 < t_end ? tile + 1 : t_begin);
      uint64_t R[1 << D];
      R[1] = (1ull << count) - 1ull;  // count <= 63
      eval_nodes<D, 1>(kmask, ns, R);
    }
    if (cur_cls != 0xFFFFFFFFu) flush();
    grid_barrier(pa.bar, g, pa.err);

    // ---- epilogue (eq. opt_all and the soft-constraint fitness)
    uint32_t nl[SL], bl[SL], n_sub = 0;
#pragma unroll
    for (int l = 0; l < SL; ++l) nl[l] = bl[l] = 0;
    for (uint32_t k = 0; k < K; ++k) {
      uint32_t reach[2 * SL];
      reach[1] = ctot[k];
      n_sub += reach[1];
#pragma unroll
      for (int t = 1; t <= SB; ++t) {
        const uint32_t left = cnt_load<true>(cnt + ((size_t)(t - 1) * K + k) * Ppad + rr);
        reach[2 * t] = left;
        reach[2 * t + 1] = reach[t] - left;
      }
#pragma unroll
      for (int l = 0; l < SL; ++l) {
        const uint32_t v = reach[SL + l];
        nl[l] += v;
        bl[l] = v > bl[l] ? v : bl[l];
      }
    }
    uint32_t correct = 0, nviol = 0;
#pragma unroll
    for (int l = 0; l < SL; ++l) {
      correct += bl[l];
      nviol += (nl[l] > 0 && nl[l] < pa.n_min) ? 1u : 0u;
    }
    double tc = (double)(n_sub - correct);
    tc = __dadd_rn(tc, __dmul_rn(pa.alpha, (double)nsplit));
    tc = __dadd_rn(tc, (double)nviol);

    // ---- selection (eq. selection; the trial wins ties), or the initial cost
    if (g == 0) {
      cost_r = tc;
    } else if (tc <= cost_r) {
      cost_r = tc;
#pragma unroll
      for (int q = 0; q < m; ++q) gp[q] = gt[q];
    }
    if (live) {
#pragma unroll
      for (int q = 0; q < m; ++q) rows[(size_t)q * P + r] = gp[q];
    }

    // ---- best: lowest index of the minimum cost
    double bc = live ? cost_r : DBL_MAX;
    uint32_t bi = r;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const double c2 = __shfl_xor(bc, o, 64);
      const uint32_t i2 = __shfl_xor(bi, o, 64);
      if (c2 < bc || (c2 == bc && i2 < bi)) {
        bc = c2;
        bi = i2;
      }
    }
    if ((threadIdx.x & 63u) == 0) {
      s_cost[threadIdx.x >> 6] = bc;
      s_idx[threadIdx.x >> 6] = bi;
    }
    __syncthreads();
    bc = s_cost[0];
    bi = s_idx[0];
#pragma unroll
    for (uint32_t x = 1; x < WAVES; ++x) {
      const double c2 = s_cost[x];
      const uint32_t i2 = s_idx[x];
      if (c2 < bc || (c2 == bc && i2 < bi)) {
        bc = c2;
        bi = i2;
      }
    }
    const uint32_t bst = bi;
    if (g == pa.G) {
      if (blockIdx.x == 0) {
        if (live) {
#pragma unroll
          for (int q = 0; q < m; ++q) pa.pop[(size_t)q * P + r] = gp[q];
          pa.cost[r] = cost_r;
        }
        if (threadIdx.x == 0) pa.best[0] = bst;
      }
      break;
    }

    // ---- DE/best/1 mutation and binomial crossover of generation g + 1
    if (live) {
      const uint32_t gg = g + 1;
      const double Mr = pa.M >= 0.0 ? pa.M : to_unit(de_draw(key, gg, r, 0));
      uint32_t r1 = to_below(de_draw(key, gg, r, 1), P - 1u);
      r1 += (r1 >= r) ? 1u : 0u;
      uint32_t r2 = to_below(de_draw(key, gg, r, 2), P - 2u);
      const uint32_t lo = r < r1 ? r : r1, hi = r < r1 ? r1 : r;
      r2 += (r2 >= lo) ? 1u : 0u;
      r2 += (r2 >= hi) ? 1u : 0u;
      const uint32_t qr = to_below(de_draw(key, gg, r, 3), m);
      const double Fp1 = (double)F + 1.0;
#pragma unroll
      for (int q = 0; q < m; ++q) {
        const double d = __dsub_rn(rows[(size_t)q * P + r1], rows[(size_t)q * P + r2]);
        double v = __dadd_rn(rows[(size_t)q * P + bst], __dmul_rn(Mr, d));
        const double hiq = q >= SB ? 1.0 : Fp1;
        if (!(v >= 0.0)) v = 0.0;
        if (v > hiq) v = hiq;
        const double u = to_unit(de_draw(key, gg, r, 4u + q));
        gt[q] = (u <= pa.CR || (uint32_t)q == qr) ? v : gp[q];
      }
    }
    set_tree(gt);
    __syncthreads();  // rows and the argmin scratch are rewritten next generation
  }
}

// Blocks per CU: the per-generation exchange (count atomics, barrier, count
// reads) grows with the block count, the tile work shrinks with it.  Measured
// at depth 3 (F = 16, P = 128 and 256, n = 5e4 .. 4e6): about 4 waves per CU
// while a CU has up to 8 tiles, then 4 more waves per further 8 tiles, up to
// 16 waves.
uint32_t persist_bpc(uint32_t max_tiles, uint32_t num_cu, uint32_t waves) {
  const uint32_t per_cu = (max_tiles + num_cu - 1) / num_cu;
  uint32_t target = 4u * ((per_cu + 7u) / 8u);
  target = target < 4u ? 4u : (target > 16u ? 16u : target);
  const uint32_t bpc = target / waves;
  return bpc ? bpc : 1u;
}

template <int D, int WAVES>
mh_status launch_w(Ctx *ctx, const PersistArgs &pa, uint32_t lds, uint32_t max_tiles, bool *used) {
  auto kern = k_deoct_persist<D, WAVES>;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, WAVES * 64, lds) != hipSuccess ||
      per_cu < 1)
    return MH_OK;  // not co-resident: the caller takes the per-generation kernels
  uint32_t bpc = ctx->persist_blocks_per_cu
                     ? ctx->persist_blocks_per_cu
                     : persist_bpc(max_tiles, (uint32_t)ctx->num_cu, WAVES);
  bpc = bpc < (uint32_t)per_cu ? bpc : (uint32_t)per_cu;
  bpc = bpc > 8u ? 8u : bpc;
  const uint32_t grid = (uint32_t)ctx->num_cu * (bpc ? bpc : 1u);
  PersistArgs a = pa;
  void *args[] = {&a};
  hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void *>(kern), dim3(grid),
                                            dim3(WAVES * 64), args, lds, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "k_deoct_persist");
  *used = true;
  return MH_OK;
}

template <int D>
mh_status launch_d(Ctx *ctx, uint32_t waves, const PersistArgs &pa, uint32_t lds,
                   uint32_t max_tiles, bool *used) {
  switch (waves) {
    case 1: return launch_w<D, 1>(ctx, pa, lds, max_tiles, used);
    case 2: return launch_w<D, 2>(ctx, pa, lds, max_tiles, used);
    case 4: return launch_w<D, 4>(ctx, pa, lds, max_tiles, used);
    default: return launch_w<D, 8>(ctx, pa, lds, max_tiles, used);
  }
}

}  // namespace

mh_status launch_deoct_persist(Ctx *ctx, const void *tiles, uint32_t F, uint32_t K,
                               uint32_t n_sub, uint32_t D, const mh_de_params *prm, uint64_t prob,
                               const uint32_t *n_unique, double *pop, double *cost,
                               uint32_t *best, uint32_t *err, bool *used) {
  *used = false;
  const uint32_t P = prm->P, SB = (1u << D) - 1u, m = 2 * SB;
  if (!ctx->coop || D < 1 || D > 5 || P > 512 || F > 80) return MH_OK;
  // barrier targets (G + 1) * blocks must fit the 32-bit arrival counters
  if ((uint64_t)(prm->G + 1) * (uint64_t)ctx->num_cu * 8u >= (1ull << 31)) return MH_OK;
  const uint32_t lds = persist_lds_bytes(F, P, m);
  if (lds > 64u * 1024u) return MH_OK;
  uint32_t waves = pad64(P) / 64;
  waves = waves > 4 ? 8 : (waves > 2 ? 4 : waves);
  const size_t cstride = (size_t)SB * K * pad64(P);
  uint32_t *cnt = (uint32_t *)arena_get(ctx, "ps_cnt", 3 * cstride * 4);
  const size_t bar_bytes = (size_t)barrier_words((uint32_t)ctx->num_cu * 8u) * 4;
  uint32_t *bar = (uint32_t *)arena_get(ctx, "ps_bar", bar_bytes);
  if (!cnt || !bar) return MH_ENOMEM;
  hipStream_t st = ctx->stream;
  MH_HIP(ctx, hipMemsetAsync(cnt, 0, 3 * cstride * 4, st));
  MH_HIP(ctx, hipMemsetAsync(bar, 0, bar_bytes, st));
  MH_HIP(ctx, hipMemsetAsync(err, 0, 4, st));
  PersistArgs pa;
  pa.hdr = reinterpret_cast<const TileHdr *>(tiles);
  pa.n_unique = n_unique;
  pa.pop = pop;
  pa.cost = cost;
  pa.best = best;
  pa.cnt = cnt;
  pa.bar = bar;
  pa.err = err;
  pa.M = prm->M;
  pa.CR = prm->CR;
  pa.alpha = prm->alpha;
  pa.seed = prm->seed;
  pa.prob = prob;
  pa.P = P;
  pa.G = prm->G;
  pa.n_min = prm->n_min;
  pa.F = F;
  pa.K = K;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const bool timed = prof_pair(ctx, &e0, &e1);
  if (timed) MH_HIP(ctx, hipEventRecord(e0, st));
  mh_status s = MH_OK;
  const uint32_t max_tiles = tile_layout(n_sub, F, K, 1).max_tiles;
  switch (D) {
    case 1: s = launch_d<1>(ctx, waves, pa, lds, max_tiles, used); break;
    case 2: s = launch_d<2>(ctx, waves, pa, lds, max_tiles, used); break;
    case 3: s = launch_d<3>(ctx, waves, pa, lds, max_tiles, used); break;
    case 4: s = launch_d<4>(ctx, waves, pa, lds, max_tiles, used); break;
    default: s = launch_d<5>(ctx, waves, pa, lds, max_tiles, used); break;
  }
  if (s) return s;
  if (timed) {
    MH_HIP(ctx, hipEventRecord(e1, st));
    if (*used) ctx->prof_launches += 1;
  }
  if (*used) ctx->prof_evals += (uint64_t)(prm->G + 1) * n_sub * P;
  return MH_OK;
}

}  // namespace mh
