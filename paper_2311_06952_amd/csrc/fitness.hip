// fitness.hip -- population fitness of classification trees (Algorithm 1;
// eq. opt_c; eq. opt_all; the soft-constraint fitness of Section 3.2).
//
// Main kernel (depth 1..5): lane = tree, 64 trees per wave, all trees of the
// block sharing one LDS-staged tile of up to 63 same-class samples.  For each
// branch node the lane finds c = #{tile ranks < tau} of its feature by a
// 6-step binary search over the tile's sorted column and takes the prefix
// mask pm[c] = the tile samples going left.  The samples reaching node t are
// a 64-bit mask R_t: R_1 = the tile, R_2t = R_t & pm, R_2t+1 = R_t & ~pm.  The
// lane accumulates popcount(R_t & pm) per node in registers; since the tile
// is single-class these are the per-(tree, node, class) left counts, and the
// leaf counts follow from them and the class totals in the epilogue:
// reach(1) = N_k, reach(2t) = left(t), reach(2t+1) = reach(t) - left(t).
//
// Walk kernel (any depth 1..10): lane = sample, the Algorithm 1 walk of one
// tree at a time with an LDS histogram per (leaf, class).
#include <hip/hip_ext.h>

#include "de_body.h"
#include "device_common.h"
#include "epilogue.h"
#include "fitness_core.h"
#include "internal.h"

namespace mh {

size_t cnt_bytes(uint32_t n_problems, uint32_t D, uint32_t K, uint32_t P) {
  return CNT_REP * cnt_copy_elems(n_problems, (1u << D) - 1u, K, P) * 4;
}

namespace {

// After its last flush, a block of the fused kernel takes a ticket on every
// problem its tiles touched; the block that completes a problem's count (all
// blocks covering its tiles have flushed) runs that problem's epilogue and
// DE step at once, with its threads as the individuals and the tile buffer as
// scratch.  The counts are the only data that cross blocks inside a launch
// and are device-coherent atomics: every wave waits for its atomics to
// complete before the ticket is taken, and the finishing block reads the
// counts with agent-scope loads (no L2 write-back or invalidate needed).
template <int D, int WAVES>
__device__ __forceinline__ void fused_tail(const FuseArgs &fa, const uint32_t *__restrict__ info,
                                           uint32_t n_tiles, uint32_t t_begin, uint32_t t_end,
                                           uint32_t K, uint8_t *lds) {
  constexpr int SB = (1 << D) - 1;
  constexpr uint32_t NT = WAVES * 64;
  __shared__ uint32_t s_last;
  const uint32_t P = fa.a.P, Ppad = pad64(P), nb = gridDim.x;
  __builtin_amdgcn_s_waitcnt(0);  // vmcnt(0) expcnt(0) lgkmcnt(0): this wave's atomics are done
  __syncthreads();
  const uint32_t s_lo = info[t_begin] >> 16, s_hi = info[t_end - 1] >> 16;
  // scratch carved from the (now free) dynamic LDS
  double *s_cost = reinterpret_cast<double *>(lds);
  uint32_t *s_idx = reinterpret_cast<uint32_t *>(lds + NT * 8);
  uint32_t *s_nu = reinterpret_cast<uint32_t *>(lds + NT * 12);
  double *rows = fa.rows_in_lds ? reinterpret_cast<double *>(lds + NT * 12 + 1024) : nullptr;
  for (uint32_t s = s_lo; s <= s_hi; ++s) {
    if (threadIdx.x == 0) {
      const uint32_t t0 = fa.segoff[s * K], t1 = fa.segoff[s * K + K];
      // blocks covering tiles [t0, t1): block b covers [T b / nb, T (b + 1) / nb),
      // at least one tile each when nb <= T, at most one when nb > T
      uint32_t covering;
      if (nb > n_tiles) {
        covering = t1 - t0;
      } else {
        const uint32_t bf = (uint32_t)(((uint64_t)(t0 + 1) * nb - 1) / n_tiles);
        const uint32_t bl = (uint32_t)(((uint64_t)t1 * nb - 1) / n_tiles);
        covering = bl - bf + 1;
      }
      const uint32_t expected = covering * gridDim.y;
      const uint32_t old = atomicAdd(&fa.done[s], 1u);
      s_last = (old + 1 == expected) ? 1u : 0u;
      if (s_last) fa.done[s] = 0;  // nobody else touches it in this launch
    }
    __syncthreads();
    if (s_last) de_gen_body<D, CNT_REP, true, false>(fa.a, fa.e, s, s_cost, s_idx, rows, s_nu);
    __syncthreads();
  }
}

// One block's share of a population evaluation on one tile set: block bx of
// nbx takes tiles [n_tiles bx / nbx, n_tiles (bx + 1) / nbx) for the trees
// by * NT .. by * NT + NT - 1.
template <int D, int WAVES, bool FUSE>
__device__ __forceinline__ void fitness_block(const TileHdr *__restrict__ hdr,
                                              const uint8_t *__restrict__ feat,
                                              const uint32_t *__restrict__ tau, uint32_t P,
                                              uint32_t *__restrict__ cnt, const FuseArgs &fa,
                                              uint32_t bx, uint32_t nbx, uint32_t by,
                                              uint8_t *lds) {
  constexpr int SB = (1 << D) - 1;
  constexpr uint32_t NT = WAVES * 64;
  const uint8_t *base = reinterpret_cast<const uint8_t *>(hdr);
  const uint32_t F = hdr->F, K = hdr->K;
  const uint32_t n_tiles = hdr->n_tiles;
  const uint32_t t_begin = (uint32_t)((uint64_t)n_tiles * bx / nbx);
  const uint32_t t_end = (uint32_t)((uint64_t)n_tiles * (bx + 1) / nbx);
  if (t_begin >= t_end) return;
  const uint32_t *__restrict__ info = reinterpret_cast<const uint32_t *>(base + hdr->off_info);
  const uint8_t *__restrict__ data = base + hdr->off_data;
  const size_t rec_bytes = tile_bytes(F);
  const uint32_t nchunk = 48u * F;
  const uint32_t r = by * NT + threadIdx.x;
  const bool live = r < P;
  const uint32_t Ppad = pad64(P);
  const uint32_t mregion = mask_region(F);
  // absolute LDS addresses: sorted column f at s0 + f * SCOL; after the
  // search a = s0 + f * SCOL + 4c, and pm[c] of column f is at kmask + 2a
  const uint32_t s0 = (uint32_t)(uintptr_t)((__attribute__((address_space(3))) uint8_t *)lds);
  const uint32_t kmask = s0 + mregion - 2u * s0;

  NodeState<D> ns;
  uint32_t cur_sub = 0xFFFFFFFFu, cur_cls = 0xFFFFFFFFu;
#pragma unroll
  for (int t = 0; t < SB; ++t) ns.acc[t] = 0;

  uint32_t *const cnt_rep =
      cnt + (bx % CNT_REP) * cnt_copy_elems(hdr->n_problems, SB, K, P);
  auto flush = [&](uint32_t sub, uint32_t cls) {
    if (!live) return;
    uint32_t *c = cnt_rep + ((size_t)sub * SB * K + cls) * Ppad + r;
#pragma unroll
    for (int t = 0; t < SB; ++t) {
      if (ns.acc[t]) atomicAdd(c + (size_t)t * K * Ppad, ns.acc[t]);
      ns.acc[t] = 0;
    }
  };

  uint4 pf[PF];
  auto prefetch = [&](uint32_t tile) {
    const uint4 *__restrict__ src = reinterpret_cast<const uint4 *>(data + (size_t)tile * rec_bytes);
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      const uint32_t c = threadIdx.x + k * NT;
      if (c < nchunk) pf[k] = src[c];
    }
  };
  // the next tile's info word travels with its prefetch
  prefetch(t_begin);
  uint32_t inf_next = info[t_begin];

  for (uint32_t tile = t_begin; tile < t_end; ++tile) {
    const uint32_t inf = inf_next;
    const uint32_t sub = inf >> 16, cls = (inf >> 8) & 0xFFu, count = inf & 0xFFu;
    if (sub != cur_sub || cls != cur_cls) {
      if (cur_sub != 0xFFFFFFFFu) flush(cur_sub, cur_cls);
      if (sub != cur_sub) {
        const uint8_t *fr = feat + ((size_t)sub * P + (live ? r : 0)) * SB;
        const uint32_t *tr = tau + ((size_t)sub * P + (live ? r : 0)) * SB;
#pragma unroll
        for (int t = 0; t < SB; ++t) {
          uint32_t f = live ? fr[t] : 0u;
          f = f <= F ? f : 0u;  // an out-of-range feature is treated as no split
          ns.col[t] = s0 + (f ? f - 1u : 0u) * SCOL;
          ns.thr[t] = f ? tr[t] : 0u;
        }
        // the parameters must have landed before the prefetch below is
        // issued, or every later wait would have to drain the prefetch too
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
      }
      cur_sub = sub;
      cur_cls = cls;
    }
    __syncthreads();  // the previous tile is no longer read
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      const uint32_t c = threadIdx.x + k * NT;
      if (c < nchunk) stage_chunk(lds, mregion, F, c, pf[k]);
    }
    if (nchunk > PF * NT) {  // wide rows: the rest without prefetch
      const uint4 *__restrict__ src =
          reinterpret_cast<const uint4 *>(data + (size_t)tile * rec_bytes);
      for (uint32_t c = threadIdx.x + PF * NT; c < nchunk; c += NT)
        stage_chunk(lds, mregion, F, c, src[c]);
    }
    __syncthreads();
    if (tile + 1 < t_end) {
      prefetch(tile + 1);
      inf_next = info[tile + 1];
    }
    uint64_t R[1 << D];
    R[1] = (1ull << count) - 1ull;  // count <= 63
    eval_nodes<D, 1>(kmask, ns, R);
  }
  flush(cur_sub, cur_cls);
  if constexpr (FUSE) {
    __syncthreads();  // the tile buffer becomes DE scratch
    fused_tail<D, WAVES>(fa, info, n_tiles, t_begin, t_end, K, lds);
  }
}

template <int D, int WAVES, bool FUSE>
__global__ __launch_bounds__(WAVES * 64) void k_fitness_bits(
    const TileHdr *__restrict__ hdr, const uint8_t *__restrict__ feat,
    const uint32_t *__restrict__ tau, uint32_t P, uint32_t *__restrict__ cnt, FuseArgs fa) {
  extern __shared__ __align__(16) uint8_t lds[];
  fitness_block<D, WAVES, FUSE>(hdr, feat, tau, P, cnt, fa, blockIdx.x, gridDim.x, blockIdx.y,
                                lds);
}

// Several independent population evaluations (one per job, each on its own
// tile set with its own trees and counters) in one launch: block b works for
// job job_of[b] as its block b - blk0 of nblk.  Every job's population fits
// one block (P <= WAVES * 64).
template <int D, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_fitness_jobs(const FitJob *__restrict__ jobs,
                                                             const uint16_t *__restrict__ job_of) {
  extern __shared__ __align__(16) uint8_t lds[];
  const FitJob jb = jobs[job_of[blockIdx.x]];
  fitness_block<D, WAVES, false>(jb.hdr, jb.feat, jb.tau, jb.P, jb.cnt, FuseArgs{},
                                 blockIdx.x - jb.blk0, jb.nblk, 0, lds);
}

// Epilogue from node left counts (tile path).  One thread per (sub, tree).
template <int D>
__global__ void k_epilogue_nodes(uint32_t *__restrict__ cnt, const uint32_t *__restrict__ ctot,
                                 const uint8_t *__restrict__ feat, uint32_t P, uint32_t K,
                                 uint32_t n_problems, uint32_t n_min, double alpha,
                                 FitnessOut out) {
  constexpr int SB = (1 << D) - 1, SL = 1 << D;
  const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= n_problems * P) return;
  const uint32_t sub = gid / P, r = gid % P;
  const uint32_t Ppad = pad64(P);
  const size_t tr = (size_t)sub * P + r;
  TreeScore sc = epilogue_node_counts<D, CNT_REP>(
      cnt + (size_t)sub * SB * K * Ppad, ctot + (size_t)sub * K, K, Ppad, r, feat + tr * SB,
      n_min, alpha, out.counts ? out.counts + tr * SL * K : nullptr,
      out.label ? out.label + tr * SL : nullptr, cnt_copy_elems(n_problems, SB, K, P));
  if (out.correct) out.correct[tr] = sc.correct;
  if (out.cost) out.cost[tr] = sc.cost;
}

// ---------------------------------------------------------------------------
// Walk kernel (any depth).  Block = 256 threads over a chunk of samples and
// every gridDim.y-th tree; for each tree: stage (feat, tau) in LDS, walk
// every sample of the chunk down the tree, histogram (leaf, class) in LDS,
// add the histogram to leafcnt.  The trees are spread over the grid's second
// dimension so that a small sample count still fills the chip.
// ---------------------------------------------------------------------------
constexpr uint32_t WALK_THREADS = 256;
constexpr uint32_t WALK_ITEMS = 8;

__global__ __launch_bounds__(WALK_THREADS) void k_fitness_walk(
    const uint32_t *__restrict__ ranks, uint32_t ld, const uint8_t *__restrict__ labels,
    const uint32_t *__restrict__ idx, uint32_t n_sub, const uint8_t *__restrict__ feat,
    const uint32_t *__restrict__ tau, uint32_t P, uint32_t D, uint32_t F, uint32_t K, uint32_t n,
    uint32_t *__restrict__ leafcnt, uint32_t hist_in_lds) {
  extern __shared__ __align__(16) uint32_t wl[];
  const uint32_t SB = (1u << D) - 1u, SL = 1u << D;
  uint32_t *s_feat = wl;
  uint32_t *s_tau = wl + SB;
  uint32_t *hist = wl + 2 * SB;
  constexpr uint32_t CHUNK = WALK_THREADS * WALK_ITEMS;
  const uint32_t n_chunks = (n_sub + CHUNK - 1) / CHUNK;
  for (uint32_t r = blockIdx.y; r < P; r += gridDim.y) {
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < SB; t += WALK_THREADS) {
      uint32_t f = feat[(size_t)r * SB + t];
      f = f <= F ? f : 0u;
      s_feat[t] = f;
      s_tau[t] = f ? tau[(size_t)r * SB + t] : 0u;
    }
    if (hist_in_lds)
      for (uint32_t e = threadIdx.x; e < SL * K; e += WALK_THREADS) hist[e] = 0;
    __syncthreads();
    uint32_t *dst = leafcnt + (size_t)r * SL * K;
    // every gridDim.x-th chunk of samples, all into the one LDS histogram
    for (uint32_t c = blockIdx.x; c < n_chunks; c += gridDim.x) {
      uint32_t ii[WALK_ITEMS];
      uint32_t yy[WALK_ITEMS];
#pragma unroll
      for (uint32_t k = 0; k < WALK_ITEMS; ++k) {
        const uint32_t j = c * CHUNK + k * WALK_THREADS + threadIdx.x;
        ii[k] = 0xFFFFFFFFu;
        yy[k] = 0;
        if (j < n_sub) {
          const uint32_t i = idx ? idx[j] : j;
          if (i < n && labels[i] < K) {  // invalid samples are left out
            ii[k] = i;
            yy[k] = labels[i];
          }
        }
      }
#pragma unroll
      for (uint32_t k = 0; k < WALK_ITEMS; ++k) {
        if (ii[k] == 0xFFFFFFFFu) continue;
        uint32_t t = 1;
        while (t <= SB) {
          uint32_t f = s_feat[t - 1];
          bool left = f != 0 && ranks[(size_t)(f - 1) * ld + ii[k]] < s_tau[t - 1];
          t = left ? 2 * t : 2 * t + 1;
        }
        uint32_t e = (t - SL) * K + yy[k];
        if (hist_in_lds)
          atomicAdd(&hist[e], 1u);
        else
          atomicAdd(&dst[e], 1u);
      }
    }
    if (hist_in_lds) {
      __syncthreads();
      for (uint32_t e = threadIdx.x; e < SL * K; e += WALK_THREADS)
        if (hist[e]) atomicAdd(&dst[e], hist[e]);
    }
  }
}

// Epilogue from leaf counts (walk path), any depth.  Block per tree: the
// threads share out the leaves (and the nodes for the split count) and the
// integer sums meet in a block reduction, so the result does not depend on
// the order.
constexpr uint32_t EPI_THREADS = 256;

__global__ __launch_bounds__(EPI_THREADS) void k_epilogue_leaves(
    uint32_t *__restrict__ leafcnt, const uint8_t *__restrict__ feat, uint32_t P, uint32_t D,
    uint32_t K, uint32_t n_min, double alpha, FitnessOut out) {
  __shared__ uint32_t s_red[4][EPI_THREADS / 64];
  const uint32_t r = blockIdx.x;
  if (r >= P) return;
  const uint32_t SB = (1u << D) - 1u, SL = 1u << D;
  uint32_t correct = 0, nviol = 0, nsplit = 0, n_sub = 0;
  for (uint32_t l = threadIdx.x; l < SL; l += EPI_THREADS) {
    uint32_t *c = leafcnt + ((size_t)r * SL + l) * K;
    uint32_t best = 0, bk = 0, nl = 0;
    for (uint32_t k = 0; k < K; ++k) {
      uint32_t v = c[k];
      c[k] = 0;
      if (out.counts) out.counts[((size_t)r * SL + l) * K + k] = v;
      nl += v;
      if (v > best) {
        best = v;
        bk = k;
      }
    }
    n_sub += nl;
    correct += best;
    nviol += (nl > 0 && nl < n_min) ? 1u : 0u;
    if (out.label) out.label[(size_t)r * SL + l] = (uint8_t)bk;
  }
  for (uint32_t t = threadIdx.x; t < SB; t += EPI_THREADS) nsplit += feat[(size_t)r * SB + t] != 0;
  uint32_t v4[4] = {correct, nviol, nsplit, n_sub};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    for (uint32_t o = 32; o > 0; o >>= 1) v4[q] += __shfl_xor(v4[q], o, 64);
    if ((threadIdx.x & 63u) == 0) s_red[q][threadIdx.x >> 6] = v4[q];
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int q = 0; q < 4; ++q) {
    v4[q] = 0;
    for (uint32_t w = 0; w < EPI_THREADS / 64; ++w) v4[q] += s_red[q][w];
  }
  correct = v4[0];
  nviol = v4[1];
  nsplit = v4[2];
  n_sub = v4[3];
  if (out.correct) out.correct[r] = correct;
  if (out.cost) {
    double v = (double)(n_sub - correct);
    v = __dadd_rn(v, __dmul_rn(alpha, (double)nsplit));
    v = __dadd_rn(v, (double)nviol);
    out.cost[r] = v;
  }
}

// Launches on st; when e0/e1 are given the launch records them at the
// kernel's start and end.
template <int D, int WAVES>
hipError_t launch_bits(const TileHdr *hdr, uint32_t F, uint32_t gx, uint32_t gy,
                       const uint8_t *feat, const uint32_t *tau, uint32_t P, uint32_t *cnt,
                       const FuseArgs *fa, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  size_t lds = (size_t)mask_region(F) + (size_t)F * MCOL;
  if (fa) {
    const size_t need = WAVES * 64 * 12 + 1024 +
                        (fa->rows_in_lds ? (size_t)P * 2 * ((1u << D) - 1u) * 8 : 0);
    lds = lds > need ? lds : need;
    hipExtLaunchKernelGGL((k_fitness_bits<D, WAVES, true>), dim3(gx, gy), dim3(WAVES * 64), lds,
                          st, e0, e1, 0, hdr, feat, tau, P, cnt, *fa);
  } else {
    hipExtLaunchKernelGGL((k_fitness_bits<D, WAVES, false>), dim3(gx, gy), dim3(WAVES * 64), lds,
                          st, e0, e1, 0, hdr, feat, tau, P, cnt, FuseArgs{});
  }
  return hipGetLastError();
}

template <int D>
hipError_t launch_bits_w(uint32_t waves, const TileHdr *hdr, uint32_t F, uint32_t gx, uint32_t gy,
                         const uint8_t *feat, const uint32_t *tau, uint32_t P, uint32_t *cnt,
                         const FuseArgs *fa, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  if (waves == 1) return launch_bits<D, 1>(hdr, F, gx, gy, feat, tau, P, cnt, fa, st, e0, e1);
  if (waves == 2) return launch_bits<D, 2>(hdr, F, gx, gy, feat, tau, P, cnt, fa, st, e0, e1);
  if (waves == 4) return launch_bits<D, 4>(hdr, F, gx, gy, feat, tau, P, cnt, fa, st, e0, e1);
  return launch_bits<D, 8>(hdr, F, gx, gy, feat, tau, P, cnt, fa, st, e0, e1);
}

template <int D>
void launch_epi(uint32_t *cnt, const uint32_t *ctot, const uint8_t *feat, uint32_t P, uint32_t K,
                uint32_t n_problems, uint32_t n_min, double alpha, const FitnessOut &out,
                hipStream_t st) {
  uint32_t n = n_problems * P;
  k_epilogue_nodes<D><<<(n + 127) / 128, 128, 0, st>>>(cnt, ctot, feat, P, K, n_problems, n_min,
                                                       alpha, out);
}

}  // namespace

// Block threads of the fitness kernel for population P, and the power of two
// (>= P, >= 64) the fused DE step needs.
uint32_t fitness_block_threads(uint32_t P) {
  uint32_t waves = pad64(P) / 64;
  waves = waves > 4 ? 8 : (waves > 2 ? 4 : waves);
  return waves * 64;
}
uint32_t fused_threads(uint32_t P) {
  uint32_t t = 64;
  while (t < P) t <<= 1;
  return t;
}

mh_status launch_fitness_count(Ctx *ctx, const void *tiles, uint32_t F, uint32_t K,
                               uint32_t n_sub, uint32_t n_problems, uint32_t max_tiles,
                               const uint8_t *feat, const uint32_t *tau, uint32_t P, uint32_t D,
                               uint32_t *cnt, const FuseArgs *fa) {
  if (D < 1 || D > 5) return fail(ctx, MH_EINVAL, "tile fitness kernel supports depth 1..5");
  const TileHdr *hdr = reinterpret_cast<const TileHdr *>(tiles);
  hipStream_t st = ctx->stream;
  const uint32_t Ppad = pad64(P);
  // one block covers up to 8 waves of 64 trees, so a tile is staged once for
  // populations up to 512
  uint32_t waves = Ppad / 64;
  waves = waves > 4 ? 8 : (waves > 2 ? 4 : waves);
  const uint32_t gy = (Ppad + waves * 64 - 1) / (waves * 64);
  // blocks: about blocks_per_cu per CU over all tree groups, each with at
  // least min_tiles tiles
  uint32_t want = (uint32_t)ctx->num_cu * ctx->fit_blocks_per_cu;
  want = (want + gy - 1) / gy;
  const uint32_t cap = (max_tiles + ctx->fit_min_tiles - 1) / ctx->fit_min_tiles;
  uint32_t gx = want < cap ? want : cap;
  if (gx == 0) gx = 1;
  if (fa && (gy != 1 || fused_threads(P) > waves * 64))
    return fail(ctx, MH_EINVAL, "fused fitness + DE needs one block per tile to hold every tree");
  hipEvent_t e0, e1;
  const bool timed = prof_pair(ctx, &e0, &e1);
  hipError_t e = hipSuccess;
  switch (D) {
    case 1: e = launch_bits_w<1>(waves, hdr, F, gx, gy, feat, tau, P, cnt, fa, st, e0, e1); break;
    case 2: e = launch_bits_w<2>(waves, hdr, F, gx, gy, feat, tau, P, cnt, fa, st, e0, e1); break;
    case 3: e = launch_bits_w<3>(waves, hdr, F, gx, gy, feat, tau, P, cnt, fa, st, e0, e1); break;
    case 4: e = launch_bits_w<4>(waves, hdr, F, gx, gy, feat, tau, P, cnt, fa, st, e0, e1); break;
    case 5: e = launch_bits_w<5>(waves, hdr, F, gx, gy, feat, tau, P, cnt, fa, st, e0, e1); break;
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "k_fitness_bits");
  if (timed) ctx->prof_launches += 1;
  ctx->prof_evals += (uint64_t)n_sub * P;
  ctx->prof_tiles += max_tiles;
  (void)K;
  (void)n_problems;
  return MH_OK;
}

mh_status launch_fitness_jobs(Ctx *ctx, uint32_t D, uint32_t waves, uint32_t F_max,
                              const FitJob *jobs, const uint16_t *job_of, uint32_t n_blocks) {
  if (n_blocks == 0) return MH_OK;
  const size_t lds = (size_t)mask_region(F_max) + (size_t)F_max * MCOL;
  hipStream_t st = ctx->stream;
  const dim3 grid(n_blocks), block(waves * 64);
#define MH_JOBS_W(DD)                                                                       \
  switch (waves) {                                                                          \
    case 1: k_fitness_jobs<DD, 1><<<grid, block, lds, st>>>(jobs, job_of); break;           \
    case 2: k_fitness_jobs<DD, 2><<<grid, block, lds, st>>>(jobs, job_of); break;           \
    case 4: k_fitness_jobs<DD, 4><<<grid, block, lds, st>>>(jobs, job_of); break;           \
    case 8: k_fitness_jobs<DD, 8><<<grid, block, lds, st>>>(jobs, job_of); break;           \
    default: return fail(ctx, MH_EINVAL, "fitness jobs: waves must be 1, 2, 4 or 8");      \
  }
  switch (D) {
    case 1: MH_JOBS_W(1) break;
    case 2: MH_JOBS_W(2) break;
    case 3: MH_JOBS_W(3) break;
    case 4: MH_JOBS_W(4) break;
    case 5: MH_JOBS_W(5) break;
    default: return fail(ctx, MH_EINVAL, "fitness jobs support depth 1..5");
  }
#undef MH_JOBS_W
  MH_LAUNCHED(ctx, "k_fitness_jobs");
  return MH_OK;
}

mh_status launch_fitness_epilogue(Ctx *ctx, const void *tiles, uint32_t F, uint32_t K,
                                  uint32_t n_sub, uint32_t n_problems, const uint8_t *feat,
                                  uint32_t P, uint32_t D, uint32_t n_min, double alpha,
                                  uint32_t *cnt, const FitnessOut &out) {
  const uint8_t *b = reinterpret_cast<const uint8_t *>(tiles);
  const TileHdr h = tile_layout(n_sub, F, K, n_problems);
  const uint32_t *ctot = reinterpret_cast<const uint32_t *>(b + h.off_ctot);
  hipStream_t st = ctx->stream;
  switch (D) {
    case 1: launch_epi<1>(cnt, ctot, feat, P, K, n_problems, n_min, alpha, out, st); break;
    case 2: launch_epi<2>(cnt, ctot, feat, P, K, n_problems, n_min, alpha, out, st); break;
    case 3: launch_epi<3>(cnt, ctot, feat, P, K, n_problems, n_min, alpha, out, st); break;
    case 4: launch_epi<4>(cnt, ctot, feat, P, K, n_problems, n_min, alpha, out, st); break;
    case 5: launch_epi<5>(cnt, ctot, feat, P, K, n_problems, n_min, alpha, out, st); break;
    default: return fail(ctx, MH_EINVAL, "tile epilogue supports depth 1..5");
  }
  MH_LAUNCHED(ctx, "k_epilogue_nodes");
  return MH_OK;
}

mh_status launch_fitness_tiles(Ctx *ctx, const void *tiles, uint32_t F, uint32_t K, uint32_t n_sub,
                               uint32_t n_problems, uint32_t max_tiles, const uint8_t *feat,
                               const uint32_t *tau, uint32_t P, uint32_t D, uint32_t n_min,
                               double alpha, uint32_t *cnt, const FitnessOut &out) {
  mh_status s = launch_fitness_count(ctx, tiles, F, K, n_sub, n_problems, max_tiles, feat, tau, P,
                                     D, cnt, nullptr);
  if (s) return s;
  return launch_fitness_epilogue(ctx, tiles, F, K, n_sub, n_problems, feat, P, D, n_min, alpha,
                                 cnt, out);
}

mh_status launch_fitness_walk(Ctx *ctx, const mh_dataset *ds, const uint32_t *idx, uint32_t n_sub,
                              const uint8_t *feat, const uint32_t *tau, uint32_t P, uint32_t D,
                              uint32_t n_min, double alpha, const FitnessOut &out,
                              uint32_t *leafcnt) {
  const uint32_t SB = (1u << D) - 1u, SL = 1u << D;
  const size_t cells = (size_t)P * SL * ds->K;
  if (!leafcnt) leafcnt = (uint32_t *)arena_get(ctx, "walk_leafcnt", cells * 4);
  if (!leafcnt) return MH_ENOMEM;
  hipStream_t st = ctx->stream;
  if (mh_status zs = launch_zero(ctx, {{leafcnt, cells * 4}})) return zs;
  const uint32_t hist_cells = SL * ds->K;
  const uint32_t in_lds = hist_cells <= 12288u ? 1u : 0u;
  size_t lds = (size_t)(2 * SB + (in_lds ? hist_cells : 0u)) * 4;
  if (n_sub > 0) {
    const uint32_t chunks = (n_sub + WALK_THREADS * WALK_ITEMS - 1) / (WALK_THREADS * WALK_ITEMS);
    // about 8 blocks per CU in all: one tree per block row where there are
    // enough trees, the chunks of samples shared out over the rest (each
    // block adds its histogram to memory once per tree)
    const uint32_t want = 8u * (uint32_t)ctx->num_cu;
    const uint32_t gy = std::max(1u, std::min(P, want));
    const uint32_t blocks = std::max(1u, std::min(chunks, (want + gy - 1) / gy));
    hipEvent_t e0, e1;
    const bool timed = prof_pair(ctx, &e0, &e1);
    hipExtLaunchKernelGGL(k_fitness_walk, dim3(blocks, gy), dim3(WALK_THREADS), lds, st, e0, e1, 0,
                          ds->ranks, ds->ld, ds->labels, idx, n_sub, feat, tau, P, D, ds->F,
                          ds->K, ds->n, leafcnt, in_lds);
    MH_LAUNCHED(ctx, "k_fitness_walk");
    if (timed) ctx->prof_launches += 1;
    ctx->prof_evals += (uint64_t)n_sub * P;
  }
  if (P > 0) {
    k_epilogue_leaves<<<P, EPI_THREADS, 0, st>>>(leafcnt, feat, P, D, ds->K, n_min, alpha, out);
    MH_LAUNCHED(ctx, "k_epilogue_leaves");
  }
  return MH_OK;
}

}  // namespace mh
