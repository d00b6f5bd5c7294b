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

size_t walk_scratch_bytes(uint32_t P, uint32_t D, uint32_t K) {
  return (size_t)P * ((size_t)1 << D) * K * 4;
}

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

constexpr uint32_t EPI_THREADS = 256;

// One tree's epilogue from its leaf counts [SL][K] (eq. opt_c, eq. opt_all
// and the soft-constraint fitness of Section 3.2), by a block of EPI_THREADS
// threads: labels (lowest class of the largest count, an empty leaf class
// 0), correct count and cost, and the counts cleared after they are read.
// COH: the counts were added by other blocks of the same launch (read with
// agent-scope loads).  Called by every thread of the block.  (Scoring a
// group's trees in the walk launch's last block instead of this separate
// launch was measured slower: that block's coherent loads ran one after
// another at the end of the launch.)
template <bool COH>
__device__ __forceinline__ void leaf_epilogue_tree(uint32_t *__restrict__ leafcnt,
                                                   const uint8_t *__restrict__ feat, uint32_t r,
                                                   uint32_t D, uint32_t K, uint32_t n_min,
                                                   double alpha, const FitnessOut &out,
                                                   uint32_t (*s_red)[EPI_THREADS / 64]) {
  const uint32_t SB = (1u << D) - 1u, SL = 1u << D;
  uint32_t correct = 0, nviol = 0, nsplit = 0, n_sub = 0;
  for (uint32_t l = threadIdx.x; l < SL; l += EPI_THREADS) {
    uint32_t *c = leafcnt + ((size_t)r * SL + l) * K;
    uint32_t best = 0, bk = 0, nl = 0;
    for (uint32_t k = 0; k < K; ++k) {
      const uint32_t v = cnt_load<COH>(c + k);
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
  __syncthreads();  // s_red may still be read from an earlier call
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

// ---------------------------------------------------------------------------
// Walk kernel (any depth): lane = sample.  A block owns a range of samples
// and a group of up to TG trees.  It stages its samples tile by tile in LDS
// (every rank column and the labels, coalesced 16-byte loads), then walks
// each tile through every tree of its group (Algorithm 1: t <- 2t if
// rank < tau else 2t + 1, D steps), adding one to the (tree, leaf, class)
// histogram in LDS; each tile is read from memory once for the whole group.
// A node is one 64-bit LDS word: tau above, and below the byte offset of its
// rank column in the tile (a no-split node reads column 0 with tau = 0, so
// every sample goes right).  A walk keeps the LDS address of its current
// node and advances it directly (node t at base + 8 (t - 1), so that child
// 2t + b sits at 2 addr - base + 8 + 8b).  With the tile in LDS as [F][T],
// lane i reads word f * T + i whatever feature its node splits on, so the
// rank reads of a wave never conflict.  Each thread walks GI trees at once
// (independent chains of dependent LDS reads).  The histogram goes to memory
// once per block (global atomics directly when it does not fit).  With many
// features (a tile of 256 samples over 48 KiB) only the labels are staged
// and the ranks are read from memory at each step (the node then holds the
// column index).
// ---------------------------------------------------------------------------
constexpr uint32_t WT_THREADS = 256;

struct WalkArgs {
  const uint32_t *ranks;
  uint32_t ld;
  const uint8_t *labels;
  const uint32_t *idx;
  uint32_t n_sub, n;
  const uint8_t *feat;
  const uint32_t *tau;
  uint32_t P, D, F, K;
  uint32_t T;       // samples per tile (a multiple of WT_THREADS)
  uint32_t TG;      // trees per block
  uint32_t ranges;  // sample ranges (gridDim.x)
  uint32_t hist_in_lds;
  uint32_t vec4;  // rank columns readable as 16-byte chunks (aligned, ld % 4 == 0)
  uint32_t *leafcnt;  // [P][2^D][K]
};

template <int IT, int GI, bool STAGED>
__global__ __launch_bounds__(WT_THREADS) void k_walk_tiles(WalkArgs a) {
  extern __shared__ __align__(16) uint32_t wl[];
  const uint32_t SB = (1u << a.D) - 1u, SL = 1u << a.D, T = a.T, K = a.K;
  const uint32_t FT = STAGED ? a.F * T : 0u;
  uint32_t *tile = wl;                                   // [F][T] when staged
  uint8_t *ylab = reinterpret_cast<uint8_t *>(wl + FT);  // [T]
  uint64_t *nodes = reinterpret_cast<uint64_t *>(wl + FT + T / 4);  // [TG][SB]
  uint32_t *hist = reinterpret_cast<uint32_t *>(nodes + (size_t)a.TG * SB);  // [TG][SL][K]
  // absolute LDS byte addresses
  const uint32_t lds0 = (uint32_t)(uintptr_t)((__attribute__((address_space(3))) uint32_t *)wl);
  const uint32_t node0 = lds0 + 4u * (FT + T / 4);
  const uint32_t r0 = blockIdx.y * a.TG;
  const uint32_t tg = min(a.TG, a.P - r0);
  // this block's trees: nodes into LDS, histogram cleared
  for (uint32_t e = threadIdx.x; e < tg * SB; e += WT_THREADS) {
    const uint32_t g = e / SB, t = e % SB;
    uint32_t f = a.feat[(size_t)(r0 + g) * SB + t];
    f = f <= a.F ? f : 0u;
    const uint32_t th = f ? a.tau[(size_t)(r0 + g) * SB + t] : 0u;
    const uint32_t col = f ? f - 1u : 0u;
    nodes[e] = ((uint64_t)th << 32) | (STAGED ? col * T * 4u : col);
  }
  if (a.hist_in_lds)
    for (uint32_t e = threadIdx.x; e < tg * SL * K; e += WT_THREADS) hist[e] = 0;
  // the block's sample range, in tiles (a whole number of tiles, so that
  // every tile starts at a multiple of 4 samples for the 16-byte loads)
  const uint32_t per = ((a.n_sub + a.ranges - 1) / a.ranges + T - 1) / T * T;
  const uint32_t s0 = blockIdx.x * per, s1 = min(a.n_sub, s0 + per);
  for (uint32_t base = s0; base < s1; base += T) {
    const uint32_t cnt = min(T, s1 - base);
    __syncthreads();  // the previous tile (and the node set-up) is done
    for (uint32_t i = threadIdx.x; i < T; i += WT_THREADS) {
      uint32_t y = 0xFFu;
      if (i < cnt) {
        const uint32_t smp = a.idx ? a.idx[base + i] : base + i;
        if (smp < a.n && a.labels[smp] < K) y = a.labels[smp];  // invalid samples are left out
      }
      ylab[i] = (uint8_t)y;
    }
    // the tile's ranks, SG loads in flight per thread before their stores
    constexpr uint32_t SG = 8;
    if (!STAGED) {
    } else if (a.idx) {
      for (uint32_t e0 = threadIdx.x; e0 < a.F * T; e0 += SG * WT_THREADS) {
        uint32_t v[SG];
#pragma unroll
        for (uint32_t u = 0; u < SG; ++u) {
          const uint32_t e = e0 + u * WT_THREADS, f = e / T, i = e % T;
          v[u] = 0;
          if (e < a.F * T && i < cnt) {
            const uint32_t smp = a.idx[base + i];
            if (smp < a.n) v[u] = a.ranks[(size_t)f * a.ld + smp];
          }
        }
#pragma unroll
        for (uint32_t u = 0; u < SG; ++u)
          if (e0 + u * WT_THREADS < a.F * T) tile[e0 + u * WT_THREADS] = v[u];
      }
    } else if (a.vec4 && cnt == T) {
      // whole tile, 16-byte chunks: chunk c is ranks 4i..4i+3 of column f
      const uint32_t T4 = T / 4, nch = a.F * T4;
      uint4 *tile4 = reinterpret_cast<uint4 *>(tile);
      for (uint32_t c0 = threadIdx.x; c0 < nch; c0 += SG * WT_THREADS) {
        uint4 v[SG];
#pragma unroll
        for (uint32_t u = 0; u < SG; ++u) {
          const uint32_t c = c0 + u * WT_THREADS;
          v[u] = make_uint4(0u, 0u, 0u, 0u);
          if (c < nch)
            v[u] = *reinterpret_cast<const uint4 *>(a.ranks + (size_t)(c / T4) * a.ld + base +
                                                    4u * (c % T4));
        }
#pragma unroll
        for (uint32_t u = 0; u < SG; ++u)
          if (c0 + u * WT_THREADS < nch) tile4[c0 + u * WT_THREADS] = v[u];
      }
    } else {
      for (uint32_t e0 = threadIdx.x; e0 < a.F * T; e0 += SG * WT_THREADS) {
        uint32_t v[SG];
#pragma unroll
        for (uint32_t u = 0; u < SG; ++u) {
          const uint32_t e = e0 + u * WT_THREADS, f = e / T, i = e % T;
          v[u] = (e < a.F * T && i < cnt) ? a.ranks[(size_t)f * a.ld + base + i] : 0u;
        }
#pragma unroll
        for (uint32_t u = 0; u < SG; ++u)
          if (e0 + u * WT_THREADS < a.F * T) tile[e0 + u * WT_THREADS] = v[u];
      }
    }
    __syncthreads();
    uint32_t yk[IT], sk[IT], lane_off[IT];
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      const uint32_t i = threadIdx.x + k * WT_THREADS;
      yk[k] = ylab[i];
      lane_off[k] = lds0 + 4u * i;  // the sample's rank in column 0
      // (unstaged ranks: the sample itself; in range whenever its label is valid)
      sk[k] = (!STAGED && yk[k] != 0xFFu) ? (a.idx ? a.idx[base + i] : base + i) : 0u;
    }
    // GI trees at a time; a group past the last tree repeats the last one
    // and leaves its count out
    for (uint32_t g0 = 0; g0 < tg; g0 += GI) {
      uint32_t nb[GI], na[GI][IT];
#pragma unroll
      for (int gg = 0; gg < GI; ++gg) {
        nb[gg] = node0 + 8u * SB * min(g0 + gg, tg - 1);
#pragma unroll
        for (int k = 0; k < IT; ++k) na[gg][k] = nb[gg];
      }
      for (uint32_t lv = 0; lv < a.D; ++lv) {
#pragma unroll
        for (int gg = 0; gg < GI; ++gg) {
#pragma unroll
          for (int k = 0; k < IT; ++k) {
            const uint64_t w = lds_rd64(na[gg][k]);
            const uint32_t lo = (uint32_t)w, th = (uint32_t)(w >> 32);
            const uint32_t rk =
                STAGED ? lds_rd32(lo + lane_off[k]) : a.ranks[(size_t)lo * a.ld + sk[k]];
            na[gg][k] = 2u * na[gg][k] - nb[gg] + (rk < th ? 8u : 16u);
          }
        }
      }
#pragma unroll
      for (int gg = 0; gg < GI; ++gg) {
        const uint32_t g = g0 + gg;
        if (g >= tg) continue;
#pragma unroll
        for (int k = 0; k < IT; ++k) {
          if (yk[k] == 0xFFu) continue;
          const uint32_t leaf = (na[gg][k] - nb[gg]) / 8u + 1u - SL;
          const uint32_t e = leaf * K + yk[k];
          if (a.hist_in_lds)
            atomicAdd(&hist[(size_t)g * SL * K + e], 1u);
          else
            atomicAdd(&a.leafcnt[(size_t)(r0 + g) * SL * K + e], 1u);
        }
      }
    }
  }
  if (a.hist_in_lds) {
    __syncthreads();
    for (uint32_t e = threadIdx.x; e < tg * SL * K; e += WT_THREADS)
      if (hist[e]) atomicAdd(&a.leafcnt[(size_t)r0 * SL * K + e], hist[e]);
  }
}

// Epilogue from leaf counts (walk path), any depth.  Block per tree: the
// threads share out the leaves (and the nodes for the split count) and the
// integer sums meet in a block reduction, so the result does not depend on
// the order.
__global__ __launch_bounds__(EPI_THREADS) void k_epilogue_leaves(
    uint32_t *__restrict__ leafcnt, const uint8_t *__restrict__ feat, uint32_t P, uint32_t D,
    uint32_t K, uint32_t n_min, double alpha, FitnessOut out) {
  __shared__ uint32_t s_red[4][EPI_THREADS / 64];
  if (blockIdx.x >= P) return;
  leaf_epilogue_tree<false>(leafcnt, feat, blockIdx.x, D, K, n_min, alpha, out, s_red);
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
  const uint32_t SB = (1u << D) - 1u, SL = 1u << D, K = ds->K, F = ds->F;
  const size_t cells = (size_t)P * SL * K;
  // only the context's own buffer is known to stay clear between calls (a
  // caller's scratch may have held anything since)
  const size_t bytes = walk_scratch_bytes(P, D, K);
  const bool own = leafcnt == nullptr;
  if (own) leafcnt = (uint32_t *)arena_get(ctx, "walk_leafcnt", bytes);
  if (!leafcnt) return MH_ENOMEM;
  hipStream_t st = ctx->stream;
  if (!(own && ctx->walk_zero == leafcnt && ctx->walk_zero_bytes >= bytes))
    if (mh_status zs = launch_zero(ctx, {{leafcnt, bytes}})) return zs;
  if (own) ctx->walk_zero = nullptr;
  if (n_sub > 0 && P > 0 && ds->n > 0) {
    WalkArgs a;
    a.ranks = ds->ranks;
    a.ld = ds->ld;
    a.labels = ds->labels;
    a.idx = idx;
    a.n_sub = n_sub;
    a.n = ds->n;
    a.feat = feat;
    a.tau = tau;
    a.P = P;
    a.D = D;
    a.F = F;
    a.K = K;
    a.leafcnt = leafcnt;
    a.vec4 = (ds->ld % 4 == 0 && ((uintptr_t)ds->ranks & 15u) == 0) ? 1u : 0u;
    // LDS: the tile ([F][T] ranks and T labels), TG trees' nodes and, when
    // it fits, their histograms, within a budget that leaves three blocks per
    // CU; samples per thread: tiles of at most 16 KiB where the features allow
    size_t budget = std::max<size_t>(48 * 1024, (ctx->max_lds - 4096) / 3);
    if (ctx->walk_lds) budget = ctx->walk_lds;
    const bool staged = (size_t)F * WT_THREADS * 4 <= 48 * 1024;
    uint32_t IT = 4;
    while (IT > 1 && (size_t)F * WT_THREADS * IT * 4 > 16 * 1024) IT /= 2;
    if (ctx->walk_it == 1 || ctx->walk_it == 2 || ctx->walk_it == 4) IT = ctx->walk_it;
    a.T = WT_THREADS * IT;
    const size_t tile_bytes = (staged ? (size_t)F * a.T * 4 : 0) + a.T;
    const size_t tree_nodes = (size_t)SB * 8, tree_hist = (size_t)SL * K * 4;
    a.hist_in_lds = 1;
    size_t TG = budget > tile_bytes ? (budget - tile_bytes) / (tree_nodes + tree_hist) : 0;
    if (TG == 0) {
      // histograms in memory: the nodes alone decide the trees per block
      a.hist_in_lds = 0;
      TG = budget > tile_bytes ? (budget - tile_bytes) / tree_nodes : 1;
    }
    TG = std::max<size_t>(1, std::min<size_t>({TG, 32, P}));
    // trees walked together per thread: 8, or 4 for small groups; a group
    // is a whole number of them where it can be
    const uint32_t GI = TG >= 8 ? 8u : 4u;
    if (TG > GI) TG -= TG % GI;
    a.TG = (uint32_t)TG;
    const uint32_t groups = (P + a.TG - 1) / a.TG;
    const size_t lds =
        tile_bytes + TG * tree_nodes + (a.hist_in_lds ? TG * tree_hist : 0);
    const size_t lds_al = (lds + 15) & ~(size_t)15;
    // sample ranges: one round of resident blocks in all, at least one tile
    // each
    const uint32_t per_cu = std::max<uint32_t>(
        1u, std::min<uint32_t>(8u, (uint32_t)(ctx->max_lds / std::max<size_t>(lds_al, 1))));
    const uint32_t want = per_cu * (uint32_t)ctx->num_cu;
    const uint32_t tiles = (n_sub + a.T - 1) / a.T;
    a.ranges = std::max(1u, std::min(tiles, want / groups));
    // a multiple of 8 ranges puts every block of one range on the same XCD
    // (blocks go round-robin over the 8 XCDs in launch order), so each XCD's
    // L2 holds only its ranges' ranks
    if (a.ranges >= 8) a.ranges &= ~7u;
    hipEvent_t e0, e1;
    const bool timed = prof_pair(ctx, &e0, &e1);
    const dim3 grid(a.ranges, groups);
#define MH_WALK2(ITV, GIV)                                                                  \
  if (staged)                                                                               \
    hipExtLaunchKernelGGL(k_walk_tiles<ITV, GIV, true>, grid, dim3(WT_THREADS), lds_al, st,  \
                          e0, e1, 0, a);                                                    \
  else                                                                                      \
    hipExtLaunchKernelGGL(k_walk_tiles<ITV, GIV, false>, grid, dim3(WT_THREADS), lds_al, st, \
                          e0, e1, 0, a);
#define MH_WALK(ITV)    \
  if (GI == 8) {        \
    MH_WALK2(ITV, 8)    \
  } else {              \
    MH_WALK2(ITV, 4)    \
  }
    if (IT == 4) {
      MH_WALK(4)
    } else if (IT == 2) {
      MH_WALK(2)
    } else {
      MH_WALK(1)
    }
#undef MH_WALK
#undef MH_WALK2
    MH_LAUNCHED(ctx, "k_walk_tiles");
    if (timed) ctx->prof_launches += 1;
    ctx->prof_evals += (uint64_t)n_sub * P;
  }
  if (P > 0) {
    k_epilogue_leaves<<<P, EPI_THREADS, 0, st>>>(leafcnt, feat, P, D, K, n_min, alpha, out);
    MH_LAUNCHED(ctx, "k_epilogue_leaves");
  }
  // (the epilogue read and cleared every count of the P trees)
  if (own && P > 0) {
    ctx->walk_zero = leafcnt;
    ctx->walk_zero_bytes = bytes;
  }
  return MH_OK;
}

}  // namespace mh
