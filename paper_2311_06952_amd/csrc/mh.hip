// mh.hip -- the moving-horizon driver (Algorithm 2; Section 4) and the exact
// depth-1 split it uses at the last levels.
//
// The tree is grown level by level.  node_of[i] is the node sample i sits at
// (heap numbering); the subset of node t is {i : node_of[i] == t}.  Nodes of a
// level have disjoint subsets and depend only on their ancestors, so solving
// them one after another (Algorithm 2's order) or all at once gives the same
// tree: the batched form runs one multi-problem DEOCT (or one batched split)
// per level, the sequential form one per node.
#include <algorithm>
#include <cstring>
#include <vector>

#include "de_body.h"
#include "device_common.h"
#include "internal.h"

namespace mh {
namespace {

__global__ void k_fill_u32(uint32_t *__restrict__ p, uint32_t n, uint32_t v) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Class histogram of the nodes of one level: hist[(t - t0) * K + y] for
// samples with node_of in [t0, t0 + width).  Block-aggregated in LDS.
__global__ __launch_bounds__(256) void k_level_hist(const uint32_t *__restrict__ node_of,
                                                    const uint8_t *__restrict__ labels, uint32_t n,
                                                    uint32_t K, uint32_t t0, uint32_t width,
                                                    uint32_t span, uint32_t *__restrict__ hist,
                                                    int in_lds) {
  extern __shared__ uint32_t h[];
  const uint32_t cells = width * K;
  if (in_lds)
    for (uint32_t c = threadIdx.x; c < cells; c += blockDim.x) h[c] = 0;
  __syncthreads();
  const uint32_t j0 = blockIdx.x * span;
  const uint32_t j1 = (uint32_t)min((uint64_t)n, (uint64_t)j0 + span);  // no wrap near 2^32
  for (uint32_t i = j0 + threadIdx.x; i < j1; i += blockDim.x) {
    const uint32_t t = node_of[i], y = labels[i];
    if (t >= t0 && t - t0 < width && y < K) atomicAdd(in_lds ? &h[(t - t0) * K + y] : &hist[(t - t0) * K + y], 1u);
  }
  __syncthreads();
  if (in_lds)
    for (uint32_t c = threadIdx.x; c < cells; c += blockDim.x)
      if (h[c]) atomicAdd(&hist[c], h[c]);
}

// Subproblem of every sample: sub_map[t - t0] for samples at a node of the
// level, else n_problems (not in any).
__global__ void k_assign_sub(const uint32_t *__restrict__ node_of, uint32_t n, uint32_t t0,
                             uint32_t width, const uint32_t *__restrict__ sub_map,
                             uint32_t n_problems, uint32_t *__restrict__ sub_of) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t t = node_of[i];
  sub_of[i] = (t >= t0 && t - t0 < width) ? sub_map[t - t0] : n_problems;
}

// Move every sample at a node of the level to its child (Section 2: left iff
// the node splits and rank < tau; a node without a split sends all right).
__global__ void k_route_level(uint32_t *__restrict__ node_of, uint32_t n, uint32_t t0,
                              uint32_t width, const uint8_t *__restrict__ feat,
                              const uint32_t *__restrict__ tau, const uint32_t *__restrict__ ranks,
                              uint32_t ld, uint32_t F) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t t = node_of[i];
  if (t < t0 || t - t0 >= width) return;
  const uint32_t f = feat[t - 1];
  const bool left = f != 0 && f <= F && ranks[(size_t)(f - 1) * ld + i] < tau[t - 1];
  node_of[i] = left ? 2 * t : 2 * t + 1;
}

// ---------------------------------------------------------------------------
// Exact depth-1 split, batched over subsets.
//
// Every (sample, feature) of every subset becomes a key
// (subset, feature, rank) with the class as payload; after a radix sort a
// (subset, feature) segment lists the subset's ranks of that feature in order.
// With per-class inclusive counts P_k over the sorted array, a threshold right
// after position j (tau = rank_j + 1, taken where the rank changes) leaves
// L_k = P_k[j] - P_k[start - 1] samples of class k on the left; its correct
// count is max_k L_k + max_k (N_k - L_k).  The winner per subset is the first
// strict maximum in the order (no split, then feature, then tau): the largest
// correct count, ties to the smallest (feature, tau), and no split unless a
// split is strictly better.
//
// The same machinery gives CART's split (Gini impurity): the candidate's
// score is sum_k L_k^2 / |L| + sum_k R_k^2 / |R| in f64 (the integer sums of
// squares divided by the side sizes, then added, each correctly rounded), the
// winner the first strict maximum over (feature, tau); a subset splits iff it
// holds two or more classes and has a candidate.  Scores are positive, so
// their bit patterns order as u64.
// ---------------------------------------------------------------------------
// The chunk of samples [c0, min(c0 + 256, j1)) of a block's range: its
// members (pred true) are numbered in thread order, their count returned and,
// for member number l, put(l, i) called before the block's next barrier.
// Must be called by all threads of a 256-thread block with the same c0, j1.
template <typename Pred, typename Fn>
__device__ __forceinline__ uint32_t chunk_members(uint32_t c0, uint32_t j1, Pred pred, Fn put,
                                                  uint32_t *s_w) {
  const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  const uint32_t i = c0 + threadIdx.x;
  const bool m = i < j1 && pred(i);
  const uint64_t bal = __ballot(m);
  const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  __syncthreads();  // the previous chunk's readers of s_w and the staged members are done
  if (lane == 0) s_w[w] = (uint32_t)__popcll(bal);
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (uint32_t q = 0; q < 4; ++q) {
    off += q < w ? s_w[q] : 0u;
    tot += s_w[q];
  }
  if (m) put(off + (uint32_t)__popcll(bal & lt), i);
  return tot;
}

// Members of [j0, j1) (pred true), counted by a 256-thread block, and the
// start of their range from one add to *cursor.
template <typename Pred>
__device__ __forceinline__ uint32_t range_reserve(uint32_t j0, uint32_t j1, Pred pred,
                                                  uint32_t *__restrict__ cursor, uint32_t *s_w,
                                                  uint32_t *s_base) {
  uint32_t c = 0;
  for (uint32_t i = j0 + threadIdx.x; i < j1; i += 256u) c += pred(i) ? 1u : 0u;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x & 63u) == 0) s_w[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t t = s_w[0] + s_w[1] + s_w[2] + s_w[3];
    *s_base = t ? atomicAdd(cursor, t) : 0u;
  }
  __syncthreads();
  return *s_base;
}

// The elements of the subsets' members: key (subset << fbits | feature) << rb
// | rank (ranks below 2^rb), the class as value.  Block b takes the samples
// [b span, (b + 1) span): one global add reserves its members' elements,
// then each chunk of 256 samples is staged in LDS and written F elements per
// member in order, so that a wave's store covers 64 consecutive elements.
__global__ __launch_bounds__(256) void k_split_keys(
    const uint32_t *__restrict__ sub_of, uint32_t n, uint32_t nsub,
    const uint32_t *__restrict__ ranks, uint32_t ld, uint32_t F,
    const uint8_t *__restrict__ labels, uint32_t K, uint32_t span, uint32_t *__restrict__ cursor,
    uint64_t *__restrict__ keys, uint32_t *__restrict__ vals, uint32_t fbits, uint32_t rb) {
  __shared__ uint32_t s_w[4], s_base;
  __shared__ uint32_t s_i[256], s_s[256];
  __shared__ uint8_t s_y[256];
  const uint32_t j0 = blockIdx.x * span;
  const uint32_t j1 = (uint32_t)min((uint64_t)n, (uint64_t)j0 + span);  // no wrap near 2^32
  auto member = [&](uint32_t i) {
    const uint32_t s = sub_of ? sub_of[i] : 0u;
    return s < nsub && labels[i] < K;
  };
  uint32_t base = range_reserve(j0, j1, member, cursor, s_w, &s_base);
  for (uint32_t c0 = j0; c0 < j1; c0 += 256u) {
    const uint32_t tot = chunk_members(c0, j1, member, [&](uint32_t l, uint32_t i) {
      s_i[l] = i;
      s_s[l] = sub_of ? sub_of[i] : 0u;
      s_y[l] = labels[i];
    }, s_w);
    __syncthreads();
    const size_t e0 = (size_t)base * F;
    for (uint32_t e = threadIdx.x; e < tot * F; e += 256u) {
      const uint32_t q = e / F, f = e - q * F;
      const uint64_t sid = (uint64_t)s_s[q] << fbits | f;
      keys[e0 + e] = sid << rb | ranks[(size_t)f * ld + s_i[q]];
      vals[e0 + e] = s_y[q];
    }
    base += tot;
  }
}
// Per-class inclusive prefix counts over the sorted classes, all classes at
// once: pk[k][j] = #{i <= j : vals[i] == k}.  A block takes 1,024 positions,
// four rounds of 256 (round q, thread t: position 1024 b + 256 q + t); a
// wave's count of class k below a lane is the popcount of the class's ballot
// under the lane.  k_split_class_sums writes the block's count of each class
// (class-major, [k][block]); after one exclusive scan of them a class's base
// for block b is its scanned entry less the entry of block 0 (the counts of
// the classes before it).
constexpr uint32_t CP_ROUNDS = 4, CP_SPAN = 256 * CP_ROUNDS;
__global__ __launch_bounds__(256) void k_split_class_sums(const uint32_t *__restrict__ vals,
                                                          uint32_t N, uint32_t K, uint32_t nb,
                                                          uint32_t *__restrict__ sums) {
  extern __shared__ uint32_t s_cnt[];  // [K]
  for (uint32_t k = threadIdx.x; k < K; k += 256u) s_cnt[k] = 0;
  __syncthreads();
  const uint32_t j0 = blockIdx.x * CP_SPAN;
  uint32_t v[CP_ROUNDS];
#pragma unroll
  for (uint32_t q = 0; q < CP_ROUNDS; ++q) {
    const uint32_t j = j0 + q * 256u + threadIdx.x;
    v[q] = j < N ? vals[j] : 0xFFFFFFFFu;
  }
  if (K <= 16) {
    // few classes: a ballot per class and round, one LDS add per wave and
    // class (adds of a whole block to one of a few words would serialise)
    for (uint32_t k = 0; k < K; ++k) {
      uint32_t c = 0;
#pragma unroll
      for (uint32_t q = 0; q < CP_ROUNDS; ++q) c += (uint32_t)__popcll(__ballot(v[q] == k));
      if ((threadIdx.x & 63u) == 0 && c) atomicAdd(&s_cnt[k], c);
    }
  } else {
#pragma unroll
    for (uint32_t q = 0; q < CP_ROUNDS; ++q)
      if (v[q] < K) atomicAdd(&s_cnt[v[q]], 1u);
  }
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < K; k += 256u) sums[(size_t)k * nb + blockIdx.x] = s_cnt[k];
}
__global__ __launch_bounds__(256) void k_split_class_prefix(const uint32_t *__restrict__ vals,
                                                            uint32_t N, uint32_t K, uint32_t nb,
                                                            const uint32_t *__restrict__ scanned,
                                                            uint32_t *__restrict__ pk) {
  extern __shared__ uint32_t s_w[];  // [CP_ROUNDS][K][4]: wave totals per round and class
  const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  const uint32_t j0 = blockIdx.x * CP_SPAN;
  uint32_t v[CP_ROUNDS];
#pragma unroll
  for (uint32_t q = 0; q < CP_ROUNDS; ++q) {
    const uint32_t j = j0 + q * 256u + threadIdx.x;
    v[q] = j < N ? vals[j] : 0xFFFFFFFFu;
  }
  for (uint32_t k = 0; k < K; ++k)
#pragma unroll
    for (uint32_t q = 0; q < CP_ROUNDS; ++q) {
      const uint64_t bal = __ballot(v[q] == k);
      if (lane == 0) s_w[(q * K + k) * 4 + w] = (uint32_t)__popcll(bal);
    }
  __syncthreads();
  for (uint32_t k = 0; k < K; ++k) {
    uint32_t run = scanned[(size_t)k * nb + blockIdx.x] - scanned[(size_t)k * nb];
#pragma unroll
    for (uint32_t q = 0; q < CP_ROUNDS; ++q) {
      const uint32_t *t = s_w + (q * K + k) * 4;
      const uint64_t bal = __ballot(v[q] == k);
      uint32_t below = 0;
#pragma unroll
      for (uint32_t x = 0; x < 4; ++x) below += x < w ? t[x] : 0u;
      const uint32_t j = j0 + q * 256u + threadIdx.x;
      if (j < N)
        pk[(size_t)k * N + j] = run + below + (uint32_t)__popcll(bal & lt) + (v[q] == k ? 1u : 0u);
      run += t[0] + t[1] + t[2] + t[3];
    }
  }
}

__global__ void k_split_bounds(const uint64_t *__restrict__ keys, uint32_t N, uint32_t rb,
                               uint32_t *__restrict__ seg_lo, uint32_t *__restrict__ seg_hi) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const uint64_t sid = keys[j] >> rb;
  if (j == 0 || (keys[j - 1] >> rb) != sid) seg_lo[sid] = j;
  if (j == N - 1 || (keys[j + 1] >> rb) != sid) seg_hi[sid] = j;
}

__device__ __forceinline__ uint32_t split_correct(const uint32_t *__restrict__ pk, uint32_t N,
                                                  uint32_t K, uint32_t lo, uint32_t j,
                                                  uint32_t hi) {
  uint32_t ml = 0, mr = 0;
  for (uint32_t k = 0; k < K; ++k) {
    const uint32_t *p = pk + (size_t)k * N;
    const uint32_t base = lo ? p[lo - 1] : 0u;
    const uint32_t L = p[j] - base, T = p[hi] - base;
    ml = L > ml ? L : ml;
    mr = T - L > mr ? T - L : mr;
  }
  return ml + mr;
}

__device__ __forceinline__ uint64_t split_gini_bits(const uint32_t *__restrict__ pk, uint32_t N,
                                                    uint32_t K, uint32_t lo, uint32_t j,
                                                    uint32_t hi) {
  uint64_t A = 0, B = 0;
  for (uint32_t k = 0; k < K; ++k) {
    const uint32_t *p = pk + (size_t)k * N;
    const uint32_t base = lo ? p[lo - 1] : 0u;
    const uint64_t L = p[j] - base, R = p[hi] - base - (uint32_t)L;
    A += L * L;
    B += R * R;
  }
  const double g = __dadd_rn(__ddiv_rn((double)A, (double)(j + 1 - lo)),
                             __ddiv_rn((double)B, (double)(hi - j)));
  return (uint64_t)__double_as_longlong(g);
}

// Pass 0 raises the subset's best score to c, pass 1 lowers its best (feature
// + 1, tau) to ft, each only when the value read is not already as good.
__device__ __forceinline__ void split_improve(uint32_t pass, unsigned long long *best_c,
                                              unsigned long long *best_ft, uint64_t c,
                                              uint64_t ft) {
  if (pass == 0) {
    if (c > __hip_atomic_load(best_c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicMax(best_c, (unsigned long long)c);
  } else {
    if (ft < __hip_atomic_load(best_ft, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicMin(best_ft, (unsigned long long)ft);
  }
}

// pass 1: the best score per subset (atomicMax over candidates): the correct
// count (GINI false) or the Gini score's bits (GINI true).
// pass 2: the smallest (feature + 1, tau) among candidates attaining it.
template <bool GINI>
__global__ void k_split_eval(const uint64_t *__restrict__ keys, uint32_t N,
                             const uint32_t *__restrict__ pk, uint32_t K,
                             const uint32_t *__restrict__ seg_lo, const uint32_t *__restrict__ seg_hi,
                             uint32_t fbits, uint32_t rb, uint32_t pass,
                             unsigned long long *__restrict__ best_c,
                             unsigned long long *__restrict__ best_ft) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  bool cand = false;
  uint32_t s = 0xFFFFFFFFu;
  uint64_t c = 0, ft = ~0ull;
  if (j < N) {
    const uint64_t key = keys[j], rmask = (1ull << rb) - 1u;
    const uint64_t sid = key >> rb;
    const uint32_t hi = seg_hi[sid];
    s = (uint32_t)(sid >> fbits);
    // a boundary: the rank changes between j and j + 1 inside the segment
    if (j != hi && (keys[j + 1] & rmask) != (key & rmask)) {
      const uint32_t f = (uint32_t)(sid & ((1u << fbits) - 1u));
      c = GINI ? split_gini_bits(pk, N, K, seg_lo[sid], j, hi)
               : (uint64_t)split_correct(pk, N, K, seg_lo[sid], j, hi);
      ft = ((uint64_t)(f + 1) << 32) | ((key & rmask) + 1);
      cand = pass == 0 || c == best_c[s];
    }
  }
  // most waves see one subset: reduce in the wave, one atomic per wave
  const uint32_t s0 = __shfl(s, 0, 64);
  const bool uniform = __ballot(j < N && s != s0) == 0ull;
  const bool any_cand = __ballot(cand) != 0ull;
  if (uniform) {
    uint64_t vc = cand ? c : 0u;
    uint64_t vf = cand ? ft : ~0ull;
    for (int d = 32; d > 0; d >>= 1) {
      const uint64_t oc = __shfl_xor(vc, d, 64);
      const uint64_t of = __shfl_xor(vf, d, 64);
      vc = oc > vc ? oc : vc;
      vf = of < vf ? of : vf;
    }
    // (only a wave that can improve the subset's value updates it: most waves
    // of a large subset see a value already better and skip the contended
    // atomic; a stale read only costs an atomic that changes nothing)
    if ((threadIdx.x & 63u) == 0 && s0 != 0xFFFFFFFFu && any_cand)
      split_improve(pass, best_c + s0, best_ft + s0, vc, vf);
  } else if (cand) {
    split_improve(pass, best_c + s, best_ft + s, c, ft);
  }
}

__global__ void k_split_init(const uint32_t *__restrict__ tot, uint32_t nsub, uint32_t K,
                             uint32_t gini, unsigned long long *__restrict__ best_c,
                             unsigned long long *__restrict__ best_ft) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsub) return;
  uint32_t m = 0;
  for (uint32_t k = 0; k < K; ++k) m = tot[(size_t)s * K + k] > m ? tot[(size_t)s * K + k] : m;
  best_c[s] = gini ? 0ull : m;  // no split (misclassification) / no candidate (Gini)
  best_ft[s] = ~0ull;           // no split unless a split is strictly better
}

__global__ void k_split_final(const uint32_t *__restrict__ tot, uint32_t nsub, uint32_t K,
                              uint32_t gini, const unsigned long long *__restrict__ best_c,
                              const unsigned long long *__restrict__ best_ft, uint8_t *__restrict__ feat,
                              uint32_t *__restrict__ tau, uint32_t *__restrict__ correct) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsub) return;
  uint32_t m = 0, classes = 0;
  for (uint32_t k = 0; k < K; ++k) {
    const uint32_t v = tot[(size_t)s * K + k];
    m = v > m ? v : m;
    classes += v ? 1u : 0u;
  }
  const uint64_t ft = best_ft[s];
  const bool split = gini ? (classes > 1 && ft != ~0ull) : (best_c[s] > m && ft != ~0ull);
  if (split) {
    feat[s] = (uint8_t)(ft >> 32);
    tau[s] = (uint32_t)ft;
  } else {
    feat[s] = 0;
    tau[s] = 0;
  }
  if (correct) correct[s] = gini ? 0u : (uint32_t)best_c[s];
}

// Scatter the root node of each problem's best tree into the full tree.
__global__ void k_put_roots(const uint8_t *__restrict__ f1, const uint32_t *__restrict__ t1,
                            uint32_t SB1, const uint32_t *__restrict__ nodes, uint32_t cnt,
                            uint8_t *__restrict__ feat, uint32_t *__restrict__ tau) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= cnt) return;
  feat[nodes[s] - 1] = f1[(size_t)s * SB1];
  tau[nodes[s] - 1] = t1[(size_t)s * SB1];
}

inline uint32_t nblk(uint32_t n, uint32_t b = 256) { return (n + b - 1) / b; }
// Samples per block of the range kernels (k_compact, k_split_keys): a
// multiple of 256, about two blocks per CU; and the blocks that cover n.
// Their loops step by 256 without wrapping for n <= RANGE_MAX_N.
constexpr uint32_t RANGE_MAX_N = 0xFFFFFF00u;
inline uint32_t range_span(const Ctx *ctx, uint32_t n) {
  const uint64_t nb = 2u * (uint64_t)(ctx->num_cu > 0 ? ctx->num_cu : 1);
  const uint64_t s = ((((uint64_t)n + nb - 1) / nb) + 255) / 256 * 256;
  return (uint32_t)(s < 256 ? 256 : s);
}
inline uint32_t range_blocks(uint32_t n, uint32_t span) {
  return (uint32_t)(((uint64_t)n + span - 1) / span);
}

// Samples at node t, in whatever order the block adds give (the counts of a
// subset do not depend on the order of its samples).  Block b takes the
// samples [b span, (b + 1) span) and reserves their slots with one add.
__global__ __launch_bounds__(256) void k_compact(const uint32_t *__restrict__ node_of, uint32_t n,
                                                 uint32_t t, uint32_t span,
                                                 uint32_t *__restrict__ cursor,
                                                 uint32_t *__restrict__ idx) {
  __shared__ uint32_t s_w[4], s_base;
  const uint32_t j0 = blockIdx.x * span;
  const uint32_t j1 = (uint32_t)min((uint64_t)n, (uint64_t)j0 + span);  // no wrap near 2^32
  auto in = [&](uint32_t i) { return node_of[i] == t; };
  uint32_t base = range_reserve(j0, j1, in, cursor, s_w, &s_base);
  for (uint32_t c0 = j0; c0 < j1; c0 += 256u)
    base += chunk_members(c0, j1, in, [&](uint32_t l, uint32_t i) { idx[base + l] = i; }, s_w);
}

// sub_of for an explicit subset: 0 for idx members, 1 for the rest; and the
// subset's class totals, counted per block in LDS (one global add per block
// and class: a million samples over a few classes would otherwise serialise
// on a few addresses).
__global__ __launch_bounds__(256) void k_mark_subset(const uint32_t *__restrict__ idx,
                                                     uint32_t n_sub, uint32_t n,
                                                     const uint8_t *__restrict__ labels,
                                                     uint32_t K, uint32_t *__restrict__ sub_of,
                                                     uint32_t *__restrict__ tot) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n_sub) {
    const uint32_t i = idx ? idx[j] : j;
    // a repeated index counts once
    if (i < n && labels[i] < K && atomicExch(&sub_of[i], 0u) != 0u) atomicAdd(&h[labels[i]], 1u);
  }
  __syncthreads();
  if (threadIdx.x < K && h[threadIdx.x]) atomicAdd(&tot[threadIdx.x], h[threadIdx.x]);
}

// ---------------------------------------------------------------------------
// CART of depth D on each of nsub subsets at once, level by level: loc[i] is
// the node (heap numbering inside its subset's tree) sample i sits at; the
// nodes of a level are split subproblems s = sub 2^l + (u - 2^l) of the
// Gini split above.
// ---------------------------------------------------------------------------
__global__ void k_cart_sub(const uint32_t *__restrict__ sub_of, uint32_t n, uint32_t nsub,
                           const uint32_t *__restrict__ loc, uint32_t l,
                           uint32_t *__restrict__ sub_l) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t s = sub_of[i];
  sub_l[i] = s < nsub ? (s << l) + loc[i] - (1u << l) : nsub << l;
}

__global__ void k_cart_put(const uint8_t *__restrict__ fl, const uint32_t *__restrict__ tl,
                           uint32_t cnt, uint32_t l, uint32_t SB, uint8_t *__restrict__ feat,
                           uint32_t *__restrict__ tau) {
  const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= cnt) return;
  const uint32_t sub = q >> l, u = (1u << l) + (q & ((1u << l) - 1u));
  feat[(size_t)sub * SB + u - 1] = fl[q];
  tau[(size_t)sub * SB + u - 1] = tl[q];
}

__global__ void k_cart_route(const uint32_t *__restrict__ sub_of, uint32_t n, uint32_t nsub,
                             uint32_t *__restrict__ loc, uint32_t l,
                             const uint8_t *__restrict__ fl, const uint32_t *__restrict__ tl,
                             const uint32_t *__restrict__ ranks, uint32_t ld, uint32_t F) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t s = sub_of[i];
  if (s >= nsub) return;
  const uint32_t u = loc[i], q = (s << l) + u - (1u << l);
  const uint32_t f = fl[q];
  const bool left = f != 0 && f <= F && ranks[(size_t)(f - 1) * ld + i] < tl[q];
  loc[i] = left ? 2 * u : 2 * u + 1;
}

}  // namespace

mh_status cart_batched(Ctx *ctx, const mh_dataset *ds, const uint32_t *sub_of, uint32_t nsub,
                       uint32_t D, uint8_t *feat, uint32_t *tau) {
  hipStream_t st = ctx->stream;
  const uint32_t n = ds->n, K = ds->K, SB = (1u << D) - 1u;
  if (nsub == 0) return MH_OK;
  const size_t maxq = (size_t)nsub << (D - 1);
  uint32_t *loc = (uint32_t *)arena_get(ctx, "ct_loc", (size_t)(n ? n : 1) * 4);
  uint32_t *sub_l = (uint32_t *)arena_get(ctx, "ct_sub", (size_t)(n ? n : 1) * 4);
  uint32_t *hist = (uint32_t *)arena_get(ctx, "ct_hist", maxq * K * 4);
  uint8_t *fl = (uint8_t *)arena_get(ctx, "ct_f", maxq);
  uint32_t *tl = (uint32_t *)arena_get(ctx, "ct_t", maxq * 4);
  if (!loc || !sub_l || !hist || !fl || !tl) return MH_ENOMEM;
  if (maxq > 0xFFFFFFFFull / 2) return fail(ctx, MH_EINVAL, "CART: too many subsets");
  if (n) {
    k_fill_u32<<<nblk(n), 256, 0, st>>>(loc, n, 1u);
    MH_LAUNCHED(ctx, "k_fill_u32");
  }
  for (uint32_t l = 0; l < D; ++l) {
    const uint32_t cnt = nsub << l;
    MH_HIP(ctx, hipMemsetAsync(hist, 0, (size_t)cnt * K * 4, st));
    if (n) {
      k_cart_sub<<<nblk(n), 256, 0, st>>>(sub_of, n, nsub, loc, l, sub_l);
      MH_LAUNCHED(ctx, "k_cart_sub");
      const bool in_lds = (size_t)cnt * K * 4 <= 32768;
      if (n > RANGE_MAX_N) return fail(ctx, MH_EINVAL, "too many samples for the level counts");
      const uint32_t span = range_span(ctx, n);
      k_level_hist<<<range_blocks(n, span), 256, in_lds ? (size_t)cnt * K * 4 : 0, st>>>(
          sub_l, ds->labels, n, K, 0, cnt, span, hist, in_lds ? 1 : 0);
      MH_LAUNCHED(ctx, "k_level_hist");
    }
    mh_status s = launch_split1(ctx, ds, sub_l, cnt, hist, fl, tl, nullptr, true);
    if (s) return s;
    k_cart_put<<<nblk(cnt), 256, 0, st>>>(fl, tl, cnt, l, SB, feat, tau);
    MH_LAUNCHED(ctx, "k_cart_put");
    if (l + 1 < D && n) {
      k_cart_route<<<nblk(n), 256, 0, st>>>(sub_of, n, nsub, loc, l, fl, tl, ds->ranks, ds->ld,
                                            ds->F);
      MH_LAUNCHED(ctx, "k_cart_route");
    }
  }
  return MH_OK;
}

mh_status cart_subset(Ctx *ctx, const mh_dataset *ds, const uint32_t *idx, uint32_t n_sub,
                      uint32_t D, uint8_t *feat, uint32_t *tau) {
  hipStream_t st = ctx->stream;
  const uint32_t n = ds->n, SB = (1u << D) - 1u;
  uint32_t *sub_of = (uint32_t *)arena_get(ctx, "s1_sub_of", (size_t)(n ? n : 1) * 4);
  uint32_t *tot = (uint32_t *)arena_get(ctx, "s1_tot", (size_t)ds->K * 4);
  uint8_t *f = (uint8_t *)arena_get(ctx, "ct_tree_f", SB);
  uint32_t *t = (uint32_t *)arena_get(ctx, "ct_tree_t", (size_t)SB * 4);
  if (!sub_of || !tot || !f || !t) return MH_ENOMEM;
  MH_HIP(ctx, hipMemsetAsync(tot, 0, (size_t)ds->K * 4, st));
  if (n) {
    k_fill_u32<<<nblk(n), 256, 0, st>>>(sub_of, n, 1u);
    MH_LAUNCHED(ctx, "k_fill_u32");
  }
  if (n_sub) {
    k_mark_subset<<<nblk(n_sub), 256, 0, st>>>(idx, n_sub, n, ds->labels, ds->K, sub_of, tot);
    MH_LAUNCHED(ctx, "k_mark_subset");
  }
  mh_status s = cart_batched(ctx, ds, sub_of, 1, D, f, t);
  if (s) return s;
  MH_HIP(ctx, hipMemcpyAsync(feat, f, SB, hipMemcpyDeviceToHost, st));
  MH_HIP(ctx, hipMemcpyAsync(tau, t, (size_t)SB * 4, hipMemcpyDeviceToHost, st));
  MH_HIP(ctx, hipStreamSynchronize(st));
  return MH_OK;
}

mh_status launch_compact(Ctx *ctx, const uint32_t *node_of, uint32_t n, uint32_t t, uint32_t *idx) {
  uint32_t *cursor = (uint32_t *)arena_get(ctx, "mh_cursor", 256);
  if (!cursor) return MH_ENOMEM;
  MH_HIP(ctx, hipMemsetAsync(cursor, 0, 4, ctx->stream));
  if (n > RANGE_MAX_N) return fail(ctx, MH_EINVAL, "too many samples for the compaction");
  if (n) {
    const uint32_t span = range_span(ctx, n);
    k_compact<<<range_blocks(n, span), 256, 0, ctx->stream>>>(node_of, n, t, span, cursor, idx);
    MH_LAUNCHED(ctx, "k_compact");
  }
  return MH_OK;
}

mh_status split1_subset(Ctx *ctx, const mh_dataset *ds, const uint32_t *idx, uint32_t n_sub,
                        uint8_t *feat, uint32_t *tau, uint32_t *correct) {
  hipStream_t st = ctx->stream;
  const uint32_t n = ds->n;
  uint32_t *sub_of = (uint32_t *)arena_get(ctx, "s1_sub_of", (size_t)(n ? n : 1) * 4);
  uint32_t *tot = (uint32_t *)arena_get(ctx, "s1_tot", (size_t)ds->K * 4);
  uint8_t *f = (uint8_t *)arena_get(ctx, "s1_f", 256);
  uint32_t *t = (uint32_t *)arena_get(ctx, "s1_t", 256);
  uint32_t *c = (uint32_t *)arena_get(ctx, "s1_c", 256);
  if (!sub_of || !tot || !f || !t || !c) return MH_ENOMEM;
  MH_HIP(ctx, hipMemsetAsync(tot, 0, (size_t)ds->K * 4, st));
  if (n) {
    k_fill_u32<<<nblk(n), 256, 0, st>>>(sub_of, n, 1u);
    MH_LAUNCHED(ctx, "k_fill_u32");
  }
  if (n_sub) {
    k_mark_subset<<<nblk(n_sub), 256, 0, st>>>(idx, n_sub, n, ds->labels, ds->K, sub_of, tot);
    MH_LAUNCHED(ctx, "k_mark_subset");
  }
  mh_status s = launch_split1(ctx, ds, sub_of, 1, tot, f, t, c);
  if (s) return s;
  MH_HIP(ctx, hipMemcpyAsync(feat, f, 1, hipMemcpyDeviceToHost, st));
  MH_HIP(ctx, hipMemcpyAsync(tau, t, 4, hipMemcpyDeviceToHost, st));
  MH_HIP(ctx, hipMemcpyAsync(correct, c, 4, hipMemcpyDeviceToHost, st));
  MH_HIP(ctx, hipStreamSynchronize(st));
  return MH_OK;
}

mh_status launch_split1(Ctx *ctx, const mh_dataset *ds, const uint32_t *sub_of, uint32_t nsub,
                        const uint32_t *tot, uint8_t *feat, uint32_t *tau, uint32_t *correct,
                        bool gini) {
  hipStream_t st = ctx->stream;
  const uint32_t n = ds->n, F = ds->F, K = ds->K;
  uint32_t fbits = 1;
  while ((1u << fbits) < F) ++fbits;
  uint32_t sbits = 0;
  while ((1u << sbits) < nsub) ++sbits;
  if (fbits + sbits > 31) return fail(ctx, MH_EINVAL, "too many subsets for split1");
  if (n > RANGE_MAX_N) return fail(ctx, MH_EINVAL, "too many samples for split1");
  // ranks lie below n: the low rb bits of a key
  uint32_t rb = 1;
  while ((1ull << rb) < n) ++rb;
  uint32_t *cursor = (uint32_t *)arena_get(ctx, "sp_cursor", 256);
  unsigned long long *best_c =
      (unsigned long long *)arena_get(ctx, "sp_best_c", (size_t)nsub * 8);
  unsigned long long *best_ft =
      (unsigned long long *)arena_get(ctx, "sp_best_ft", (size_t)nsub * 8);
  if (!cursor || !best_c || !best_ft) return MH_ENOMEM;
  MH_HIP(ctx, hipMemsetAsync(cursor, 0, 4, st));
  if (nsub == 0) return MH_OK;
  k_split_init<<<nblk(nsub), 256, 0, st>>>(tot, nsub, K, gini ? 1u : 0u, best_c, best_ft);
  MH_LAUNCHED(ctx, "k_split_init");
  // elements: (member sample, feature) pairs; members counted on the host
  uint32_t members = 0;
  {
    std::vector<uint32_t> h((size_t)nsub * K);
    MH_HIP(ctx, hipMemcpyAsync(h.data(), tot, h.size() * 4, hipMemcpyDeviceToHost, st));
    MH_HIP(ctx, hipStreamSynchronize(st));
    for (uint32_t v : h) members += v;
  }
  const uint64_t N64 = (uint64_t)members * F;
  if (N64 >= 0xFFFFFFFFull) return fail(ctx, MH_EINVAL, "split1: too many elements");
  const uint32_t N = (uint32_t)N64;
  if (N > 0) {
    uint64_t *ka = (uint64_t *)arena_get(ctx, "sp_keys_a", (size_t)N * 8);
    uint64_t *kb = (uint64_t *)arena_get(ctx, "sp_keys_b", (size_t)N * 8);
    uint32_t *va = (uint32_t *)arena_get(ctx, "sp_vals_a", (size_t)N * 4);
    uint32_t *vb = (uint32_t *)arena_get(ctx, "sp_vals_b", (size_t)N * 4);
    uint32_t *pk = (uint32_t *)arena_get(ctx, "sp_prefix", (size_t)N * K * 4);
    const size_t nseg = (size_t)nsub << fbits;
    uint32_t *seg_lo = (uint32_t *)arena_get(ctx, "sp_seg_lo", nseg * 4);
    uint32_t *seg_hi = (uint32_t *)arena_get(ctx, "sp_seg_hi", nseg * 4);
    if (!ka || !kb || !va || !vb || !pk || !seg_lo || !seg_hi) return MH_ENOMEM;
    const uint32_t span = range_span(ctx, n);
    k_split_keys<<<range_blocks(n, span), 256, 0, st>>>(sub_of, n, nsub, ds->ranks, ds->ld, F,
                                                         ds->labels, K, span, cursor, ka, va,
                                                         fbits, rb);
    MH_LAUNCHED(ctx, "k_split_keys");
    uint64_t *keys = ka;
    uint32_t *vals = va;
    const uint32_t key_bits = ((rb + fbits + sbits + 7) / 8) * 8;
    mh_status s = radix_sort_pairs(ctx, &keys, &vals, keys == ka ? kb : ka, vals == va ? vb : va,
                                   N, key_bits);
    if (s) return s;
    // per-class inclusive prefix counts, all classes in two passes over vals
    {
      const uint32_t nbc = (uint32_t)(((uint64_t)N + CP_SPAN - 1) / CP_SPAN);
      if ((uint64_t)nbc * K >= 0xFFFFFFFFull) return fail(ctx, MH_EINVAL, "split1: too many elements");
      uint32_t *csum = (uint32_t *)arena_get(ctx, "sp_csum", (size_t)nbc * K * 4);
      if (!csum) return MH_ENOMEM;
      k_split_class_sums<<<nbc, 256, (size_t)K * 4, st>>>(vals, N, K, nbc, csum);
      MH_LAUNCHED(ctx, "k_split_class_sums");
      s = scan_u32(ctx, csum, csum, nbc * K, false);
      if (s) return s;
      k_split_class_prefix<<<nbc, 256, (size_t)CP_ROUNDS * K * 4 * 4, st>>>(vals, N, K, nbc, csum,
                                                                             pk);
      MH_LAUNCHED(ctx, "k_split_class_prefix");
    }
    k_split_bounds<<<nblk(N), 256, 0, st>>>(keys, N, rb, seg_lo, seg_hi);
    MH_LAUNCHED(ctx, "k_split_bounds");
    for (uint32_t pass = 0; pass < 2; ++pass) {
      if (gini)
        k_split_eval<true><<<nblk(N), 256, 0, st>>>(keys, N, pk, K, seg_lo, seg_hi, fbits, rb, pass,
                                                    best_c, best_ft);
      else
        k_split_eval<false><<<nblk(N), 256, 0, st>>>(keys, N, pk, K, seg_lo, seg_hi, fbits, rb, pass,
                                                     best_c, best_ft);
      MH_LAUNCHED(ctx, "k_split_eval");
    }
  }
  k_split_final<<<nblk(nsub), 256, 0, st>>>(tot, nsub, K, gini ? 1u : 0u, best_c, best_ft, feat,
                                             tau, correct);
  MH_LAUNCHED(ctx, "k_split_final");
  return MH_OK;
}

// Multi-problem DEOCT: one tile set over all problems, one fitness launch and
// one fused epilogue + DE step (a block per problem) per generation.
mh_status deoct_batched(Ctx *ctx, const mh_dataset *ds, const uint32_t *sub_of,
                        uint32_t n_problems, const uint64_t *prob_ids, uint32_t D,
                        const mh_de_params *prm, const uint32_t *class_counts,
                        const double *warm, uint32_t W, uint8_t *feat_out, uint32_t *tau_out) {
  const uint32_t P = prm->P, SB = (1u << D) - 1u, m = 2 * SB, K = ds->K, F = ds->F;
  if (D > 5 || F > 80) return fail(ctx, MH_EINVAL, "batched DEOCT needs depth <= 5 and F <= 80");
  hipStream_t st = ctx->stream;
  TileHdr h = tile_layout(ds->n, F, K, n_problems);
  void *tiles = arena_get(ctx, "mb_tiles", h.total_bytes);
  const size_t cb = cnt_bytes(n_problems, D, K, P);
  uint32_t *cnt = (uint32_t *)arena_get(ctx, "mb_cnt", cb);
  double *pop = (double *)arena_get(ctx, "mb_pop", (size_t)n_problems * P * m * 8);
  double *trial = (double *)arena_get(ctx, "mb_trial", (size_t)n_problems * P * m * 8);
  double *cost = (double *)arena_get(ctx, "mb_cost", (size_t)n_problems * P * 8);
  uint8_t *feat = (uint8_t *)arena_get(ctx, "mb_feat", (size_t)n_problems * P * SB);
  uint32_t *tau = (uint32_t *)arena_get(ctx, "mb_tau", (size_t)n_problems * P * SB * 4);
  uint32_t *best = (uint32_t *)arena_get(ctx, "mb_best", (size_t)n_problems * 4);
  if (!tiles || !cnt || !pop || !trial || !cost || !feat || !tau || !best) return MH_ENOMEM;
  mh_status s = launch_tile_build(ctx, ds, nullptr, sub_of, ds->n, n_problems, tiles, h.total_bytes);
  if (s) return s;
  MH_HIP(ctx, hipMemsetAsync(cnt, 0, cb, st));
  const uint32_t *ctot =
      reinterpret_cast<const uint32_t *>(reinterpret_cast<const uint8_t *>(tiles) + h.off_ctot);
  DeDev de{P, D, F, prm->G, prm->M, prm->CR, prm->seed, ds->n_unique, true};
  s = launch_de_init(ctx, P, D, F, prm->seed, prob_ids, 0, n_problems, warm, W, pop, true);
  if (s) return s;
  if (class_counts && ctx->persist) {
    // every problem's whole run in one cooperative launch (a block group
    // per problem)
    uint32_t *err = (uint32_t *)arena_get(ctx, "mb_err", 256);
    if (!err) return MH_ENOMEM;
    bool used = false;
    s = launch_deoct_persist_multi(ctx, tiles, F, K, ds->n, n_problems, class_counts, D, prm,
                                   prob_ids, ds->n_unique, pop, cost, best, err, &used);
    if (s) return s;
    if (used) {
      s = launch_decode(ctx, pop, P, D, F, ds->n_unique, feat_out, tau_out, n_problems, best, true);
      if (s) return s;
      uint32_t h_err = 0;
      MH_HIP(ctx, hipMemcpyAsync(&h_err, err, 4, hipMemcpyDeviceToHost, st));
      MH_HIP(ctx, hipStreamSynchronize(st));
      if (!h_err) return MH_OK;
      // the cooperative grid did not run all at once: not again; the level
      // runs on the per-generation kernels from a fresh start
      coop_note_failure(ctx);
      MH_HIP(ctx, hipMemsetAsync(cnt, 0, cb, st));
      s = launch_de_init(ctx, P, D, F, prm->seed, prob_ids, 0, n_problems, warm, W, pop, true);
      if (s) return s;
    }
  }
  s = launch_decode(ctx, pop, P, D, F, ds->n_unique, feat, tau, n_problems, nullptr, true);
  if (s) return s;
  const bool fuse = ctx->fuse_de && fusable(P, D, F);
  uint32_t *done = (uint32_t *)arena_get(ctx, "mb_done", (size_t)n_problems * 4);
  if (!done) return MH_ENOMEM;
  MH_HIP(ctx, hipMemsetAsync(done, 0, (size_t)n_problems * 4, st));
  const uint32_t *segoff =
      reinterpret_cast<const uint32_t *>(reinterpret_cast<const uint8_t *>(tiles) + h.off_segoff);
  for (uint32_t g = 0; g <= prm->G; ++g) {
    if (fuse) {
      // one launch per generation for every problem of the level: the block
      // that completes a problem's counts runs its DE step
      FuseArgs fa = make_fuse(de, prob_ids, 0, n_problems, g + 1, g == 0, pop, cost, trial, best,
                              g < prm->G ? trial : nullptr, feat, tau, cnt, ctot, K, prm->n_min,
                              prm->alpha, done, segoff);
      s = launch_fitness_count(ctx, tiles, F, K, ds->n, n_problems, h.max_tiles, feat, tau, P, D,
                               cnt, &fa);
      if (s) return s;
      continue;
    }
    s = launch_fitness_count(ctx, tiles, F, K, ds->n, n_problems, h.max_tiles, feat, tau, P, D, cnt,
                             nullptr);
    if (s) return s;
    s = launch_de_gen(ctx, de, prob_ids, 0, n_problems, g + 1, g == 0, pop, cost, trial, best,
                      g < prm->G ? trial : nullptr, feat, tau, cnt, ctot, K, prm->n_min,
                      prm->alpha);
    if (s) return s;
  }
  return launch_decode(ctx, pop, P, D, F, ds->n_unique, feat_out, tau_out, n_problems, best, true);
}

// Warm-start genes of na nodes of a level (Algorithm 2's warm-start branch):
// per node, the whole-tree run's subtree of depth De at the node (when whole
// is given; subtree node u at depth k is tree node t 2^k + u - 2^k) and then
// the node's CART subtree (cf / ct, device [na][2^De - 1], when given),
// encoded into genes (device [na][W][2 (2^De - 1)]).
static mh_status level_warm(Ctx *ctx, const mh_dataset *ds, const uint32_t *nodes, uint32_t na,
                            uint32_t D, uint32_t De, const mh_tree *whole, const uint8_t *cf,
                            const uint32_t *ct, uint32_t W, double *genes) {
  hipStream_t st = ctx->stream;
  const uint32_t SBe = (1u << De) - 1u, SB = (1u << D) - 1u;
  uint8_t *wf = (uint8_t *)arena_get(ctx, "mh_wf", (size_t)na * W * SBe);
  uint32_t *wt = (uint32_t *)arena_get(ctx, "mh_wt", (size_t)na * W * SBe * 4);
  if (!wf || !wt) return MH_ENOMEM;
  if (whole) {
    std::vector<uint8_t> hf((size_t)na * W * SBe, 0);
    std::vector<uint32_t> ht((size_t)na * W * SBe, 0);
    for (uint32_t a = 0; a < na; ++a)
      for (uint32_t u = 1; u <= SBe; ++u) {
        uint32_t k = 0;
        while ((2u << k) <= u) ++k;
        const uint64_t v = ((uint64_t)nodes[a] << k) + (u - (1u << k));
        if (v > SB) continue;
        hf[(size_t)a * W * SBe + u - 1] = whole->feat[v - 1];
        ht[(size_t)a * W * SBe + u - 1] = whole->tau[v - 1];
      }
    MH_HIP(ctx, hipMemcpyAsync(wf, hf.data(), hf.size(), hipMemcpyHostToDevice, st));
    MH_HIP(ctx, hipMemcpyAsync(wt, ht.data(), ht.size() * 4, hipMemcpyHostToDevice, st));
    MH_HIP(ctx, hipStreamSynchronize(st));  // the host vectors go out of scope
  }
  if (cf) {
    const size_t w = W - 1;
    MH_HIP(ctx, hipMemcpy2DAsync(wf + w * SBe, (size_t)W * SBe, cf, SBe, SBe, na,
                                 hipMemcpyDeviceToDevice, st));
    MH_HIP(ctx, hipMemcpy2DAsync(wt + w * SBe, (size_t)W * SBe * 4, ct, (size_t)SBe * 4,
                                 (size_t)SBe * 4, na, hipMemcpyDeviceToDevice, st));
  }
  return launch_tree_encode(ctx, wf, wt, na * W, De, ds->F, ds->n_unique, genes);
}

// Algorithm 2.  flags: MH_SEQUENTIAL or MH_BATCHED, and the warm starts
// MH_WS_CART, MH_WS_DEOCT, MH_WS_DEOCT_CART.
// solve_one(ctx, ds, node_of, t, depth, prm, warm, W, &feat, &tau): the root
// of the DEOCT subtree of node t (sequential form), warm-started with the
// device genes warm [W][2 SB].
// solve_all(ctx, ds, D, prm, warm, W, &tree): DEOCT of the whole tree on
// every sample (problem id 0).
mh_status mh_train_impl(Ctx *ctx, const mh_dataset *ds, uint32_t D, uint32_t D_MH,
                        const mh_de_params *prm, uint32_t flags, mh_tree *out,
                        SolveNodeFn solve_one, SolveAllFn solve_all) {
  hipStream_t st = ctx->stream;
  const uint32_t n = ds->n, K = ds->K, SB = (1u << D) - 1u, SL = 1u << D;
  const bool batched = (flags & MH_BATCHED) != 0;
  const bool ws_cart = (flags & MH_WS_CART) != 0, ws_deoct = (flags & MH_WS_DEOCT) != 0;
  const uint32_t W = (ws_cart ? 1u : 0u) + (ws_deoct ? 1u : 0u);
  uint32_t *node_of = (uint32_t *)arena_get(ctx, "mh_node_of", (size_t)(n ? n : 1) * 4);
  uint32_t *sub_of = (uint32_t *)arena_get(ctx, "mh_sub_of", (size_t)(n ? n : 1) * 4);
  uint8_t *tfeat = (uint8_t *)arena_get(ctx, "mh_feat", SB);
  uint32_t *ttau = (uint32_t *)arena_get(ctx, "mh_tau", (size_t)SB * 4);
  const uint32_t maxw = 1u << (D - 1);
  uint32_t *hist = (uint32_t *)arena_get(ctx, "mh_hist", (size_t)maxw * K * 4);
  uint32_t *smap = (uint32_t *)arena_get(ctx, "mh_smap", (size_t)maxw * 4);
  uint64_t *pids = (uint64_t *)arena_get(ctx, "mh_pids", (size_t)maxw * 8);
  uint32_t *nodes_d = (uint32_t *)arena_get(ctx, "mh_nodes", (size_t)maxw * 4);
  uint8_t *rf = (uint8_t *)arena_get(ctx, "mh_rf", (size_t)maxw * 31);
  uint32_t *rt = (uint32_t *)arena_get(ctx, "mh_rt", (size_t)maxw * 31 * 4);
  uint32_t *scorr = (uint32_t *)arena_get(ctx, "mh_scorr", (size_t)maxw * 4);
  uint32_t *idx = (uint32_t *)arena_get(ctx, "mh_idx", (size_t)(n ? n : 1) * 4);
  if (!node_of || !sub_of || !tfeat || !ttau || !hist || !smap || !pids || !nodes_d || !rf || !rt ||
      !scorr || !idx)
    return MH_ENOMEM;
  MH_HIP(ctx, hipMemsetAsync(tfeat, 0, SB, st));
  MH_HIP(ctx, hipMemsetAsync(ttau, 0, (size_t)SB * 4, st));
  if (n) {
    k_fill_u32<<<nblk(n), 256, 0, st>>>(node_of, n, 1u);
    MH_LAUNCHED(ctx, "k_fill_u32");
  }
  // the whole-tree DEOCT run whose subtrees warm-start the nodes
  mh_tree whole;
  if (ws_deoct) {
    const double *wg = nullptr;
    uint32_t Wd = 0;
    if (flags & MH_WS_DEOCT_CART) {
      uint8_t *cf = (uint8_t *)arena_get(ctx, "mh_cf", SB);
      uint32_t *ct = (uint32_t *)arena_get(ctx, "mh_ct", (size_t)SB * 4);
      double *g = (double *)arena_get(ctx, "mh_wgenes", (size_t)2 * SB * 8);
      if (!cf || !ct || !g) return MH_ENOMEM;
      if (n) {
        k_fill_u32<<<nblk(n), 256, 0, st>>>(sub_of, n, 0u);
        MH_LAUNCHED(ctx, "k_fill_u32");
      }
      mh_status s = cart_batched(ctx, ds, sub_of, 1, D, cf, ct);
      if (!s) s = launch_tree_encode(ctx, cf, ct, 1, D, ds->F, ds->n_unique, g);
      if (s) return s;
      wg = g;
      Wd = 1;
    }
    mh_status s = solve_all(ctx, ds, D, prm, wg, Wd, &whole);
    if (s) return s;
  }
  std::vector<uint32_t> hh((size_t)maxw * K);
  for (uint32_t L = 0; L < D; ++L) {
    const uint32_t t0 = 1u << L, width = 1u << L;
    // class histogram of the level's nodes
    MH_HIP(ctx, hipMemsetAsync(hist, 0, (size_t)width * K * 4, st));
    if (n) {
      const bool in_lds = (size_t)width * K * 4 <= 32768;
      // a range of samples per block (about two blocks per CU): the few
      // cells of a shallow level take a few hundred global adds each
      if (n > RANGE_MAX_N) return fail(ctx, MH_EINVAL, "too many samples for the level counts");
      const uint32_t span = range_span(ctx, n);
      k_level_hist<<<range_blocks(n, span), 256, in_lds ? (size_t)width * K * 4 : 0, st>>>(
          node_of, ds->labels, n, K, t0, width, span, hist, in_lds ? 1 : 0);
      MH_LAUNCHED(ctx, "k_level_hist");
    }
    MH_HIP(ctx, hipMemcpyAsync(hh.data(), hist, (size_t)width * K * 4, hipMemcpyDeviceToHost, st));
    MH_HIP(ctx, hipStreamSynchronize(st));
    // which nodes are solved (more than n_min samples of more than one class)
    std::vector<uint32_t> active, map(width, 0xFFFFFFFFu);
    for (uint32_t w = 0; w < width; ++w) {
      uint32_t size = 0, classes = 0;
      for (uint32_t k = 0; k < K; ++k) {
        size += hh[(size_t)w * K + k];
        classes += hh[(size_t)w * K + k] ? 1u : 0u;
      }
      if (size > prm->n_min && classes > 1) {
        map[w] = (uint32_t)active.size();
        active.push_back(t0 + w);
      }
    }
    const uint32_t De = std::min(D_MH, D - L);
    const uint32_t na = (uint32_t)active.size();
    if (na > 0) {
      for (uint32_t w = 0; w < width; ++w)
        if (map[w] == 0xFFFFFFFFu) map[w] = na;
      MH_HIP(ctx, hipMemcpyAsync(smap, map.data(), (size_t)width * 4, hipMemcpyHostToDevice, st));
      MH_HIP(ctx, hipMemcpyAsync(nodes_d, active.data(), (size_t)na * 4, hipMemcpyHostToDevice, st));
      std::vector<uint64_t> pid(active.begin(), active.end());
      MH_HIP(ctx, hipMemcpyAsync(pids, pid.data(), (size_t)na * 8, hipMemcpyHostToDevice, st));
      MH_HIP(ctx, hipStreamSynchronize(st));  // map / pid host buffers are reused below
      // roots land in rf/rt with stride SB1 (batched trees) or 1 (one root)
      uint32_t SB1 = (De == 1 || !batched) ? 1u : (1u << De) - 1u;
      if (batched || De == 1) {
        k_assign_sub<<<nblk(n), 256, 0, st>>>(node_of, n, t0, width, smap, na, sub_of);
        MH_LAUNCHED(ctx, "k_assign_sub");
      }
      if (De == 1) {
        // exact split of every active node (one batched launch; the result of
        // a node does not depend on the others)
        std::vector<uint32_t> tot((size_t)na * K);
        for (uint32_t a = 0; a < na; ++a)
          for (uint32_t k = 0; k < K; ++k) tot[(size_t)a * K + k] = hh[(size_t)(active[a] - t0) * K + k];
        MH_HIP(ctx, hipMemcpyAsync(hist, tot.data(), tot.size() * 4, hipMemcpyHostToDevice, st));
        MH_HIP(ctx, hipStreamSynchronize(st));
        mh_status s = launch_split1(ctx, ds, sub_of, na, hist, rf, rt, scorr);
        if (s) return s;
      } else if (batched) {
        std::vector<uint32_t> cc((size_t)na * K);
        for (uint32_t a = 0; a < na; ++a)
          for (uint32_t k = 0; k < K; ++k) cc[(size_t)a * K + k] = hh[(size_t)(active[a] - t0) * K + k];
        const uint32_t SBe = (1u << De) - 1u;
        double *wg = nullptr;
        if (W) {
          uint8_t *cf = (uint8_t *)arena_get(ctx, "mh_cf", (size_t)na * SBe);
          uint32_t *ct = (uint32_t *)arena_get(ctx, "mh_ct", (size_t)na * SBe * 4);
          wg = (double *)arena_get(ctx, "mh_wgenes", (size_t)na * W * 2 * SBe * 8);
          if (!cf || !ct || !wg) return MH_ENOMEM;
          mh_status s = ws_cart ? cart_batched(ctx, ds, sub_of, na, De, cf, ct) : MH_OK;
          if (!s)
            s = level_warm(ctx, ds, active.data(), na, D, De, ws_deoct ? &whole : nullptr,
                           ws_cart ? cf : nullptr, ct, W, wg);
          if (s) return s;
        }
        mh_status s = deoct_batched(ctx, ds, sub_of, na, pids, De, prm, cc.data(), wg, W, rf, rt);
        if (s) return s;
      } else {
        std::vector<uint8_t> hf(na);
        std::vector<uint32_t> ht(na);
        const uint32_t SBe = (1u << De) - 1u;
        for (uint32_t a = 0; a < na; ++a) {
          double *wg = nullptr;
          if (W) {
            // node t's own subset (subset 0) for its CART subtree
            uint32_t *one = (uint32_t *)arena_get(ctx, "mh_smap1", 4);
            uint8_t *cf = (uint8_t *)arena_get(ctx, "mh_cf", SBe);
            uint32_t *ct = (uint32_t *)arena_get(ctx, "mh_ct", (size_t)SBe * 4);
            wg = (double *)arena_get(ctx, "mh_wgenes", (size_t)W * 2 * SBe * 8);
            if (!one || !cf || !ct || !wg) return MH_ENOMEM;
            mh_status s = MH_OK;
            if (ws_cart) {
              MH_HIP(ctx, hipMemsetAsync(one, 0, 4, st));
              if (n) {
                k_assign_sub<<<nblk(n), 256, 0, st>>>(node_of, n, active[a], 1, one, 1, sub_of);
                MH_LAUNCHED(ctx, "k_assign_sub");
              }
              s = cart_batched(ctx, ds, sub_of, 1, De, cf, ct);
            }
            if (!s)
              s = level_warm(ctx, ds, &active[a], 1, D, De, ws_deoct ? &whole : nullptr,
                             ws_cart ? cf : nullptr, ct, W, wg);
            if (s) return s;
          }
          mh_status s = solve_one(ctx, ds, node_of, active[a], De, prm, wg, W, &hf[a], &ht[a]);
          if (s) return s;
        }
        MH_HIP(ctx, hipMemcpyAsync(rf, hf.data(), na, hipMemcpyHostToDevice, st));
        MH_HIP(ctx, hipMemcpyAsync(rt, ht.data(), (size_t)na * 4, hipMemcpyHostToDevice, st));
        MH_HIP(ctx, hipStreamSynchronize(st));  // host vectors go out of scope
      }
      k_put_roots<<<nblk(na), 256, 0, st>>>(rf, rt, SB1, nodes_d, na, tfeat, ttau);
      MH_LAUNCHED(ctx, "k_put_roots");
    }
    if (L + 1 < D && n) {
      k_route_level<<<nblk(n), 256, 0, st>>>(node_of, n, t0, width, tfeat, ttau, ds->ranks, ds->ld,
                                             ds->F);
      MH_LAUNCHED(ctx, "k_route_level");
    }
  }
  // leaf classes and objective of the final tree over all training samples
  uint8_t *lab = (uint8_t *)arena_get(ctx, "mh_lab", SL);
  uint32_t *corr = (uint32_t *)arena_get(ctx, "mh_corr", 256);
  double *cst = (double *)arena_get(ctx, "mh_cost", 256);
  if (!lab || !corr || !cst) return MH_ENOMEM;
  FitnessOut fo;
  fo.label = lab;
  fo.correct = corr;
  fo.cost = cst;
  mh_status s = launch_fitness_walk(ctx, ds, nullptr, n, tfeat, ttau, 1, D, prm->n_min, prm->alpha, fo);
  if (s) return s;
  std::memset(out, 0, sizeof(*out));
  out->D = D;
  MH_HIP(ctx, hipMemcpyAsync(out->feat, tfeat, SB, hipMemcpyDeviceToHost, st));
  MH_HIP(ctx, hipMemcpyAsync(out->tau, ttau, (size_t)SB * 4, hipMemcpyDeviceToHost, st));
  MH_HIP(ctx, hipMemcpyAsync(out->label, lab, SL, hipMemcpyDeviceToHost, st));
  MH_HIP(ctx, hipMemcpyAsync(&out->correct, corr, 4, hipMemcpyDeviceToHost, st));
  MH_HIP(ctx, hipMemcpyAsync(&out->cost, cst, 8, hipMemcpyDeviceToHost, st));
  MH_HIP(ctx, hipStreamSynchronize(st));
  return MH_OK;
}

}  // namespace mh
