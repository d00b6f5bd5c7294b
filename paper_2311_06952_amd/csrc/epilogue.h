// epilogue.h -- from per-(node, class) left counts to leaf counts, leaf
// classes, correct count and cost (eq. opt_c; eq. opt_all; Section 3.2).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mh {

// Result of one tree's epilogue.
struct TreeScore {
  uint32_t correct;
  double cost;
};

// cnt: NREP copies (stride rep_stride) of [SB][K][Ppad] left counts of this
// problem (entry for tree r at ((t * K + k) * Ppad + r)); ctot: [K] class
// totals.  The reach of node 1 is the class total, reach(2t) = left(t),
// reach(2t+1) = reach(t) - left(t); the leaves are the reaches of nodes
// 2^D .. 2^(D+1)-1.  Consumed counters are set back to zero (after all loads,
// so that the loads are not ordered behind stores).  counts / label (may be
// null) receive [SL][K] and [SL].
// Counts written by other blocks of the same launch are read with
// agent-scope (coherent) loads when COH is set.
template <bool COH>
__device__ __forceinline__ uint32_t cnt_load(const uint32_t *p) {
  if constexpr (COH)
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    return *p;
}

template <int D, int NREP, bool COH = false>
__device__ __forceinline__ TreeScore epilogue_node_counts(
    uint32_t *__restrict__ cnt, const uint32_t *__restrict__ ctot, uint32_t K, uint32_t Ppad,
    uint32_t r, const uint8_t *__restrict__ feat_r, uint32_t n_min, double alpha,
    uint32_t *__restrict__ counts, uint8_t *__restrict__ label, size_t rep_stride,
    uint32_t tpi = 1) {
  // With tpi > 1 the tree is handled by tpi adjacent lanes: lane j takes the
  // classes k = j, j + tpi, ...; the per-leaf maxima and sizes are then merged
  // across the group (ties to the lower class), and every lane of the group
  // returns the same score.
  constexpr int SB = (1 << D) - 1, SL = 1 << D;
  const uint32_t j0 = tpi > 1 ? (threadIdx.x % tpi) : 0u;
  uint32_t nl[SL], best[SL], bk[SL];
#pragma unroll
  for (int l = 0; l < SL; ++l) nl[l] = best[l] = bk[l] = 0;
  uint32_t n_sub = 0;
  // With up to KB classes per lane every count load is issued before the
  // first one is used (one memory round trip); more classes loop.
  constexpr uint32_t KB = (SB * NREP <= 32) ? 4u : 2u;
  uint32_t pre[KB][SB];
#pragma unroll
  for (uint32_t kk = 0; kk < KB; ++kk) {
    // classes past K load class K-1 (in bounds, K >= 1) and are zeroed, so
    // that the loads carry no branch
    const uint32_t k = j0 + kk * tpi;
    const uint32_t kc = k < K ? k : K - 1u;
#pragma unroll
    for (int t = 0; t < SB; ++t) {
      uint32_t v = 0;
#pragma unroll
      for (int q = 0; q < NREP; ++q)
        v += cnt_load<COH>(cnt + q * rep_stride + ((size_t)t * K + kc) * Ppad + r);
      pre[kk][t] = k < K ? v : 0u;
    }
  }
  for (uint32_t k = j0, kk = 0; k < K; k += tpi, ++kk) {
    uint32_t reach[2 * SL];
    uint32_t left[SB];
    if (kk < KB) {
#pragma unroll
      for (int t = 0; t < SB; ++t) left[t] = 0;
#pragma unroll
      for (uint32_t c = 0; c < KB; ++c)
        if (c == kk)
#pragma unroll
          for (int t = 0; t < SB; ++t) left[t] = pre[c][t];
    } else {
#pragma unroll
      for (int t = 0; t < SB; ++t) {
        uint32_t v = 0;
#pragma unroll
        for (int q = 0; q < NREP; ++q)
          v += cnt_load<COH>(cnt + q * rep_stride + ((size_t)t * K + k) * Ppad + r);
        left[t] = v;
      }
    }
    reach[1] = ctot[k];
    n_sub += reach[1];
#pragma unroll
    for (int t = 1; t <= SB; ++t) {
      reach[2 * t] = left[t - 1];
      reach[2 * t + 1] = reach[t] - left[t - 1];
    }
#pragma unroll
    for (int l = 0; l < SL; ++l) {
      const uint32_t v = reach[SL + l];
      if (counts) counts[(size_t)l * K + k] = v;
      nl[l] += v;
      if (v > best[l]) {  // classes ascend in this lane: ties keep the lower one
        best[l] = v;
        bk[l] = k;
      }
    }
  }
  if (tpi > 1) {
    // merge the lanes' partial results: sizes add; the larger maximum wins,
    // equal maxima keep the lower class (an empty leaf keeps class 0)
    for (uint32_t d = 1; d < tpi; d <<= 1) {
      n_sub += __shfl_xor(n_sub, (int)d, 64);
#pragma unroll
      for (int l = 0; l < SL; ++l) {
        const uint32_t ob = __shfl_xor(best[l], (int)d, 64);
        const uint32_t ok = __shfl_xor(bk[l], (int)d, 64);
        nl[l] += __shfl_xor(nl[l], (int)d, 64);
        if (ob > best[l] || (ob == best[l] && ob > 0 && ok < bk[l])) {
          best[l] = ob;
          bk[l] = ok;
        }
        if (best[l] == 0) bk[l] = 0;
      }
    }
  }
  uint32_t correct = 0, nviol = 0, nsplit = 0;
#pragma unroll
  for (int l = 0; l < SL; ++l) {
    correct += best[l];
    nviol += (nl[l] > 0 && nl[l] < n_min) ? 1u : 0u;
    if (label && j0 == 0) label[l] = (uint8_t)bk[l];
  }
#pragma unroll
  for (int t = 0; t < SB; ++t) nsplit += feat_r[t] != 0;
  for (uint32_t k = j0; k < K; k += tpi) {
#pragma unroll
    for (int q = 0; q < NREP; ++q)
#pragma unroll
      for (int t = 0; t < SB; ++t) cnt[q * rep_stride + ((size_t)t * K + k) * Ppad + r] = 0;
  }
  double v = (double)(n_sub - correct);
  v = __dadd_rn(v, __dmul_rn(alpha, (double)nsplit));
  v = __dadd_rn(v, (double)nviol);
  return TreeScore{correct, v};
}

}  // namespace mh
