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
template <int D, int NREP>
__device__ __forceinline__ TreeScore epilogue_node_counts(
    uint32_t *__restrict__ cnt, const uint32_t *__restrict__ ctot, uint32_t K, uint32_t Ppad,
    uint32_t r, const uint8_t *__restrict__ feat_r, uint32_t n_min, double alpha,
    uint32_t *__restrict__ counts, uint8_t *__restrict__ label, size_t rep_stride) {
  constexpr int SB = (1 << D) - 1, SL = 1 << D;
  uint32_t nl[SL], best[SL], bk[SL];
#pragma unroll
  for (int l = 0; l < SL; ++l) nl[l] = best[l] = bk[l] = 0;
  uint32_t n_sub = 0;
  // all NREP x SB loads of a class are independent (one round trip per class)
#pragma unroll 2
  for (uint32_t k = 0; k < K; ++k) {
    uint32_t reach[2 * SL];
    uint32_t part[NREP][SB];
#pragma unroll
    for (int q = 0; q < NREP; ++q)
#pragma unroll
      for (int t = 0; t < SB; ++t) part[q][t] = cnt[q * rep_stride + ((size_t)t * K + k) * Ppad + r];
    uint32_t left[SB];
#pragma unroll
    for (int t = 0; t < SB; ++t) {
      left[t] = part[0][t];
#pragma unroll
      for (int q = 1; q < NREP; ++q) left[t] += part[q][t];
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
      if (v > best[l]) {
        best[l] = v;
        bk[l] = k;
      }
    }
  }
  uint32_t correct = 0, nviol = 0, nsplit = 0;
#pragma unroll
  for (int l = 0; l < SL; ++l) {
    correct += best[l];
    nviol += (nl[l] > 0 && nl[l] < n_min) ? 1u : 0u;
    if (label) label[l] = (uint8_t)bk[l];
  }
#pragma unroll
  for (int t = 0; t < SB; ++t) nsplit += feat_r[t] != 0;
  for (uint32_t k = 0; k < K; ++k) {
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
