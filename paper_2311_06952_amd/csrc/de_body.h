// de_body.h -- the DE step (Section 2 eqs. mutation, crossover, selection;
// Section 3.3; Algorithm 4) as a block-wide device routine, shared by the
// stand-alone DE kernels and the fused fitness + DE kernel.
#pragma once

#include <cfloat>

#include "device_common.h"
#include "epilogue.h"
#include "internal.h"

namespace mh {

__device__ __forceinline__ uint64_t prob_of(const uint64_t *prob_ids, uint64_t prob_base,
                                            uint32_t sub) {
  return prob_ids ? prob_ids[sub] : prob_base + sub;
}

struct StepArgs {
  uint32_t P, SB, F, g;
  double M, CR;
  uint64_t seed;
  const uint32_t *n_unique;
  const uint64_t *prob_ids;
  uint64_t prob_base;
  double *pop, *cost;
  const double *trial, *trial_cost;
  uint32_t *best;
  double *next_trial;
  uint8_t *feat;
  uint32_t *tau;
  int rows_in_lds;
  uint32_t rs, qs;  // gene (r, q) of a problem at r * rs + q * qs
};

// Phases of one DE step for problem `sub`.  Individual r is handled by the
// tpi adjacent threads r * tpi + j (j < tpi):
//  1. selection (eq. selection; ties go to the trial) when `select`, with
//     the trial's cost tc; or, when `init`, cost[r] = tc (generation 0);
//  2. best = lowest index of the minimum cost;
//  3. DE/best/1 mutation and binomial crossover of generation g into
//     next_trial (thread j makes the genes of nodes t = j, j + tpi, ...),
//     decoded into (feat, tau) when those are given.
// With `rows` (LDS, gene-major [m][P]) the post-selection population is also
// kept in LDS so that phase 3 reads its three parents there; s_nu caches
// n_unique.
__device__ __forceinline__ void de_step_body(const StepArgs &a, uint32_t sub, uint32_t r,
                                             uint32_t j, uint32_t tpi, bool select, bool init,
                                             double tc, double *s_cost, uint32_t *s_idx,
                                             double *rows, uint32_t *s_nu) {
  const uint32_t P = a.P, m = 2 * a.SB;
  double *pop = a.pop + (size_t)sub * P * m;
  double *cost = a.cost + (size_t)sub * P;
  if (a.feat && a.n_unique)
    for (uint32_t f = threadIdx.x; f < a.F; f += blockDim.x) s_nu[f] = a.n_unique[f];
  const uint32_t rs = a.rs, qs = a.qs;
  double my_cost = 0.0;
  if (r < P) {
    my_cost = cost[r];
    const bool take = select && tc <= my_cost;
    if (init || take) my_cost = tc;
    const double *tr = a.trial + (size_t)sub * P * m + (size_t)r * rs;
    double *pr = pop + (size_t)r * rs;
    const double *src = take ? tr : pr;
    if (rows || take) {
      // genes move in batches of 16 loads issued together (one round trip
      // per batch); through LDS (gene-major [m][P]) when rows is given
      for (uint32_t q0 = j; q0 < m; q0 += 16 * tpi) {
        double v[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const uint32_t q = q0 + i * tpi;
          v[i] = q < m ? src[(size_t)q * qs] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const uint32_t q = q0 + i * tpi;
          if (q < m) {
            if (rows) rows[(size_t)q * P + r] = v[i];
            if (take) pr[(size_t)q * qs] = v[i];
          }
        }
      }
    }
    if ((init || take) && j == 0) cost[r] = my_cost;
  }
  const uint32_t nr = blockDim.x / tpi;  // a power of two >= P
  if (j == 0) {
    s_cost[r] = r < P ? my_cost : DBL_MAX;
    s_idx[r] = r;
  }
  __syncthreads();
  for (uint32_t d = nr >> 1; d > 0; d >>= 1) {
    const uint32_t x = threadIdx.x;
    if (x < d) {
      const double c2 = s_cost[x + d];
      const uint32_t i2 = s_idx[x + d];
      if (c2 < s_cost[x] || (c2 == s_cost[x] && i2 < s_idx[x])) {
        s_cost[x] = c2;
        s_idx[x] = i2;
      }
    }
    __syncthreads();
  }
  const uint32_t best = s_idx[0];
  if (threadIdx.x == 0 && a.best) a.best[sub] = best;
  if (!a.next_trial || r >= P) return;
  const uint64_t key = de_key(a.seed, prob_of(a.prob_ids, a.prob_base, sub));
  const uint32_t g = a.g;
  const double Mr = a.M >= 0.0 ? a.M : to_unit(de_draw(key, g, r, 0));
  uint32_t r1 = to_below(de_draw(key, g, r, 1), P - 1u);
  r1 += (r1 >= r) ? 1u : 0u;
  uint32_t r2 = to_below(de_draw(key, g, r, 2), P - 2u);
  const uint32_t lo = r < r1 ? r : r1, hi = r < r1 ? r1 : r;
  r2 += (r2 >= lo) ? 1u : 0u;
  r2 += (r2 >= hi) ? 1u : 0u;
  const uint32_t qr = to_below(de_draw(key, g, r, 3), m);
  // parents: LDS rows are gene-major [m][P]; global ones use (rs, qs)
  const double *src = rows ? rows : pop;
  const uint32_t prs = rows ? 1u : rs, pqs = rows ? P : qs;
  const double *sb = src + (size_t)best * prs;
  const double *s1 = src + (size_t)r1 * prs;
  const double *s2 = src + (size_t)r2 * prs;
  const double *sr = src + (size_t)r * prs;
  double *out = a.next_trial + (size_t)sub * P * m + (size_t)r * rs;
  const double Fp1 = (double)a.F + 1.0;
  uint8_t *fo = a.feat ? a.feat + ((size_t)sub * P + r) * a.SB : nullptr;
  uint32_t *to = a.feat ? a.tau + ((size_t)sub * P + r) * a.SB : nullptr;
  // a feature gene q < SB and its threshold gene SB + q are made together so
  // that the node can be decoded at once
  for (uint32_t q = j; q < a.SB; q += tpi) {
    double gq[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint32_t qq = q + (h ? a.SB : 0u);
      const size_t o = (size_t)qq * pqs;
      const double d = __dsub_rn(s1[o], s2[o]);
      double v = __dadd_rn(sb[o], __dmul_rn(Mr, d));
      const double hiq = h ? 1.0 : Fp1;
      if (!(v >= 0.0)) v = 0.0;
      if (v > hiq) v = hiq;
      const double u = to_unit(de_draw(key, g, r, 4u + qq));
      gq[h] = (u <= a.CR || qq == qr) ? v : sr[o];
      out[(size_t)qq * qs] = gq[h];
    }
    if (fo) {
      uint32_t f, th;
      decode_node(gq[0], gq[1], a.F, s_nu, f, th);
      fo[q] = (uint8_t)f;
      to[q] = th;
    }
  }
}

// The same step fused with the fitness epilogue of the population just
// evaluated (tile path): thread r turns its tree's node counts into the
// cost, then steps.  In generation 0 (init) the cost is the population's own.
struct GenArgs {
  uint32_t *cnt;          // [n_problems][SB][K][Ppad], re-zeroed here
  const uint32_t *ctot;   // [n_problems][K]
  uint32_t K, n_min;
  double alpha;
  int init;
  uint32_t tpi;         // threads per individual
  uint32_t n_problems;  // problems in the count buffer (replica stride)
};

// One problem's DE generation inside a multi-job launch (k_de_jobs): the
// epilogue of its counts, then the DE step; e.n_problems is 1.
struct GenJob {
  StepArgs a;
  GenArgs e;
};

// Everything the fused fitness + DE kernel needs besides the fitness inputs.
struct FuseArgs {
  StepArgs a;               // prob_ids / prob_base select the problem ids
  GenArgs e;                // counts, class totals, penalties, init flag
  uint32_t *done;           // [n_problems] finished-block tickets, zero between launches
  const uint32_t *segoff;   // tile set: first tile of segment (sub * K + class)
  uint32_t rows_in_lds;     // keep the post-selection population in LDS
};

}  // namespace mh
