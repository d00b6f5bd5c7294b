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

// A whole DE generation of one problem by one block, thread r = individual
// r (blockDim.x a power of two >= P): the epilogue of the just evaluated
// population's node counts (its cost; eq. opt_all and the soft-constraint
// fitness), then selection (eq. selection) or, when init, the initial cost,
// best = lowest index of the minimum cost, and the trial of generation a.g
// (eqs. mutation and crossover, decoded into feat/tau).  Same arithmetic and
// results as epilogue_node_counts followed by de_step_body with tpi = 1, but
// every global load of the step (counts, class totals, feature bytes, the
// parent's cost and both gene rows, n_unique) is issued before the first
// store, so the step waits for memory once before the argmin; the argmin
// reduces in registers within each wave, then once across waves.
// ROOMY: the kernel has registers to spare (at most 256 threads per block),
// so both gene rows are loaded up front too.
template <int D, int NREP, bool COH, bool ROOMY>
__device__ __forceinline__ void de_gen_body(const StepArgs &a, const GenArgs &e, uint32_t sub,
                                            double *s_cost, uint32_t *s_idx, double *rows,
                                            uint32_t *s_nu) {
  constexpr int SB = (1 << D) - 1, SL = 1 << D, m = 2 * SB;
  // classes whose counts are loaded per batch (a second batch is in flight
  // while the first is used)
  constexpr uint32_t KB = (SB * NREP <= 8) ? 4u : (SB * NREP <= 16 ? 2u : 1u);
  constexpr bool GENES_EARLY = ROOMY && m <= 32;
  const uint32_t P = a.P, Ppad = pad64(P), K = e.K, r = threadIdx.x;
  const bool live = r < P;
  const uint32_t rr = live ? r : 0u;  // loads of idle threads stay in bounds
  const size_t rep = cnt_copy_elems(e.n_problems, SB, K, P);
  uint32_t *cnt = e.cnt + (size_t)sub * SB * K * Ppad + rr;
  const uint32_t *ctot = e.ctot + (size_t)sub * K;
  double *pop = a.pop + (size_t)sub * P * m + (size_t)rr * a.rs;
  const double *tr = a.trial + (size_t)sub * P * m + (size_t)rr * a.rs;
  double *cost = a.cost + (size_t)sub * P;
  const uint32_t qs = a.qs;
  const bool init = e.init != 0;

  // ---- loads
  if (a.feat && a.n_unique)
    for (uint32_t f = threadIdx.x; f < a.F; f += blockDim.x) s_nu[f] = a.n_unique[f];
  // a batch: the left counts of KB classes and their class totals
  auto load_batch = [&](uint32_t k0, uint32_t (&v)[KB][SB], uint32_t (&ct)[KB]) {
#pragma unroll
    for (uint32_t kk = 0; kk < KB; ++kk) {
      const uint32_t k = k0 + kk < K ? k0 + kk : K - 1u;
      ct[kk] = ctot[k];
#pragma unroll
      for (int t = 0; t < SB; ++t) {
        uint32_t x = 0;
#pragma unroll
        for (int q = 0; q < NREP; ++q) x += cnt_load<COH>(cnt + q * rep + ((size_t)t * K + k) * Ppad);
        v[kk][t] = x;
      }
    }
  };
  uint32_t cur[KB][SB], nxt[KB][SB], ccur[KB], cnxt[KB];
  load_batch(0, cur, ccur);
  if (KB < K) load_batch(KB, nxt, cnxt);
  uint32_t nsplit = 0;
  if (a.feat) {
    const uint8_t *fr = a.feat + ((size_t)sub * P + rr) * SB;
#pragma unroll
    for (int t = 0; t < SB; ++t) nsplit += fr[t] != 0;
  }
  const double c_old = cost[rr];
  double gp[GENES_EARLY ? m : 1], gt[GENES_EARLY ? m : 1];
  if constexpr (GENES_EARLY) {
#pragma unroll
    for (int q = 0; q < m; ++q) gp[q] = pop[(size_t)q * qs];
    if (!init) {
#pragma unroll
      for (int q = 0; q < m; ++q) gt[q] = tr[(size_t)q * qs];
    }
  }

  // ---- epilogue: leaf sizes, per-leaf maxima, cost
  uint32_t nl[SL], best[SL], n_sub = 0;
#pragma unroll
  for (int l = 0; l < SL; ++l) nl[l] = best[l] = 0;
  auto use_class = [&](uint32_t total, const uint32_t (&left)[SB]) {
    uint32_t reach[2 * SL];
    reach[1] = total;
    n_sub += reach[1];
#pragma unroll
    for (int t = 1; t <= SB; ++t) {
      reach[2 * t] = left[t - 1];
      reach[2 * t + 1] = reach[t] - left[t - 1];
    }
#pragma unroll
    for (int l = 0; l < SL; ++l) {
      const uint32_t v = reach[SL + l];
      nl[l] += v;
      best[l] = v > best[l] ? v : best[l];
    }
  };
  for (uint32_t k0 = 0; k0 < K; k0 += KB) {
#pragma unroll
    for (uint32_t kk = 0; kk < KB; ++kk)
      if (k0 + kk < K) use_class(ccur[kk], cur[kk]);
    if (k0 + KB < K) {
#pragma unroll
      for (uint32_t kk = 0; kk < KB; ++kk) {
        ccur[kk] = cnxt[kk];
#pragma unroll
        for (int t = 0; t < SB; ++t) cur[kk][t] = nxt[kk][t];
      }
      if (k0 + 2 * KB < K) load_batch(k0 + 2 * KB, nxt, cnxt);
    }
  }
  uint32_t correct = 0, nviol = 0;
#pragma unroll
  for (int l = 0; l < SL; ++l) {
    correct += best[l];
    nviol += (nl[l] > 0 && nl[l] < e.n_min) ? 1u : 0u;
  }
  double tc = (double)(n_sub - correct);
  tc = __dadd_rn(tc, __dmul_rn(e.alpha, (double)nsplit));
  tc = __dadd_rn(tc, (double)nviol);

  // ---- stores: consumed counters back to zero; selection
  if (live) {
    for (uint32_t k = 0; k < K; ++k)
#pragma unroll
      for (int q = 0; q < NREP; ++q)
#pragma unroll
        for (int t = 0; t < SB; ++t) cnt[q * rep + ((size_t)t * K + k) * Ppad] = 0;
  }
  double my_cost = DBL_MAX;
  if (live) {
    const bool take = !init && tc <= c_old;
    my_cost = (init || take) ? tc : c_old;
    if (init || take) cost[r] = my_cost;
    if constexpr (GENES_EARLY) {
#pragma unroll
      for (int q = 0; q < m; ++q) {
        const double v = take ? gt[q] : gp[q];
        if (rows) rows[(size_t)q * P + r] = v;
        if (take) pop[(size_t)q * qs] = v;
      }
    } else {
      // batches of loads issued together: a store into pop may alias a later
      // load of it, so unbatched loads would each wait for the previous store
      const double *src = take ? tr : pop;
      constexpr int QB = 10;
#pragma unroll
      for (int q0 = 0; q0 < m; q0 += QB) {
        double v[QB];
#pragma unroll
        for (int i = 0; i < QB; ++i)
          if (q0 + i < m) v[i] = src[(size_t)(q0 + i) * qs];
#pragma unroll
        for (int i = 0; i < QB; ++i) {
          if (q0 + i < m) {
            if (rows) rows[(size_t)(q0 + i) * P + r] = v[i];
            if (take) pop[(size_t)(q0 + i) * qs] = v[i];
          }
        }
      }
    }
  }

  // ---- best: lowest index of the minimum cost
  double bc = my_cost;
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
  const uint32_t w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63u) == 0) {
    s_cost[w] = bc;
    s_idx[w] = bi;
  }
  __syncthreads();
  bc = s_cost[0];
  bi = s_idx[0];
  for (uint32_t x = 1; x < nw; ++x) {
    const double c2 = s_cost[x];
    const uint32_t i2 = s_idx[x];
    if (c2 < bc || (c2 == bc && i2 < bi)) {
      bc = c2;
      bi = i2;
    }
  }
  const uint32_t bst = bi;
  if (threadIdx.x == 0 && a.best) a.best[sub] = bst;
  if (!a.next_trial || !live) return;

  // ---- DE/best/1 mutation, binomial crossover, decode
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
  const double *src = rows ? rows : a.pop + (size_t)sub * P * m;
  const uint32_t prs = rows ? 1u : a.rs, pqs = rows ? P : qs;
  const double *sb = src + (size_t)bst * prs;
  const double *s1 = src + (size_t)r1 * prs;
  const double *s2 = src + (size_t)r2 * prs;
  const double *sr = src + (size_t)r * prs;
  double *out = a.next_trial + (size_t)sub * P * m + (size_t)r * a.rs;
  const double Fp1 = (double)a.F + 1.0;
  uint8_t *fo = a.feat ? a.feat + ((size_t)sub * P + r) * SB : nullptr;
  uint32_t *to = a.feat ? a.tau + ((size_t)sub * P + r) * SB : nullptr;
#pragma unroll
  for (int q = 0; q < SB; ++q) {
    double gq[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint32_t qq = q + (h ? SB : 0);
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

// Everything the fused fitness + DE kernel needs besides the fitness inputs.
struct FuseArgs {
  StepArgs a;               // prob_ids / prob_base select the problem ids
  GenArgs e;                // counts, class totals, penalties, init flag
  uint32_t *done;           // [n_problems] finished-block tickets, zero between launches
  const uint32_t *segoff;   // tile set: first tile of segment (sub * K + class)
  uint32_t rows_in_lds;     // keep the post-selection population in LDS
};

}  // namespace mh
