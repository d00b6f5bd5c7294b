// de.hip -- differential evolution on the device (Section 2 eqs. mutation,
// crossover and selection; Section 3.3; Algorithm 4).
//
// The population never leaves HBM: initialisation, decoding, selection, the
// best-of-generation reduction, DE/best/1 mutation and binomial crossover all
// run here, one block per DE problem.  Every random number is a function of
// (seed, problem, generation, individual, slot), so results do not depend on
// launch shape or on which other problems share a launch.  f64 arithmetic
// uses explicitly rounded operations (no contraction) in a fixed order.
#include <cfloat>

#include "device_common.h"
#include "epilogue.h"
#include "internal.h"

namespace mh {
namespace {

__device__ __forceinline__ uint64_t prob_of(const uint64_t *prob_ids, uint64_t prob_base,
                                            uint32_t sub) {
  return prob_ids ? prob_ids[sub] : prob_base + sub;
}

// Algorithm 4, first loop: warm starts, then uniform draws inside the range
// limits (slot q of generation 0 for gene q).
__global__ void k_de_init(uint32_t P, uint32_t SB, uint32_t F, uint64_t seed,
                          const uint64_t *__restrict__ prob_ids, uint64_t prob_base,
                          uint32_t n_problems, const double *__restrict__ warm, uint32_t W,
                          double *__restrict__ pop) {
  const uint32_t m = 2 * SB;
  const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (uint64_t)n_problems * P * m) return;
  const uint32_t q = (uint32_t)(e % m);
  const uint32_t r = (uint32_t)((e / m) % P);
  const uint32_t sub = (uint32_t)(e / ((uint64_t)m * P));
  double v;
  if (r < W) {
    v = warm[(size_t)r * m + q];
  } else {
    const uint64_t key = de_key(seed, prob_of(prob_ids, prob_base, sub));
    const double u = to_unit(de_draw(key, 0, r, q));
    v = (q < SB) ? __dmul_rn(u, (double)F + 1.0) : u;
  }
  pop[e] = v;
}

// Decode [n_problems][P][2 SB] genes into (feat, tau).  With row_sel, decode
// only row row_sel[sub] of each problem into [n_problems][1][SB].
__global__ void k_decode(const double *__restrict__ genes, uint32_t P, uint32_t SB, uint32_t F,
                         const uint32_t *__restrict__ n_unique, uint8_t *__restrict__ feat,
                         uint32_t *__restrict__ tau, uint32_t n_problems,
                         const uint32_t *__restrict__ row_sel) {
  const uint32_t rows = row_sel ? 1u : P;
  const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (uint64_t)n_problems * rows * SB) return;
  const uint32_t t = (uint32_t)(e % SB);
  const uint32_t rr = (uint32_t)((e / SB) % rows);
  const uint32_t sub = (uint32_t)(e / ((uint64_t)SB * rows));
  const uint32_t r = row_sel ? row_sel[sub] : rr;
  const double *g = genes + ((size_t)sub * P + r) * 2 * SB;
  uint32_t f, th;
  decode_node(g[t], g[SB + t], F, n_unique, f, th);
  feat[e] = (uint8_t)f;
  tau[e] = th;
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
};

// Phases of one DE step for problem `sub`, thread r = individual r:
//  1. selection (eq. selection; ties go to the trial) when `select`, with
//     the trial's cost tc; or, when `init`, cost[r] = tc (generation 0);
//  2. best = lowest index of the minimum cost;
//  3. DE/best/1 mutation and binomial crossover of generation g into
//     next_trial, decoded into (feat, tau) when those are given.
// With `rows` (LDS, [P][m]) the post-selection population is also kept in
// LDS so that phase 3 reads its three parents there; s_nu caches n_unique.
__device__ __forceinline__ void de_step_body(const StepArgs &a, uint32_t sub, uint32_t r,
                                             bool select, bool init, double tc,
                                             double *s_cost, uint32_t *s_idx, double *rows,
                                             uint32_t *s_nu) {
  const uint32_t P = a.P, m = 2 * a.SB;
  double *pop = a.pop + (size_t)sub * P * m;
  double *cost = a.cost + (size_t)sub * P;
  if (a.feat && a.n_unique)
    for (uint32_t f = r; f < a.F; f += blockDim.x) s_nu[f] = a.n_unique[f];
  double my_cost = 0.0;
  if (r < P) {
    my_cost = cost[r];
    const bool take = select && tc <= my_cost;
    if (init || take) my_cost = tc;
    const double *tr = a.trial + ((size_t)sub * P + r) * m;
    double *pr = pop + (size_t)r * m;
    if (rows) {
      // through LDS, so that the global loads are not ordered behind stores
      double *row = rows + (size_t)r * m;
      const double *src = take ? tr : pr;
      for (uint32_t q = 0; q < m; ++q) row[q] = src[q];
      if (take)
        for (uint32_t q = 0; q < m; ++q) pr[q] = row[q];
    } else if (take) {
      for (uint32_t q = 0; q < m; ++q) pr[q] = tr[q];
    }
    if (init || take) cost[r] = my_cost;
  }
  s_cost[r] = r < P ? my_cost : DBL_MAX;
  s_idx[r] = r;
  __syncthreads();
  for (uint32_t d = blockDim.x >> 1; d > 0; d >>= 1) {
    if (r < d) {
      const double c2 = s_cost[r + d];
      const uint32_t i2 = s_idx[r + d];
      if (c2 < s_cost[r] || (c2 == s_cost[r] && i2 < s_idx[r])) {
        s_cost[r] = c2;
        s_idx[r] = i2;
      }
    }
    __syncthreads();
  }
  const uint32_t best = s_idx[0];
  if (r == 0 && a.best) a.best[sub] = best;
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
  const double *src = rows ? rows : pop;
  const double *sb = src + (size_t)best * m;
  const double *s1 = src + (size_t)r1 * m;
  const double *s2 = src + (size_t)r2 * m;
  const double *sr = src + (size_t)r * m;
  double *out = a.next_trial + ((size_t)sub * P + r) * m;
  const double Fp1 = (double)a.F + 1.0;
  uint8_t *fo = a.feat ? a.feat + ((size_t)sub * P + r) * a.SB : nullptr;
  uint32_t *to = a.feat ? a.tau + ((size_t)sub * P + r) * a.SB : nullptr;
  // a feature gene q < SB and its threshold gene SB + q are made together so
  // that the node can be decoded at once
  for (uint32_t q = 0; q < a.SB; ++q) {
    double gq[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint32_t qq = q + (h ? a.SB : 0u);
      const double d = __dsub_rn(s1[qq], s2[qq]);
      double v = __dadd_rn(sb[qq], __dmul_rn(Mr, d));
      const double hiq = h ? 1.0 : Fp1;
      if (!(v >= 0.0)) v = 0.0;
      if (v > hiq) v = hiq;
      const double u = to_unit(de_draw(key, g, r, 4u + qq));
      gq[h] = (u <= a.CR || qq == qr) ? v : sr[qq];
      out[qq] = gq[h];
    }
    if (fo) {
      uint32_t f, th;
      decode_node(gq[0], gq[1], a.F, s_nu, f, th);
      fo[q] = (uint8_t)f;
      to[q] = th;
    }
  }
}

// One block per problem, thread r = individual r; trial costs from memory.
__global__ __launch_bounds__(1024) void k_de_step(StepArgs a) {
  __shared__ double s_cost[1024];
  __shared__ uint32_t s_idx[1024];
  __shared__ uint32_t s_nu[256];
  extern __shared__ double rows[];
  const uint32_t sub = blockIdx.x, r = threadIdx.x;
  const bool select = a.trial != nullptr;
  const double tc = (select && r < a.P) ? a.trial_cost[(size_t)sub * a.P + r] : 0.0;
  de_step_body(a, sub, r, select, false, tc, s_cost, s_idx, a.rows_in_lds ? rows : nullptr, s_nu);
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
};

template <int D>
__global__ __launch_bounds__(1024) void k_de_gen(StepArgs a, GenArgs e) {
  constexpr int SB = (1 << D) - 1;
  __shared__ double s_cost[1024];
  __shared__ uint32_t s_idx[1024];
  __shared__ uint32_t s_nu[256];
  extern __shared__ double rows[];
  const uint32_t sub = blockIdx.x, r = threadIdx.x, P = a.P, Ppad = pad64(P);
  double tc = 0.0;
  if (r < P) {
    tc = epilogue_node_counts<D, CNT_REP>(e.cnt + (size_t)sub * SB * e.K * Ppad, e.ctot + (size_t)sub * e.K,
                                 e.K, Ppad, r, a.feat + ((size_t)sub * P + r) * SB, e.n_min,
                                 e.alpha, nullptr, nullptr, cnt_copy_elems(gridDim.x, SB, e.K, P))
             .cost;
  }
  de_step_body(a, sub, r, !e.init, e.init != 0, tc, s_cost, s_idx, a.rows_in_lds ? rows : nullptr,
               s_nu);
}

}  // namespace

mh_status launch_de_init(Ctx *ctx, uint32_t P, uint32_t D, uint32_t F, uint64_t seed,
                         const uint64_t *prob_ids, uint64_t prob_base, uint32_t n_problems,
                         const double *warm, uint32_t W, double *pop) {
  const uint32_t SB = (1u << D) - 1u;
  const uint64_t total = (uint64_t)n_problems * P * 2 * SB;
  if (total == 0) return MH_OK;
  const uint32_t blocks = (uint32_t)((total + 255) / 256);
  k_de_init<<<blocks, 256, 0, ctx->stream>>>(P, SB, F, seed, prob_ids, prob_base, n_problems, warm,
                                             W, pop);
  MH_LAUNCHED(ctx, "k_de_init");
  return MH_OK;
}

mh_status launch_decode(Ctx *ctx, const double *genes, uint32_t P, uint32_t D, uint32_t F,
                        const uint32_t *n_unique, uint8_t *feat, uint32_t *tau,
                        uint32_t n_problems, const uint32_t *row_sel) {
  const uint32_t SB = (1u << D) - 1u;
  const uint64_t total = (uint64_t)n_problems * (row_sel ? 1u : P) * SB;
  if (total == 0) return MH_OK;
  const uint32_t blocks = (uint32_t)((total + 255) / 256);
  k_decode<<<blocks, 256, 0, ctx->stream>>>(genes, P, SB, F, n_unique, feat, tau, n_problems,
                                            row_sel);
  MH_LAUNCHED(ctx, "k_decode");
  return MH_OK;
}

// LDS for the post-selection population when it fits in 48 KiB, else 0.
static size_t rows_lds_bytes(uint32_t P, uint32_t D) {
  const size_t b = (size_t)P * 2 * ((1u << D) - 1u) * 8;
  return b <= 48 * 1024 ? b : 0;
}

static StepArgs make_args(const DeDev &de, const uint64_t *prob_ids, uint64_t prob_base,
                          uint32_t g, double *pop, double *cost, const double *trial,
                          const double *trial_cost, uint32_t *best, double *next_trial,
                          uint8_t *feat, uint32_t *tau) {
  StepArgs a;
  a.P = de.P;
  a.SB = (1u << de.D) - 1u;
  a.F = de.F;
  a.g = g;
  a.M = de.M;
  a.CR = de.CR;
  a.seed = de.seed;
  a.n_unique = de.n_unique;
  a.prob_ids = prob_ids;
  a.prob_base = prob_base;
  a.pop = pop;
  a.cost = cost;
  a.trial = trial;
  a.trial_cost = trial_cost;
  a.best = best;
  a.next_trial = next_trial;
  a.feat = feat;
  a.tau = tau;
  a.rows_in_lds = rows_lds_bytes(de.P, de.D) > 0;
  return a;
}

static uint32_t step_threads(uint32_t P) {
  uint32_t threads = 64;
  while (threads < P) threads <<= 1;  // power of two for the argmin tree
  return threads;
}

mh_status launch_de_gen(Ctx *ctx, const DeDev &de, const uint64_t *prob_ids, uint64_t prob_base,
                        uint32_t n_problems, uint32_t g, bool init, double *pop, double *cost,
                        const double *trial, uint32_t *best, double *next_trial, uint8_t *feat,
                        uint32_t *tau, uint32_t *cnt, const uint32_t *ctot, uint32_t K,
                        uint32_t n_min, double alpha) {
  StepArgs a = make_args(de, prob_ids, prob_base, g, pop, cost, trial, nullptr, best, next_trial,
                         feat, tau);
  GenArgs e{cnt, ctot, K, n_min, alpha, init ? 1 : 0};
  const uint32_t threads = step_threads(de.P);
  const size_t lds = rows_lds_bytes(de.P, de.D);
  hipStream_t st = ctx->stream;
  switch (de.D) {
    case 1: k_de_gen<1><<<n_problems, threads, lds, st>>>(a, e); break;
    case 2: k_de_gen<2><<<n_problems, threads, lds, st>>>(a, e); break;
    case 3: k_de_gen<3><<<n_problems, threads, lds, st>>>(a, e); break;
    case 4: k_de_gen<4><<<n_problems, threads, lds, st>>>(a, e); break;
    case 5: k_de_gen<5><<<n_problems, threads, lds, st>>>(a, e); break;
    default: return fail(ctx, MH_EINVAL, "fused DE step supports depth 1..5");
  }
  MH_LAUNCHED(ctx, "k_de_gen");
  return MH_OK;
}

mh_status launch_de_step(Ctx *ctx, const DeDev &de, const uint64_t *prob_ids, uint64_t prob_base,
                         uint32_t n_problems, uint32_t g, double *pop, double *cost,
                         const double *trial, const double *trial_cost, uint32_t *best,
                         double *next_trial, uint8_t *feat, uint32_t *tau) {
  StepArgs a = make_args(de, prob_ids, prob_base, g, pop, cost, trial, trial_cost, best,
                         next_trial, feat, tau);
  const uint32_t threads = step_threads(de.P);
  k_de_step<<<n_problems, threads, rows_lds_bytes(de.P, de.D), ctx->stream>>>(a);
  MH_LAUNCHED(ctx, "k_de_step");
  return MH_OK;
}

}  // namespace mh
