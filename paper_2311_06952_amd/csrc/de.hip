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

#include "de_body.h"
#include "device_common.h"
#include "epilogue.h"
#include "internal.h"

namespace mh {
namespace {

// Algorithm 4, first loop: warm starts, then uniform draws inside the range
// limits (slot q of generation 0 for gene q).
// Gene (r, q) of a problem's population lives at r * rs + q * qs: rs = m,
// qs = 1 is the row-major [P][m] layout of the C ABI; rs = 1, qs = P the
// gene-major layout used inside the DE loops (consecutive individuals at
// consecutive addresses, so that a wave's accesses coalesce).
__global__ void k_de_init(uint32_t P, uint32_t SB, uint32_t F, uint64_t seed,
                          const uint64_t *__restrict__ prob_ids, uint64_t prob_base,
                          uint32_t n_problems, const double *__restrict__ warm, uint32_t W,
                          double *__restrict__ pop, uint32_t rs, uint32_t qs) {
  const uint32_t m = 2 * SB;
  const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (uint64_t)n_problems * P * m) return;
  // e enumerates (sub, q, r) with r fastest
  const uint32_t r = (uint32_t)(e % P);
  const uint32_t q = (uint32_t)((e / P) % m);
  const uint32_t sub = (uint32_t)(e / ((uint64_t)m * P));
  double v;
  if (r < W) {
    v = warm[((size_t)sub * W + r) * m + q];  // each problem's own warm starts
  } else {
    const uint64_t key = de_key(seed, prob_of(prob_ids, prob_base, sub));
    const double u = to_unit(de_draw(key, 0, r, q));
    v = (q < SB) ? __dmul_rn(u, (double)F + 1.0) : u;
  }
  pop[(size_t)sub * P * m + (size_t)r * rs + (size_t)q * qs] = v;
}

// Decode [n_problems][P][2 SB] genes into (feat, tau).  With row_sel, decode
// only row row_sel[sub] of each problem into [n_problems][1][SB].
__global__ void k_decode(const double *__restrict__ genes, uint32_t P, uint32_t SB, uint32_t F,
                         const uint32_t *__restrict__ n_unique, uint8_t *__restrict__ feat,
                         uint32_t *__restrict__ tau, uint32_t n_problems,
                         const uint32_t *__restrict__ row_sel, uint32_t rs, uint32_t qs) {
  const uint32_t rows = row_sel ? 1u : P;
  const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (uint64_t)n_problems * rows * SB) return;
  const uint32_t t = (uint32_t)(e % SB);
  const uint32_t rr = (uint32_t)((e / SB) % rows);
  const uint32_t sub = (uint32_t)(e / ((uint64_t)SB * rows));
  const uint32_t r = row_sel ? row_sel[sub] : rr;
  const double *g = genes + (size_t)sub * P * 2 * SB + (size_t)r * rs;
  uint32_t f, th;
  decode_node(g[(size_t)t * qs], g[(size_t)(SB + t) * qs], F, n_unique, f, th);
  feat[e] = (uint8_t)f;
  tau[e] = th;
}

// One block per problem; tpi threads per individual (individual r =
// threadIdx.x % nr, its lane j = threadIdx.x / nr, nr = blockDim.x / tpi a
// power of two >= P); trial costs from memory.
__global__ __launch_bounds__(1024) void k_de_step(StepArgs a, uint32_t tpi) {
  __shared__ double s_cost[1024];
  __shared__ uint32_t s_idx[1024];
  __shared__ uint32_t s_nu[256];
  extern __shared__ double rows[];
  const uint32_t nr = blockDim.x / tpi;
  const uint32_t sub = blockIdx.x, r = threadIdx.x % nr, j = threadIdx.x / nr;
  const bool select = a.trial != nullptr;
  const double tc = (select && r < a.P) ? a.trial_cost[(size_t)sub * a.P + r] : 0.0;
  de_step_body(a, sub, r, j, tpi, select, false, tc, s_cost, s_idx, a.rows_in_lds ? rows : nullptr,
               s_nu);
}

template <int D, int LB>
__global__ __launch_bounds__(LB) void k_de_gen(StepArgs a, GenArgs e) {
  constexpr int SB = (1 << D) - 1;
  __shared__ double s_cost[1024];
  __shared__ uint32_t s_idx[1024];
  __shared__ uint32_t s_nu[256];
  extern __shared__ double rows[];
  (void)SB;
  de_gen_body<D, CNT_REP, false, (LB <= 256)>(a, e, blockIdx.x, s_cost, s_idx,
                                              a.rows_in_lds ? rows : nullptr, s_nu);
}

// The same generation split over the chip for large populations (one block
// of de_gen_body would make every individual's draws and float64 work one
// after another on a single CU).  Same arithmetic and results.
//
// Part 1, individual r of problem blockIdx.y on e.tpi adjacent lanes (lane j
// of the group takes classes j, j + tpi, ... of the epilogue and genes j,
// j + tpi, ... of the copy): the epilogue of the evaluated population's node
// counts (its cost), then selection (eq. selection, ties to the trial) or, in
// generation 0, the initial cost; the consumed counters go back to zero.
constexpr uint32_t SPLIT_THREADS = 256;

template <int D, int TPI>
__global__ __launch_bounds__(SPLIT_THREADS) void k_de_select(StepArgs a, GenArgs e) {
  constexpr int SB = (1 << D) - 1, m = 2 * SB;
  constexpr uint32_t tpi = TPI;
  const uint32_t sub = blockIdx.y, P = a.P, Ppad = pad64(P), K = e.K;
  const uint32_t r = (blockIdx.x * SPLIT_THREADS + threadIdx.x) / tpi, j = threadIdx.x % tpi;
  if (r >= P) return;  // whole groups leave together
  double *cost = a.cost + (size_t)sub * P;
  // the parent's cost and this lane's share of the trial genes are loaded
  // with the counts, before the selection is known, so that the step waits
  // for memory once
  constexpr int QM = (m + TPI - 1) / TPI;  // genes per lane
  double v[QM];
  double pc = 0.0;
  if (!e.init) {
    pc = cost[r];
    const double *tr = a.trial + (size_t)sub * P * m + (size_t)r * a.rs;
#pragma unroll
    for (int i = 0; i < QM; ++i) {
      const uint32_t q = j + (uint32_t)i * tpi;
      if (q < (uint32_t)m) v[i] = tr[(size_t)q * a.qs];
    }
  }
  const size_t rep = cnt_copy_elems(e.n_problems, SB, K, P);
  const TreeScore sc = epilogue_node_counts<D, CNT_REP>(
      e.cnt + (size_t)sub * SB * K * Ppad, e.ctot + (size_t)sub * K, K, Ppad, r,
      a.feat + ((size_t)sub * P + r) * SB, e.n_min, e.alpha, nullptr, nullptr, rep, tpi);
  if (e.init) {
    if (j == 0) cost[r] = sc.cost;
    return;
  }
  if (!(sc.cost <= pc)) return;
  double *pr = a.pop + (size_t)sub * P * m + (size_t)r * a.rs;
#pragma unroll
  for (int i = 0; i < QM; ++i) {
    const uint32_t q = j + (uint32_t)i * tpi;
    if (q < (uint32_t)m) pr[(size_t)q * a.qs] = v[i];
  }
  if (j == 0) cost[r] = sc.cost;
}

// Part 2, one thread per (node t, individual r) of problem blockIdx.y, r
// fastest so that a wave's gene reads coalesce (gene-major population):
// every block first finds best (lowest index of the minimum cost) itself,
// block 0 writes it; then DE/best/1 mutation of the node's two genes, clamp,
// binomial crossover, the trial genes, and the node decoded into (feat, tau).
// Any depth (SB = a.SB).
__global__ __launch_bounds__(SPLIT_THREADS) void k_de_mutate(StepArgs a) {
  const uint32_t SB = a.SB;
  __shared__ double s_c[SPLIT_THREADS / 64];
  __shared__ uint32_t s_i[SPLIT_THREADS / 64];
  const uint32_t sub = blockIdx.y, P = a.P;
  const double *cost = a.cost + (size_t)sub * P;
  double bc = DBL_MAX;
  uint32_t bi = 0xFFFFFFFFu;
  for (uint32_t i = threadIdx.x; i < P; i += SPLIT_THREADS) {
    const double c = cost[i];
    if (c < bc) {  // ascending i in this thread: ties keep the lower index
      bc = c;
      bi = i;
    }
  }
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
    s_c[threadIdx.x >> 6] = bc;
    s_i[threadIdx.x >> 6] = bi;
  }
  __syncthreads();
  bc = s_c[0];
  bi = s_i[0];
  for (uint32_t x = 1; x < SPLIT_THREADS / 64; ++x) {
    if (s_c[x] < bc || (s_c[x] == bc && s_i[x] < bi)) {
      bc = s_c[x];
      bi = s_i[x];
    }
  }
  const uint32_t bst = bi;
  if (blockIdx.x == 0 && threadIdx.x == 0 && a.best) a.best[sub] = bst;
  if (!a.next_trial) return;
  const uint32_t e = blockIdx.x * SPLIT_THREADS + threadIdx.x;
  if (e >= P * SB) return;
  const uint32_t t = e / P, r = e % P;
  const uint32_t m = 2 * SB;
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
  const double *pop = a.pop + (size_t)sub * P * m;
  double *out = a.next_trial + (size_t)sub * P * m;
  const double Fp1 = (double)a.F + 1.0;
  double gq[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const uint32_t qq = t + (h ? SB : 0u);
    const double *row = pop + (size_t)qq * a.qs;
    const double d = __dsub_rn(row[(size_t)r1 * a.rs], row[(size_t)r2 * a.rs]);
    double v = __dadd_rn(row[(size_t)bst * a.rs], __dmul_rn(Mr, d));
    const double hiq = h ? 1.0 : Fp1;
    if (!(v >= 0.0)) v = 0.0;
    if (v > hiq) v = hiq;
    const double u = to_unit(de_draw(key, g, r, 4u + qq));
    gq[h] = (u <= a.CR || qq == qr) ? v : row[(size_t)r * a.rs];
    out[(size_t)qq * a.qs + (size_t)r * a.rs] = gq[h];
  }
  if (a.feat) {
    uint32_t f, th;
    decode_node(gq[0], gq[1], a.F, a.n_unique, f, th);
    a.feat[((size_t)sub * P + r) * SB + t] = (uint8_t)f;
    a.tau[((size_t)sub * P + r) * SB + t] = th;
  }
}

// One DE generation of a problem whose trial costs are already in memory
// (the walk path), one thread per (node t, individual r), r fastest: the
// selection of generation g - 1 (eq. selection, ties to the trial) and the
// trial of generation g in one launch.  Selection is applied where it is
// read: individual j's post-selection gene is trial[j] when
// cost_t[j] <= cost[j], else pop[j], and its post-selection cost the smaller
// rule's pick; every block finds best from those, block 0 writes it.  The
// thread of (t, r) also stores r's two selected genes into pop (and, for
// t = 0, r's cost into cost) when the trial won.  These stores race with no
// read: a taken individual's genes and cost are read from the trial side, and
// an individual whose trial lost is never written; the cost rule picks the
// same value before and after its store.  The trial population is read from
// `trial` and the next one written to a different buffer, next_trial
// (generation g; null: only the selection and best).  Without trial
// (generation 1 from the initial population) nothing is selected.
__global__ __launch_bounds__(SPLIT_THREADS) void k_de_select_mutate(StepArgs a) {
  const uint32_t SB = a.SB, P = a.P, m = 2 * SB;
  __shared__ double s_c[SPLIT_THREADS / 64];
  __shared__ uint32_t s_i[SPLIT_THREADS / 64];
  double *cost = a.cost;
  const double *ct = a.trial_cost;
  const bool sel = a.trial != nullptr;
  auto post_cost = [&](uint32_t j) {
    const double c = cost[j];
    if (!sel) return c;
    const double t = ct[j];
    return t <= c ? t : c;
  };
  double bc = DBL_MAX;
  uint32_t bi = 0xFFFFFFFFu;
  for (uint32_t i = threadIdx.x; i < P; i += SPLIT_THREADS) {
    const double c = post_cost(i);
    if (c < bc) {  // ascending i in this thread: ties keep the lower index
      bc = c;
      bi = i;
    }
  }
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
    s_c[threadIdx.x >> 6] = bc;
    s_i[threadIdx.x >> 6] = bi;
  }
  __syncthreads();
  bc = s_c[0];
  bi = s_i[0];
  for (uint32_t x = 1; x < SPLIT_THREADS / 64; ++x) {
    if (s_c[x] < bc || (s_c[x] == bc && s_i[x] < bi)) {
      bc = s_c[x];
      bi = s_i[x];
    }
  }
  const uint32_t bst = bi;
  if (blockIdx.x == 0 && threadIdx.x == 0 && a.best) a.best[0] = bst;
  const uint32_t e = blockIdx.x * SPLIT_THREADS + threadIdx.x;
  if (e >= P * SB) return;
  const uint32_t t = e / P, r = e % P;
  double *pop = a.pop;
  const double *tr = a.trial;
  auto taken = [&](uint32_t j) { return sel && ct[j] <= cost[j]; };
  // gene q of individual j after selection (gene-major: q * P + j)
  auto gene = [&](uint32_t j, bool tk, uint32_t q) {
    const size_t o = (size_t)q * P + j;
    return tk ? tr[o] : pop[o];
  };
  const bool tk_r = taken(r);
  if (!a.next_trial) {
    if (tk_r) {
      pop[(size_t)t * P + r] = tr[(size_t)t * P + r];
      pop[(size_t)(SB + t) * P + r] = tr[(size_t)(SB + t) * P + r];
      if (t == 0) cost[r] = ct[r];
    }
    return;
  }
  const uint64_t key = de_key(a.seed, a.prob_base);
  const uint32_t g = a.g;
  const double Mr = a.M >= 0.0 ? a.M : to_unit(de_draw(key, g, r, 0));
  uint32_t r1 = to_below(de_draw(key, g, r, 1), P - 1u);
  r1 += (r1 >= r) ? 1u : 0u;
  uint32_t r2 = to_below(de_draw(key, g, r, 2), P - 2u);
  const uint32_t lo = r < r1 ? r : r1, hi = r < r1 ? r1 : r;
  r2 += (r2 >= lo) ? 1u : 0u;
  r2 += (r2 >= hi) ? 1u : 0u;
  const uint32_t qr = to_below(de_draw(key, g, r, 3), m);
  const bool tk_b = taken(bst), tk_1 = taken(r1), tk_2 = taken(r2);
  const double Fp1 = (double)a.F + 1.0;
  double gq[2], own[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const uint32_t qq = t + (h ? SB : 0u);
    own[h] = gene(r, tk_r, qq);
    const double d = __dsub_rn(gene(r1, tk_1, qq), gene(r2, tk_2, qq));
    double v = __dadd_rn(gene(bst, tk_b, qq), __dmul_rn(Mr, d));
    const double hiq = h ? 1.0 : Fp1;
    if (!(v >= 0.0)) v = 0.0;
    if (v > hiq) v = hiq;
    const double u = to_unit(de_draw(key, g, r, 4u + qq));
    gq[h] = (u <= a.CR || qq == qr) ? v : own[h];
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const uint32_t qq = t + (h ? SB : 0u);
    a.next_trial[(size_t)qq * P + r] = gq[h];
    if (tk_r) pop[(size_t)qq * P + r] = own[h];
  }
  if (tk_r && t == 0) cost[r] = ct[r];
  if (a.feat) {
    uint32_t f, th;
    decode_node(gq[0], gq[1], a.F, a.n_unique, f, th);
    a.feat[(size_t)r * SB + t] = (uint8_t)f;
    a.tau[(size_t)r * SB + t] = th;
  }
}

// One block per job (problem), each with its own population, tile-set
// counts and generation; threads r < P of the job are its individuals.
template <int D, int LB>
__global__ __launch_bounds__(LB) void k_de_jobs(const GenJob *__restrict__ jobs) {
  constexpr int SB = (1 << D) - 1;
  __shared__ double s_cost[1024];
  __shared__ uint32_t s_idx[1024];
  __shared__ uint32_t s_nu[256];
  extern __shared__ double rows[];
  (void)SB;
  const GenJob jb = jobs[blockIdx.x];
  de_gen_body<D, CNT_REP, false, (LB <= 256)>(jb.a, jb.e, 0, s_cost, s_idx,
                                              jb.a.rows_in_lds ? rows : nullptr, s_nu);
}

}  // namespace

mh_status launch_de_init(Ctx *ctx, uint32_t P, uint32_t D, uint32_t F, uint64_t seed,
                         const uint64_t *prob_ids, uint64_t prob_base, uint32_t n_problems,
                         const double *warm, uint32_t W, double *pop, bool gene_major) {
  const uint32_t SB = (1u << D) - 1u;
  const uint64_t total = (uint64_t)n_problems * P * 2 * SB;
  if (total == 0) return MH_OK;
  const uint32_t blocks = (uint32_t)((total + 255) / 256);
  k_de_init<<<blocks, 256, 0, ctx->stream>>>(P, SB, F, seed, prob_ids, prob_base, n_problems, warm,
                                             W, pop, gene_major ? 1u : 2 * SB,
                                             gene_major ? P : 1u);
  MH_LAUNCHED(ctx, "k_de_init");
  return MH_OK;
}

mh_status launch_decode(Ctx *ctx, const double *genes, uint32_t P, uint32_t D, uint32_t F,
                        const uint32_t *n_unique, uint8_t *feat, uint32_t *tau,
                        uint32_t n_problems, const uint32_t *row_sel, bool gene_major) {
  const uint32_t SB = (1u << D) - 1u;
  const uint64_t total = (uint64_t)n_problems * (row_sel ? 1u : P) * SB;
  if (total == 0) return MH_OK;
  const uint32_t blocks = (uint32_t)((total + 255) / 256);
  k_decode<<<blocks, 256, 0, ctx->stream>>>(genes, P, SB, F, n_unique, feat, tau, n_problems,
                                            row_sel, gene_major ? 1u : 2 * SB,
                                            gene_major ? P : 1u);
  MH_LAUNCHED(ctx, "k_decode");
  return MH_OK;
}

// LDS for the post-selection population when it fits in `limit` bytes
// (48 KiB unless the launch has more to give), else 0.
static size_t rows_lds_bytes(uint32_t P, uint32_t D, size_t limit = 48 * 1024) {
  const size_t b = (size_t)P * 2 * ((1u << D) - 1u) * 8;
  return b <= limit ? b : 0;
}
// The most dynamic LDS a one-block-per-problem DE kernel may take: the
// device's per-block limit less its static arrays (argmin scratch, n_unique).
static size_t de_rows_limit(const Ctx *ctx) {
  const size_t stat = 1024 * 8 + 1024 * 4 + 256 * 4 + 1024;
  return ctx->max_lds > stat ? ctx->max_lds - stat : 0;
}

static StepArgs make_args(const DeDev &de, const uint64_t *prob_ids, uint64_t prob_base,
                          uint32_t g, double *pop, double *cost, const double *trial,
                          const double *trial_cost, uint32_t *best, double *next_trial,
                          uint8_t *feat, uint32_t *tau) {
  StepArgs a;
  const uint32_t m = 2 * ((1u << de.D) - 1u);
  a.rs = de.gene_major ? 1u : m;
  a.qs = de.gene_major ? de.P : 1u;
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

// From this population size on a generation's DE work runs as two launches
// spread over the chip instead of one block per problem.
constexpr uint32_t DE_SPLIT_MIN_P = 256;

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
  const uint32_t rp = step_threads(de.P);
  const uint32_t tpi = 1;  // more threads per individual measured slower
  GenArgs e{cnt, ctot, K, n_min, alpha, init ? 1 : 0, tpi, n_problems};
  if (de.P >= DE_SPLIT_MIN_P) {
    // large populations: the generation as two launches spread over the chip;
    // the epilogue and selection of an individual on up to 4 lanes (one per
    // class), so that its count loads and gene copies are spread out
    hipStream_t st = ctx->stream;
    const uint32_t SB = (1u << de.D) - 1u;
    uint32_t stpi = 1;
    while (stpi < K && stpi < 4) stpi <<= 1;
    if (ctx->de_select_tpi) stpi = ctx->de_select_tpi;
    e.tpi = stpi;
    const dim3 g1((de.P * stpi + SPLIT_THREADS - 1) / SPLIT_THREADS, n_problems);
    const dim3 g2((de.P * SB + SPLIT_THREADS - 1) / SPLIT_THREADS, n_problems);
#define MH_SPLIT(DD)                                                          \
  if (stpi == 1) k_de_select<DD, 1><<<g1, SPLIT_THREADS, 0, st>>>(a, e);      \
  else if (stpi == 2) k_de_select<DD, 2><<<g1, SPLIT_THREADS, 0, st>>>(a, e); \
  else if (stpi == 4) k_de_select<DD, 4><<<g1, SPLIT_THREADS, 0, st>>>(a, e); \
  else k_de_select<DD, 8><<<g1, SPLIT_THREADS, 0, st>>>(a, e);                \
  k_de_mutate<<<g2, SPLIT_THREADS, 0, st>>>(a);
    switch (de.D) {
      case 1: MH_SPLIT(1) break;
      case 2: MH_SPLIT(2) break;
      case 3: MH_SPLIT(3) break;
      case 4: MH_SPLIT(4) break;
      case 5: MH_SPLIT(5) break;
      default: return fail(ctx, MH_EINVAL, "fused DE step supports depth 1..5");
    }
#undef MH_SPLIT
    MH_LAUNCHED(ctx, "k_de_select/k_de_mutate");
    return MH_OK;
  }
  const uint32_t threads = rp * tpi;
  const size_t lds = rows_lds_bytes(de.P, de.D, de_rows_limit(ctx));
  a.rows_in_lds = lds > 0;
  hipStream_t st = ctx->stream;
#define MH_GEN(DD)                                                            \
  if (threads <= 256)                                                         \
    k_de_gen<DD, 256><<<n_problems, threads, lds, st>>>(a, e);                \
  else                                                                        \
    k_de_gen<DD, 1024><<<n_problems, threads, lds, st>>>(a, e);
  switch (de.D) {
    case 1: MH_GEN(1) break;
    case 2: MH_GEN(2) break;
    case 3: MH_GEN(3) break;
    case 4: MH_GEN(4) break;
    case 5: MH_GEN(5) break;
    default: return fail(ctx, MH_EINVAL, "fused DE step supports depth 1..5");
  }
#undef MH_GEN
  MH_LAUNCHED(ctx, "k_de_gen");
  return MH_OK;
}

GenJob make_gen_job(const DeDev &de, uint64_t prob, uint32_t g, bool init, double *pop,
                    double *cost, const double *trial, uint32_t *best, double *next_trial,
                    uint8_t *feat, uint32_t *tau, uint32_t *cnt, const uint32_t *ctot,
                    uint32_t K, uint32_t n_min, double alpha, uint32_t P_max) {
  GenJob j;
  j.a = make_args(de, nullptr, prob, g, pop, cost, trial, nullptr, best, next_trial, feat, tau);
  // every job of a launch shares the dynamic LDS sized for the largest one
  j.a.rows_in_lds = rows_lds_bytes(P_max, de.D) > 0;
  j.e = GenArgs{cnt, ctot, K, n_min, alpha, init ? 1 : 0, 1u, 1u};
  return j;
}

mh_status launch_de_jobs(Ctx *ctx, uint32_t D, const GenJob *jobs, uint32_t n_jobs,
                         uint32_t P_max) {
  if (n_jobs == 0) return MH_OK;
  if (P_max > 1024) return fail(ctx, MH_EINVAL, "DE jobs support P <= 1024");
  const uint32_t threads = step_threads(P_max);
  const size_t lds = rows_lds_bytes(P_max, D);
  hipStream_t st = ctx->stream;
#define MH_JOBS(DD)                                                           \
  if (threads <= 256)                                                         \
    k_de_jobs<DD, 256><<<n_jobs, threads, lds, st>>>(jobs);                   \
  else                                                                        \
    k_de_jobs<DD, 1024><<<n_jobs, threads, lds, st>>>(jobs);
  switch (D) {
    case 1: MH_JOBS(1) break;
    case 2: MH_JOBS(2) break;
    case 3: MH_JOBS(3) break;
    case 4: MH_JOBS(4) break;
    case 5: MH_JOBS(5) break;
    default: return fail(ctx, MH_EINVAL, "DE jobs support depth 1..5");
  }
#undef MH_JOBS
  MH_LAUNCHED(ctx, "k_de_jobs");
  return MH_OK;
}

FuseArgs make_fuse(const DeDev &de, const uint64_t *prob_ids, uint64_t prob_base,
                   uint32_t n_problems, uint32_t g, bool init, double *pop, double *cost,
                   const double *trial, uint32_t *best, double *next_trial, uint8_t *feat,
                   uint32_t *tau, uint32_t *cnt, const uint32_t *ctot, uint32_t K, uint32_t n_min,
                   double alpha, uint32_t *done, const uint32_t *segoff) {
  FuseArgs f;
  f.a = make_args(de, prob_ids, prob_base, g, pop, cost, trial, nullptr, best, next_trial, feat,
                  tau);
  f.e = GenArgs{cnt, ctot, K, n_min, alpha, init ? 1 : 0, 1u, n_problems};
  f.done = done;
  f.segoff = segoff;
  f.rows_in_lds = rows_lds_bytes(de.P, de.D) > 0 ? 1u : 0u;
  f.a.rows_in_lds = (int)f.rows_in_lds;
  return f;
}

bool fusable(uint32_t P, uint32_t D, uint32_t F) {
  return D >= 1 && D <= 5 && F <= 80 && fused_threads(P) <= fitness_block_threads(P) &&
         fitness_block_threads(P) >= pad64(P);
}

mh_status launch_de_select_mutate(Ctx *ctx, const DeDev &de, uint64_t prob, uint32_t g,
                                 double *pop, double *cost, const double *trial,
                                 const double *trial_cost, uint32_t *best, double *next_trial,
                                 uint8_t *feat, uint32_t *tau) {
  StepArgs a = make_args(de, nullptr, prob, g, pop, cost, trial, trial_cost, best, next_trial,
                         feat, tau);
  const uint32_t SB = (1u << de.D) - 1u;
  const uint32_t blocks = (de.P * SB + SPLIT_THREADS - 1) / SPLIT_THREADS;
  k_de_select_mutate<<<blocks, SPLIT_THREADS, 0, ctx->stream>>>(a);
  MH_LAUNCHED(ctx, "k_de_select_mutate");
  return MH_OK;
}

mh_status launch_de_step(Ctx *ctx, const DeDev &de, const uint64_t *prob_ids, uint64_t prob_base,
                         uint32_t n_problems, uint32_t g, double *pop, double *cost,
                         const double *trial, const double *trial_cost, uint32_t *best,
                         double *next_trial, uint8_t *feat, uint32_t *tau) {
  StepArgs a = make_args(de, prob_ids, prob_base, g, pop, cost, trial, trial_cost, best,
                         next_trial, feat, tau);
  const uint32_t nr = step_threads(de.P);
  // deep trees: several threads per individual share its nodes (about 32
  // genes each); shallow ones keep one
  const uint32_t m = 2u * ((1u << de.D) - 1u);
  uint32_t tpi = 1;
  while (tpi * 2u * nr <= 1024u && tpi * 2u * 32u <= m) tpi *= 2u;
  k_de_step<<<n_problems, nr * tpi, rows_lds_bytes(de.P, de.D), ctx->stream>>>(a, tpi);
  MH_LAUNCHED(ctx, "k_de_step");
  return MH_OK;
}

namespace {
// Transpose of a gene-major population into rows: element e = r * m + q.
__global__ void k_pop_rows(const double *__restrict__ gm, uint32_t P, uint32_t m,
                           double *__restrict__ rows) {
  const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (uint64_t)P * m) return;
  const uint32_t r = (uint32_t)(e / m), q = (uint32_t)(e % m);
  rows[e] = gm[(size_t)q * P + r];
}
}  // namespace

mh_status launch_pop_rows(Ctx *ctx, const double *gene_major, uint32_t P, uint32_t m,
                          double *rows) {
  const uint64_t total = (uint64_t)P * m;
  if (total == 0) return MH_OK;
  k_pop_rows<<<(uint32_t)((total + 255) / 256), 256, 0, ctx->stream>>>(gene_major, P, m, rows);
  MH_LAUNCHED(ctx, "k_pop_rows");
  return MH_OK;
}

namespace {
// One solved tree, its labels, correct count, cost and a status word, copied
// into one record (pinned host memory) so that the host waits once.
__global__ void k_pack_result(uint32_t D, uint32_t SB, uint32_t SL, const uint8_t *__restrict__ f1,
                              const uint32_t *__restrict__ t1, const uint8_t *__restrict__ lab1,
                              const uint32_t *__restrict__ corr1, const double *__restrict__ cost1,
                              const uint32_t *__restrict__ flag_a,
                              const uint32_t *__restrict__ flag_b, ResultOut *out) {
  for (uint32_t i = threadIdx.x; i < SL; i += blockDim.x) {
    if (i < SB) {
      out->tree.feat[i] = f1[i];
      out->tree.tau[i] = t1[i];
    }
    out->tree.label[i] = lab1[i];
  }
  if (threadIdx.x == 0) {
    out->tree.D = D;
    out->tree.correct = *corr1;
    out->tree.cost = *cost1;
    const uint32_t a = flag_a ? *flag_a : 0u, b = flag_b ? *flag_b : 0u;
    out->flag = (a ? 1u : 0u) | (b << 1);
  }
}
}  // namespace

mh_status launch_pack_result(Ctx *ctx, uint32_t D, const uint8_t *f1, const uint32_t *t1,
                             const uint8_t *lab1, const uint32_t *corr1, const double *cost1,
                             const uint32_t *flag_a, const uint32_t *flag_b, ResultOut *out) {
  const uint32_t SB = (1u << D) - 1u, SL = 1u << D;
  k_pack_result<<<1, 64, 0, ctx->stream>>>(D, SB, SL, f1, t1, lab1, corr1, cost1, flag_a, flag_b,
                                            out);
  MH_LAUNCHED(ctx, "k_pack_result");
  return MH_OK;
}

}  // namespace mh
