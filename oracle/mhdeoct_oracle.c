/*
 * mhdeoct_oracle.c -- plain, slow CPU oracle for the
 * MH-DEOCT fitness-evaluation path (Ren et al., "A GPU-Accelerated
 * Moving-Horizon Algorithm for Training Deep Classification Trees on Large
 * Datasets", arXiv 2311.06952).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the CPU implementation that the HIP
 * library's results are compared against.  Only the test suite, the smoke entry point and the CPU
 * baseline leg of the benchmark may load it.  The product library never links,
 * loads or calls it, and it shares no code, header, table or helper with the
 * HIP path.
 *
 * Every function follows the paper's definitions in the paper's order, with no
 * blocking, fusion or reordering.  Where the paper leaves a choice open the
 * reading taken is stated at the function (readings R1..R12 in the design
 * notes).  Indices are 0-based here; tree nodes use the paper's 1-based heap
 * numbering t = 1..T internally and are stored at array slot t-1.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no FMA contraction,
 * so that every f64 operation is a single IEEE rounding, exactly as written).
 * The one parallel loop is oracle_fitness's loop over individuals: each
 * individual's counts, labels and cost are its own, so the thread count
 * (OMP_NUM_THREADS) never changes a result; everything else is sequential.
 *
 * Parity status per function (pins live in tests/test_oracle_*.py):
 *   oracle_rank_encode   pinned (numpy.unique special case, -0/+0, NaN)
 *   oracle_decode        pinned (closed form, ulp edges)
 *   oracle_route         pinned (hand-worked trees, brute force)
 *   oracle_fitness       pinned (hand-worked golden example, brute force,
 *                        invariants)
 *   oracle_split1        pinned (brute force over all (f, tau))
 *   oracle_opt2          pinned (brute force over all 3-node trees)
 *   oracle_greedy_tree   pinned (equals MH with horizon 1; brute force at D=1)
 *   oracle_splitmix64_*  pinned (published SplitMix64 output sequence)
 *   oracle_de_*          trajectories: parity unpinned against the paper
 *                        (the paper prints no trajectory); pinned by
 *                        properties (monotone best, CR=0, M=0, <= opt2)
 *   oracle_mh_train      parity unpinned against the paper; pinned by the
 *                        horizon-1 special case (greedy tree)
 *   oracle_tree_encode   pinned (decode(encode(tree)) == tree, hand-worked
 *                        genes)
 *   oracle_tree_thresholds, oracle_predict
 *                        pinned (the paper's scaled midpoint sets in exact
 *                        rationals; equal to rank routing on training rows)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)

/* ------------------------------------------------------------------------ */
/* Counter-based random numbers: SplitMix64 (Steele, Lea and Flood, "Fast   */
/* splittable pseudorandom number generators", OOPSLA 2014).  The k-th      */
/* output (k >= 1) of the generator seeded with s is mix(s + k * gamma).    */
/* ------------------------------------------------------------------------ */
#define OR_GAMMA 0x9E3779B97F4A7C15ULL

static uint64_t or_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* Sequential SplitMix64: advance the state by gamma, return the mix. */
uint64_t oracle_splitmix64_next(uint64_t *state) {
  *state += OR_GAMMA;
  return or_mix64(*state);
}

/* Output number (c + 1) of SplitMix64 seeded with s. */
static uint64_t or_sm_at(uint64_t s, uint64_t c) {
  return or_mix64(s + (c + 1u) * OR_GAMMA);
}

/* The DE random stream (reading R8): a per-problem key is output (prob + 1)
 * of SplitMix64 seeded with `seed`; draw (g, r, slot) is output
 * ((g << 40 | r << 20 | slot) + 1) of SplitMix64 seeded with that key.
 * Requires g < 2^24, r < 2^20, slot < 2^20. */
uint64_t oracle_draw(uint64_t seed, uint64_t prob, uint32_t g, uint32_t r,
                     uint32_t slot) {
  uint64_t key = or_sm_at(seed, prob);
  uint64_t ctr = ((uint64_t)g << 40) | ((uint64_t)r << 20) | (uint64_t)slot;
  return or_sm_at(key, ctr);
}

/* Uniform double in [0, 1): the top 53 bits times 2^-53. */
double oracle_u01(uint64_t u) { return (double)(u >> 11) * (1.0 / 9007199254740992.0); }

/* Uniform integer in [0, m): the top 32 bits scaled by m (multiply-shift). */
uint32_t oracle_uint(uint64_t u, uint32_t m) {
  return (uint32_t)(((u >> 32) * (uint64_t)m) >> 32);
}

/* ------------------------------------------------------------------------ */
/* Threshold sets (Section 3.1, the sets B_p; reading R1): the sorted unique */
/* values of each feature, generated once.  Realised as dense ranks: rank   */
/* of x[i][p] = its index among the sorted unique values of feature p.      */
/* Equality is IEEE equality (-0 == +0); NaN is rejected.                    */
/* ------------------------------------------------------------------------ */
typedef struct {
  float v;
  uint32_t i;
} or_vi;

static int or_cmp_vi(const void *a, const void *b) {
  const or_vi *x = (const or_vi *)a, *y = (const or_vi *)b;
  if (x->v < y->v) return -1;
  if (x->v > y->v) return 1;
  return (x->i < y->i) ? -1 : (x->i > y->i);
}

/* X is row-major [n][F]; ranks is column-major [F][n]; n_unique is [F]. */
int oracle_rank_encode(const float *X, uint32_t n, uint32_t F, uint32_t *ranks,
                       uint32_t *n_unique) {
  if (F == 0) return OR_EINVAL;
  or_vi *buf = (or_vi *)malloc(sizeof(or_vi) * (n ? n : 1));
  if (!buf) return OR_ENOMEM;
  for (uint32_t f = 0; f < F; ++f) {
    for (uint32_t i = 0; i < n; ++i) {
      float v = X[(size_t)i * F + f];
      if (v != v) {
        free(buf);
        return OR_EINVAL;
      }
      if (v == 0.0f) v = 0.0f; /* -0 and +0 are one value */
      buf[i].v = v;
      buf[i].i = i;
    }
    qsort(buf, n, sizeof(or_vi), or_cmp_vi);
    uint32_t r = 0;
    for (uint32_t j = 0; j < n; ++j) {
      if (j > 0 && buf[j].v != buf[j - 1].v) r += 1;
      ranks[(size_t)f * n + buf[j].i] = r;
    }
    n_unique[f] = n ? r + 1 : 0;
  }
  free(buf);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Decoding an individual (Section 3.1, eq. aenc and eq. benc).             */
/* Individual layout: [a^_1 .. a^_SB, b^_1 .. b^_SB], SB = 2^D - 1.          */
/*   a_t = floor(a^_t), a^_t in [0, F+1]  (0 = no split), clamped to F.      */
/*   threshold index i = floor(b^_t (n_p + 1)) + 1 (1-based into B_p);       */
/*   reading R2/R4: tau = i - 1 clamped to n_p, left iff rank < tau.         */
/*   a_t = 0 forces b_t = 0, i.e. tau = 0 (everything goes right).           */
/* ------------------------------------------------------------------------ */
void oracle_decode(const double *genes, uint32_t P, uint32_t D, uint32_t F,
                   const uint32_t *n_unique, uint8_t *feat, uint32_t *tau) {
  uint32_t SB = (1u << D) - 1u;
  uint32_t m = 2u * SB;
  for (uint32_t r = 0; r < P; ++r) {
    for (uint32_t t = 0; t < SB; ++t) {
      double a = genes[(size_t)r * m + t];
      double b = genes[(size_t)r * m + SB + t];
      if (!(a >= 0.0)) a = 0.0;
      if (a > (double)F + 1.0) a = (double)F + 1.0;
      if (!(b >= 0.0)) b = 0.0;
      if (b > 1.0) b = 1.0;
      double fa = floor(a);
      uint32_t f = (fa >= (double)F) ? F : (uint32_t)fa;
      uint32_t th = 0;
      if (f != 0) {
        uint32_t np = n_unique[f - 1];
        double x = floor(b * (double)(np + 1u));
        th = (x >= (double)np) ? np : (uint32_t)x;
      }
      feat[(size_t)r * SB + t] = (uint8_t)f;
      tau[(size_t)r * SB + t] = th;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Routing one sample (Section 2 tree semantics; Algorithm 1 walk).          */
/* t <- 1; while t <= SB: t <- (x_{a_t} < b_t) ? 2t : 2t + 1.  Returns the   */
/* 0-based leaf t - 2^D.  A node with a_t = 0 sends the sample right.        */
/* ------------------------------------------------------------------------ */
uint32_t oracle_route(const uint32_t *ranks, size_t ld, uint32_t i,
                      const uint8_t *feat, const uint32_t *tau, uint32_t D) {
  uint32_t SB = (1u << D) - 1u;
  uint32_t t = 1;
  while (t <= SB) {
    uint32_t f = feat[t - 1];
    int left = (f != 0) && (ranks[(size_t)(f - 1) * ld + i] < tau[t - 1]);
    t = left ? 2u * t : 2u * t + 1u;
  }
  return t - (1u << D);
}

/* ------------------------------------------------------------------------ */
/* Fitness of P trees (eq. opt_c, eq. opt_all, and the soft-constraint      */
/* fitness of Section 3.2; reading R7).                                      */
/*   counts[r][l][k] = # samples of class k routed to leaf l by tree r       */
/*   label[r][l]     = lowest k attaining max_k counts (empty leaf -> 0)     */
/*   correct[r]      = sum_l max_k counts[r][l][k]                           */
/*   cost[r]         = (n - correct) + alpha * #{t: a_t != 0}                */
/*                     + #{l : 0 < n_l < n_min}                              */
/* idx (may be NULL) selects the n_sub samples; otherwise samples 0..n_sub-1.*/
/* ------------------------------------------------------------------------ */
void oracle_tree_epilogue(const uint32_t *counts, uint32_t K, uint32_t D,
                          const uint8_t *feat, uint32_t n_sub, uint32_t n_min,
                          double alpha, uint8_t *label, uint32_t *correct,
                          double *cost) {
  uint32_t SL = 1u << D, SB = SL - 1u;
  uint32_t corr = 0, nviol = 0, nsplit = 0;
  for (uint32_t l = 0; l < SL; ++l) {
    const uint32_t *c = counts + (size_t)l * K;
    uint32_t best = c[0], bk = 0, nl = c[0];
    for (uint32_t k = 1; k < K; ++k) {
      nl += c[k];
      if (c[k] > best) {
        best = c[k];
        bk = k;
      }
    }
    if (label) label[l] = (uint8_t)bk;
    corr += best;
    if (nl > 0 && nl < n_min) nviol += 1;
  }
  for (uint32_t t = 0; t < SB; ++t) nsplit += (feat[t] != 0);
  if (correct) *correct = corr;
  if (cost) {
    double v = (double)(n_sub - corr);
    v = v + alpha * (double)nsplit;
    v = v + (double)nviol;
    *cost = v;
  }
}

/* Threads the parallel fitness loop uses (1 without OpenMP). */
int oracle_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

int oracle_fitness(const uint32_t *ranks, size_t ld, const uint8_t *labels,
                   uint32_t K, const uint32_t *idx, uint32_t n_sub,
                   const uint8_t *feat, const uint32_t *tau, uint32_t P,
                   uint32_t D, uint32_t n_min, double alpha, uint32_t *counts,
                   uint32_t *correct, uint8_t *label, double *cost) {
  if (K < 1 || D < 1 || D > 10) return OR_EINVAL;
  uint32_t SL = 1u << D, SB = SL - 1u;
#pragma omp parallel for schedule(dynamic, 1)
  for (uint32_t r = 0; r < P; ++r) {
    uint32_t *c = counts + (size_t)r * SL * K;
    memset(c, 0, sizeof(uint32_t) * SL * K);
    const uint8_t *fr = feat + (size_t)r * SB;
    const uint32_t *tr = tau + (size_t)r * SB;
    for (uint32_t j = 0; j < n_sub; ++j) {
      uint32_t i = idx ? idx[j] : j;
      uint32_t l = oracle_route(ranks, ld, i, fr, tr, D);
      c[(size_t)l * K + labels[i]] += 1;
    }
    oracle_tree_epilogue(c, K, D, fr, n_sub, n_min, alpha,
                         label ? label + (size_t)r * SL : NULL,
                         correct ? correct + r : NULL, cost ? cost + r : NULL);
  }
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Depth-1 exact split with the misclassification loss (Algorithm 2, the    */
/* horizon-1 branch; reading R10).  Candidates in order: no split first,    */
/* then f = 1..F, tau = 1..n_f - 1; the first strict maximum of correct is  */
/* kept.  correct(f, tau) = max_k L_k + max_k (N_k - L_k), L_k = # samples  */
/* of class k with rank_f < tau.                                             */
/* ------------------------------------------------------------------------ */
int oracle_split1(const uint32_t *ranks, size_t ld, const uint32_t *n_unique,
                  uint32_t F, const uint8_t *labels, uint32_t K,
                  const uint32_t *idx, uint32_t n_sub, uint8_t *feat_out,
                  uint32_t *tau_out, uint32_t *correct_out) {
  uint32_t *tot = (uint32_t *)calloc(K, sizeof(uint32_t));
  uint32_t *left = (uint32_t *)calloc(K, sizeof(uint32_t));
  if (!tot || !left) {
    free(tot);
    free(left);
    return OR_ENOMEM;
  }
  for (uint32_t j = 0; j < n_sub; ++j) tot[labels[idx ? idx[j] : j]] += 1;
  uint32_t best = 0;
  for (uint32_t k = 0; k < K; ++k)
    if (tot[k] > best) best = tot[k];
  uint32_t bf = 0, bt = 0;
  for (uint32_t f = 1; f <= F; ++f) {
    uint32_t nf = n_unique[f - 1];
    if (nf < 2) continue;
    uint32_t *hist = (uint32_t *)calloc((size_t)nf * K, sizeof(uint32_t));
    if (!hist) {
      free(tot);
      free(left);
      return OR_ENOMEM;
    }
    for (uint32_t j = 0; j < n_sub; ++j) {
      uint32_t i = idx ? idx[j] : j;
      hist[(size_t)ranks[(size_t)(f - 1) * ld + i] * K + labels[i]] += 1;
    }
    memset(left, 0, sizeof(uint32_t) * K);
    for (uint32_t t = 1; t <= nf - 1; ++t) {
      /* move the samples with rank t-1 to the left side */
      for (uint32_t k = 0; k < K; ++k) left[k] += hist[(size_t)(t - 1) * K + k];
      uint32_t ml = 0, mr = 0;
      for (uint32_t k = 0; k < K; ++k) {
        if (left[k] > ml) ml = left[k];
        if (tot[k] - left[k] > mr) mr = tot[k] - left[k];
      }
      if (ml + mr > best) {
        best = ml + mr;
        bf = f;
        bt = t;
      }
    }
    free(hist);
  }
  free(tot);
  free(left);
  if (feat_out) *feat_out = (uint8_t)bf;
  if (tau_out) *tau_out = bt;
  if (correct_out) *correct_out = best;
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Exhaustive depth-2 optimum (test only; reading R11): the best root split */
/* (no split, or any (f, tau), tau in [0, n_f]) followed by the exact best  */
/* depth-1 split on each side.  Returns the 3-node tree in heap order.      */
/* ------------------------------------------------------------------------ */
int oracle_opt2(const uint32_t *ranks, size_t ld, const uint32_t *n_unique,
                uint32_t F, const uint8_t *labels, uint32_t K,
                const uint32_t *idx, uint32_t n_sub, uint32_t *correct_out,
                uint8_t *feat3, uint32_t *tau3) {
  uint32_t *L = (uint32_t *)malloc(sizeof(uint32_t) * (n_sub ? n_sub : 1));
  uint32_t *R = (uint32_t *)malloc(sizeof(uint32_t) * (n_sub ? n_sub : 1));
  if (!L || !R) {
    free(L);
    free(R);
    return OR_ENOMEM;
  }
  uint8_t f2, f3;
  uint32_t t2, t3, c2, c3;
  /* root without a split: everything goes right */
  for (uint32_t j = 0; j < n_sub; ++j) R[j] = idx ? idx[j] : j;
  oracle_split1(ranks, ld, n_unique, F, labels, K, R, n_sub, &f3, &t3, &c3);
  uint32_t best = c3;
  uint8_t bf[3] = {0, 0, f3};
  uint32_t bt[3] = {0, 0, t3};
  for (uint32_t f = 1; f <= F; ++f) {
    uint32_t nf = n_unique[f - 1];
    for (uint32_t t = 0; t <= nf; ++t) {
      uint32_t nl = 0, nr = 0;
      for (uint32_t j = 0; j < n_sub; ++j) {
        uint32_t i = idx ? idx[j] : j;
        if (ranks[(size_t)(f - 1) * ld + i] < t)
          L[nl++] = i;
        else
          R[nr++] = i;
      }
      c2 = 0;
      c3 = 0;
      f2 = f3 = 0;
      t2 = t3 = 0;
      if (nl) oracle_split1(ranks, ld, n_unique, F, labels, K, L, nl, &f2, &t2, &c2);
      if (nr) oracle_split1(ranks, ld, n_unique, F, labels, K, R, nr, &f3, &t3, &c3);
      if (c2 + c3 > best) {
        best = c2 + c3;
        bf[0] = (uint8_t)f;
        bt[0] = t;
        bf[1] = f2;
        bt[1] = t2;
        bf[2] = f3;
        bt[2] = t3;
      }
    }
  }
  free(L);
  free(R);
  if (correct_out) *correct_out = best;
  if (feat3) memcpy(feat3, bf, 3);
  if (tau3) memcpy(tau3, bt, sizeof(bt));
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Greedy top-down tree with the 0-1 loss (test only).  Written as a plain  */
/* recursion over explicit subsets so that it shares no structure with the  */
/* moving-horizon driver below; with horizon 1 the two must agree.          */
/* ------------------------------------------------------------------------ */
static int or_greedy_rec(const uint32_t *ranks, size_t ld,
                         const uint32_t *n_unique, uint32_t F,
                         const uint8_t *labels, uint32_t K, uint32_t *S,
                         uint32_t nS, uint32_t t, uint32_t depth, uint32_t D,
                         uint32_t n_min, uint8_t *feat, uint32_t *tau) {
  if (depth == D) return OR_OK;
  uint8_t f = 0;
  uint32_t th = 0;
  int pure = 1;
  for (uint32_t j = 1; j < nS; ++j)
    if (labels[S[j]] != labels[S[0]]) pure = 0;
  if (nS > n_min && !pure) {
    int rc = oracle_split1(ranks, ld, n_unique, F, labels, K, S, nS, &f, &th, NULL);
    if (rc) return rc;
  }
  feat[t - 1] = f;
  tau[t - 1] = th;
  uint32_t *A = (uint32_t *)malloc(sizeof(uint32_t) * (nS ? nS : 1));
  uint32_t *B = (uint32_t *)malloc(sizeof(uint32_t) * (nS ? nS : 1));
  if (!A || !B) {
    free(A);
    free(B);
    return OR_ENOMEM;
  }
  uint32_t na = 0, nb = 0;
  for (uint32_t j = 0; j < nS; ++j) {
    uint32_t i = S[j];
    if (f != 0 && ranks[(size_t)(f - 1) * ld + i] < th)
      A[na++] = i;
    else
      B[nb++] = i;
  }
  int rc = or_greedy_rec(ranks, ld, n_unique, F, labels, K, A, na, 2 * t,
                         depth + 1, D, n_min, feat, tau);
  if (!rc)
    rc = or_greedy_rec(ranks, ld, n_unique, F, labels, K, B, nb, 2 * t + 1,
                       depth + 1, D, n_min, feat, tau);
  free(A);
  free(B);
  return rc;
}

int oracle_greedy_tree(const uint32_t *ranks, size_t ld,
                       const uint32_t *n_unique, uint32_t F,
                       const uint8_t *labels, uint32_t K, uint32_t n,
                       uint32_t D, uint32_t n_min, uint8_t *feat,
                       uint32_t *tau) {
  uint32_t *S = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
  if (!S) return OR_ENOMEM;
  for (uint32_t i = 0; i < n; ++i) S[i] = i;
  int rc = or_greedy_rec(ranks, ld, n_unique, F, labels, K, S, n, 1, 0, D,
                         n_min, feat, tau);
  free(S);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* CART, the warm start of Algorithm 2 (the CART solution of a moving-      */
/* horizon subtree) and of the plain DEOCT runs of Section 4.  The paper    */
/* names the CART package it uses, not the impurity; reading R15: Gini.     */
/* Top down in heap order, each node u on its subset S: when S holds more   */
/* than one class and some threshold sends samples both ways, u takes the   */
/* first strict maximum, over features f = 1..F and thresholds              */
/* tau = 1..n_f - 1 with both sides non-empty, of the Gini score            */
/*   g = sum_k L_k^2 / |L| + sum_k R_k^2 / |R|                               */
/* (|S| minus the children's weighted Gini impurity), in float64 as         */
/* (double)A / (double)|L| + (double)B / (double)|R| with A and B the       */
/* integer sums of squares.  Otherwise u gets no split (every sample goes   */
/* right, so its right child sees the same subset).                         */
/* ------------------------------------------------------------------------ */
static int or_cart_split(const uint32_t *ranks, size_t ld, const uint32_t *n_unique,
                         uint32_t F, const uint8_t *labels, uint32_t K, const uint32_t *S,
                         uint32_t nS, uint8_t *f_out, uint32_t *t_out) {
  *f_out = 0;
  *t_out = 0;
  uint32_t *tot = (uint32_t *)calloc(K, sizeof(uint32_t));
  uint32_t *left = (uint32_t *)calloc(K, sizeof(uint32_t));
  if (!tot || !left) {
    free(tot);
    free(left);
    return OR_ENOMEM;
  }
  for (uint32_t j = 0; j < nS; ++j) tot[labels[S[j]]] += 1;
  uint32_t classes = 0;
  for (uint32_t k = 0; k < K; ++k) classes += tot[k] ? 1u : 0u;
  double best = -1.0;
  for (uint32_t f = 1; f <= F && classes > 1; ++f) {
    uint32_t nf = n_unique[f - 1];
    if (nf < 2) continue;
    uint32_t *hist = (uint32_t *)calloc((size_t)nf * K, sizeof(uint32_t));
    if (!hist) {
      free(tot);
      free(left);
      return OR_ENOMEM;
    }
    for (uint32_t j = 0; j < nS; ++j) {
      uint32_t i = S[j];
      hist[(size_t)ranks[(size_t)(f - 1) * ld + i] * K + labels[i]] += 1;
    }
    memset(left, 0, sizeof(uint32_t) * K);
    uint32_t nL = 0;
    for (uint32_t th = 1; th < nf; ++th) {
      for (uint32_t k = 0; k < K; ++k) {
        left[k] += hist[(size_t)(th - 1) * K + k];
        nL += hist[(size_t)(th - 1) * K + k];
      }
      uint32_t nR = nS - nL;
      if (nL == 0 || nR == 0) continue;
      uint64_t A = 0, B = 0;
      for (uint32_t k = 0; k < K; ++k) {
        uint64_t l = left[k], r = tot[k] - left[k];
        A += l * l;
        B += r * r;
      }
      double g = (double)A / (double)nL + (double)B / (double)nR;
      if (g > best) {
        best = g;
        *f_out = (uint8_t)f;
        *t_out = th;
      }
    }
    free(hist);
  }
  free(tot);
  free(left);
  return OR_OK;
}

static int or_cart_rec(const uint32_t *ranks, size_t ld, const uint32_t *n_unique, uint32_t F,
                       const uint8_t *labels, uint32_t K, uint32_t *S, uint32_t nS, uint32_t u,
                       uint32_t depth, uint32_t D, uint8_t *feat, uint32_t *tau) {
  if (depth == D) return OR_OK;
  uint8_t f = 0;
  uint32_t th = 0;
  int rc = or_cart_split(ranks, ld, n_unique, F, labels, K, S, nS, &f, &th);
  if (rc) return rc;
  feat[u - 1] = f;
  tau[u - 1] = th;
  uint32_t *A = (uint32_t *)malloc(sizeof(uint32_t) * (nS ? nS : 1));
  uint32_t *B = (uint32_t *)malloc(sizeof(uint32_t) * (nS ? nS : 1));
  if (!A || !B) {
    free(A);
    free(B);
    return OR_ENOMEM;
  }
  uint32_t na = 0, nb = 0;
  for (uint32_t j = 0; j < nS; ++j) {
    uint32_t i = S[j];
    if (f != 0 && ranks[(size_t)(f - 1) * ld + i] < th)
      A[na++] = i;
    else
      B[nb++] = i;
  }
  rc = or_cart_rec(ranks, ld, n_unique, F, labels, K, A, na, 2 * u, depth + 1, D, feat, tau);
  if (!rc)
    rc = or_cart_rec(ranks, ld, n_unique, F, labels, K, B, nb, 2 * u + 1, depth + 1, D, feat,
                     tau);
  free(A);
  free(B);
  return rc;
}

/* The CART tree of depth D on the samples idx[0..n_sub) (all n if idx is
 * NULL): feat / tau [2^D - 1]. */
int oracle_cart(const uint32_t *ranks, size_t ld, const uint32_t *n_unique, uint32_t F,
                const uint8_t *labels, uint32_t K, const uint32_t *idx, uint32_t n_sub,
                uint32_t D, uint8_t *feat, uint32_t *tau) {
  if (D < 1 || D > 10 || K < 1) return OR_EINVAL;
  uint32_t SB = (1u << D) - 1u;
  memset(feat, 0, SB);
  memset(tau, 0, sizeof(uint32_t) * SB);
  uint32_t *S = (uint32_t *)malloc(sizeof(uint32_t) * (n_sub ? n_sub : 1));
  if (!S) return OR_ENOMEM;
  for (uint32_t j = 0; j < n_sub; ++j) S[j] = idx ? idx[j] : j;
  int rc = or_cart_rec(ranks, ld, n_unique, F, labels, K, S, n_sub, 1, 0, D, feat, tau);
  free(S);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Differential evolution for OCT (Section 2 eqs. mutation / crossover /    */
/* selection; Section 3.3; Algorithm 4; reading R8).                         */
/* ------------------------------------------------------------------------ */
typedef struct {
  uint32_t P, G;
  double M;  /* mutation factor; M < 0 draws M_r ~ U[0,1) per (g, r) */
  double CR; /* crossover probability */
  uint64_t seed;
  uint32_t n_min;
  double alpha;
} oracle_de_params;

/* Initialisation (Algorithm 4, first loop): warm starts fill slots 0..W-1;
 * the rest are drawn uniformly inside the range limits at g = 0:
 * a^ = U * (F + 1), b^ = U, gene q using slot q. */
void oracle_de_init(uint32_t P, uint32_t D, uint32_t F, uint64_t seed,
                    uint64_t prob, const double *warm, uint32_t W,
                    double *pop) {
  uint32_t SB = (1u << D) - 1u, m = 2u * SB;
  for (uint32_t r = 0; r < P; ++r) {
    for (uint32_t q = 0; q < m; ++q) {
      double v;
      if (r < W) {
        v = warm[(size_t)r * m + q];
      } else {
        double u = oracle_u01(oracle_draw(seed, prob, 0, r, q));
        v = (q < SB) ? u * ((double)F + 1.0) : u;
      }
      pop[(size_t)r * m + q] = v;
    }
  }
}

/* The lowest index attaining the minimum cost. */
uint32_t oracle_argmin(const double *cost, uint32_t P) {
  uint32_t b = 0;
  for (uint32_t r = 1; r < P; ++r)
    if (cost[r] < cost[b]) b = r;
  return b;
}

/* Mutation (DE/best/1) and binomial crossover for generation g >= 1.
 * Slots: 0 = M_r (if M < 0), 1 = r1, 2 = r2, 3 = q_rand, 4 + q = crossover
 * draw of gene q.  r1 != r and r2 not in {r, r1} are drawn without
 * rejection.  v = s_best + M_r (s_r1 - s_r2), clamped to [0, F+1] for the
 * feature genes and [0, 1] for the threshold genes; u_q = v_q if
 * U_q <= CR or q == q_rand, else s_q. */
void oracle_de_pick(uint32_t P, uint32_t m, uint64_t seed, uint64_t prob,
                    uint32_t g, uint32_t r, uint32_t *r1_out, uint32_t *r2_out,
                    uint32_t *qr_out) {
  uint32_t r1 = oracle_uint(oracle_draw(seed, prob, g, r, 1), P - 1u);
  if (r1 >= r) r1 += 1u;
  uint32_t r2 = oracle_uint(oracle_draw(seed, prob, g, r, 2), P - 2u);
  uint32_t lo = r < r1 ? r : r1, hi = r < r1 ? r1 : r;
  if (r2 >= lo) r2 += 1u;
  if (r2 >= hi) r2 += 1u;
  *r1_out = r1;
  *r2_out = r2;
  *qr_out = oracle_uint(oracle_draw(seed, prob, g, r, 3), m);
}

void oracle_de_trial(uint32_t P, uint32_t D, uint32_t F, double M, double CR,
                     uint64_t seed, uint64_t prob, uint32_t g,
                     const double *pop, uint32_t best, double *trial) {
  uint32_t SB = (1u << D) - 1u, m = 2u * SB;
  for (uint32_t r = 0; r < P; ++r) {
    double Mr = (M >= 0.0) ? M : oracle_u01(oracle_draw(seed, prob, g, r, 0));
    uint32_t r1, r2, qr;
    oracle_de_pick(P, m, seed, prob, g, r, &r1, &r2, &qr);
    for (uint32_t q = 0; q < m; ++q) {
      double d = pop[(size_t)r1 * m + q] - pop[(size_t)r2 * m + q];
      double md = Mr * d;
      double v = pop[(size_t)best * m + q] + md;
      double hiq = (q < SB) ? ((double)F + 1.0) : 1.0;
      if (!(v >= 0.0)) v = 0.0;
      if (v > hiq) v = hiq;
      double uq = oracle_u01(oracle_draw(seed, prob, g, r, 4u + q));
      trial[(size_t)r * m + q] = (uq <= CR || q == qr) ? v : pop[(size_t)r * m + q];
    }
  }
}

/* Greedy selection (eq. selection): the trial replaces the parent when its
 * cost is less than or equal to the parent's. */
void oracle_de_select(uint32_t P, uint32_t m, double *pop, double *cost,
                      const double *trial, const double *trial_cost) {
  for (uint32_t r = 0; r < P; ++r) {
    if (trial_cost[r] <= cost[r]) {
      memcpy(pop + (size_t)r * m, trial + (size_t)r * m, sizeof(double) * m);
      cost[r] = trial_cost[r];
    }
  }
}

/* Evaluate the cost of P individuals: decode, then fitness. */
static int or_eval_pop(const uint32_t *ranks, size_t ld,
                       const uint32_t *n_unique, uint32_t F,
                       const uint8_t *labels, uint32_t K, const uint32_t *idx,
                       uint32_t n_sub, uint32_t D, uint32_t P, uint32_t n_min,
                       double alpha, const double *genes, uint8_t *feat,
                       uint32_t *tau, uint32_t *counts, double *cost) {
  oracle_decode(genes, P, D, F, n_unique, feat, tau);
  return oracle_fitness(ranks, ld, labels, K, idx, n_sub, feat, tau, P, D,
                        n_min, alpha, counts, NULL, NULL, cost);
}

/* DEOCT (Algorithm 4): initialise, evaluate, pick the best; then for
 * g = 1..G build every trial from the best of the previous generation,
 * evaluate the trial population at once, select, and pick the new best.
 * Outputs the best individual, its decoded tree, leaf labels, correct count
 * and cost.  best_trace (optional) receives the best cost after the
 * initial evaluation and after each generation ([G + 1]); final_pop
 * (optional) receives the last population ([P][m]). */
int oracle_deoct(const uint32_t *ranks, size_t ld, const uint32_t *n_unique,
                 uint32_t F, const uint8_t *labels, uint32_t K,
                 const uint32_t *idx, uint32_t n_sub, uint32_t D,
                 const oracle_de_params *prm, const double *warm, uint32_t W,
                 uint64_t prob, double *best_genes, uint8_t *feat_out,
                 uint32_t *tau_out, uint8_t *label_out, uint32_t *correct_out,
                 double *cost_out, double *best_trace, double *final_pop) {
  uint32_t P = prm->P;
  if (P < 3 || D < 1 || D > 10 || W > P) return OR_EINVAL;
  uint32_t SB = (1u << D) - 1u, SL = SB + 1u, m = 2u * SB;
  double *pop = (double *)malloc(sizeof(double) * P * m);
  double *trial = (double *)malloc(sizeof(double) * P * m);
  double *cost = (double *)malloc(sizeof(double) * P);
  double *tcost = (double *)malloc(sizeof(double) * P);
  uint8_t *feat = (uint8_t *)malloc((size_t)P * SB);
  uint32_t *tau = (uint32_t *)malloc(sizeof(uint32_t) * P * SB);
  uint32_t *counts = (uint32_t *)malloc(sizeof(uint32_t) * P * SL * K);
  int rc = OR_OK;
  if (!pop || !trial || !cost || !tcost || !feat || !tau || !counts) {
    rc = OR_ENOMEM;
    goto done;
  }
  oracle_de_init(P, D, F, prm->seed, prob, warm, W, pop);
  rc = or_eval_pop(ranks, ld, n_unique, F, labels, K, idx, n_sub, D, P,
                   prm->n_min, prm->alpha, pop, feat, tau, counts, cost);
  if (rc) goto done;
  uint32_t best = oracle_argmin(cost, P);
  if (best_trace) best_trace[0] = cost[best];
  for (uint32_t g = 1; g <= prm->G; ++g) {
    oracle_de_trial(P, D, F, prm->M, prm->CR, prm->seed, prob, g, pop, best,
                    trial);
    rc = or_eval_pop(ranks, ld, n_unique, F, labels, K, idx, n_sub, D, P,
                     prm->n_min, prm->alpha, trial, feat, tau, counts, tcost);
    if (rc) goto done;
    oracle_de_select(P, m, pop, cost, trial, tcost);
    best = oracle_argmin(cost, P);
    if (best_trace) best_trace[g] = cost[best];
  }
  /* the best tree, re-evaluated for its labels and correct count */
  {
    uint8_t bf[1023];
    uint32_t bt[1023];
    oracle_decode(pop + (size_t)best * m, 1, D, F, n_unique, bf, bt);
    /* counts has room for P >= 1 trees */
    oracle_fitness(ranks, ld, labels, K, idx, n_sub, bf, bt, 1, D, prm->n_min,
                   prm->alpha, counts, correct_out, label_out, cost_out);
    if (feat_out) memcpy(feat_out, bf, SB);
    if (tau_out) memcpy(tau_out, bt, sizeof(uint32_t) * SB);
    if (best_genes) memcpy(best_genes, pop + (size_t)best * m, sizeof(double) * m);
    if (final_pop) memcpy(final_pop, pop, sizeof(double) * P * m);
  }
done:
  free(pop);
  free(trial);
  free(cost);
  free(tcost);
  free(feat);
  free(tau);
  free(counts);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Moving-horizon DEOCT (Algorithm 2; Section 4; reading R9).               */
/* For each branch node t in index order: the subset reaching t through the */
/* already fixed ancestors; if it has more than n_min samples and more than */
/* one class, the effective horizon D_t = min(D_MH, D - depth(t)) decides:  */
/* DEOCT on a depth-D_t subtree (problem id t) when D_t != 1, the exact     */
/* depth-1 split otherwise; the subtree's first node is kept.  Otherwise    */
/* the artificial node {a_t = 0, b_t = 0}.  No warm starts (the paper's     */
/* no-warm-start variant).  Leaf labels come from the final tree over all   */
/* training samples.                                                         */
/* ------------------------------------------------------------------------ */
void oracle_tree_encode(const uint8_t *feat, const uint32_t *tau, uint32_t P, uint32_t D,
                        uint32_t F, const uint32_t *n_unique, double *genes);

/* The subtree of depth De rooted at heap node t of a depth-D tree (the
 * shape and location a moving-horizon subproblem at t covers): subtree node
 * u at depth k of the subtree (2^k <= u < 2^(k+1)) is tree node
 * t 2^k + (u - 2^k).  Subtree nodes below the tree's last split level get
 * no split. */
void oracle_subtree(const uint8_t *feat, const uint32_t *tau, uint32_t D, uint32_t t,
                    uint32_t De, uint8_t *sf, uint32_t *st) {
  uint32_t SB = (1u << D) - 1u, SBe = (1u << De) - 1u;
  for (uint32_t u = 1; u <= SBe; ++u) {
    uint32_t k = 0;
    while ((2u << k) <= u) k += 1u;
    uint64_t v = ((uint64_t)t << k) + (u - (1u << k));
    sf[u - 1] = v <= SB ? feat[v - 1] : 0;
    st[u - 1] = v <= SB ? tau[v - 1] : 0;
  }
}

/* Warm starts of the moving horizon (Algorithm 2's warm-start branch and
 * the variants of Section 4's ablation), bits of `flags`:
 *   2 (CART)        the CART tree of each DE-solved node's subtree, on the
 *                   node's subset, is added to its DEOCT warm starts;
 *   4 (DEOCT)       a DEOCT run on the whole tree (depth D, all samples,
 *                   problem id 0) gives warm-start trees: node t's DEOCT gets
 *                   the run's subtree with the same shape and location;
 *   8 (DEOCT_CART)  that whole-tree run is itself warm-started with the
 *                   CART tree of depth D.
 * A node's warm starts come in the order of Algorithm 2: the retrieved
 * subtree first, then the CART solution. */
int oracle_mh_train(const uint32_t *ranks, size_t ld, const uint32_t *n_unique,
                    uint32_t F, const uint8_t *labels, uint32_t K, uint32_t n,
                    uint32_t D, uint32_t D_MH, const oracle_de_params *prm, uint32_t flags,
                    uint8_t *feat, uint32_t *tau, uint8_t *label_out,
                    uint32_t *correct_out, double *cost_out) {
  if (D < 1 || D > 10 || D_MH < 1) return OR_EINVAL;
  uint32_t SB = (1u << D) - 1u;
  uint32_t *S = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
  if (!S) return OR_ENOMEM;
  memset(feat, 0, SB);
  memset(tau, 0, sizeof(uint32_t) * SB);
  int rc = OR_OK;
  /* the whole-tree DEOCT warm-start tree */
  uint8_t wf[1023];
  uint32_t wt[1023];
  if (flags & 4u) {
    double wg[2 * 1023];
    uint32_t Wd = 0;
    if (flags & 8u) {
      uint8_t cf[1023];
      uint32_t ct[1023];
      rc = oracle_cart(ranks, ld, n_unique, F, labels, K, NULL, n, D, cf, ct);
      if (rc) {
        free(S);
        return rc;
      }
      oracle_tree_encode(cf, ct, 1, D, F, n_unique, wg);
      Wd = 1;
    }
    rc = oracle_deoct(ranks, ld, n_unique, F, labels, K, NULL, n, D, prm, Wd ? wg : NULL, Wd, 0,
                      NULL, wf, wt, NULL, NULL, NULL, NULL, NULL);
    if (rc) {
      free(S);
      return rc;
    }
  }
  for (uint32_t t = 1; t <= SB && rc == OR_OK; ++t) {
    uint32_t dt = 0;
    while ((2u << dt) <= t) dt += 1u; /* depth of node t: floor(log2 t) */
    /* the subset reaching t: walk each sample dt steps from the root */
    uint32_t nS = 0;
    for (uint32_t i = 0; i < n; ++i) {
      uint32_t u = 1;
      for (uint32_t s = 0; s < dt; ++s) {
        uint32_t f = feat[u - 1];
        int left = (f != 0) && (ranks[(size_t)(f - 1) * ld + i] < tau[u - 1]);
        u = left ? 2u * u : 2u * u + 1u;
      }
      if (u == t) S[nS++] = i;
    }
    int multi = 0;
    for (uint32_t j = 1; j < nS; ++j)
      if (labels[S[j]] != labels[S[0]]) multi = 1;
    if (nS > prm->n_min && multi) {
      uint32_t De = D - dt < D_MH ? D - dt : D_MH;
      if (De != 1) {
        uint8_t sf[1023];
        uint32_t st[1023];
        /* warm starts: the whole-tree run's subtree at t (node u of depth k
         * of the subtree is node t 2^k + u - 2^k of the tree), then CART */
        uint32_t SBe = (1u << De) - 1u, W = 0;
        double warm[2 * 2 * 1023];
        if (flags & 4u) {
          oracle_subtree(wf, wt, D, t, De, sf, st);
          oracle_tree_encode(sf, st, 1, De, F, n_unique, warm + (size_t)W * 2 * SBe);
          W += 1;
        }
        if (flags & 2u) {
          rc = oracle_cart(ranks, ld, n_unique, F, labels, K, S, nS, De, sf, st);
          if (rc) break;
          oracle_tree_encode(sf, st, 1, De, F, n_unique, warm + (size_t)W * 2 * SBe);
          W += 1;
        }
        rc = oracle_deoct(ranks, ld, n_unique, F, labels, K, S, nS, De, prm,
                          W ? warm : NULL, W, (uint64_t)t, NULL, sf, st, NULL, NULL, NULL,
                          NULL, NULL);
        feat[t - 1] = sf[0];
        tau[t - 1] = st[0];
      } else {
        rc = oracle_split1(ranks, ld, n_unique, F, labels, K, S, nS,
                           &feat[t - 1], &tau[t - 1], NULL);
      }
    } else {
      feat[t - 1] = 0;
      tau[t - 1] = 0;
    }
  }
  free(S);
  if (rc) return rc;
  uint32_t SL = SB + 1u;
  uint32_t *counts = (uint32_t *)malloc(sizeof(uint32_t) * SL * K);
  if (!counts) return OR_ENOMEM;
  rc = oracle_fitness(ranks, ld, labels, K, NULL, n, feat, tau, 1, D,
                      prm->n_min, prm->alpha, counts, correct_out, label_out,
                      cost_out);
  free(counts);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Applying a trained tree to samples it was not trained on (Section 2 tree */
/* semantics with the Section 3.1 threshold sets; the test accuracy of      */
/* Section 4; reading R13).  The threshold set of feature p is the midpoints */
/* of adjacent sorted unique training values, with the scaled 0 (the        */
/* training minimum) in front.  A split of rank threshold tau therefore     */
/* sends x left iff x < beta, where, with u_0 < u_1 < ... the unique        */
/* training values of the feature and n_p their number:                     */
/*   tau = 0           beta = u_0   (-inf when n_p = 0)                     */
/*   0 < tau < n_p     beta = (u_{tau-1} + u_tau) / 2                       */
/*   tau >= n_p        beta = +inf  (reading R2: every sample goes left)    */
/* Min-max scaling is affine and increasing, so comparing in raw units is   */
/* the same decision as comparing scaled values.  beta and the comparison   */
/* are in f64.  A node with a_t = 0 (or a_t > F) gets beta = 0 and sends    */
/* every sample right.                                                      */
/* ------------------------------------------------------------------------ */
static int or_cmp_f(const void *a, const void *b) {
  float x = *(const float *)a, y = *(const float *)b;
  return (x < y) ? -1 : (x > y);
}

/* X: training features, row-major [n][F].  feat / tau: one tree [SB].
 * thr: out [SB]. */
int oracle_tree_thresholds(const float *X, uint32_t n, uint32_t F,
                           const uint8_t *feat, const uint32_t *tau, uint32_t D,
                           double *thr) {
  uint32_t SB = (1u << D) - 1u;
  float *u = (float *)malloc(sizeof(float) * (n ? n : 1));
  if (!u) return OR_ENOMEM;
  for (uint32_t t = 0; t < SB; ++t) {
    uint32_t f = feat[t];
    thr[t] = 0.0;
    if (f == 0 || f > F) continue;
    for (uint32_t i = 0; i < n; ++i) {
      float v = X[(size_t)i * F + (f - 1)];
      if (v != v) {
        free(u);
        return OR_EINVAL;
      }
      u[i] = (v == 0.0f) ? 0.0f : v;
    }
    qsort(u, n, sizeof(float), or_cmp_f);
    uint32_t m = 0; /* unique values, compacted in place */
    for (uint32_t i = 0; i < n; ++i)
      if (m == 0 || u[i] != u[m - 1]) u[m++] = u[i];
    uint32_t k = tau[t];
    if (k == 0)
      thr[t] = m ? (double)u[0] : -INFINITY;
    else if (k >= m)
      thr[t] = INFINITY;
    else
      thr[t] = ((double)u[k - 1] + (double)u[k]) / 2.0;
  }
  free(u);
  return OR_OK;
}

/* Routes each row of X (row-major [n][F]) through the tree: t <- 1; while
 * t <= SB: t <- (x_{a_t} < beta_t) ? 2t : 2t + 1; the prediction is the
 * label of leaf t - 2^D.  Writes pred [n] (if not NULL) and returns the
 * number of rows whose prediction equals y (0 when y is NULL). */
uint32_t oracle_predict(const float *X, uint32_t n, uint32_t F, const uint8_t *feat,
                        const double *thr, const uint8_t *label, uint32_t D,
                        const uint8_t *y, uint8_t *pred) {
  uint32_t SB = (1u << D) - 1u, correct = 0;
  for (uint32_t i = 0; i < n; ++i) {
    uint32_t t = 1;
    while (t <= SB) {
      uint32_t f = feat[t - 1];
      int left = (f != 0) && (f <= F) && ((double)X[(size_t)i * F + (f - 1)] < thr[t - 1]);
      t = left ? 2u * t : 2u * t + 1u;
    }
    uint8_t p = label[t - (1u << D)];
    if (pred) pred[i] = p;
    if (y && y[i] == p) correct += 1;
  }
  return correct;
}

/* ------------------------------------------------------------------------ */
/* Encoding a tree into genes (the inverse of eq. aenc and eq. benc), for   */
/* warm starts (Section 4 warm-start variants; reading R14).  Each gene is  */
/* the centre of the interval that decodes to the node's value:             */
/*   a^_t = a_t + 0.5,  b^_t = (tau_t + 0.5) / (n_f + 1) for a_t != 0       */
/* and a^_t = 0.5, b^_t = 0 for a_t = 0 (also for a_t > F, not a feature).   */
/* feat / tau: [P][SB]; genes: out [P][2*SB] as [a^_1..a^_SB, b^_1..b^_SB]. */
/* ------------------------------------------------------------------------ */
void oracle_tree_encode(const uint8_t *feat, const uint32_t *tau, uint32_t P, uint32_t D,
                        uint32_t F, const uint32_t *n_unique, double *genes) {
  uint32_t SB = (1u << D) - 1u;
  for (uint32_t r = 0; r < P; ++r) {
    double *g = genes + (size_t)r * 2 * SB;
    for (uint32_t t = 0; t < SB; ++t) {
      uint32_t f = feat[(size_t)r * SB + t];
      if (f == 0 || f > F) {
        g[t] = 0.5;
        g[SB + t] = 0.0;
      } else {
        g[t] = (double)f + 0.5;
        g[SB + t] = ((double)tau[(size_t)r * SB + t] + 0.5) / ((double)n_unique[f - 1] + 1.0);
      }
    }
  }
}
