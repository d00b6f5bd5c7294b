/*
 * mhdeoct.h -- C ABI of the MI355X (gfx950) library for the data-parallel hot
 * path of MH-DEOCT: differential-evolution fitness evaluation of
 * classification trees (Ren et al., arXiv 2311.06952).
 *
 * Conventions
 * -----------
 *  - Plain C: no C++ types, no exceptions cross this boundary.
 *  - Every array argument is a DEVICE pointer (HBM of the context's GPU)
 *    unless its comment says "host".  The caller owns every buffer it passes
 *    in; the library never frees or keeps a caller pointer past the call
 *    (the serving calls keep the dataset pointers of a request until it
 *    completes; see mh_server_submit).
 *  - A context (mh_ctx) is bound to one device and one HIP stream.  Calls
 *    queue their kernels on that stream and return without waiting, except
 *    those that fill host memory (subtree_solve, mh_train, mh_server_poll,
 *    mh_ctx_stats), which synchronise the stream before returning.
 *  - The context owns an internal device arena for its scratch (tile
 *    layouts, DE state, counters).  It grows on demand with hipMalloc and is
 *    released by mh_ctx_destroy.
 *  - Errors: every call returns an mh_status; a negative value is an error
 *    and mh_last_error() gives a message.  Invalid arguments are reported
 *    before any kernel is queued.  MH_EDEVICE carries the HIP error string.
 *    A context is not thread-safe: use one per host thread.
 *  - Indices are 0-based.  Tree nodes are stored in the paper's heap order
 *    (node t = 1..2^D-1 at slot t-1; children of t are 2t and 2t+1); leaves
 *    are numbered left to right, 0..2^D-1.  A node's feature is 0 for "no
 *    split", else f + 1 for feature f.
 */
#ifndef MHDEOCT_H
#define MHDEOCT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mh_status;
enum {
  MH_OK = 0,
  MH_EINVAL = -1,    /* invalid argument (bad size, depth, null pointer, NaN) */
  MH_ENOMEM = -2,    /* device allocation failed */
  MH_EDEVICE = -3,   /* a HIP call or kernel launch failed */
  MH_EBUSY = -4,     /* serving: admission refused (no slot or HBM budget) */
  MH_ECANCELED = -5  /* serving: request cancelled */
};

/* Limits.  Depth covers the paper's deepest trees (D = 8) with margin. */
#define MH_MAX_DEPTH 10
#define MH_MAX_POP 1024     /* population size P per DE problem */
#define MH_MAX_CLASSES 255
#define MH_MAX_FEATURES 255
#define MH_MAX_BRANCH ((1 << MH_MAX_DEPTH) - 1)

typedef struct mh_ctx mh_ctx;

/* A rank-encoded training set (Section 2 notation: n samples, F features,
 * K classes).  ranks[f * ld + i] is the dense rank of x[i][f] among the
 * sorted unique values of feature f (the threshold sets of Section 3.1,
 * generated once); 0 <= rank < n_unique[f].  labels[i] < K. */
typedef struct {
  uint32_t n, F, K;
  uint32_t ld;               /* column stride of ranks, >= n */
  const uint32_t *ranks;     /* device, column-major [F][ld] */
  const uint8_t *labels;     /* device, [n] */
  const uint32_t *n_unique;  /* device, [F] */
  /* device word written by an asynchronous mh_rank_encode, or NULL.
   * subtree_solve and mh_autotune fail with MH_EINVAL when its bit 0 is set
   * (X held a NaN) and with MH_EDEVICE when a higher bit is (the encoding
   * failed on the device); subtree_solve reads it with its result, mh_train
   * and mh_autotune before they start.  The other calls do not read it. */
  const uint32_t *status;
} mh_dataset;

/* DE parameters (Section 2 eqs. mutation / crossover / selection; Section
 * 3.3; Algorithm 4).  M < 0 draws M_r ~ U[0,1) per individual and
 * generation (the paper's DEOCT setting); M >= 0 is a fixed factor. */
typedef struct {
  uint32_t P;      /* population size, 3 <= P <= MH_MAX_POP */
  uint32_t G;      /* generations; P * (G + 1) trees are evaluated */
  double M;        /* mutation factor */
  double CR;       /* crossover probability */
  uint64_t seed;   /* DE seed; draws are keyed by (seed, problem, g, r, slot) */
  uint32_t n_min;  /* minimum leaf size of the soft constraint (>= 1) */
  double alpha;    /* complexity penalty per split (>= 0) */
} mh_de_params;

/* A decoded tree with its leaf classes and objective (host struct). */
typedef struct {
  uint32_t D;
  uint8_t feat[MH_MAX_BRANCH];     /* 0 = no split, else feature + 1 */
  uint32_t tau[MH_MAX_BRANCH];     /* left iff rank < tau */
  uint8_t label[1 << MH_MAX_DEPTH];
  uint32_t correct;                /* correctly classified training samples */
  double cost;                     /* objective of the Section 3.2 fitness */
} mh_tree;

/* ---------------------------------------------------------------------- */
/* Context                                                                  */
/* ---------------------------------------------------------------------- */

/* Create a context on `device`, queuing work on `hip_stream` (a
 * hipStream_t; NULL = the default stream).  *out receives the handle. */
mh_status mh_ctx_create(int device, void *hip_stream, mh_ctx **out);
void mh_ctx_destroy(mh_ctx *ctx);
/* Message of the last error on this context (never NULL; static storage
 * owned by the context).  With ctx == NULL: the last mh_ctx_create error. */
const char *mh_last_error(const mh_ctx *ctx);
/* Library version string (static). */
const char *mh_version(void);

/* Timing of the fitness kernel.  When enabled, every population-evaluation
 * launch of the fitness kernel records a start and a stop HIP event itself
 * on the context's stream (nothing waits on them; the single-tree
 * evaluation at the end of subtree_solve is not timed).  mh_ctx_stats
 * synchronises the stream and reports the totals since the last reset:
 * timed launches and their milliseconds, and, over every fitness launch of
 * the context whether timed or not, sample-tree evaluations (trees x
 * samples) and scanned tiles. */
mh_status mh_ctx_profile(mh_ctx *ctx, int enable);
mh_status mh_ctx_stats(mh_ctx *ctx, uint64_t *launches, double *ms,
                       uint64_t *evals, uint64_t *tiles, int reset);

/* ---------------------------------------------------------------------- */
/* a1. Threshold sets as dense ranks (Section 3.1: the sets B_p of sorted    */
/* unique values, generated once; min-max scaling does not change ranks).    */
/* ---------------------------------------------------------------------- */

/* X: device, row-major [n][F] float32.  Writes ranks (device [F][ld],
 * ld >= n; columns n..ld-1 are left unwritten) and n_unique (device [F]).
 * -0 and +0 are one value.
 * status == NULL: synchronises the stream and returns MH_EINVAL if X holds
 * a NaN (MH_EDEVICE if the encoding failed on the device).
 * status != NULL (a device word): returns once the work is queued; the
 * device sets *status to 0 when the ranks are valid, bit 0 if X holds a
 * NaN, and higher bits if the encoding failed on the device.  Pass it on in
 * mh_dataset.status to have the solving calls check it. */
mh_status mh_rank_encode(mh_ctx *ctx, const float *X, uint32_t n, uint32_t F,
                         uint32_t ld, uint32_t *ranks, uint32_t *n_unique,
                         uint32_t *status);

/* ---------------------------------------------------------------------- */
/* a2. Decoding individuals (Section 3.1, eq. aenc and eq. benc).           */
/* ---------------------------------------------------------------------- */

/* genes: device [P][2*SB] float64, SB = 2^D - 1, laid out
 * [a^_1..a^_SB, b^_1..b^_SB].  feat_t = min(floor(clamp(a^_t, 0, F+1)), F);
 * tau_t = min(floor(clamp(b^_t, 0, 1) * (n_unique[feat_t - 1] + 1)),
 * n_unique[feat_t - 1]) for feat_t != 0, else 0.  Writes feat (device
 * [P][SB] uint8) and tau (device [P][SB] uint32). */
mh_status tree_decode(mh_ctx *ctx, const double *genes, uint32_t P, uint32_t D,
                      uint32_t F, const uint32_t *n_unique, uint8_t *feat,
                      uint32_t *tau);

/* The inverse of tree_decode, for warm starts (the warm-started variants
 * of Section 4): feat / tau device [P][SB] -> genes device [P][2*SB]
 * float64 with a^_t = feat_t + 0.5 and b^_t = (tau_t + 0.5) / (n_unique[
 * feat_t - 1] + 1), the centre of the interval that decodes to the node;
 * (0.5, 0) for feat_t = 0 or feat_t > F.  tree_decode of the result gives
 * (feat, tau) back for every tau in [0, n_unique].  Only queues work on the
 * context's stream.  MH_EINVAL for bad sizes or null pointers. */
mh_status tree_encode(mh_ctx *ctx, const uint8_t *feat, const uint32_t *tau, uint32_t P,
                      uint32_t D, uint32_t F, const uint32_t *n_unique, double *genes);

/* ---------------------------------------------------------------------- */
/* a3-a5. Fitness of P trees (Algorithm 1; eq. opt_c; eq. opt_all; the      */
/* soft-constraint fitness of Section 3.2).                                  */
/* ---------------------------------------------------------------------- */

/* Routes each of the n_sub samples (idx[j] if idx != NULL, else j) through
 * every tree (left iff feat != 0 and rank < tau) and counts, per tree, leaf
 * and class.  Outputs (device; any may be NULL except cost):
 *   counts  [P][2^D][K] uint32
 *   correct [P] uint32   sum over leaves of the largest class count
 *   label   [P][2^D] uint8 lowest class attaining the largest count
 *   cost    [P] float64  (n_sub - correct) + alpha * #splits
 *                        + #{leaves with 0 < size < n_min}
 * feat / tau: device [P][SB] as written by tree_decode.  1 <= D <= 10,
 * 1 <= P <= MH_MAX_POP, n_sub >= 0.  Builds the tiled sample layout in the
 * context arena on every call (see mh_tileset_build to reuse it). */
mh_status fitness_eval(mh_ctx *ctx, const mh_dataset *ds, const uint32_t *idx,
                       uint32_t n_sub, const uint8_t *feat, const uint32_t *tau,
                       uint32_t P, uint32_t D, uint32_t n_min, double alpha,
                       uint32_t *counts, uint32_t *correct, uint8_t *label,
                       double *cost);

/* fitness_eval for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, outputs and errors as fitness_eval, but the tile layout
 * and counters (tile path: depth <= 5 and F <= 80) or the per-(tree, leaf,
 * class) counts (walk path) live in one static device array of 64 MiB that
 * each GPU holds from the library's load until the process ends; the call
 * calls no allocating routine and only queues kernels on the context's
 * stream (no memset nodes, no timing events).  An evaluation that needs more
 * than 64 MiB of that scratch (the tile path needs about 13.2 * F bytes per
 * sample plus 4 * (2^D - 1) * K * P rounded up; the walk path 4 * P * 2^D * K
 * bytes) fails with MH_EINVAL and queues nothing.  Every call on one GPU
 * shares that GPU's array: calls in flight at the same time on different
 * streams of one GPU race (calls on one stream are ordered).  Each call
 * clears what it reads before use, so no call depends on an earlier one's
 * contents.  MH_EDEVICE if the array's device address could not be looked
 * up. */
mh_status fitness_eval_static(mh_ctx *ctx, const mh_dataset *ds, const uint32_t *idx,
                              uint32_t n_sub, const uint8_t *feat, const uint32_t *tau,
                              uint32_t P, uint32_t D, uint32_t n_min, double alpha,
                              uint32_t *counts, uint32_t *correct, uint8_t *label,
                              double *cost);

/* The tiled sample layout the fitness kernel reads: samples grouped by
 * class into tiles of at most 63, each tile holding, per feature, its ranks
 * in ascending order and the prefix bitmasks of the sample positions in
 * that order, and beside the records the positions themselves (one byte per
 * sorted rank).  mh_tileset_bytes gives the device bytes a layout for n_sub
 * samples needs; mh_tileset_build fills a caller-owned device buffer of at
 * least that size (256-byte aligned).  The layout stays valid as long as
 * the dataset's ranks and labels do not change.  The layout needs
 * ds->n < 2^31 (MH_EINVAL otherwise; fitness_eval then takes the per-sample
 * walk). */
mh_status mh_tileset_bytes(uint32_t n_sub, uint32_t F, uint32_t K, size_t *bytes);
mh_status mh_tileset_build(mh_ctx *ctx, const mh_dataset *ds, const uint32_t *idx,
                           uint32_t n_sub, void *tiles, size_t bytes);
/* fitness_eval over a prebuilt layout (same outputs as fitness_eval). */
mh_status fitness_eval_tiles(mh_ctx *ctx, const void *tiles, const uint32_t *n_unique,
                             const uint8_t *feat, const uint32_t *tau, uint32_t P,
                             uint32_t D, uint32_t n_min, double alpha,
                             uint32_t *counts, uint32_t *correct, uint8_t *label,
                             double *cost);

/* ---------------------------------------------------------------------- */
/* a6. DE step (Section 2 eqs. mutation / crossover / selection; Section    */
/* 3.3; Algorithm 4).                                                        */
/* ---------------------------------------------------------------------- */

/* Initial population (Algorithm 4, first loop): rows 0..W-1 copied from
 * warm (device [W][2*SB], may be NULL when W == 0), the rest drawn inside
 * the range limits: a^ = U (F + 1), b^ = U with U ~ U[0,1).  pop: device
 * [P][2*SB] float64. */
mh_status de_init(mh_ctx *ctx, uint32_t P, uint32_t D, uint32_t F, uint64_t seed,
                  uint64_t problem_id, const double *warm, uint32_t W, double *pop);

/* One DE step for generation g >= 1 of problem `problem_id`:
 *  1. if trial != NULL: selection, pop[r] <- trial[r] and cost[r] <-
 *     trial_cost[r] when trial_cost[r] <= cost[r];
 *  2. best = lowest index of the minimum cost, written to *best (device);
 *  3. if next_trial != NULL: DE/best/1 mutation v = pop[best] + M_r
 *     (pop[r1] - pop[r2]) with r1 != r, r2 not in {r, r1}, clamped to the
 *     range limits, and binomial crossover with CR and q_rand, writing the
 *     trial population of generation g to next_trial (device [P][2*SB]).
 * pop, cost ([P] float64), trial, trial_cost, next_trial: device. */
mh_status de_step(mh_ctx *ctx, const mh_de_params *prm, uint32_t D, uint32_t F,
                  uint64_t problem_id, uint32_t g, double *pop, double *cost,
                  const double *trial, const double *trial_cost, uint32_t *best,
                  double *next_trial);

/* DEOCT (Algorithm 4) on the samples idx[0..n_sub) (all n if idx == NULL):
 * initialise (warm: HOST [W][2*SB] float64, may be NULL), evaluate, then G
 * generations of trial construction from the previous best, population-wide
 * evaluation and selection, all on the device.  Fills *out (host) with the
 * best tree, its leaf labels, correct count and cost.  Synchronises. */
mh_status subtree_solve(mh_ctx *ctx, const mh_dataset *ds, const uint32_t *idx,
                        uint32_t n_sub, uint32_t D, const mh_de_params *prm,
                        const double *warm, uint32_t W, uint64_t problem_id,
                        mh_tree *out);

/* subtree_solve, and the whole final population of the run (Algorithm 4:
 * the population after the selection of generation G): pop_out device
 * [P][2*SB] float64 in the layout of de_init, cost_out device [P] float64,
 * each individual's objective after that selection.  Either may be NULL.
 * Same arguments, errors and synchronisation as subtree_solve; the caller
 * owns both buffers. */
mh_status subtree_solve_pop(mh_ctx *ctx, const mh_dataset *ds, const uint32_t *idx,
                            uint32_t n_sub, uint32_t D, const mh_de_params *prm,
                            const double *warm, uint32_t W, uint64_t problem_id, mh_tree *out,
                            double *pop_out, double *cost_out);

/* Launch-configuration autotuning for DEOCT runs on a dataset shape: times
 * short runs (G = generations, on all of ds) of each candidate (the whole-run
 * cooperative kernel with one or two tile streams per block and 1, 2 or 4
 * blocks per CU; the per-generation kernels with 1, 2 or 4 fitness blocks per
 * CU) and keeps the fastest in the context for this shape (depth, P, F, K and
 * the power-of-two bucket of tiles per CU); later subtree_solve calls of that
 * shape use it.  Configurations change timing only: results are identical.
 * Fills *out (host).  Synchronises. */
typedef struct {
  uint32_t persist, halves, persist_blocks_per_cu, fit_blocks_per_cu;  /* the winner */
  double ms_per_generation;   /* its time per generation */
  uint32_t n_candidates;
  double ms[16];              /* median run time of each candidate, ms */
} mh_tune_result;
mh_status mh_autotune(mh_ctx *ctx, const mh_dataset *ds, uint32_t D,
                      const mh_de_params *prm, uint32_t generations,
                      mh_tune_result *out);

/* ---------------------------------------------------------------------- */
/* a7. Moving-horizon DEOCT (Algorithm 2; Section 4).                       */
/* ---------------------------------------------------------------------- */

#define MH_SEQUENTIAL 0u  /* node by node in heap order, as in Algorithm 2 */
#define MH_BATCHED 1u     /* every node of a level in one batched launch */
/* Warm starts of the subtree solves (Algorithm 2's warm-start branch; the
 * warm-start factors of Section 4's ablation table), OR-ed into flags: */
#define MH_WS_CART 2u       /* the CART subtree (cart_tree) of the node's subset */
#define MH_WS_DEOCT 4u      /* the subtree at the node's location of a DEOCT
                               run on the whole tree (depth D, all samples,
                               problem id 0) made before the first level */
#define MH_WS_DEOCT_CART 8u /* that whole-tree run warm-started with the
                               depth-D CART tree; needs MH_WS_DEOCT */

/* Trains a depth-D tree node by node: each branch node whose subset has
 * more than n_min samples and more than one class gets the first node of a
 * DEOCT subtree of depth min(D_MH, D - depth(t)) (problem id t), or the
 * exact best depth-1 split when that depth is 1; other nodes get no split.
 * A subtree solve's warm starts, by the MH_WS_* bits of flags, come in the
 * order: whole-tree run's subtree, then CART subtree.  The batched form
 * solves all nodes of a level together and returns the identical tree.
 * Fills *out (host).  Synchronises.  MH_EINVAL for unknown flags or
 * MH_WS_DEOCT_CART without MH_WS_DEOCT. */
mh_status mh_train(mh_ctx *ctx, const mh_dataset *ds, uint32_t D, uint32_t D_MH,
                   const mh_de_params *prm, uint32_t flags, mh_tree *out);

/* Exact best depth-1 split under the 0-1 loss (Algorithm 2, horizon-1
 * branch): candidates no-split first, then features ascending, thresholds
 * 1..n_f-1 ascending; the first strict maximum of correct wins.  Writes
 * feat/tau/correct to host.  Synchronises. */
mh_status split1(mh_ctx *ctx, const mh_dataset *ds, const uint32_t *idx,
                 uint32_t n_sub, uint8_t *feat, uint32_t *tau, uint32_t *correct);

/* CART of depth D with the Gini impurity (Breiman et al., the method the
 * paper's DEOCT and MH-DEOCT take warm starts from; Section 4, Algorithm 2)
 * on the samples idx[0..n_sub) (device, distinct indices < n; all of ds
 * when idx is NULL and n_sub == n).  Top down in heap order a node whose
 * subset holds two or more classes takes the first strict maximum, over
 * features 1..F and thresholds 1..n_f-1 ascending that send samples both
 * ways, of sum_k L_k^2/|L| + sum_k R_k^2/|R| in float64 (each division and
 * the sum correctly rounded); other nodes get no split (feat = tau = 0).
 * Writes feat [2^D - 1] and tau [2^D - 1] to HOST memory the caller owns.
 * Synchronises.  MH_EINVAL for bad sizes or null pointers. */
mh_status cart_tree(mh_ctx *ctx, const mh_dataset *ds, const uint32_t *idx,
                    uint32_t n_sub, uint32_t D, uint8_t *feat, uint32_t *tau);

/* ---------------------------------------------------------------------- */
/* Applying a trained tree to held-out samples (Section 2 split rule with   */
/* the Section 3.1 threshold sets; the test accuracy of Section 4).          */
/* ---------------------------------------------------------------------- */

/* Raw-unit thresholds of one tree trained on ds.  X: device, row-major
 * [ds->n][ds->F] float32, the rows ds was rank-encoded from.  feat / tau:
 * device [SB] (SB = 2^D - 1) as in mh_tree or tree_decode.  Writes thr
 * (device [SB] float64): with u_0 < u_1 < ... the unique training values of
 * the node's feature and n_f their number, thr = u_0 for tau = 0 (-inf when
 * n_f = 0), (u_{tau-1} + u_tau) / 2 in float64 for 0 < tau < n_f, +inf for
 * tau >= n_f (every sample left, as the rank rule does), and 0 for a node
 * with feat = 0 or feat > F.  Finite feature values give exactly the rank
 * rule on the training rows.  The caller owns every buffer; the call only
 * queues work on the context's stream.  1 <= D <= 10, ds->n <= 2^31;
 * MH_EINVAL for bad sizes or null pointers. */
mh_status mh_tree_thresholds(mh_ctx *ctx, const mh_dataset *ds, const float *X,
                             const uint8_t *feat, const uint32_t *tau, uint32_t D,
                             double *thr);

/* Routes each row of X (device, row-major [n][F] float32) through the tree
 * (feat device [SB], thr device [SB] from mh_tree_thresholds, label device
 * [2^D]): a row goes left at a node iff feat != 0, feat <= F and
 * (double)x[feat - 1] < thr; it is predicted the label of the leaf it
 * reaches.  NaN values compare false (right).  Writes pred (device [n]
 * uint8) unless NULL.  With y (device [n] uint8) and correct (device
 * uint32) given, *correct receives the number of rows whose prediction
 * equals y; correct needs y when n > 0.  Only queues work on the context's stream.
 * n <= 2^31; MH_EINVAL for bad sizes or null pointers. */
mh_status mh_predict(mh_ctx *ctx, const float *X, uint32_t n, uint32_t F, const uint8_t *feat,
                     const double *thr, const uint8_t *label, uint32_t D, const uint8_t *y,
                     uint8_t *pred, uint32_t *correct);

/* ---------------------------------------------------------------------- */
/* a8. Served subtree solves: DEOCT (Algorithm 4) per request on the problem */
/* of eq. opt_all, with continuous batching.                                 */
/* ---------------------------------------------------------------------- */

typedef struct mh_server mh_server;

/* Result of one request (host struct). */
typedef struct {
  uint64_t req_id;
  mh_status status;      /* MH_OK, MH_EINVAL when the request's X held a NaN, MH_EDEVICE
                            when its cooperative launch gave up at a grid barrier,
                            MH_ECANCELED when it was cancelled (mh_server_cancel or the
                            time limit of mh_server_set_limits; tree then unset) */
  uint32_t n, F, K;
  mh_tree tree;          /* equal to subtree_solve on the same data, problem id 0 */
  uint64_t t_submit_ns;  /* host steady clock: mh_server_submit */
  uint64_t t_admit_ns;   /* admission (device state allocated, work queued) */
  uint64_t t_done_ns;    /* completion observed by mh_server_pump / _poll */
} mh_result;

/* A server on the context's device and stream.  hbm_budget bytes of device
 * memory are allocated once, here, as the pool that holds the resident
 * state of admitted requests (tile layout, population, counters); the
 * context's arena additionally holds the rank-encoding scratch of the
 * largest request.  At most max_slots (1..256) requests are resident at a
 * time.  The context must not be used for other calls while the server
 * exists (they would share its stream and arena). */
mh_status mh_server_create(mh_ctx *ctx, uint64_t hbm_budget, uint32_t max_slots,
                           mh_server **out);
/* Waits for the server's queued work and frees its pool. */
void mh_server_destroy(mh_server *srv);

/* Queues a request: DEOCT of depth D (1..5) with parameters *prm
 * (3 <= P <= 512) on the n samples of X (device, row-major [n][F] float32,
 * F <= 80) with labels (device [n], < K, 2 <= K <= 255).  X and labels must
 * stay valid and unchanged until the request's result has been returned by
 * mh_server_poll.  Requests are admitted in submission order when a slot is
 * free and the pool has room for the request's footprint (the head of the
 * queue waits; later requests do not pass it).  Returns MH_ENOMEM when the
 * footprint exceeds the whole pool, MH_EBUSY when the queue holds the
 * limit set by mh_server_set_limits, MH_EINVAL for invalid arguments.
 * Host-only: queues nothing on the device. */
mh_status mh_server_submit(mh_server *srv, uint64_t req_id, const float *X,
                           const uint8_t *labels, uint32_t n, uint32_t F, uint32_t K,
                           uint32_t D, const mh_de_params *prm);
/* Back-pressure and time limit of a server (both 0 at creation: none).
 * max_queued > 0: mh_server_submit refuses a request with MH_EBUSY (and
 * queues nothing) while max_queued requests wait for admission.
 * timeout_ns > 0: a request not finished timeout_ns after its submission is
 * cancelled at the next scheduling round (as by mh_server_cancel).  Host-only. */
mh_status mh_server_set_limits(mh_server *srv, uint32_t max_queued, uint64_t timeout_ns);
/* Cancels request req_id.  A queued request leaves the queue; a resident one
 * stepped generation by generation is dropped at the next scheduling round
 * (mh_server_pump), and its slot and pool room go to other requests; a
 * request already running as one whole-request launch, or whose result is
 * being copied out, finishes on the device.  Either way its result arrives
 * through mh_server_poll with status MH_ECANCELED.  MH_EINVAL when no queued
 * or running request has this id (unknown, or already finished).
 * Host-only: queues nothing on the device. */
mh_status mh_server_cancel(mh_server *srv, uint64_t req_id);
/* Device bytes of the pool a request of this shape occupies while resident. */
mh_status mh_server_footprint(uint32_t n, uint32_t F, uint32_t K, uint32_t D,
                              uint32_t P, uint64_t *bytes);
/* Runs up to `ticks` scheduling rounds.  A round collects the requests
 * whose device work has finished, admits queued requests while slots and
 * pool allow (rank encoding, tile layout, initial population, queued on the
 * stream), then queues one generation of every resident request: one
 * fitness launch per depth for all of them together, and one DE launch per
 * depth (epilogue, selection, best, next trial), each request at its own
 * generation.  A request whose tile layout has at least two tiles per CU
 * (about 32,000 samples on 256 CUs; MHDEOCT_SERVE_SOLO_TILES sets the tile
 * count, 0 never) fills the device by itself: it runs whole at admission as
 * one cooperative launch, the plain form's kernel.  Requests that ran their
 * G generations get their best tree evaluated and copied to pinned host
 * memory.  At most a few rounds are in
 * flight on the device; a round waits for older ones as needed.  Stops
 * early when nothing is resident or queued.  *n_active / *n_queued (may be
 * NULL) receive the counts after the last round. */
mh_status mh_server_pump(mh_server *srv, uint32_t ticks, uint32_t *n_active,
                         uint32_t *n_queued);
/* Moves up to `max` completed results (in completion order) to out (host)
 * and sets *n_done.  Does not wait. */
mh_status mh_server_poll(mh_server *srv, mh_result *out, uint32_t max, uint32_t *n_done);

#ifdef __cplusplus
}
#endif

#endif /* MHDEOCT_H */
