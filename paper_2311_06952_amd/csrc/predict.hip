// predict.hip -- applying a trained tree to samples it was not trained on
// (Section 2 split rule with the Section 3.1 threshold sets; the test
// accuracy of Section 4).
//
// A tree from the solvers holds rank thresholds: a split (p, tau) sends a
// training sample left iff its rank in feature p is below tau.  For a new
// sample the split needs a value.  The threshold set of feature p is the
// midpoints of adjacent sorted unique training values, headed by the
// training minimum (the scaled 0); the last entry is read as +inf, so that
// tau = n_p still sends every sample left.  With u_0 < u_1 < ... the unique
// training values:
//   tau = 0         beta = u_0   (-inf when n_p = 0)
//   0 < tau < n_p   beta = (u_{tau-1} + u_tau) / 2   in f64
//   tau >= n_p      beta = +inf
// and a sample goes left iff (double)x < beta.
//
// k_thr_scan finds u_{tau-1} and u_tau for every split by scanning the
// feature's rank column: every rank below n_p occurs, and all samples of
// one rank hold the same value (-0 and +0 are one value and give the same
// midpoint), so any matching sample supplies it.  The two floats are staged
// in the two halves of the node's own f64 output word, which k_thr_finish
// then overwrites with beta: no scratch memory.
//
// k_predict stages tiles of rows in LDS, routes each row through the tree
// (also in LDS) and writes the leaf label; with labels given it counts the
// matches (a register count per thread, one atomic per block).  It reads
// each row once, with nontemporal loads: HBM-bound at 4F + 2 bytes per
// sample.
#include "internal.h"

namespace mh {
namespace {

constexpr uint32_t PRED_THREADS = 256;

struct ThrArgs {
  const uint32_t *ranks;
  const uint32_t *n_unique;
  const float *X;
  const uint8_t *feat;
  const uint32_t *tau;
  double *thr;
  uint32_t n, F, ld, SB;
};

__global__ __launch_bounds__(PRED_THREADS) void k_thr_scan(ThrArgs a) {
  const uint32_t t = blockIdx.y;
  const uint32_t f = a.feat[t];
  if (f == 0 || f > a.F) return;
  const uint32_t k = a.tau[t];
  const uint32_t nu = a.n_unique[f - 1];
  if (k >= nu) return;
  float *half = reinterpret_cast<float *>(a.thr + t);
  const uint32_t *col = a.ranks + (size_t)(f - 1) * a.ld;
  const uint32_t stride = gridDim.x * PRED_THREADS;
  for (uint32_t i = blockIdx.x * PRED_THREADS + threadIdx.x; i < a.n; i += stride) {
    const uint32_t r = col[i];
    if (r == k) half[1] = a.X[(size_t)i * a.F + (f - 1)];
    else if (r + 1 == k) half[0] = a.X[(size_t)i * a.F + (f - 1)];
  }
}

__global__ __launch_bounds__(PRED_THREADS) void k_thr_finish(ThrArgs a) {
  const uint32_t t = blockIdx.x * PRED_THREADS + threadIdx.x;
  if (t >= a.SB) return;
  const uint32_t f = a.feat[t];
  double beta = 0.0;
  if (f != 0 && f <= a.F) {
    const uint32_t k = a.tau[t];
    const uint32_t nu = a.n_unique[f - 1];
    const float *half = reinterpret_cast<const float *>(a.thr + t);
    if (k >= nu)
      beta = k == 0 ? -__builtin_inf() : __builtin_inf();
    else if (k == 0)
      beta = (double)half[1];
    else
      beta = __dmul_rn(__dadd_rn((double)half[0], (double)half[1]), 0.5);
  }
  a.thr[t] = beta;
}

struct PredArgs {
  const float *X;
  const uint8_t *feat;
  const double *thr;
  const uint8_t *label;
  const uint8_t *y;
  uint8_t *pred;
  uint32_t *correct;
  uint32_t n, F, D;
  uint32_t tile_rows;  // rows staged per tile: tile_rows * (F + 1) <= PRED_TILE_FLOATS
  uint32_t div_w;      // words (float4 in the vector form, float otherwise) per row
  uint32_t div_m;      // ceil(2^32 / div_w) when div_w > 1: q = umulhi(j, div_m) = j / div_w
};

constexpr uint32_t PRED_TILE_FLOATS = 4096;  // 16 KB of staged rows per block
// the streaming loads of X are nontemporal (each row is read once)
typedef float f4v __attribute__((ext_vector_type(4)));

// j / w for j < 2^16 (a tile holds fewer than 2^16 words) and w < 2^8:
// the multiply-high by ceil(2^32 / w) is exact there.
__device__ __forceinline__ uint32_t tile_div(uint32_t j, uint32_t w, uint32_t m) {
  return w == 1u ? j : __umulhi(j, m);
}

// Rows staged through LDS: a tile of consecutive rows is one contiguous
// stretch of X, read with coalesced loads (float4 when rows are whole
// float4s and X is 16-byte aligned, else single floats); the next tile is
// loaded into registers while the current one is walked, and the walk's
// dependent loads hit LDS.  Rows are padded to F + 1 words so
// that lanes reading the same column of different rows fall in different
// banks.
template <bool VEC>
__global__ __launch_bounds__(PRED_THREADS) void k_predict(PredArgs a) {
  __shared__ float s_x[PRED_TILE_FLOATS];
  __shared__ double s_thr[(1u << MH_MAX_DEPTH) - 1];
  __shared__ uint8_t s_feat[(1u << MH_MAX_DEPTH) - 1];
  __shared__ uint8_t s_label[1u << MH_MAX_DEPTH];
  __shared__ uint32_t s_red[PRED_THREADS / 64];
  const uint32_t SB = (1u << a.D) - 1u;
  const uint32_t F = a.F, ldr = a.F + 1u;
  for (uint32_t t = threadIdx.x; t < SB; t += PRED_THREADS) {
    const uint32_t f = a.feat[t];
    s_feat[t] = (uint8_t)(f <= F ? f : 0u);
    s_thr[t] = a.thr[t];
  }
  for (uint32_t l = threadIdx.x; l <= SB; l += PRED_THREADS) s_label[l] = a.label[l];
  uint32_t ok_count = 0;
  const uint32_t n_tiles = (a.n + a.tile_rows - 1u) / a.tile_rows;
  // the staged rows of a tile through the tree: prediction and count
  auto walk = [&](uint32_t base, uint32_t rows) {
    for (uint32_t r = threadIdx.x; r < rows; r += PRED_THREADS) {
      const float *row = s_x + r * ldr;
      uint32_t t = 0;
      for (uint32_t d = 0; d < a.D; ++d) {
        const uint32_t f = s_feat[t];
        const bool left = f != 0 && (double)row[f - 1] < s_thr[t];
        t = 2u * t + (left ? 1u : 2u);
      }
      const uint8_t p = s_label[t - SB];
      if (a.pred) a.pred[base + r] = p;
      if (a.y) ok_count += a.y[base + r] == p ? 1u : 0u;
    }
  };
  if constexpr (VEC) {
    // A tile is at most PRED_TILE_FLOATS / 4 float4s, PF per lane: the next
    // tile's words are loaded into registers while this one is walked.
    constexpr uint32_t PF = PRED_TILE_FLOATS / 4 / PRED_THREADS;
    f4v nv[PF];
    auto fetch = [&](uint32_t tl) {
      if (tl >= n_tiles) return;
      const uint32_t base = tl * a.tile_rows;
      const uint32_t cnt = min(a.tile_rows, a.n - base) * a.div_w;  // float4 words
      const f4v *src4 = reinterpret_cast<const f4v *>(a.X + (size_t)base * F);
#pragma unroll
      for (uint32_t u = 0; u < PF; ++u) {
        const uint32_t j = threadIdx.x + u * PRED_THREADS;
        if (j < cnt) nv[u] = __builtin_nontemporal_load(src4 + j);
      }
    };
    fetch(blockIdx.x);
    for (uint32_t tl = blockIdx.x; tl < n_tiles; tl += gridDim.x) {
      const uint32_t base = tl * a.tile_rows;
      const uint32_t rows = min(a.tile_rows, a.n - base);
      const uint32_t cnt = rows * a.div_w;
      __syncthreads();  // the previous tile's walk is done (and the tree is staged)
#pragma unroll
      for (uint32_t u = 0; u < PF; ++u) {
        const uint32_t j = threadIdx.x + u * PRED_THREADS;
        if (j < cnt) {
          const uint32_t r = tile_div(j, a.div_w, a.div_m);
          float *dst = s_x + r * ldr + 4u * (j - r * a.div_w);
          dst[0] = nv[u].x;
          dst[1] = nv[u].y;
          dst[2] = nv[u].z;
          dst[3] = nv[u].w;
        }
      }
      __syncthreads();
      fetch(tl + gridDim.x);
      walk(base, rows);
    }
  } else {
    // the same with single floats, PFS per lane
    constexpr uint32_t PFS = PRED_TILE_FLOATS / PRED_THREADS;
    float nv[PFS];
    auto fetch = [&](uint32_t tl) {
      if (tl >= n_tiles) return;
      const uint32_t base = tl * a.tile_rows;
      const uint32_t cnt = min(a.tile_rows, a.n - base) * F;
      const float *src = a.X + (size_t)base * F;
#pragma unroll
      for (uint32_t u = 0; u < PFS; ++u) {
        const uint32_t j = threadIdx.x + u * PRED_THREADS;
        if (j < cnt) nv[u] = __builtin_nontemporal_load(src + j);
      }
    };
    fetch(blockIdx.x);
    for (uint32_t tl = blockIdx.x; tl < n_tiles; tl += gridDim.x) {
      const uint32_t base = tl * a.tile_rows;
      const uint32_t rows = min(a.tile_rows, a.n - base);
      const uint32_t cnt = rows * F;
      __syncthreads();  // the previous tile's walk is done (and the tree is staged)
#pragma unroll
      for (uint32_t u = 0; u < PFS; ++u) {
        const uint32_t j = threadIdx.x + u * PRED_THREADS;
        if (j < cnt) {
          const uint32_t r = tile_div(j, a.div_w, a.div_m);
          s_x[r * ldr + (j - r * F)] = nv[u];
        }
      }
      __syncthreads();
      fetch(tl + gridDim.x);
      walk(base, rows);
    }
  }
  if (a.correct) {
    // one atomic per block: wave sums, then the block's
    for (uint32_t o = 32; o > 0; o >>= 1) ok_count += __shfl_xor(ok_count, o, 64);
    if ((threadIdx.x & 63u) == 0) s_red[threadIdx.x >> 6] = ok_count;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t sum = 0;
      for (uint32_t w = 0; w < PRED_THREADS / 64; ++w) sum += s_red[w];
      if (sum) atomicAdd(a.correct, sum);
    }
  }
}

}  // namespace
}  // namespace mh

using namespace mh;

#define PRED_CTX_OR_FAIL(ctx)                                          \
  do {                                                                 \
    if (!(ctx)) return fail(nullptr, MH_EINVAL, "context is null");    \
    hipError_t e_ = hipSetDevice((ctx)->c.device);                     \
    if (e_ != hipSuccess) return hip_fail(&(ctx)->c, e_, "hipSetDevice"); \
  } while (0)

extern "C" {

mh_status mh_tree_thresholds(mh_ctx *ctx, const mh_dataset *ds, const float *X,
                             const uint8_t *feat, const uint32_t *tau, uint32_t D,
                             double *thr) {
  PRED_CTX_OR_FAIL(ctx);
  Ctx *c = &ctx->c;
  if (!ds) return fail(c, MH_EINVAL, "dataset is null");
  if (ds->F == 0 || ds->F > MH_MAX_FEATURES) return fail(c, MH_EINVAL, "F must be in 1..255");
  if (ds->ld < ds->n) return fail(c, MH_EINVAL, "ld must be >= n");
  if (D < 1 || D > MH_MAX_DEPTH) return fail(c, MH_EINVAL, "D must be in 1..10");
  if (!ds->n_unique || !feat || !tau || !thr) return fail(c, MH_EINVAL, "null pointer");
  if (ds->n > 0 && (!ds->ranks || !X)) return fail(c, MH_EINVAL, "null ranks or X");
  // 32-bit grid-stride indices: i + stride must not wrap
  if (ds->n > (1u << 31)) return fail(c, MH_EINVAL, "n must be <= 2^31");
  ThrArgs a{ds->ranks, ds->n_unique, X, feat, tau, thr, ds->n, ds->F, ds->ld, (1u << D) - 1u};
  if (ds->n > 0) {
    const uint32_t bx = std::min<uint32_t>((ds->n + PRED_THREADS - 1) / PRED_THREADS, 64u);
    k_thr_scan<<<dim3(bx, a.SB), PRED_THREADS, 0, c->stream>>>(a);
    MH_LAUNCHED(c, "k_thr_scan");
  }
  k_thr_finish<<<(a.SB + PRED_THREADS - 1) / PRED_THREADS, PRED_THREADS, 0, c->stream>>>(a);
  MH_LAUNCHED(c, "k_thr_finish");
  return MH_OK;
}

mh_status mh_predict(mh_ctx *ctx, const float *X, uint32_t n, uint32_t F, const uint8_t *feat,
                     const double *thr, const uint8_t *label, uint32_t D, const uint8_t *y,
                     uint8_t *pred, uint32_t *correct) {
  PRED_CTX_OR_FAIL(ctx);
  Ctx *c = &ctx->c;
  if (F == 0 || F > MH_MAX_FEATURES) return fail(c, MH_EINVAL, "F must be in 1..255");
  if (D < 1 || D > MH_MAX_DEPTH) return fail(c, MH_EINVAL, "D must be in 1..10");
  if (!feat || !thr || !label) return fail(c, MH_EINVAL, "null tree pointer");
  if (correct && !y && n > 0) return fail(c, MH_EINVAL, "correct needs y");
  if (n > 0 && !X) return fail(c, MH_EINVAL, "X is null");
  if (n > (1u << 31)) return fail(c, MH_EINVAL, "n must be <= 2^31");
  if (correct) {
    mh_status s = launch_zero(c, {{correct, 4}});
    if (s) return s;
  }
  if (n == 0 || (!pred && !correct)) return MH_OK;
  const uint32_t tile_rows = std::min<uint32_t>(PRED_THREADS, PRED_TILE_FLOATS / (F + 1));
  const bool vec = F % 4u == 0 && reinterpret_cast<uintptr_t>(X) % 16u == 0;
  const uint32_t w = vec ? F / 4u : F;
  const uint32_t m = w > 1 ? (uint32_t)(((1ull << 32) + w - 1) / w) : 0u;
  PredArgs a{X, feat, thr, label, y, pred, correct, n, F, D, tile_rows, w, m};
  const uint32_t tiles = (n + tile_rows - 1) / tile_rows;
  // about 27 KB of LDS per block: five resident blocks per CU, one round
  // (measured: faster than 32 KB tiles at three per CU and 8 KB or 12 KB
  // tiles at seven; with the next tile prefetched into registers one round
  // took 0.183 ms for 16M rows of 16 features, two 0.185 and four 0.186)
  const uint32_t blocks = std::min<uint32_t>(tiles, 5u * (uint32_t)c->num_cu);
  if (vec)
    k_predict<true><<<blocks, PRED_THREADS, 0, c->stream>>>(a);
  else
    k_predict<false><<<blocks, PRED_THREADS, 0, c->stream>>>(a);
  MH_LAUNCHED(c, "k_predict");
  return MH_OK;
}

}  // extern "C"
