// rank_encode.hip -- threshold sets as dense ranks (Section 3.1: the sorted
// unique values of each feature, generated once at the start).
//
// All F columns are sorted together by the composite key
// (feature << 32 | order-preserving bits of the value) with the sample index
// as payload, by a stable LSD radix sort (8 bits per pass, 5 passes).  A flag
// marks every position whose key differs from its predecessor; the inclusive
// scan of the flags counts distinct (feature, value) pairs, and a sample's
// rank is that count minus the count at its feature's first position.
#include "device_common.h"
#include "internal.h"

namespace mh {
namespace {

constexpr uint32_t RS_THREADS = 256;
constexpr uint32_t RS_ITEMS = 16;
constexpr uint32_t RS_CHUNK = RS_THREADS * RS_ITEMS;  // keys per block
constexpr uint32_t RS_BINS = 256;

// ---------------------------------------------------------------------------
// u32 scan (exclusive or inclusive) in three kernels
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(RS_THREADS) void k_scan_sums(const uint32_t *__restrict__ in, uint32_t n,
                                                          uint32_t *__restrict__ sums) {
  __shared__ uint32_t red[RS_THREADS];
  const uint32_t b0 = blockIdx.x * RS_CHUNK;
  uint32_t s = 0;
  for (uint32_t k = 0; k < RS_ITEMS; ++k) {
    uint32_t j = b0 + k * RS_THREADS + threadIdx.x;
    if (j < n) s += in[j];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (uint32_t d = RS_THREADS / 2; d > 0; d >>= 1) {
    if (threadIdx.x < d) red[threadIdx.x] += red[threadIdx.x + d];
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = red[0];
}

// Exclusive scan of nb block sums in place (one block).
__global__ __launch_bounds__(1024) void k_scan_top(uint32_t *__restrict__ sums, uint32_t nb) {
  __shared__ uint32_t part[1024];
  __shared__ uint32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (uint32_t b0 = 0; b0 < nb; b0 += 1024) {
    uint32_t b = b0 + threadIdx.x;
    uint32_t v = b < nb ? sums[b] : 0u;
    part[threadIdx.x] = v;
    __syncthreads();
    for (uint32_t d = 1; d < 1024; d <<= 1) {
      uint32_t t = threadIdx.x >= d ? part[threadIdx.x - d] : 0u;
      __syncthreads();
      part[threadIdx.x] += t;
      __syncthreads();
    }
    if (b < nb) sums[b] = carry + part[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry += part[1023];
    __syncthreads();
  }
}

// Blocked local scan: thread t owns items [t*ITEMS, (t+1)*ITEMS) of the chunk.
__global__ __launch_bounds__(RS_THREADS) void k_scan_apply(const uint32_t *__restrict__ in,
                                                           uint32_t *__restrict__ out, uint32_t n,
                                                           const uint32_t *__restrict__ sums,
                                                           int inclusive) {
  __shared__ uint32_t part[RS_THREADS];
  const uint32_t b0 = blockIdx.x * RS_CHUNK + threadIdx.x * RS_ITEMS;
  uint32_t v[RS_ITEMS];
  uint32_t tot = 0;
#pragma unroll
  for (uint32_t k = 0; k < RS_ITEMS; ++k) {
    uint32_t j = b0 + k;
    v[k] = j < n ? in[j] : 0u;
    tot += v[k];
  }
  part[threadIdx.x] = tot;
  __syncthreads();
  for (uint32_t d = 1; d < RS_THREADS; d <<= 1) {
    uint32_t t = threadIdx.x >= d ? part[threadIdx.x - d] : 0u;
    __syncthreads();
    part[threadIdx.x] += t;
    __syncthreads();
  }
  uint32_t run = sums[blockIdx.x] + part[threadIdx.x] - tot;
#pragma unroll
  for (uint32_t k = 0; k < RS_ITEMS; ++k) {
    uint32_t j = b0 + k;
    if (inclusive) run += v[k];
    if (j < n) out[j] = run;
    if (!inclusive) run += v[k];
  }
}

// ---------------------------------------------------------------------------
// radix sort passes
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(RS_THREADS) void k_rs_hist(const uint64_t *__restrict__ keys, uint32_t n,
                                                        uint32_t shift, uint32_t nb,
                                                        uint32_t *__restrict__ hist) {
  __shared__ uint32_t h[RS_BINS];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t b0 = blockIdx.x * RS_CHUNK;
  for (uint32_t k = 0; k < RS_ITEMS; ++k) {
    uint32_t j = b0 + k * RS_THREADS + threadIdx.x;
    if (j < n) atomicAdd(&h[(uint32_t)(keys[j] >> shift) & 0xFFu], 1u);
  }
  __syncthreads();
  hist[threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter.  Keys of the block are taken in order, 256 at a time (a
// round); inside a round wave w holds keys [64w, 64w + 64).  A key's
// destination is its digit's global offset for this block plus the number
// of earlier keys of the block with the same digit: earlier rounds (running),
// earlier waves of this round, and earlier lanes of this wave (ballot match).
__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(
    const uint64_t *__restrict__ keys, const uint32_t *__restrict__ vals, uint32_t n, uint32_t shift,
    uint32_t nb, const uint32_t *__restrict__ offs, uint64_t *__restrict__ okeys,
    uint32_t *__restrict__ ovals) {
  __shared__ uint32_t running[RS_BINS];
  __shared__ uint32_t wcnt[RS_THREADS / 64][RS_BINS];
  const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  running[threadIdx.x] = offs[threadIdx.x * nb + blockIdx.x];
  for (uint32_t q = 0; q < RS_THREADS / 64; ++q) wcnt[q][threadIdx.x] = 0;
  __syncthreads();
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const uint32_t b0 = blockIdx.x * RS_CHUNK;
  for (uint32_t k = 0; k < RS_ITEMS; ++k) {
    const uint32_t j = b0 + k * RS_THREADS + threadIdx.x;
    const bool valid = j < n;
    uint64_t key = valid ? keys[j] : 0ull;
    uint32_t val = valid ? vals[j] : 0u;
    const uint32_t d = (uint32_t)(key >> shift) & 0xFFu;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (uint32_t b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bal = __ballot(bit);
      peers &= bit ? bal : ~bal;
    }
    const uint32_t below = (uint32_t)__popcll(peers & lt_mask);
    if (valid && below == 0) wcnt[w][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pre = running[d] + below;
      for (uint32_t q = 0; q < w; ++q) pre += wcnt[q][d];
      okeys[pre] = key;
      ovals[pre] = val;
    }
    __syncthreads();
    uint32_t add = 0;
    for (uint32_t q = 0; q < RS_THREADS / 64; ++q) {
      add += wcnt[q][threadIdx.x];
      wcnt[q][threadIdx.x] = 0;
    }
    running[threadIdx.x] += add;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// rank encoding
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t orderable_bits(float x) {
  uint32_t u = __float_as_uint(x);
  if (x == 0.0f) u = 0u;  // -0 == +0
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__global__ void k_rank_keys(const float *__restrict__ X, uint32_t n, uint32_t F,
                            uint64_t *__restrict__ keys, uint32_t *__restrict__ vals,
                            uint32_t *__restrict__ nan_flag) {
  uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (uint64_t)n * F) return;
  uint32_t f = (uint32_t)(e / n), i = (uint32_t)(e % n);
  float x = X[(size_t)i * F + f];
  if (x != x) atomicOr(nan_flag, 1u);
  keys[e] = ((uint64_t)f << 32) | orderable_bits(x);
  vals[e] = i;
}

__global__ void k_rank_flags(const uint64_t *__restrict__ keys, uint32_t total,
                             uint32_t *__restrict__ flags) {
  uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= total) return;
  flags[j] = (j == 0 || keys[j] != keys[j - 1]) ? 1u : 0u;
}

__global__ void k_rank_write(const uint32_t *__restrict__ vals, const uint32_t *__restrict__ U,
                             uint32_t n, uint32_t total, uint32_t ld, uint32_t *__restrict__ ranks,
                             uint32_t *__restrict__ n_unique) {
  uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= total) return;
  uint32_t f = j / n;
  uint32_t first = U[f * n];
  ranks[(size_t)f * ld + vals[j]] = U[j] - first;
  if (j == f * n + n - 1) n_unique[f] = U[j] - first + 1u;
}

}  // namespace

mh_status scan_u32(Ctx *ctx, const uint32_t *in, uint32_t *out, uint32_t n, bool inclusive) {
  uint32_t nb = (n + RS_CHUNK - 1) / RS_CHUNK;
  uint32_t *sums = (uint32_t *)arena_get(ctx, "scan_sums", (size_t)(nb ? nb : 1) * 4);
  if (!sums) return MH_ENOMEM;
  hipStream_t st = ctx->stream;
  k_scan_sums<<<nb, RS_THREADS, 0, st>>>(in, n, sums);
  MH_LAUNCHED(ctx, "k_scan_sums");
  k_scan_top<<<1, 1024, 0, st>>>(sums, nb);
  MH_LAUNCHED(ctx, "k_scan_top");
  k_scan_apply<<<nb, RS_THREADS, 0, st>>>(in, out, n, sums, inclusive ? 1 : 0);
  MH_LAUNCHED(ctx, "k_scan_apply");
  return MH_OK;
}

mh_status radix_sort_pairs(Ctx *ctx, uint64_t **keys, uint32_t **vals, uint64_t *keys_alt,
                           uint32_t *vals_alt, uint32_t count, uint32_t key_bits) {
  if (count == 0) return MH_OK;
  uint32_t nb = (count + RS_CHUNK - 1) / RS_CHUNK;
  uint32_t nh = nb * RS_BINS;
  uint32_t *hist = (uint32_t *)arena_get(ctx, "rs_hist", (size_t)nh * 4);
  if (!hist) return MH_ENOMEM;
  hipStream_t st = ctx->stream;
  uint64_t *k0 = *keys, *k1 = keys_alt;
  uint32_t *v0 = *vals, *v1 = vals_alt;
  for (uint32_t shift = 0; shift < key_bits; shift += 8) {
    k_rs_hist<<<nb, RS_THREADS, 0, st>>>(k0, count, shift, nb, hist);
    MH_LAUNCHED(ctx, "k_rs_hist");
    mh_status s = scan_u32(ctx, hist, hist, nh, false);
    if (s) return s;
    k_rs_scatter<<<nb, RS_THREADS, 0, st>>>(k0, v0, count, shift, nb, hist, k1, v1);
    MH_LAUNCHED(ctx, "k_rs_scatter");
    uint64_t *tk = k0;
    k0 = k1;
    k1 = tk;
    uint32_t *tv = v0;
    v0 = v1;
    v1 = tv;
  }
  *keys = k0;
  *vals = v0;
  return MH_OK;
}

mh_status launch_rank_encode(Ctx *ctx, const float *X, uint32_t n, uint32_t F, uint32_t ld,
                             uint32_t *ranks, uint32_t *n_unique, uint32_t *nan_out) {
  uint64_t total64 = (uint64_t)n * F;
  if (total64 >= 0xFFFFFFFFull) return fail(ctx, MH_EINVAL, "n * F too large");
  uint32_t total = (uint32_t)total64;
  if (total == 0) {
    MH_HIP(ctx, hipMemsetAsync(n_unique, 0, (size_t)F * 4, ctx->stream));
    if (nan_out) MH_HIP(ctx, hipMemsetAsync(nan_out, 0, 4, ctx->stream));
    return MH_OK;
  }
  uint64_t *ka = (uint64_t *)arena_get(ctx, "re_keys_a", (size_t)total * 8);
  uint64_t *kb = (uint64_t *)arena_get(ctx, "re_keys_b", (size_t)total * 8);
  uint32_t *va = (uint32_t *)arena_get(ctx, "re_vals_a", (size_t)total * 4);
  uint32_t *vb = (uint32_t *)arena_get(ctx, "re_vals_b", (size_t)total * 4);
  uint32_t *flags = (uint32_t *)arena_get(ctx, "re_flags", (size_t)total * 4 + 256);
  if (!ka || !kb || !va || !vb || !flags) return MH_ENOMEM;
  uint32_t *nan_flag = nan_out ? nan_out : flags + ((total + 63u) & ~63u);
  hipStream_t st = ctx->stream;
  MH_HIP(ctx, hipMemsetAsync(nan_flag, 0, 4, st));
  uint32_t blocks = (total + 255) / 256;
  k_rank_keys<<<blocks, 256, 0, st>>>(X, n, F, ka, va, nan_flag);
  MH_LAUNCHED(ctx, "k_rank_keys");
  uint32_t fbits = 32;
  while ((1u << (fbits - 32)) < F && fbits < 40) fbits += 1;  // bits for the feature id
  uint32_t key_bits = ((fbits + 7) / 8) * 8;
  uint64_t *keys = ka;
  uint32_t *vals = va;
  mh_status s = radix_sort_pairs(ctx, &keys, &vals, kb, vb, total, key_bits);
  if (s) return s;
  k_rank_flags<<<blocks, 256, 0, st>>>(keys, total, flags);
  MH_LAUNCHED(ctx, "k_rank_flags");
  s = scan_u32(ctx, flags, flags, total, true);
  if (s) return s;
  k_rank_write<<<blocks, 256, 0, st>>>(vals, flags, n, total, ld, ranks, n_unique);
  MH_LAUNCHED(ctx, "k_rank_write");
  if (nan_out) return MH_OK;
  uint32_t h_nan = 0;
  MH_HIP(ctx, hipMemcpyAsync(&h_nan, nan_flag, 4, hipMemcpyDeviceToHost, st));
  MH_HIP(ctx, hipStreamSynchronize(st));
  if (h_nan) return fail(ctx, MH_EINVAL, "X holds a NaN");
  return MH_OK;
}

}  // namespace mh
