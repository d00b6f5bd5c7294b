// rank_encode.hip -- threshold sets as dense ranks (Section 3.1: the sorted
// unique values of each feature, generated once at the start).
//
// A sample's rank in feature f is the number of distinct values of f below
// its value.  Two forms compute it:
//
// * one cooperative launch (inputs of up to a few million values): block b
//   owns a contiguous range of one feature's samples, held in LDS as
//   (order-preserving value bits << 32 | sample) pairs.  Four stable LSD
//   radix passes of 8 bits sort every feature's column; per pass each block
//   publishes its digit histogram and, while a grid barrier completes them,
//   sorts its pairs by digit in LDS; then it derives its digit offsets
//   (totals over the feature's blocks, plus the counts of the blocks before
//   it) and writes each digit's pairs as one contiguous run, and a second
//   barrier precedes the reload of its range in the new order.  A last pass
//   flags every position whose value differs from its predecessor, counts the
//   flags per block, and after a barrier writes each sample's rank (the
//   flags up to it, minus one) and each feature's distinct-value count.
// * separate launches (any size): feature f's (value bits << 32 | sample)
//   pairs form segment f of one array, transposed from X through LDS.  Four
//   stable LSD radix passes of 8 bits sort every segment: per pass a
//   histogram launch (block digit counts, digit-major per feature), one
//   exclusive scan over them all (feature f's part starts at f n, the first
//   position of its segment), and a scatter launch in which a block sorts its
//   pairs by digit in LDS and writes each digit's run contiguously.  Then
//   distinct-value flags, an inclusive scan, and the rank scatter.
#include "device_common.h"
#include "grid_sync.h"
#include "internal.h"
#include "xcd.h"

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
// round); inside a round wave w holds keys [64w, 64w + 64).  A key's rank
// among the block's keys of its digit counts the earlier ones: earlier rounds
// (running), earlier waves of this round, and earlier lanes of this wave
// (ballot match); its destination is its digit's global offset for this
// block plus that rank.  The keys are first placed in LDS in digit order (the
// digit's start inside the block plus the rank) and then written out in that
// order, so that consecutive threads store consecutive slots of a digit's run.
__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(
    const uint64_t *__restrict__ keys, const uint32_t *__restrict__ vals, uint32_t n, uint32_t shift,
    uint32_t nb, const uint32_t *__restrict__ offs, uint64_t *__restrict__ okeys,
    uint32_t *__restrict__ ovals) {
  static_assert(RS_BINS == RS_THREADS, "one digit per thread");
  __shared__ uint64_t s_key[RS_CHUNK];
  __shared__ uint32_t s_val[RS_CHUNK];
  __shared__ uint32_t running[RS_BINS], lstart[RS_BINS], gstart[RS_BINS];
  __shared__ uint32_t wcnt[RS_THREADS / 64][RS_BINS];
  __shared__ uint32_t wsum[RS_THREADS / 64];
  const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  const uint32_t b0 = blockIdx.x * RS_CHUNK;
  // this block's count of digit d = threadIdx.x: the next entry of the scanned
  // [digit][block] offsets less its own (the last entry's next is n)
  const uint32_t o = threadIdx.x * nb + blockIdx.x;
  const uint32_t g = offs[o];
  const uint32_t c = (o + 1 < RS_BINS * nb ? offs[o + 1] : n) - g;
  uint32_t x = c;
#pragma unroll
  for (uint32_t d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  uint32_t ex = x - c;
  for (uint32_t q = 0; q < w; ++q) ex += wsum[q];
  lstart[threadIdx.x] = ex;
  gstart[threadIdx.x] = g;
  running[threadIdx.x] = ex;
  for (uint32_t q = 0; q < RS_THREADS / 64; ++q) wcnt[q][threadIdx.x] = 0;
  __syncthreads();
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  // the block's keys and values loaded up front (one round trip)
  uint64_t kr[RS_ITEMS];
  uint32_t vr[RS_ITEMS];
#pragma unroll
  for (uint32_t k = 0; k < RS_ITEMS; ++k) {
    const uint32_t j = b0 + k * RS_THREADS + threadIdx.x;
    kr[k] = j < n ? keys[j] : 0ull;
    vr[k] = j < n ? vals[j] : 0u;
  }
#pragma unroll
  for (uint32_t k = 0; k < RS_ITEMS; ++k) {
    const uint32_t j = b0 + k * RS_THREADS + threadIdx.x;
    const bool valid = j < n;
    const uint64_t key = kr[k];
    const uint32_t val = vr[k];
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
      s_key[pre] = key;
      s_val[pre] = val;
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
  const uint32_t cnt = n - b0 < RS_CHUNK ? n - b0 : RS_CHUNK;
  for (uint32_t p = threadIdx.x; p < cnt; p += RS_THREADS) {
    const uint64_t key = s_key[p];
    const uint32_t d = (uint32_t)(key >> shift) & 0xFFu;
    const uint32_t dst = gstart[d] + (p - lstart[d]);
    okeys[dst] = key;
    ovals[dst] = s_val[p];
  }
}

// ---------------------------------------------------------------------------
// cooperative form
// ---------------------------------------------------------------------------
constexpr uint32_t RC_THREADS = 256;
constexpr uint32_t RC_WAVES = RC_THREADS / 64;
constexpr uint32_t RC_MAX_R = 8192;  // samples per block (a multiple of 256)
constexpr uint32_t RC_BARRIERS = 9;  // 2 per radix pass, 1 before the rank write

__host__ __device__ __forceinline__ uint32_t rc_lds_bytes(uint32_t R) {
  return R * 16 + RC_WAVES * 256 * 4 + 256 * 4 + 64;
}

struct RankCoopArgs {
  const float *X;  // [n][F]
  uint32_t n, F, ld;
  uint32_t R, nbf;       // samples per block, blocks per feature
  uint64_t *buf0, *buf1;  // [F][n] pairs, ping-pong
  uint32_t *hist;         // [F][nbf][256]
  uint32_t *dcount;       // [F][nbf]
  uint32_t *bar, *err, *nan_flag;
  uint32_t *ranks, *n_unique;
  uint64_t wait_ticks;  // barrier time limit, device wall-clock ticks
};

// Cross-block stores and loads go through agent-scope accesses (the L2s of
// the XCDs are not coherent for ordinary ones).
template <typename T>
__device__ __forceinline__ void xst(T *p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T xld(const T *p) {
  return __hip_atomic_load(const_cast<T *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exclusive scan of one value per thread over the block (256 threads);
// *total receives the sum.  `tmp` holds RC_WAVES + 1 words of LDS.
__device__ __forceinline__ uint32_t rc_block_exscan(uint32_t v, uint32_t *tmp, uint32_t *total) {
  const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (uint32_t d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) tmp[w] = x;
  __syncthreads();
  uint32_t before = 0, all = 0;
#pragma unroll
  for (uint32_t q = 0; q < RC_WAVES; ++q) {
    const uint32_t t = tmp[q];
    before += q < w ? t : 0u;
    all += t;
  }
  __syncthreads();
  *total = all;
  return before + x - v;
}

// ---------------------------------------------------------------------------
// separate launches, per-feature segments
// ---------------------------------------------------------------------------
constexpr uint32_t SG_THREADS = 256;
constexpr uint32_t SG_ITEMS = 16;                  // pairs per thread
constexpr uint32_t SG_R = SG_THREADS * SG_ITEMS;   // positions per block
constexpr uint32_t SG_WSPAN = SG_R / (SG_THREADS / 64);  // positions per wave

// The segment kernels work through the (feature, chunk) list in XCD order
// (xcd.h): the chunks of a feature meet in one XCD's L2.

// Pairs of rows [r0, r0 + rows) for every feature: the rows come in
// coalesced (row-major X) into LDS, padded to F + 1 words per row, and each
// feature's run of positions f n + r0 .. goes out contiguously.
__global__ __launch_bounds__(SG_THREADS) void k_seg_keys(const float *__restrict__ X, uint32_t n,
                                                         uint32_t F, uint32_t rows,
                                                         uint64_t *__restrict__ out,
                                                         uint32_t *__restrict__ nan_flag) {
  extern __shared__ __align__(16) uint32_t sk[];
  const uint32_t r0 = blockIdx.x * rows;
  const uint32_t cnt = min(rows, n - r0);
  bool nan = false;
  // eight loads in flight per lane, then their transforms into LDS
  constexpr uint32_t KU = 8;
  const float *src = X + (size_t)r0 * F;
  const uint32_t tot = cnt * F;
  for (uint32_t e0 = threadIdx.x; e0 < tot; e0 += KU * SG_THREADS) {
    float x[KU];
#pragma unroll
    for (uint32_t u = 0; u < KU; ++u) {
      const uint32_t e = e0 + u * SG_THREADS;
      x[u] = e < tot ? __builtin_nontemporal_load(src + e) : 0.0f;
    }
#pragma unroll
    for (uint32_t u = 0; u < KU; ++u) {
      const uint32_t e = e0 + u * SG_THREADS;
      if (e < tot) {
        nan |= x[u] != x[u];
        uint32_t v = __float_as_uint(x[u]);
        if (x[u] == 0.0f) v = 0u;  // -0 == +0
        v = (v & 0x80000000u) ? ~v : (v | 0x80000000u);
        sk[(e / F) * (F + 1) + e % F] = v;
      }
    }
  }
  if (__ballot(nan) && (threadIdx.x & 63u) == 0) atomicOr(nan_flag, 1u);
  __syncthreads();
  for (uint32_t e = threadIdx.x; e < cnt * F; e += SG_THREADS) {
    const uint32_t f = e / cnt, r = e % cnt;
    out[(size_t)f * n + r0 + r] = ((uint64_t)sk[r * (F + 1) + f] << 32) | (uint64_t)(r0 + r);
  }
}

// One wave's digits d (valid lanes only) into its LDS histogram h.  Lanes
// that share the digit of the lowest pending lane add once, by popcount, while
// such groups hold four lanes or more (the top bytes of real data repeat
// within a wave, and adds of many lanes to one word serialise); the rest add
// one by one.
__device__ __forceinline__ void wave_hist_add(uint32_t *h, uint32_t d, bool valid) {
  const uint32_t lane = threadIdx.x & 63u;
  uint64_t pending = __ballot(valid);
  while (pending) {
    const int leader = __builtin_ctzll(pending);
    const uint32_t dl = (uint32_t)__builtin_amdgcn_readlane((int)d, leader);
    const uint64_t same = __ballot(valid && d == dl) & pending;
    const uint32_t c = (uint32_t)__popcll(same);
    if (c < 4) break;
    if (lane == (uint32_t)leader) atomicAdd(&h[dl], c);
    pending &= ~same;
  }
  if ((pending >> lane) & 1ull) atomicAdd(&h[d], 1u);
}

// Digit counts of block (f, j): positions [j SG_R, (j + 1) SG_R) of segment f,
// into hist[(f 256 + digit) nbf + j].
__global__ __launch_bounds__(SG_THREADS) void k_seg_hist(const uint64_t *__restrict__ src,
                                                         uint32_t n, uint32_t F, uint32_t nbf,
                                                         uint32_t shift,
                                                         uint32_t *__restrict__ hist) {
  __shared__ uint32_t h[SG_THREADS / 64][256];
  const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  const uint32_t bi = xcd_order(blockIdx.x, gridDim.x);
  if (bi >= F * nbf) return;
  const uint32_t f = bi / nbf, j = bi % nbf;
  const uint32_t lo = j * SG_R, hi = min(n, lo + SG_R);
#pragma unroll
  for (uint32_t q = 0; q < 4; ++q) h[w][q * 64 + lane] = 0;
  __syncthreads();
  const uint64_t *seg = src + (size_t)f * n;
  uint32_t d[SG_ITEMS];
#pragma unroll
  for (uint32_t k = 0; k < SG_ITEMS; ++k) {
    const uint32_t q = lo + k * SG_THREADS + threadIdx.x;
    d[k] = q < hi ? (uint32_t)(seg[q] >> shift) & 0xFFu : 256u;
  }
#pragma unroll
  for (uint32_t k = 0; k < SG_ITEMS; ++k)
    wave_hist_add(h[w], d[k], d[k] < 256u);
  __syncthreads();
  uint32_t t = 0;
#pragma unroll
  for (uint32_t q = 0; q < SG_THREADS / 64; ++q) t += h[q][threadIdx.x];
  hist[((size_t)f * 256 + threadIdx.x) * nbf + j] = t;
}

// Block (f, j) of a pass: its pairs (wave w holds the span of SG_WSPAN
// positions w SG_WSPAN ..., 64 at a time in registers) stably sorted by digit
// into LDS (a wave's digit counts and their offsets in the block's order,
// then each pair's rank among the earlier pairs of its wave with the same
// digit by ballot match), and written out: digit d's run goes to offs[(f 256
// + d) nbf + j], the global position the scan gave it.
__global__ __launch_bounds__(SG_THREADS) void k_seg_scatter(const uint64_t *__restrict__ src,
                                                            uint64_t *__restrict__ dst,
                                                            uint32_t n, uint32_t F, uint32_t nbf,
                                                            uint32_t shift,
                                                            const uint32_t *__restrict__ offs) {
  __shared__ uint64_t kv[SG_R];
  __shared__ uint32_t wc[SG_THREADS / 64][256];
  __shared__ uint32_t gpos[256];
  __shared__ uint32_t tmp[SG_THREADS / 64 + 1];
  const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  const uint32_t bi = xcd_order(blockIdx.x, gridDim.x);
  if (bi >= F * nbf) return;
  const uint32_t f = bi / nbf, j = bi % nbf;
  const uint32_t lo = j * SG_R, cnt = min(n - lo, SG_R);
  const uint64_t *seg = src + (size_t)f * n + lo;
  const uint64_t lt_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
  constexpr uint32_t RND = SG_WSPAN / 64;
  uint64_t v[RND];
  uint32_t d[RND];
#pragma unroll
  for (uint32_t k = 0; k < 4; ++k) wc[w][k * 64 + lane] = 0;
#pragma unroll
  for (uint32_t k = 0; k < RND; ++k) {
    const uint32_t q = w * SG_WSPAN + k * 64 + lane;
    v[k] = q < cnt ? seg[q] : 0ull;
    d[k] = q < cnt ? (uint32_t)(v[k] >> shift) & 0xFFu : 256u;
  }
  __syncthreads();
#pragma unroll
  for (uint32_t k = 0; k < RND; ++k)
    if (d[k] < 256u) atomicAdd(&wc[w][d[k]], 1u);
  __syncthreads();
  // block order: digit-major, then wave; wc[w][d] becomes wave w's first slot
  // of digit d, gpos[d] the global position of the block's slot 0 of digit d
  {
    uint32_t c[SG_THREADS / 64], tot = 0;
#pragma unroll
    for (uint32_t q = 0; q < SG_THREADS / 64; ++q) {
      c[q] = wc[q][threadIdx.x];
      tot += c[q];
    }
    uint32_t all;
    const uint32_t start = rc_block_exscan(tot, tmp, &all);
    uint32_t run = start;
#pragma unroll
    for (uint32_t q = 0; q < SG_THREADS / 64; ++q) {
      wc[q][threadIdx.x] = run;
      run += c[q];
    }
    gpos[threadIdx.x] = offs[((size_t)f * 256 + threadIdx.x) * nbf + j] - start;
  }
  __syncthreads();
#pragma unroll
  for (uint32_t k = 0; k < RND; ++k) {
    const bool valid = d[k] < 256u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (uint32_t bit = 0; bit < 8; ++bit) {
      const bool on = (d[k] >> bit) & 1u;
      const uint64_t bal = __ballot(on);
      peers &= on ? bal : ~bal;
    }
    const uint32_t below = (uint32_t)__popcll(peers & lt_mask);
    const uint32_t slot = valid ? wc[w][d[k]] : 0u;
    __builtin_amdgcn_wave_barrier();
    if (valid) {
      kv[slot + below] = v[k];
      if (below == 0) wc[w][d[k]] = slot + (uint32_t)__popcll(peers);
    }
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  for (uint32_t q = threadIdx.x; q < cnt; q += SG_THREADS) {
    const uint64_t x = kv[q];
    dst[gpos[(uint32_t)(x >> shift) & 0xFFu] + q] = x;
  }
}

// Ranks from the sorted segments.  Position p of segment f starts a new value
// when it is the segment's first or its value bits differ from position
// p - 1's; a sample's rank is the number of such starts up to and including
// its position, minus one.  Block (f, j) covers positions [j SG_R, (j + 1)
// SG_R) of segment f, wave w the span of SG_WSPAN positions from j SG_R +
// w SG_WSPAN, 64 at a time: the starts among a chunk's lanes come from one
// ballot, so a lane's count is a popcount of the bits below it.
//
// Pass 1: starts per block, ucnt[f nbf + j].
__global__ __launch_bounds__(SG_THREADS) void k_seg_ucount(const uint64_t *__restrict__ src,
                                                           uint32_t n, uint32_t F, uint32_t nbf,
                                                           uint32_t *__restrict__ ucnt) {
  __shared__ uint32_t wsum[SG_THREADS / 64];
  const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  const uint32_t bi = xcd_order(blockIdx.x, gridDim.x);
  if (bi >= F * nbf) return;
  const uint32_t f = bi / nbf, j = bi % nbf;
  const uint64_t *seg = src + (size_t)f * n;
  const uint32_t q0 = j * SG_R + w * SG_WSPAN;
  const uint32_t q1 = min(n, q0 + SG_WSPAN);
  uint32_t starts = 0;
  // value bits of the position before the chunk (none before the segment)
  uint32_t prev = (q0 > 0 && q0 < n) ? (uint32_t)(seg[q0 - 1] >> 32) : 0u;
  bool prev_ok = q0 > 0;
  // the wave's span loaded up front (one round trip), then scanned 64 at a time
  constexpr uint32_t RND = SG_WSPAN / 64;
  uint32_t vv[RND];
#pragma unroll
  for (uint32_t k = 0; k < RND; ++k) {
    const uint32_t q = q0 + k * 64 + lane;
    vv[k] = q < q1 ? (uint32_t)(seg[q] >> 32) : 0u;
  }
#pragma unroll
  for (uint32_t k = 0; k < RND; ++k) {
    const uint32_t q = q0 + k * 64 + lane;
    const bool valid = q < q1;
    const uint32_t v = vv[k];
    uint32_t left = __shfl_up(v, 1, 64);
    if (lane == 0) left = prev;
    const bool start = valid && (lane == 0 ? (!prev_ok || v != left) : v != left);
    starts += (uint32_t)__popcll(__ballot(start));
    prev = __shfl(v, 63, 64);
    prev_ok = true;
  }
  if (lane == 0) wsum[w] = starts;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
#pragma unroll
    for (uint32_t q = 0; q < SG_THREADS / 64; ++q) t += wsum[q];
    ucnt[bi] = t;
  }
}

// Pass 2, block f: exclusive scan of segment f's block counts in place, and
// its number of distinct values.
__global__ __launch_bounds__(SG_THREADS) void k_seg_ubase(uint32_t *__restrict__ ucnt, uint32_t nbf,
                                                          uint32_t *__restrict__ n_unique) {
  __shared__ uint32_t tmp[SG_THREADS / 64 + 1];
  uint32_t *u = ucnt + (size_t)blockIdx.x * nbf;
  uint32_t run = 0;
  for (uint32_t c = 0; c < nbf; c += SG_THREADS) {
    const uint32_t i = c + threadIdx.x;
    const uint32_t v = i < nbf ? u[i] : 0u;
    uint32_t all;
    const uint32_t ex = rc_block_exscan(v, tmp, &all);
    if (i < nbf) u[i] = run + ex;
    run += all;
  }
  if (threadIdx.x == 0) n_unique[blockIdx.x] = run;
}

// Pass 3: each position's rank, written to its sample: ranks[f ld + sample].
__global__ __launch_bounds__(SG_THREADS) void k_seg_rank_scatter(
    const uint64_t *__restrict__ src, uint32_t n, uint32_t F, uint32_t nbf,
    const uint32_t *__restrict__ ubase, uint32_t ld, uint32_t id_lo, uint32_t id_hi,
    uint32_t *__restrict__ ranks) {
  __shared__ uint32_t wsum[SG_THREADS / 64];
  const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  const uint32_t bi = xcd_order(blockIdx.x, gridDim.x);
  if (bi >= F * nbf) return;
  const uint32_t f = bi / nbf, j = bi % nbf;
  const uint64_t *seg = src + (size_t)f * n;
  const uint32_t q0 = j * SG_R + w * SG_WSPAN;
  const uint32_t q1 = min(n, q0 + SG_WSPAN);
  constexpr uint32_t RND = SG_WSPAN / 64;
  const uint64_t lt_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
  uint32_t loc[RND], idx[RND];
  uint32_t starts = 0;
  uint32_t prev = (q0 > 0 && q0 < n) ? (uint32_t)(seg[q0 - 1] >> 32) : 0u;
  bool prev_ok = q0 > 0;
#pragma unroll
  for (uint32_t k = 0; k < RND; ++k) {
    const uint32_t q = q0 + k * 64 + lane;
    const bool valid = q < q1;
    const uint64_t x = valid ? __builtin_nontemporal_load(seg + q) : 0ull;
    const uint32_t v = (uint32_t)(x >> 32);
    uint32_t left = __shfl_up(v, 1, 64);
    if (lane == 0) left = prev;
    const bool start = valid && (lane == 0 ? (!prev_ok || v != left) : v != left);
    const uint64_t b = __ballot(start);
    // starts of the wave's span up to and including this position
    loc[k] = starts + (uint32_t)__popcll(b & lt_mask) + (start ? 1u : 0u);
    idx[k] = valid ? (uint32_t)x : 0xFFFFFFFFu;
    starts += (uint32_t)__popcll(b);
    prev = __shfl(v, 63, 64);
    prev_ok = true;
  }
  if (lane == 0) wsum[w] = starts;
  __syncthreads();
  uint32_t base = ubase[bi];
  for (uint32_t q = 0; q < w; ++q) base += wsum[q];
  uint32_t *rk = ranks + (size_t)f * ld;
#pragma unroll
  for (uint32_t k = 0; k < RND; ++k)
    if (idx[k] - id_lo < id_hi - id_lo) rk[idx[k]] = base + loc[k] - 1u;
}

__global__ __launch_bounds__(RC_THREADS) void k_rank_coop(RankCoopArgs a) {
  extern __shared__ __align__(16) uint8_t rc_lds[];
  uint64_t *kv = reinterpret_cast<uint64_t *>(rc_lds);                // [R] the block's range
  uint64_t *kv2 = kv + a.R;                                          // [R] sorted by digit
  uint32_t *wcnt = reinterpret_cast<uint32_t *>(rc_lds + a.R * 16);  // [RC_WAVES][256]
  uint32_t *hb = wcnt + RC_WAVES * 256;                              // [256]
  uint32_t *tmp = hb + 256;                                          // [16]
  const uint32_t tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
  const uint32_t nb = gridDim.x, b = blockIdx.x;
  const uint32_t f = b / a.nbf, j = b % a.nbf;
  const uint32_t n = a.n;
  const uint32_t lo = min(n, j * a.R), hi = min(n, lo + a.R), cnt = hi - lo;
  const uint64_t lt_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
  const size_t seg = (size_t)f * n;
  uint32_t k = 0;  // barriers passed

  // load: order-preserving bits of X[i][f] (-0 as +0) with the sample index
  bool nan = false;
  for (uint32_t q = tid; q < cnt; q += RC_THREADS) {
    const float x = a.X[(size_t)(lo + q) * a.F + f];
    nan |= x != x;
    uint32_t u = __float_as_uint(x);
    if (x == 0.0f) u = 0u;
    u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    kv[q] = ((uint64_t)u << 32) | (uint64_t)(lo + q);
  }
  if (__ballot(nan) && lane == 0)
    __hip_atomic_fetch_or(a.nan_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // wave w handles the span [w0, w1) of S consecutive positions
  const uint32_t S = ((cnt + RC_THREADS - 1) / RC_THREADS) * 64;
  const uint32_t w0 = min(cnt, w * S), w1 = min(cnt, w0 + S);

  const uint64_t *src = nullptr;
  uint64_t *dst = a.buf0;
  for (uint32_t pass = 0; pass < 4; ++pass) {
    const uint32_t shift = 32 + 8 * pass;
    // digit histogram of each wave's span
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) wcnt[w * 256 + q * 64 + lane] = 0;
    __syncthreads();
    for (uint32_t q = w0 + lane; q < w1; q += 64)
      atomicAdd(&wcnt[w * 256 + ((uint32_t)(kv[q] >> shift) & 0xFFu)], 1u);
    __syncthreads();
    // the block's histogram is published; in the block's digit-sorted order
    // digit d starts at hb[d], and wave w's keys of digit d at wcnt[w][d]
    {
      uint32_t c[RC_WAVES], tot = 0;
#pragma unroll
      for (uint32_t q = 0; q < RC_WAVES; ++q) {
        c[q] = wcnt[q * 256 + tid];
        tot += c[q];
      }
      xst(a.hist + ((size_t)b * 256 + tid), tot);
      uint32_t all;
      const uint32_t loc = rc_block_exscan(tot, tmp, &all);
      hb[tid] = loc;
      uint32_t run = loc;
#pragma unroll
      for (uint32_t q = 0; q < RC_WAVES; ++q) {
        wcnt[q * 256 + tid] = run;
        run += c[q];
      }
    }
    barrier_arrive(a.bar, k, b, nb);
    // meanwhile: the block's keys, stably sorted by digit, into kv2 (a
    // position's rank among the earlier positions of its wave's span with
    // the same digit: ballot match over the digit's bits)
    for (uint32_t q0 = w0; q0 < w1; q0 += 64) {
      const uint32_t q = q0 + lane;
      const bool valid = q < w1;
      const uint64_t v = valid ? kv[q] : 0ull;
      const uint32_t d = (uint32_t)(v >> shift) & 0xFFu;
      uint64_t peers = __ballot(valid);
#pragma unroll
      for (uint32_t bit = 0; bit < 8; ++bit) {
        const bool on = (d >> bit) & 1u;
        const uint64_t bal = __ballot(on);
        peers &= on ? bal : ~bal;
      }
      const uint32_t below = (uint32_t)__popcll(peers & lt_mask);
      const uint32_t c = valid ? wcnt[w * 256 + d] : 0u;
      __builtin_amdgcn_wave_barrier();
      if (valid) {
        if (c + below < cnt) kv2[c + below] = v;
        if (below == 0) wcnt[w * 256 + d] = c + (uint32_t)__popcll(peers);
      }
      __builtin_amdgcn_wave_barrier();
    }
    barrier_wait(a.bar, k, a.err, a.wait_ticks);
    ++k;
    // global start of the block's keys of digit tid: all smaller digits of
    // the feature, plus digit tid in the feature's earlier blocks
    {
      uint32_t pre = 0, tot = 0;
      const uint32_t *h = a.hist + (size_t)f * a.nbf * 256 + tid;
      for (uint32_t j0 = 0; j0 < a.nbf; j0 += 16) {
        uint32_t v[16];
#pragma unroll
        for (uint32_t u = 0; u < 16; ++u) v[u] = j0 + u < a.nbf ? xld(h + (size_t)(j0 + u) * 256) : 0u;
#pragma unroll
        for (uint32_t u = 0; u < 16; ++u) {
          tot += v[u];
          pre += j0 + u < j ? v[u] : 0u;
        }
      }
      uint32_t all;
      const uint32_t gb = rc_block_exscan(tot, tmp, &all) + pre;
      hb[tid] = gb - hb[tid];  // kv2[q] of digit d goes to position hb[d] + q
    }
    __syncthreads();
    for (uint32_t q = tid; q < cnt; q += RC_THREADS) {
      const uint64_t v = kv2[q];
      const uint32_t pos = hb[(uint32_t)(v >> shift) & 0xFFu] + q;
      if (pos < n)
        xst(dst + seg + pos, v);
      else
        __hip_atomic_fetch_or(a.err, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    barrier_arrive(a.bar, k, b, nb);
    barrier_wait(a.bar, k, a.err, a.wait_ticks);
    ++k;
    for (uint32_t q = tid; q < cnt; q += RC_THREADS) kv[q] = xld(dst + seg + lo + q);
    src = dst;
    dst = dst == a.buf0 ? a.buf1 : a.buf0;
  }
  __syncthreads();

  // distinct-value flags of the sorted column: a position starts a new value
  // when it is the feature's first or its value differs from the previous one
  const uint64_t prev_lo = lo > 0 ? xld(src + seg + lo - 1) : 0ull;
  auto flag_at = [&](uint32_t q) -> uint32_t {
    const uint32_t v = (uint32_t)(kv[q] >> 32);
    if (q == 0) return (lo == 0 || (uint32_t)(prev_lo >> 32) != v) ? 1u : 0u;
    return (uint32_t)(kv[q - 1] >> 32) != v ? 1u : 0u;
  };
  uint32_t mine = 0;
  for (uint32_t q = tid; q < cnt; q += RC_THREADS) mine += flag_at(q);
  uint32_t count;
  (void)rc_block_exscan(mine, tmp, &count);
  if (tid == 0) xst(a.dcount + b, count);
  barrier_arrive(a.bar, k, b, nb);
  barrier_wait(a.bar, k, a.err, a.wait_ticks);
  ++k;
  uint32_t base = 0;
  {
    uint32_t part = 0;
    for (uint32_t jj = tid; jj < j; jj += RC_THREADS)
      part += xld(a.dcount + (size_t)f * a.nbf + jj);
    uint32_t all;
    (void)rc_block_exscan(part, tmp, &all);
    base = all;
  }
  // rank = distinct values up to and including this position, minus one
  uint32_t carry = base;
  for (uint32_t c0 = 0; c0 < cnt; c0 += RC_THREADS) {
    const uint32_t q = c0 + tid;
    const uint32_t fl = q < cnt ? flag_at(q) : 0u;
    uint32_t chunk;
    const uint32_t ex = rc_block_exscan(fl, tmp, &chunk);
    if (q < cnt) {
      const uint32_t i = (uint32_t)kv[q];
      if (i < n)
        a.ranks[(size_t)f * a.ld + i] = carry + ex + fl - 1u;
      else
        __hip_atomic_fetch_or(a.err, 4u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    carry += chunk;
  }
  if (j == a.nbf - 1 && tid == 0) a.n_unique[f] = base + count;
  // a caller that takes the NaN flag sees a failure there too (bit 1 and up)
  if (tid == 0) {
    const uint32_t e = xld(a.err);
    if (e) __hip_atomic_fetch_or(a.nan_flag, e << 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  (void)RC_BARRIERS;
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

namespace {
// Samples per block of the cooperative form for an n x F input, or 0 when it
// does not apply: the smallest power of two from 256 that keeps the grid
// within four blocks per CU (grids of six blocks per CU, although accepted
// by the launch, did not all become resident together) and within what the
// occupancy query allows.
uint32_t rank_coop_R(Ctx *ctx, uint32_t n, uint32_t F) {
  if (!ctx->coop || !ctx->rank_coop) return 0;
  const uint64_t target = (uint64_t)ctx->num_cu * 4u;
  for (uint32_t R = 256; R <= RC_MAX_R; R *= 2) {
    if (ctx->rank_coop_R && R != ctx->rank_coop_R) continue;
    const uint64_t grid = (uint64_t)F * ((n + R - 1) / R);
    if (grid > target) continue;
    const void *kern = reinterpret_cast<const void *>(k_rank_coop);
    const int per_cu = coop_per_cu(ctx, kern, RC_THREADS, rc_lds_bytes(R));
    if (per_cu < 1) return 0;
    if ((uint64_t)per_cu * ctx->num_cu >= grid && !coop_is_bad(ctx, kern, (uint32_t)grid))
      return R;
  }
  return 0;
}

// The cooperative form; *used = false leaves the work to the separate
// launches (a shape the cooperative launch refuses).
mh_status rank_encode_coop(Ctx *ctx, const float *X, uint32_t n, uint32_t F, uint32_t ld,
                           uint32_t R, uint32_t *ranks, uint32_t *n_unique, uint32_t *nan_flag,
                           uint32_t *err, uint32_t *bar, bool *used) {
  *used = false;
  const uint32_t nbf = (n + R - 1) / R, grid = F * nbf;
  const size_t total = (size_t)n * F;
  RankCoopArgs a;
  a.X = X;
  a.n = n;
  a.F = F;
  a.ld = ld;
  a.R = R;
  a.nbf = nbf;
  a.buf0 = (uint64_t *)arena_get(ctx, "re_keys_a", total * 8);
  a.buf1 = (uint64_t *)arena_get(ctx, "re_keys_b", total * 8);
  a.hist = (uint32_t *)arena_get(ctx, "re_hist", (size_t)grid * 256 * 4);
  a.dcount = (uint32_t *)arena_get(ctx, "re_dcount", (size_t)grid * 4);
  a.bar = bar;
  if (!a.buf0 || !a.buf1 || !a.hist || !a.dcount) return MH_ENOMEM;
  a.err = err;
  a.nan_flag = nan_flag;
  a.ranks = ranks;
  a.n_unique = n_unique;
  a.wait_ticks = ctx->wait_ticks;
  void *args[] = {&a};
  hipError_t e = launch_grid_sync(ctx, reinterpret_cast<const void *>(k_rank_coop), dim3(grid),
                                  dim3(RC_THREADS), args, rc_lds_bytes(R));
  if (e == hipErrorInvalidValue || e == hipErrorCooperativeLaunchTooLarge ||
      e == hipErrorInvalidConfiguration) {
    (void)hipGetLastError();
    return MH_OK;
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "k_rank_coop");
  ctx->last_coop_kern = reinterpret_cast<const void *>(k_rank_coop);
  ctx->last_coop_grid = grid;
  *used = true;
  return MH_OK;
}
}  // namespace

mh_status launch_rank_encode(Ctx *ctx, const float *X, uint32_t n, uint32_t F, uint32_t ld,
                             uint32_t *ranks, uint32_t *n_unique, uint32_t *nan_out, bool retry) {
  uint64_t total64 = (uint64_t)n * F;
  if (total64 >= 0xFFFFFFFFull) return fail(ctx, MH_EINVAL, "n * F too large");
  uint32_t total = (uint32_t)total64;
  hipStream_t st = ctx->stream;
  if (total == 0) {
    MH_HIP(ctx, hipMemsetAsync(n_unique, 0, (size_t)F * 4, st));
    if (nan_out) MH_HIP(ctx, hipMemsetAsync(nan_out, 0, 4, st));
    return MH_OK;
  }
  // [0] NaN seen (unless the caller takes it); [1] cooperative-form failure
  // bits: 1 a grid barrier wait gave up, 2 and 4 an index out of range
  uint32_t *words = (uint32_t *)arena_get(ctx, "re_words", 256);
  if (!words) return MH_ENOMEM;
  uint32_t *nan_flag = nan_out ? nan_out : words;
  // the cooperative form's barrier words are cleared with the flags
  const uint32_t R = rank_coop_R(ctx, n, F);
  const size_t bar_bytes = R ? (size_t)barrier_words(F * ((n + R - 1) / R)) * 4 : 0;
  uint32_t *bar = R ? (uint32_t *)arena_get(ctx, "re_bar", bar_bytes) : nullptr;
  if (R && !bar) return MH_ENOMEM;
  mh_status zs = launch_zero(ctx, {{words, 8}, {nan_out, nan_out ? 4u : 0u}, {bar, bar_bytes}});
  if (zs) return zs;
  bool done = false;
  if (R) {
    mh_status s =
        rank_encode_coop(ctx, X, n, F, ld, R, ranks, n_unique, nan_flag, words + 1, bar, &done);
    if (s) return s;
  }
  if (!done) {
    uint64_t *ka = (uint64_t *)arena_get(ctx, "re_keys_a", (size_t)total * 8);
    uint64_t *kb = (uint64_t *)arena_get(ctx, "re_keys_b", (size_t)total * 8);
    const uint32_t nbf = (n + SG_R - 1) / SG_R, nh = F * 256 * nbf;
    uint32_t *hist = (uint32_t *)arena_get(ctx, "re_seg_hist", (size_t)nh * 4);
    uint32_t *ucnt = (uint32_t *)arena_get(ctx, "re_ucnt", (size_t)F * nbf * 4);
    if (!ka || !kb || !hist || !ucnt) return MH_ENOMEM;
    // rows per transposing block: an LDS tile of rows x (F + 1) words
    const uint32_t rows = std::max(1u, std::min(256u, (uint32_t)(16384u / (F + 1u))));
    const uint32_t kblocks = (n + rows - 1) / rows;
    k_seg_keys<<<kblocks, SG_THREADS, (size_t)rows * (F + 1) * 4, st>>>(X, n, F, rows, ka,
                                                                        nan_flag);
    MH_LAUNCHED(ctx, "k_seg_keys");
    uint64_t *a = ka, *b = kb;
    for (uint32_t pass = 0; pass < 4; ++pass) {
      const uint32_t shift = 32 + 8 * pass;
      k_seg_hist<<<xcd_grid(F * nbf), SG_THREADS, 0, st>>>(a, n, F, nbf, shift, hist);
      MH_LAUNCHED(ctx, "k_seg_hist");
      mh_status s = scan_u32(ctx, hist, hist, nh, false);
      if (s) return s;
      k_seg_scatter<<<xcd_grid(F * nbf), SG_THREADS, 0, st>>>(a, b, n, F, nbf, shift, hist);
      MH_LAUNCHED(ctx, "k_seg_scatter");
      std::swap(a, b);
    }
    k_seg_ucount<<<xcd_grid(F * nbf), SG_THREADS, 0, st>>>(a, n, F, nbf, ucnt);
    MH_LAUNCHED(ctx, "k_seg_ucount");
    k_seg_ubase<<<F, SG_THREADS, 0, st>>>(ucnt, nbf, n_unique);
    MH_LAUNCHED(ctx, "k_seg_ubase");
    // The scatter's 4-byte writes land at random in a feature's row of ranks,
    // and an XCD works through its features one after another.  With rows of
    // 2 to 8 MB (an XCD's L2 holds 4 MB) the launch runs twice, each time
    // writing only the ranks of one half of the sample ids, so that the lines
    // of that half fill in the L2 before they are written back: measured at
    // n = 10^6, F = 32, 399 us in one launch, 264 in two halves (the sorted
    // pairs read twice), 314 and 377 in three and four parts.
    const uint64_t row_bytes = (uint64_t)n * 4;
    const uint32_t W = (row_bytes > (2u << 20) && row_bytes <= (8u << 20)) ? 2u : 1u;
    for (uint32_t wi = 0; wi < W; ++wi) {
      const uint32_t lo = (uint32_t)((uint64_t)n * wi / W), hi = (uint32_t)((uint64_t)n * (wi + 1) / W);
      k_seg_rank_scatter<<<xcd_grid(F * nbf), SG_THREADS, 0, st>>>(a, n, F, nbf, ucnt, ld, lo, hi,
                                                                     ranks);
      MH_LAUNCHED(ctx, "k_seg_rank_scatter");
    }
  }
  if (nan_out) return MH_OK;
  uint32_t *h = host_words(ctx);
  if (!h) return MH_ENOMEM;
  MH_HIP(ctx, hipMemcpyAsync(h, words, 8, hipMemcpyDeviceToHost, st));
  MH_HIP(ctx, hipStreamSynchronize(st));
  if ((h[1] & 1u) && done && retry) {
    // the cooperative grid did not run all at once: not again, and the
    // encoding is redone
    coop_note_failure(ctx);
    const bool coop = ctx->rank_coop;
    ctx->rank_coop = false;  // the separate launches redo it
    const mh_status r = launch_rank_encode(ctx, X, n, F, ld, ranks, n_unique, nullptr, false);
    ctx->rank_coop = coop;
    return r;
  }
  if (h[1])
    return fail(ctx, MH_EDEVICE, "rank encoding failed on the device (" +
                                     std::string(h[1] & 1u ? "a grid barrier wait gave up" : "an index out of range") +
                                     ", code " + std::to_string(h[1]) + ")");
  if (h[0]) return fail(ctx, MH_EINVAL, "X holds a NaN");
  return MH_OK;
}

}  // namespace mh
