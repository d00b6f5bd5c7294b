// tiles.hip -- builds the tiled sample layout the fitness kernel reads.
//
// The fitness of a tree only depends on how many samples of each class reach
// each leaf (eq. opt_c), so samples may be regrouped freely.  They are grouped
// by (subproblem, class) and cut into tiles of at most 63.  For every tile and
// feature the 63 ranks are sorted once; the set of tile samples with
// rank < tau is then a prefix of that order, i.e. one of 64 precomputed
// bitmasks, selected by a 6-step binary search.  Every tree of the population
// reuses the same tile, so the sort cost is paid once per dataset (or once
// per moving-horizon level), not once per evaluation.
#include <algorithm>
#include <type_traits>

#include "device_common.h"
#include "internal.h"
#include "xcd.h"

namespace mh {

TileHdr tile_layout(uint32_t n_sub, uint32_t F, uint32_t K, uint32_t n_problems) {
  TileHdr h{};
  h.magic = TILE_MAGIC;
  h.F = F;
  h.K = K;
  h.n_sub = n_sub;
  h.n_tiles = 0;
  h.max_tiles = max_tiles_for(n_sub, n_problems, K);
  h.n_problems = n_problems;
  size_t off = 256;
  h.off_info = off;
  off = align256(off + (size_t)h.max_tiles * 4);
  h.off_ctot = off;
  off = align256(off + (size_t)n_problems * K * 4);
  h.off_data = off;
  off = align256(off + (size_t)h.max_tiles * tile_bytes(F));
  h.off_order = off;
  off = align256(off + (size_t)h.max_tiles * TILE_W * 4);
  h.off_segoff = off;
  off = align256(off + ((size_t)n_problems * K + 1) * 4);
  h.off_cursor = off;
  off = align256(off + (size_t)n_problems * K * 4);
  h.off_perm = off;
  off = align256(off + (size_t)h.max_tiles * F * TILE_W);
  h.total_bytes = off;
  return h;
}

namespace {

// The header travels as a kernel argument (no host buffer outlives the call);
// the per-(subproblem, class) counts that follow start at zero.
__global__ void k_tile_hdr(TileHdr *__restrict__ dst, TileHdr h, uint32_t *__restrict__ ctot,
                           uint32_t nseg) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *dst = h;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nseg; i += gridDim.x * blockDim.x)
    ctot[i] = 0u;
}

// Per-(subproblem, class) sample counts.
// Samples with an index >= n, a label >= K or a subproblem >= n_problems are
// invalid input and are left out (here and in the scatter).
__device__ __forceinline__ bool sample_ok(const uint8_t *__restrict__ labels,
                                          const uint32_t *__restrict__ idx,
                                          const uint32_t *__restrict__ sub_of, uint32_t j,
                                          uint32_t n, uint32_t K, uint32_t n_problems,
                                          uint32_t &i, uint32_t &seg) {
  i = idx ? idx[j] : j;
  if (i >= n) return false;
  const uint32_t y = labels[i];
  const uint32_t s = sub_of ? sub_of[j] : 0u;
  if (y >= K || s >= n_problems) return false;
  seg = s * K + y;
  return true;
}

// Block-aggregated segment counts: LDS histogram when the segments fit,
// then one global atomic per (block, segment).  Block b takes the samples
// [b span, (b + 1) span), span a multiple of its 256 threads: with about two
// blocks per CU the segments' totals take a few hundred global adds each
// rather than one per 256 samples (adds to one address serialise).
constexpr uint32_t LDS_SEGS = 2048;

__global__ __launch_bounds__(256) void k_tile_count(
    const uint8_t *__restrict__ labels, const uint32_t *__restrict__ idx,
    const uint32_t *__restrict__ sub_of, uint32_t n_sub, uint32_t n, uint32_t K,
    uint32_t n_problems, uint32_t span, uint32_t *__restrict__ ctot) {
  __shared__ uint32_t h[LDS_SEGS];
  const uint32_t nseg = n_problems * K;
  const bool local = nseg <= LDS_SEGS;
  if (local)
    for (uint32_t s = threadIdx.x; s < nseg; s += blockDim.x) h[s] = 0;
  __syncthreads();
  const uint32_t j0 = blockIdx.x * span;
  const uint32_t j1 = (uint32_t)min((uint64_t)n_sub, (uint64_t)j0 + span);  // no wrap near 2^32
  for (uint32_t j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
    uint32_t i, seg;
    if (!sample_ok(labels, idx, sub_of, j, n, K, n_problems, i, seg)) continue;
    if (local) atomicAdd(&h[seg], 1u);
    else atomicAdd(&ctot[seg], 1u);
  }
  __syncthreads();
  if (local)
    for (uint32_t s = threadIdx.x; s < nseg; s += blockDim.x)
      if (h[s]) atomicAdd(&ctot[s], h[s]);
}

// Segment plan: tiles per (subproblem, class) segment, their first tile, and
// the info word of every tile.  One block; segments are few (<= 128 * 255).
__global__ void k_tile_plan(TileHdr *__restrict__ hdr, uint32_t nseg) {
  uint8_t *base = reinterpret_cast<uint8_t *>(hdr);
  const uint32_t *ctot = reinterpret_cast<const uint32_t *>(base + hdr->off_ctot);
  uint32_t *segoff = reinterpret_cast<uint32_t *>(base + hdr->off_segoff);
  uint32_t *cursor = reinterpret_cast<uint32_t *>(base + hdr->off_cursor);
  uint32_t *info = reinterpret_cast<uint32_t *>(base + hdr->off_info);
  const uint32_t K = hdr->K;
  __shared__ uint32_t carry;
  __shared__ uint32_t part[1024];
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  // exclusive scan of tiles-per-segment, in chunks of blockDim
  for (uint32_t s0 = 0; s0 < nseg; s0 += blockDim.x) {
    uint32_t s = s0 + threadIdx.x;
    uint32_t v = (s < nseg) ? (ctot[s] + TILE_CAP - 1) / TILE_CAP : 0u;
    part[threadIdx.x] = v;
    __syncthreads();
    for (uint32_t d = 1; d < blockDim.x; d <<= 1) {
      uint32_t t = (threadIdx.x >= d) ? part[threadIdx.x - d] : 0u;
      __syncthreads();
      part[threadIdx.x] += t;
      __syncthreads();
    }
    if (s < nseg) {
      segoff[s] = carry + part[threadIdx.x] - v;
      cursor[s] = 0;
    }
    __syncthreads();
    if (threadIdx.x == blockDim.x - 1) carry += part[threadIdx.x];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    segoff[nseg] = carry;
    hdr->n_tiles = carry;
  }
  (void)info;
  (void)K;
}

// Info word of every tile: thread per tile, its segment found by binary
// search over the segment offsets.
__global__ void k_tile_info(TileHdr *__restrict__ hdr, uint32_t nseg) {
  uint8_t *base = reinterpret_cast<uint8_t *>(hdr);
  const uint32_t *ctot = reinterpret_cast<const uint32_t *>(base + hdr->off_ctot);
  const uint32_t *segoff = reinterpret_cast<const uint32_t *>(base + hdr->off_segoff);
  uint32_t *info = reinterpret_cast<uint32_t *>(base + hdr->off_info);
  const uint32_t K = hdr->K, n_tiles = hdr->n_tiles;
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tiles) return;
  // the last segment s with segoff[s] <= t (empty segments share offsets)
  uint32_t lo = 0, hi = nseg;  // segoff[lo] <= t < segoff[hi]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (segoff[mid] <= t) lo = mid;
    else hi = mid;
  }
  const uint32_t q = t - segoff[lo];
  const uint32_t cnt = min(TILE_CAP, ctot[lo] - q * TILE_CAP);
  info[t] = ((lo / K) << 16) | ((lo % K) << 8) | cnt;
}

// Scatter sample ids into their tile slots.  Block b takes the samples
// [b span, (b + 1) span) (as k_tile_count): it counts them per segment in
// LDS, reserves one range per segment with a single global atomic, and
// fills the ranges from LDS cursors in a second pass over its samples.  The
// order inside a segment is whatever the atomics give; counts do not depend
// on it.
__global__ __launch_bounds__(256) void k_tile_scatter(
    const uint8_t *__restrict__ labels, const uint32_t *__restrict__ idx,
    const uint32_t *__restrict__ sub_of, uint32_t n_sub, uint32_t n, uint32_t span,
    TileHdr *__restrict__ hdr) {
  __shared__ uint32_t h[LDS_SEGS];
  uint8_t *base = reinterpret_cast<uint8_t *>(hdr);
  const uint32_t *segoff = reinterpret_cast<const uint32_t *>(base + hdr->off_segoff);
  uint32_t *cursor = reinterpret_cast<uint32_t *>(base + hdr->off_cursor);
  uint32_t *order = reinterpret_cast<uint32_t *>(base + hdr->off_order);
  const uint32_t K = hdr->K, n_problems = hdr->n_problems, nseg = n_problems * K;
  const bool local = nseg <= LDS_SEGS;
  const uint32_t j0 = blockIdx.x * span;
  const uint32_t j1 = (uint32_t)min((uint64_t)n_sub, (uint64_t)j0 + span);  // no wrap near 2^32
  auto put = [&](uint32_t i, uint32_t s, uint32_t pos) {
    const uint32_t tile = segoff[s] + pos / TILE_CAP;
    order[tile * TILE_W + pos % TILE_CAP] = i;
  };
  if (!local) {
    for (uint32_t j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
      uint32_t i, s;
      if (sample_ok(labels, idx, sub_of, j, n, K, n_problems, i, s)) put(i, s, atomicAdd(&cursor[s], 1u));
    }
    return;
  }
  for (uint32_t s = threadIdx.x; s < nseg; s += blockDim.x) h[s] = 0;
  __syncthreads();
  for (uint32_t j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
    uint32_t i, s;
    if (sample_ok(labels, idx, sub_of, j, n, K, n_problems, i, s)) atomicAdd(&h[s], 1u);
  }
  __syncthreads();
  for (uint32_t q = threadIdx.x; q < nseg; q += blockDim.x)
    if (h[q]) h[q] = atomicAdd(&cursor[q], h[q]);
  __syncthreads();
  for (uint32_t j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
    uint32_t i, s;
    if (sample_ok(labels, idx, sub_of, j, n, K, n_problems, i, s)) put(i, s, atomicAdd(&h[s], 1u));
  }
}

// v of lane ^ J.  J = 1, 2 by a quad permutation, J = 4, 8 by shifts within
// rows of 16 (lane + J where lane & J is zero, else lane - J; the lanes whose
// shift leaves the row are the ones that take the other shift), all DPP moves
// without the LDS pipe; J = 16, 32 by a permute through it.
template <uint32_t J>
__device__ __forceinline__ uint32_t xor_lane32(uint32_t v, uint32_t lane) {
  if constexpr (J == 1) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);
  else if constexpr (J == 2) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);
  else if constexpr (J == 4 || J == 8) {
    const uint32_t up = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x100 + (int)J, 0xF, 0xF, false);
    const uint32_t dn = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x110 + (int)J, 0xF, 0xF, false);
    return (lane & J) ? dn : up;
  } else {
    return (uint32_t)__shfl_xor((int)v, (int)J, 64);
  }
}
template <uint32_t J, typename KT>
__device__ __forceinline__ KT xor_lane(KT v, uint32_t lane) {
  if constexpr (sizeof(KT) == 4) {
    return (KT)xor_lane32<J>((uint32_t)v, lane);
  } else {
    const uint32_t lo = xor_lane32<J>((uint32_t)v, lane);
    const uint32_t hi = xor_lane32<J>((uint32_t)(v >> 32), lane);
    return ((KT)hi << 32) | lo;
  }
}
// One compare-exchange stage of the bitonic network: merge size K, distance J.
template <uint32_t K, uint32_t J, typename KT>
__device__ __forceinline__ KT bitonic_stage(KT v, uint32_t lane) {
  const KT o = xor_lane<J>(v, lane);
  const bool up = (lane & K) == 0, lo = (lane & J) == 0;
  const KT mn = v < o ? v : o, mx = v < o ? o : v;
  return (lo == up) ? mn : mx;
}
// Inclusive OR-scan of a 64-bit value over the wave: within rows of 16 by
// row shifts of 1, 2, 4 and 8 (a lane without a source in the row ORs zero),
// then the row totals across rows (row broadcasts of lanes 15 and 31).
__device__ __forceinline__ uint64_t or_scan64(uint64_t x) {
  uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
  auto step = [&](auto ctrl_tag, auto mask_tag) {
    constexpr int ctrl = decltype(ctrl_tag)::value, rmask = decltype(mask_tag)::value;
    lo |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)lo, ctrl, rmask, 0xF, false);
    hi |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)hi, ctrl, rmask, 0xF, false);
  };
  step(std::integral_constant<int, 0x111>{}, std::integral_constant<int, 0xF>{});  // row_shr:1
  step(std::integral_constant<int, 0x112>{}, std::integral_constant<int, 0xF>{});  // row_shr:2
  step(std::integral_constant<int, 0x114>{}, std::integral_constant<int, 0xF>{});  // row_shr:4
  step(std::integral_constant<int, 0x118>{}, std::integral_constant<int, 0xF>{});  // row_shr:8
  step(std::integral_constant<int, 0x142>{}, std::integral_constant<int, 0xA>{});  // row_bcast:15
  step(std::integral_constant<int, 0x143>{}, std::integral_constant<int, 0xC>{});  // row_bcast:31
  return ((uint64_t)hi << 32) | lo;
}

// One wave per (tile, feature): sort the tile's ranks with their positions
// (bitonic network across the 64 lanes), write the sorted ranks and the
// prefix masks of the positions in sorted order.  The composite key (rank,
// position) is 32 bits wide when every rank is below 2^26 (fewer than 2^26
// samples), else 64.
//
// Block b works on feature f and tiles 4 q .. 4 q + 3 (one per wave), with
// (f, q) = block xcd_order(b) of the feature-major list (xcd.h), so that an
// XCD's random reads of a feature's ranks stay in its own L2.
template <typename KT>
__global__ __launch_bounds__(256) void k_tile_sort(const uint32_t *__restrict__ ranks, uint32_t ld,
                                                   TileHdr *__restrict__ hdr) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t F = hdr->F;
  const uint32_t tq = (hdr->max_tiles + 3u) / 4u;  // tile quads per feature
  const uint32_t bi = xcd_order(blockIdx.x, gridDim.x);
  const uint32_t f = bi / tq, tile = (bi % tq) * 4u + (threadIdx.x >> 6);
  if (f >= F || tile >= hdr->n_tiles) return;
  uint8_t *base = reinterpret_cast<uint8_t *>(hdr);
  const uint32_t info = reinterpret_cast<const uint32_t *>(base + hdr->off_info)[tile];
  const uint32_t *order = reinterpret_cast<const uint32_t *>(base + hdr->off_order);
  const uint32_t cnt = info & 0xFFu;
  // unused lanes sort last: all ones
  constexpr uint32_t KB = sizeof(KT) * 8;
  uint32_t key = (uint32_t)(~KT(0) >> 6);
  if (lane < cnt) key = ranks[(size_t)f * ld + order[tile * TILE_W + lane]];
  // composite (key, position): distinct, so the network sorts a total order
  KT v = ((KT)key << 6) | lane;
  (void)KB;
  // the network: merges of size 2, 4, ..., 64, each halving its distance
  v = bitonic_stage<2, 1>(v, lane);
  v = bitonic_stage<4, 2>(v, lane);
  v = bitonic_stage<4, 1>(v, lane);
  v = bitonic_stage<8, 4>(v, lane);
  v = bitonic_stage<8, 2>(v, lane);
  v = bitonic_stage<8, 1>(v, lane);
  v = bitonic_stage<16, 8>(v, lane);
  v = bitonic_stage<16, 4>(v, lane);
  v = bitonic_stage<16, 2>(v, lane);
  v = bitonic_stage<16, 1>(v, lane);
  v = bitonic_stage<32, 16>(v, lane);
  v = bitonic_stage<32, 8>(v, lane);
  v = bitonic_stage<32, 4>(v, lane);
  v = bitonic_stage<32, 2>(v, lane);
  v = bitonic_stage<32, 1>(v, lane);
  v = bitonic_stage<64, 32>(v, lane);
  v = bitonic_stage<64, 16>(v, lane);
  v = bitonic_stage<64, 8>(v, lane);
  v = bitonic_stage<64, 4>(v, lane);
  v = bitonic_stage<64, 2>(v, lane);
  v = bitonic_stage<64, 1>(v, lane);
  // unused entries: 0x7FFFFFFF, above every rank and threshold (n < 2^31)
  const uint32_t skey = lane < cnt ? (uint32_t)(v >> 6) : 0x7FFFFFFFu;
  const uint32_t pos = (uint32_t)(v & 63u);
  // inclusive OR-scan over lanes: pm[lane + 1]
  const uint64_t bit = or_scan64((lane < cnt) ? (1ull << pos) : 0ull);
  uint8_t *rec = base + hdr->off_data + (size_t)tile * tile_bytes(F);
  uint32_t *sorted = reinterpret_cast<uint32_t *>(rec) + f * TILE_W;
  uint64_t *pm = reinterpret_cast<uint64_t *>(rec + (size_t)F * TILE_W * 4) + f * TILE_W;
  sorted[lane] = skey;
  if (lane < 63u) pm[lane + 1] = bit;
  else pm[0] = 0ull;
  // the compact form: past the count the last sample's position again, so
  // that a running union of (1 << position) stays correct without a test
  const uint32_t last = (uint32_t)__shfl((int)pos, (int)(cnt ? cnt - 1u : 0u), 64);
  base[hdr->off_perm + ((size_t)tile * F + f) * TILE_W + lane] = (uint8_t)(lane < cnt ? pos : last);
}

}  // namespace

mh_status launch_tile_build(Ctx *ctx, const mh_dataset *ds, const uint32_t *idx,
                            const uint32_t *sub_of, uint32_t n_sub, uint32_t n_problems,
                            void *base, size_t bytes) {
  TileHdr h = tile_layout(n_sub, ds->F, ds->K, n_problems);
  if (bytes < h.total_bytes) return fail(ctx, MH_EINVAL, "tile buffer too small");
  if (((uintptr_t)base & 255u) != 0) return fail(ctx, MH_EINVAL, "tile buffer not 256-byte aligned");
  if (n_problems == 0 || n_problems > 65535) return fail(ctx, MH_EINVAL, "bad subproblem count");
  // the search takes v < tau from the sign of v - tau: ranks and thresholds
  // below 2^31
  if (ds->n >= (1u << 31)) return fail(ctx, MH_EINVAL, "tile layout needs fewer than 2^31 samples");
  // the count and scatter loops step their sample index by 256 without wrapping
  if (n_sub > 0xFFFFFF00u) return fail(ctx, MH_EINVAL, "too many (sample, subproblem) pairs");
  hipStream_t st = ctx->stream;
  TileHdr *dh = reinterpret_cast<TileHdr *>(base);
  uint8_t *b = reinterpret_cast<uint8_t *>(base);
  const uint32_t nseg = n_problems * ds->K;
  k_tile_hdr<<<std::min<uint32_t>((nseg + 255) / 256, 256u), 256, 0, st>>>(
      dh, h, reinterpret_cast<uint32_t *>(b + h.off_ctot), nseg);
  MH_LAUNCHED(ctx, "k_tile_hdr");
  // samples per block of the count and scatter: a multiple of 256, about two
  // blocks per CU
  const uint32_t nb_max = 2u * (uint32_t)std::max(1, ctx->num_cu);
  const uint32_t span = (uint32_t)(((((uint64_t)n_sub + nb_max - 1) / nb_max) + 255) / 256 * 256);
  const uint32_t nb = n_sub ? (uint32_t)(((uint64_t)n_sub + span - 1) / span) : 0u;
  if (n_sub > 0) {
    k_tile_count<<<nb, 256, 0, st>>>(ds->labels, idx, sub_of, n_sub, ds->n, ds->K, n_problems, span,
                                     reinterpret_cast<uint32_t *>(b + h.off_ctot));
    MH_LAUNCHED(ctx, "k_tile_count");
  }
  k_tile_plan<<<1, 1024, 0, st>>>(dh, nseg);
  MH_LAUNCHED(ctx, "k_tile_plan");
  k_tile_info<<<(h.max_tiles + 255) / 256, 256, 0, st>>>(dh, nseg);
  MH_LAUNCHED(ctx, "k_tile_info");
  if (n_sub > 0) {
    k_tile_scatter<<<nb, 256, 0, st>>>(ds->labels, idx, sub_of, n_sub, ds->n, span, dh);
    MH_LAUNCHED(ctx, "k_tile_scatter");
    // F blocks per quad of tiles (see k_tile_sort)
    const uint64_t quads = ((uint64_t)h.max_tiles + 3) / 4;
    const uint32_t blocks = xcd_grid((uint32_t)(quads * ds->F));
    if (ds->n < (1u << 26))
      k_tile_sort<uint32_t><<<blocks, 256, 0, st>>>(ds->ranks, ds->ld, dh);
    else
      k_tile_sort<uint64_t><<<blocks, 256, 0, st>>>(ds->ranks, ds->ld, dh);
    MH_LAUNCHED(ctx, "k_tile_sort");
  }
  return MH_OK;
}

}  // namespace mh
