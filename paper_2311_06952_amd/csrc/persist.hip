// persist.hip -- a whole DEOCT run (Algorithm 4) of one problem as a single
// launch whose blocks synchronise through a grid barrier.
//
// Every block evaluates its share of the tiles for all P trees (lane = tree,
// as in the per-generation fitness kernel) and adds its left counts into a
// device counter set.  After a grid barrier, every block reads all counts and
// runs the same epilogue, selection, argmin and mutation for the whole
// population, redundantly: the DE state is a few kilobytes and identical
// arithmetic on identical inputs gives every block the same next population,
// so the counts are the only data that cross blocks.  Thread r of each wave
// group keeps individual r's cost and the trial genes of the group's nodes in
// registers; the post-selection population sits in LDS (the parents of the
// mutation, and individual r's own genes).
//
// Counters rotate over three copies: generation g adds into copy g % 3, all
// blocks read it between barriers g and g + 1, and each block zeroes its share
// of copy (g + 1) % 3 during generation g (that copy was last read before
// barrier g - 1 and is next added into after barrier g).  Cross-block data
// (counts, the barrier words) moves only through device-scope atomics and
// agent-scope loads; each wave waits for its own atomics before arriving at a
// barrier.  A barrier wait gives up after a time limit and raises the error
// flag instead of spinning forever.
//
// The results are those of the per-generation kernels: the same epilogue,
// the same selection and argmin rules, the same random draws and float64
// operations.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cstdio>
#include <type_traits>
#include <vector>

#include "device_common.h"
#include "epilogue.h"
#include "fitness_core.h"
#include "grid_sync.h"
#include "internal.h"

namespace mh {
namespace {

struct PersistArgs {
  const TileHdr *hdr;        // tile set of the problem (one subproblem)
  const uint32_t *n_unique;  // [F]
  double *pop;               // gene-major [m][P]: initial population in, final out
  double *cost;              // [P] out
  uint32_t *best;            // [1] out
  uint32_t *cnt;             // 3 copies of [SB][K][Ppad], zero on entry
  uint32_t *bar;             // barrier arrivals, zero on entry
  uint32_t *err;             // non-zero after a barrier wait gave up
  double M, CR, alpha;
  uint64_t seed, prob;
  uint32_t P, G, n_min, F, K;
  // several problems of one multi-problem tile set (null for one problem):
  // problem of each block, and per problem {first tile, end tile, first
  // block, blocks}; pop, cost, best, cnt and bar hold one area per problem
  const uint16_t *prob_of_block;
  const uint4 *ranges;
  const uint64_t *prob_ids;  // [problems]
  uint32_t bar_stride;       // barrier words per problem
  // > 0: every half keeps its (at most tph) tiles resident in LDS, staged in
  // generation 0 only; 0: tiles are staged every generation
  uint32_t tph;
  // the best tree after the last generation (one problem; null: not wanted):
  // nodes [SB], leaf classes [SL], correct count and cost
  uint8_t *out_feat;
  uint32_t *out_tau;
  uint8_t *out_label;
  uint32_t *out_correct;
  double *out_cost;
  uint64_t wait_ticks;  // barrier time limit, device wall-clock ticks
};

__host__ __device__ __forceinline__ uint32_t align16u(uint32_t x) { return (x + 15u) & ~15u; }

// (cost, index) of the wave's smallest cost, ties to the lower index: DPP
// row shifts (1, 2, 4, 8) reduce each row of 16 lanes into its last lane,
// two row broadcasts fold the four rows into lane 63, which is read back.
// A lane with no source in a step sees the (largest cost, largest index)
// sentinel, which never wins.
__device__ __forceinline__ void wave_argmin(double &c, uint32_t &i) {
  auto step = [&](auto ctrl_tag, auto mask_tag) {
    constexpr int ctrl = decltype(ctrl_tag)::value, rmask = decltype(mask_tag)::value;
    const uint32_t lo = (uint32_t)__double2loint(c), hi = (uint32_t)__double2hiint(c);
    const uint32_t nlo = (uint32_t)__builtin_amdgcn_update_dpp((int)0xFFFFFFFFu, (int)lo, ctrl,
                                                               rmask, 0xF, false);
    const uint32_t nhi = (uint32_t)__builtin_amdgcn_update_dpp((int)0x7FEFFFFFu, (int)hi, ctrl,
                                                               rmask, 0xF, false);
    const uint32_t ni = (uint32_t)__builtin_amdgcn_update_dpp((int)0xFFFFFFFFu, (int)i, ctrl,
                                                              rmask, 0xF, false);
    const double cn = __hiloint2double((int)nhi, (int)nlo);
    const bool better = (cn < c) | ((cn == c) & (ni < i));
    c = better ? cn : c;
    i = better ? ni : i;
  };
  step(std::integral_constant<int, 0x111>{}, std::integral_constant<int, 0xF>{});  // row_shr:1
  step(std::integral_constant<int, 0x112>{}, std::integral_constant<int, 0xF>{});  // row_shr:2
  step(std::integral_constant<int, 0x114>{}, std::integral_constant<int, 0xF>{});  // row_shr:4
  step(std::integral_constant<int, 0x118>{}, std::integral_constant<int, 0xF>{});  // row_shr:8
  step(std::integral_constant<int, 0x142>{}, std::integral_constant<int, 0xA>{});  // row_bcast:15
  step(std::integral_constant<int, 0x143>{}, std::integral_constant<int, 0xC>{});  // row_bcast:31
  const int lo = __builtin_amdgcn_readlane(__double2loint(c), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(c), 63);
  c = __hiloint2double(hi, lo);
  i = (uint32_t)__builtin_amdgcn_readlane((int)i, 63);
}

// LDS after n_unique: argmin scratch (32 costs, 32 indices) and the info
// words of resident tiles (MAX_TPH per group, 4 groups at most).
constexpr uint32_t MAX_TPH = 32;
constexpr uint32_t PERSIST_TAIL = 32 * 8 + 32 * 4 + 4 * MAX_TPH * 4;

// Bytes of one count-merge slot: a group's open class and its counts per
// tree.
__host__ __device__ __forceinline__ uint32_t persist_merge_slot(uint32_t SB, uint32_t P) {
  return align16u(P * 4 + SB * P * 4);
}
// Bytes the exchanges need in the first tile buffer: decoded nodes (feature
// byte and threshold per node and tree), or two count-merge slots (H > 1).
__host__ __device__ __forceinline__ uint32_t persist_exchange_bytes(uint32_t SB, uint32_t P,
                                                                   uint32_t H) {
  const uint32_t nodes = align16u(SB * P) + SB * P * 4;
  const uint32_t counts = (H > 1 ? 2u : 0u) * persist_merge_slot(SB, P);
  return nodes > counts ? nodes : counts;
}
// The first tile buffer, large enough for the exchanges.
__host__ __device__ __forceinline__ uint32_t persist_slot_a(uint32_t F, uint32_t SB, uint32_t P,
                                                           uint32_t H) {
  const uint32_t tile = align16u(mask_region(F) + F * MCOL);
  const uint32_t x = align16u(persist_exchange_bytes(SB, P, H));
  return tile > x ? tile : x;
}
// LDS: first tile buffer (also the exchange area) | H - 1 more tile buffers
// | rows [m][P] f64 | n_unique [F] | argmin scratch.
__host__ __device__ __forceinline__ uint32_t persist_lds_bytes(uint32_t F, uint32_t P, uint32_t SB,
                                                              uint32_t H) {
  const uint32_t tile = align16u(mask_region(F) + F * MCOL);
  return persist_slot_a(F, SB, P, H) + (H - 1) * tile + align16u(2 * SB * P * 8) +
         align16u(F * 4) + PERSIST_TAIL;
}

// Features from which tiles staged every generation come in the compact form.
constexpr uint32_t PERSIST_COMPACT_MIN_F = 16;

// Prefix masks of a tile from its compact form: chunk q of the positions
// holds, for feature f = q / 4, the tile positions of sorted entries
// 16 (q % 4) .. 16 (q % 4) + 15 (past the tile's count the last sample's
// position again, so the running union needs no test).  The four
// chunks of a feature sit on the four lanes of an aligned quad (the chunk
// index and the lane advance together and the chunk ranges start at
// multiples of 4), which exchange their chunks' unions so that each lane
// writes its 16 masks pm[16 (q % 4) + j + 1] = positions of the first
// 16 (q % 4) + j + 1 sorted entries; lane 0 of the quad writes pm[0] = 0.
// All four lanes of a quad call this together.
__device__ __forceinline__ void stage_positions(uint8_t *__restrict__ lds, uint32_t mregion,
                                                uint32_t q, const uint4 &v) {
  const uint32_t f = q >> 2, part = q & 3u;
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
  uint64_t run = 0;
  uint64_t m[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const uint32_t pos = (w[j >> 2] >> (8 * (j & 3))) & 63u;
    run |= 1ull << pos;
    m[j] = run;
  }
  // union of the earlier chunks of the feature (lanes part - 1 .. part - 3)
  const uint64_t u1 = __shfl_up(run, 1, 4), u2 = __shfl_up(run, 2, 4), u3 = __shfl_up(run, 3, 4);
  const uint64_t e = (part >= 1 ? u1 : 0ull) | (part >= 2 ? u2 : 0ull) | (part >= 3 ? u3 : 0ull);
  uint64_t *pm = reinterpret_cast<uint64_t *>(lds + mregion + f * MCOL) + part * 16u;
#pragma unroll
  for (int j = 0; j < 16; ++j) pm[j + 1] = e | m[j];
  if (part == 0) pm[0] = 0ull;
}

// Wave groups (H = 1, 2 or 4): the block holds H copies of the population's
// lanes; group h (threads h * NTH ..) counts every H-th tile of the block's
// range in its own staging buffer, so H tiles are in flight per block, and
// in the DE phase group h makes the genes of its share of the nodes (nodes
// h * NA .. with NA = ceil(SB / H)).  Decoded nodes are exchanged through
// LDS so that every group evaluates whole trees.
// CMP (staged tiles only): the tiles come in the compact form (sorted ranks
// and positions, the masks rebuilt in LDS) rather than as whole records.
template <int D, int WAVES, int H, bool RES, bool CMP = false>
__global__ __launch_bounds__(H * WAVES * 64) void k_deoct_persist(PersistArgs pa) {
  constexpr int SB = (1 << D) - 1, SL = 1 << D, m = 2 * SB;
  constexpr uint32_t NTH = WAVES * 64, NT = H * NTH;
  constexpr int NA = (SB + H - 1) / H;  // nodes per group (the last may have fewer)
  extern __shared__ __align__(16) uint8_t lds[];
  const uint32_t P = pa.P, Ppad = pad64(P), K = pa.K, F = pa.F;
  // wave groups are whole waves, so the group index is wave-uniform
  const uint32_t h = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x / NTH));
  uint32_t r = threadIdx.x % NTH;
  const bool live = r < P;
  const uint32_t rr = live ? r : 0u;
  const int n_lo = (int)h * NA < SB ? (int)h * NA : SB;  // this group's nodes
  const int n_hi = n_lo + NA < SB ? n_lo + NA : SB;

  const uint8_t *base = reinterpret_cast<const uint8_t *>(pa.hdr);
  uint32_t s_prob = 0, b = blockIdx.x, nb = gridDim.x, T0 = 0, T1 = pa.hdr->n_tiles;
  if (pa.prob_of_block) {
    s_prob = pa.prob_of_block[blockIdx.x];
    const uint4 rg = pa.ranges[s_prob];
    // the ranges come from host-side counts; never past the built tiles
    T0 = rg.x < T1 ? rg.x : T1;
    T1 = rg.y < T1 ? rg.y : T1;
    b = blockIdx.x - rg.z;
    nb = rg.w;
  }
  const uint32_t *__restrict__ info = reinterpret_cast<const uint32_t *>(base + pa.hdr->off_info);
  const uint8_t *__restrict__ data = base + pa.hdr->off_data;
  const uint32_t *__restrict__ ctot =
      reinterpret_cast<const uint32_t *>(base + pa.hdr->off_ctot) + (size_t)s_prob * pa.K;
  const size_t rec_bytes = tile_bytes(F);
  const uint32_t nchunk = 48u * F;
  // tiles staged every generation in the compact form: the record's sorted
  // ranks (16 F chunks) and the tile positions in sorted order (4 F chunks),
  // the masks rebuilt in LDS (stage_positions); else the whole record
  const uint8_t *__restrict__ perm = base + pa.hdr->off_perm;
  constexpr bool compact = CMP && !RES;
  const uint32_t nchunk_c = compact ? 20u * F : nchunk;
  const uint32_t t_begin = T0 + (uint32_t)((uint64_t)(T1 - T0) * b / nb);
  const uint32_t t_end = T0 + (uint32_t)((uint64_t)(T1 - T0) * (b + 1) / nb);
  uint32_t rounds = (t_end - t_begin + H - 1) / H;  // tile steps, same for both halves
  if ((RES || pa.tph) && rounds > pa.tph) {
    // more tiles than resident slots: cannot happen with the host's bound;
    // stay inside the LDS and report
    rounds = pa.tph;
    if (threadIdx.x == 0) __hip_atomic_store(pa.err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }

  const uint32_t mregion = mask_region(F);
  const uint32_t tile_lds = align16u(mregion + F * MCOL);
  const uint32_t tph = pa.tph;
  // staged every generation: one buffer per half, the first also the
  // exchange area; resident: the exchange area, then tph slots per half
  const uint32_t slot_a = persist_slot_a(F, SB, P, H);
  const uint32_t x_bytes = align16u(persist_exchange_bytes(SB, P, H));
  const uint32_t tile_off =
      tph ? x_bytes + h * tph * tile_lds : (h == 0 ? 0u : slot_a + (h - 1) * tile_lds);
  const uint32_t rows_off = tph ? x_bytes + H * tph * tile_lds : slot_a + (H - 1) * tile_lds;
  double *rows = reinterpret_cast<double *>(lds + rows_off);
  uint32_t *s_nu = reinterpret_cast<uint32_t *>(lds + rows_off + align16u(m * P * 8));
  double *s_cost = reinterpret_cast<double *>(reinterpret_cast<uint8_t *>(s_nu) + align16u(F * 4));
  uint32_t *s_idx = reinterpret_cast<uint32_t *>(s_cost + 32);
  uint32_t *s_info = s_idx + 32;  // [H][MAX_TPH] info words of resident tiles
  // exchanges at the start of LDS
  uint8_t *x_feat = lds;                                              // [SB][P]
  uint32_t *x_thr = reinterpret_cast<uint32_t *>(lds + align16u(SB * P));  // [SB][P]
  const uint32_t mslot = persist_merge_slot(SB, P);  // count-merge slot i at lds + i * mslot:
                                                     // class [P], then counts [SB][P]
  const uint32_t s0 =
      (uint32_t)(uintptr_t)((__attribute__((address_space(3))) uint8_t *)lds) + tile_off;
  const uint32_t kmask = s0 + mregion - 2u * s0;

  for (uint32_t f = threadIdx.x; f < F; f += NT) s_nu[f] = pa.n_unique[f];
  // The post-selection population lives in LDS (rows, gene-major [m][P]);
  // a thread keeps in registers only the trial genes of its half's nodes:
  // gt[j] and gt[NA + j] are the feature and threshold genes of node
  // n_lo + j.  Each half writes the rows of its own nodes.
  double *pop_s = pa.pop + (size_t)s_prob * P * m;
  double gt[2 * NA];
#pragma unroll
  for (int j = 0; j < NA; ++j) {
    const int t = n_lo + j;
    gt[j] = gt[NA + j] = 0.0;
    if (t < n_hi && live) {
      gt[j] = pop_s[(size_t)t * P + r];
      gt[NA + j] = pop_s[(size_t)(SB + t) * P + r];
      rows[(size_t)t * P + r] = gt[j];
      rows[(size_t)(SB + t) * P + r] = gt[NA + j];
    }
  }
  __syncthreads();

  NodeState<D> ns;
  uint32_t nsplit = 0;
  // decode this half's nodes of `gen`, publish them, then take the whole tree
  // (callers: every thread; contains barriers)
  auto set_tree = [&](const double (&gen)[2 * NA]) {
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int t = n_lo + j;
      if (t < n_hi && live) {
        uint32_t f = 0, th = 0;
        decode_node(gen[j], gen[NA + j], F, s_nu, f, th);
        x_feat[t * P + r] = (uint8_t)f;
        x_thr[t * P + r] = th;
      }
    }
    __syncthreads();
    nsplit = 0;
#pragma unroll
    for (int t = 0; t < SB; ++t) {
      const uint32_t f = live ? x_feat[t * P + r] : 0u;
      const uint32_t th = live ? x_thr[t * P + r] : 0u;
      ns.col[t] = s0 + (f ? f - 1u : 0u) * SCOL;
      ns.thr[t] = f ? th : 0u;
      nsplit += f != 0;
    }
    // staged tiles: the exchange area is a tile buffer again
    if constexpr (!RES) __syncthreads();
  };
  set_tree(gt);

  const size_t cstride = (size_t)SB * K * Ppad;
  const uint64_t key = de_key(pa.seed, pa.prob_ids ? pa.prob_ids[s_prob] : pa.prob);
  uint32_t *cnt3 = pa.cnt + (size_t)s_prob * 3 * cstride;
  uint32_t *bar = pa.bar + (size_t)s_prob * pa.bar_stride;
  double cost_r = 0.0;
  constexpr int NPF = RES ? 1 : PF;
  uint4 pf[NPF];
  auto prefetch = [&](uint32_t tile) {
    const uint4 *__restrict__ src = reinterpret_cast<const uint4 *>(data + (size_t)tile * rec_bytes);
    const uint4 *__restrict__ psrc = reinterpret_cast<const uint4 *>(perm + (size_t)tile * F * TILE_W);
#pragma unroll
    for (int k = 0; k < NPF; ++k) {
      const uint32_t c = r + k * NTH;
      if (c < 16u * F || (!compact && c < nchunk_c)) pf[k] = src[c];
      else if (c < nchunk_c) pf[k] = psrc[c - 16u * F];
    }
  };
  uint32_t inf_next = 0;
  if constexpr (RES) {
    // resident tiles: group h's tiles (t_begin + h, + H, ...) go to its slots
    // once, with their info words
    for (uint32_t i = 0; i < rounds; ++i) {
      const uint32_t tile = t_begin + i * H + h;
      if (tile >= t_end) break;
      uint8_t *dst = lds + tile_off + i * tile_lds;
      const uint4 *__restrict__ src = reinterpret_cast<const uint4 *>(data + (size_t)tile * rec_bytes);
      for (uint32_t c = r; c < nchunk; c += NTH) stage_chunk(dst, mregion, F, c, src[c]);
      if (r == 0) s_info[h * MAX_TPH + i] = info[tile];
    }
    __syncthreads();
  } else if (t_begin + h < t_end) {
    // the next tile's info word travels with its prefetch, so that the loop
    // never waits on it
    prefetch(t_begin + h);
    inf_next = info[t_begin + h];
  }

  // generation G + 1, when the best tree is wanted, counts that tree alone
  const uint32_t g_end = pa.out_label ? pa.G + 1 : pa.G;
  uint32_t bst_fin = 0;
  double cost_fin = 0.0;
  for (uint32_t g = 0; g <= g_end; ++g) {
    // with four groups or deep trees the lane index is re-read each
    // generation, so that the compiler recomputes the addresses derived from
    // it instead of holding them in registers across the whole loop (1024
    // threads leave 128 registers per lane; deep trees spill otherwise)
    if constexpr (H == 4 || D >= 4) asm volatile("" : "+v"(r));
    uint32_t *cnt = cnt3 + (size_t)(g % 3) * cstride;
    {
      uint32_t *z = cnt3 + (size_t)((g + 1) % 3) * cstride;
      for (size_t i = (size_t)b * NT + threadIdx.x; i < cstride; i += (size_t)nb * NT)
        __hip_atomic_store(z + i, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }

    // ---- counts of this block's tiles (half h: tiles t_begin + h, + H, ...)
#pragma unroll
    for (int t = 0; t < SB; ++t) ns.acc[t] = 0;
    uint32_t cur_cls = 0xFFFFFFFFu;
    // (in the pass for the best tree every lane holds that tree; lane 0 adds)
    const bool adds = live && (g <= pa.G || r == 0);
    auto flush = [&]() {
      if (!live || cur_cls == 0xFFFFFFFFu) return;
      uint32_t *c = cnt + (size_t)cur_cls * Ppad + r;
#pragma unroll
      for (int t = 0; t < SB; ++t) {
        if (ns.acc[t] && adds) atomicAdd(c + (size_t)t * K * Ppad, ns.acc[t]);
        ns.acc[t] = 0;
      }
    };
    if constexpr (RES) {
      for (uint32_t i = 0; i < rounds;) {
        const uint32_t tile = t_begin + i * H + h;
        if (tile >= t_end) break;
        const uint32_t inf = s_info[h * MAX_TPH + i];
        const uint32_t cls = (inf >> 8) & 0xFFu;
        if (cls != cur_cls) {
          flush();
          cur_cls = cls;
        }
        uint64_t R[1 << D];
        R[1] = (1ull << (inf & 0xFFu)) - 1ull;  // count <= 63
        // (the pair test is uniform over the group: the tile list is)
        const uint32_t inf2 = i + 1 < rounds && tile + H < t_end ? s_info[h * MAX_TPH + i + 1]
                                                                 : 0xFFFFFFFFu;
        if (D <= 3 && inf2 != 0xFFFFFFFFu && ((inf2 >> 8) & 0xFFu) == cls) {
          // two tiles of the same class at once
          uint64_t R2[1 << D];
          R2[1] = (1ull << (inf2 & 0xFFu)) - 1ull;
          eval_nodes2<D, 1>(kmask, ns, R, R2, i * tile_lds, (i + 1) * tile_lds);
          i += 2;
        } else {
          eval_nodes<D, 1>(kmask, ns, R, i * tile_lds);
          i += 1;
        }
      }
    } else {
      for (uint32_t i = 0; i < rounds; ++i) {
        const uint32_t tile = t_begin + i * H + h;
        const bool act = tile < t_end;
        uint8_t *my_tile = lds + tile_off;
        uint32_t count = 0;
        if (act) {
          const uint32_t inf = inf_next;
          const uint32_t cls = (inf >> 8) & 0xFFu;
          count = inf & 0xFFu;
          if (cls != cur_cls) {
            flush();
            cur_cls = cls;
          }
        }
        __syncthreads();  // the previous tiles are no longer read
        if (act) {
#pragma unroll
          for (int k = 0; k < NPF; ++k) {
            const uint32_t c = r + k * NTH;
            if (c < 16u * F || (!compact && c < nchunk_c)) stage_chunk(my_tile, mregion, F, c, pf[k]);
            else if (c < nchunk_c) stage_positions(my_tile, mregion, c - 16u * F, pf[k]);
          }
          if (nchunk_c > NPF * NTH) {
            const uint4 *__restrict__ src =
                reinterpret_cast<const uint4 *>(data + (size_t)tile * rec_bytes);
            const uint4 *__restrict__ psrc =
                reinterpret_cast<const uint4 *>(perm + (size_t)tile * F * TILE_W);
            for (uint32_t c = r + NPF * NTH; c < nchunk_c; c += NTH) {
              if (c < 16u * F || !compact) stage_chunk(my_tile, mregion, F, c, src[c]);
              else stage_positions(my_tile, mregion, c - 16u * F, psrc[c - 16u * F]);
            }
          }
        }
        __syncthreads();
        if (act) {
          // the next tile, or this group's first tile again for the next
          // generation (the layout does not change)
          const uint32_t nxt = tile + H < t_end ? tile + H : t_begin + h;
          prefetch(nxt);
          inf_next = info[nxt];
          uint64_t R[1 << D];
          R[1] = (1ull << count) - 1ull;  // count <= 63
          eval_nodes<D, 1>(kmask, ns, R, 0u);
        }
      }
    }
    if constexpr (H == 2) {
      // both groups publish their open class and counts; then group h adds
      // both groups' counts of its own nodes and flushes them (each group
      // issues half the atomics).  When the two groups end on different
      // classes each flushes its own counts instead.  (The first barrier also
      // keeps the slots, which overlap the node exchange, from being written
      // while a slower wave still reads the exchanged nodes.)
      __syncthreads();
      if (live) {
        uint8_t *sl = lds + h * mslot;
        reinterpret_cast<uint32_t *>(sl)[r] = cur_cls;
#pragma unroll
        for (int t = 0; t < SB; ++t) reinterpret_cast<uint32_t *>(sl + P * 4)[t * P + r] = ns.acc[t];
      }
      __syncthreads();
      if (live) {
        const uint8_t *so = lds + (1u - h) * mslot;
        const uint32_t co = reinterpret_cast<const uint32_t *>(so)[r];
        const uint32_t *xo = reinterpret_cast<const uint32_t *>(so + P * 4);
        if (co == cur_cls || co == 0xFFFFFFFFu || cur_cls == 0xFFFFFFFFu) {
          const uint32_t cls = cur_cls != 0xFFFFFFFFu ? cur_cls : co;
          if (cls != 0xFFFFFFFFu && adds) {
            uint32_t *c = cnt + (size_t)cls * Ppad + r;
#pragma unroll
            for (int t = 0; t < SB; ++t) {
              if (t < n_lo || t >= n_hi) continue;
              const uint32_t v = ns.acc[t] + xo[t * P + r];
              if (v) atomicAdd(c + (size_t)t * K * Ppad, v);
            }
          }
        } else {
          flush();
        }
      }
#pragma unroll
      for (int t = 0; t < SB; ++t) ns.acc[t] = 0;
      cur_cls = 0xFFFFFFFFu;
    } else if constexpr (H > 2) {
      // merge the groups' open counts pairwise (group h + w into group h for
      // w = H / 2, .., 1), adding them when both end on the same class (the
      // usual case: tiles are grouped by class) and flushing otherwise
#pragma unroll
      for (uint32_t w = H / 2; w >= 1; w /= 2) {
        __syncthreads();
        if (h >= w && h < 2 * w && live) {
          uint8_t *sl = lds + (h - w) * mslot;
          reinterpret_cast<uint32_t *>(sl)[r] = cur_cls;
#pragma unroll
          for (int t = 0; t < SB; ++t) reinterpret_cast<uint32_t *>(sl + P * 4)[t * P + r] = ns.acc[t];
        }
        __syncthreads();
        if (h < w && live) {
          const uint8_t *sl = lds + h * mslot;
          const uint32_t c1 = reinterpret_cast<const uint32_t *>(sl)[r];
          const uint32_t *xa = reinterpret_cast<const uint32_t *>(sl + P * 4);
          if (c1 == cur_cls || cur_cls == 0xFFFFFFFFu) {
            if (c1 != 0xFFFFFFFFu) cur_cls = c1;
#pragma unroll
            for (int t = 0; t < SB; ++t) ns.acc[t] += xa[t * P + r];
          } else if (c1 != 0xFFFFFFFFu) {
            flush();
            cur_cls = c1;
#pragma unroll
            for (int t = 0; t < SB; ++t) ns.acc[t] = xa[t * P + r];
          }
        }
        if (h >= w && h < 2 * w) {
#pragma unroll
          for (int t = 0; t < SB; ++t) ns.acc[t] = 0;
          cur_cls = 0xFFFFFFFFu;
        }
      }
    }
    flush();
    barrier_arrive(bar, g, b, nb);

    // ---- the random draws of generation g + 1 (they depend only on the
    // seed, the generation, the individual and the slot), made while the
    // other blocks finish: M_r, r1, r2, q_rand, and one crossover decision
    // per gene of this half's nodes
    const uint32_t gg = g + 1;
    double Mr = pa.M;
    uint32_t r1 = 0, r2 = 0, qr = 0;
    uint64_t cross = 0;
    if (live && g < pa.G) {
      // draw (gg, r, slot) is SplitMix64 output (base counter + slot)
      const uint64_t cbase =
          key + ((((uint64_t)gg << 40) | ((uint64_t)r << 20)) + 1ull) * 0x9E3779B97F4A7C15ull;
      auto draw = [&](uint32_t slot) {
        return sm64_fmix(cbase + (uint64_t)slot * 0x9E3779B97F4A7C15ull);
      };
      if (pa.M < 0.0) Mr = to_unit(draw(0));
      r1 = to_below(draw(1), P - 1u);
      r1 += (r1 >= r) ? 1u : 0u;
      r2 = to_below(draw(2), P - 2u);
      const uint32_t lo = r < r1 ? r : r1, hi = r < r1 ? r1 : r;
      r2 += (r2 >= lo) ? 1u : 0u;
      r2 += (r2 >= hi) ? 1u : 0u;
      qr = to_below(draw(3), m);
#pragma unroll
      for (int t = 0; t < SB; ++t) {
        if (t < n_lo || t >= n_hi) continue;
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
          const int q = t + (hh ? SB : 0);
          const double u = to_unit(draw(4u + q));
          if (u <= pa.CR || (uint32_t)q == qr) cross |= 1ull << q;
        }
      }
    }
    barrier_wait(bar, g, pa.err, pa.wait_ticks);

    if (g > pa.G) {
      // ---- the best tree's nodes, leaf classes (the largest count, ties to
      // the lower class, an empty leaf class 0), correct count and cost
      if (b == 0 && threadIdx.x == 0) {
        uint32_t nl[SL], bv[SL], bk[SL];
#pragma unroll
        for (int l = 0; l < SL; ++l) nl[l] = bv[l] = bk[l] = 0;
        for (uint32_t k = 0; k < K; ++k) {
          uint32_t reach[2 * SL];
          reach[1] = ctot[k];
#pragma unroll
          for (int t = 1; t <= SB; ++t) {
            const uint32_t left = cnt_load<true>(cnt + ((size_t)(t - 1) * K + k) * Ppad);
            reach[2 * t] = left;
            reach[2 * t + 1] = reach[t] - left;
          }
#pragma unroll
          for (int l = 0; l < SL; ++l) {
            const uint32_t v = reach[SL + l];
            nl[l] += v;
            if (v > bv[l]) {
              bv[l] = v;
              bk[l] = k;
            }
          }
        }
        uint32_t correct = 0;
#pragma unroll
        for (int l = 0; l < SL; ++l) {
          correct += bv[l];
          pa.out_label[l] = (uint8_t)bk[l];
        }
#pragma unroll
        for (int t = 0; t < SB; ++t) {
          uint32_t f = 0, th = 0;
          decode_node(rows[(size_t)t * P + bst_fin], rows[(size_t)(SB + t) * P + bst_fin], F,
                      s_nu, f, th);
          pa.out_feat[t] = (uint8_t)f;
          pa.out_tau[t] = th;
        }
        *pa.out_correct = correct;
        *pa.out_cost = cost_fin;
      }
      break;
    }

    // ---- epilogue (eq. opt_all and the soft-constraint fitness); the counts
    // of up to KB classes are loaded together
    constexpr uint32_t KB = SB <= 7 ? 4u : (SB <= 15 ? 2u : 1u);
    uint32_t nl[SL], bl[SL], n_sub = 0;
#pragma unroll
    for (int l = 0; l < SL; ++l) nl[l] = bl[l] = 0;
    for (uint32_t k0 = 0; k0 < K; k0 += KB) {
      uint32_t left[KB][SB], tot[KB];
#pragma unroll
      for (uint32_t kk = 0; kk < KB; ++kk) {
        const uint32_t k = k0 + kk < K ? k0 + kk : K - 1u;
        tot[kk] = ctot[k];
#pragma unroll
        for (int t = 0; t < SB; ++t)
          left[kk][t] = cnt_load<true>(cnt + ((size_t)t * K + k) * Ppad + rr);
      }
#pragma unroll
      for (uint32_t kk = 0; kk < KB; ++kk) {
        if (k0 + kk >= K) continue;
        uint32_t reach[2 * SL];
        reach[1] = tot[kk];
        n_sub += reach[1];
#pragma unroll
        for (int t = 1; t <= SB; ++t) {
          reach[2 * t] = left[kk][t - 1];
          reach[2 * t + 1] = reach[t] - left[kk][t - 1];
        }
#pragma unroll
        for (int l = 0; l < SL; ++l) {
          const uint32_t v = reach[SL + l];
          nl[l] += v;
          bl[l] = v > bl[l] ? v : bl[l];
        }
      }
    }
    uint32_t correct = 0, nviol = 0;
#pragma unroll
    for (int l = 0; l < SL; ++l) {
      correct += bl[l];
      nviol += (nl[l] > 0 && nl[l] < pa.n_min) ? 1u : 0u;
    }
    double tc = (double)(n_sub - correct);
    tc = __dadd_rn(tc, __dmul_rn(pa.alpha, (double)nsplit));
    tc = __dadd_rn(tc, (double)nviol);

    // ---- selection (eq. selection; the trial wins ties), or the initial cost
    if (g == 0) {
      cost_r = tc;
    } else if (tc <= cost_r) {
      cost_r = tc;
      if (live) {
#pragma unroll
        for (int j = 0; j < NA; ++j) {
          const int t = n_lo + j;
          if (t < n_hi) {
            rows[(size_t)t * P + r] = gt[j];
            rows[(size_t)(SB + t) * P + r] = gt[NA + j];
          }
        }
      }
    }

    // ---- best: lowest index of the minimum cost (both halves hold every
    // individual's cost; duplicates do not change the result)
    double bc = live ? cost_r : DBL_MAX;
    uint32_t bi = r;
    // (every group holds the same costs: the first group's waves reduce them)
    if (h == 0) {
      wave_argmin(bc, bi);
      if ((threadIdx.x & 63u) == 0) {
        s_cost[threadIdx.x >> 6] = bc;
        s_idx[threadIdx.x >> 6] = bi;
      }
    }
    __syncthreads();
    bc = s_cost[0];
    bi = s_idx[0];
#pragma unroll
    for (uint32_t x = 1; x < NTH / 64; ++x) {
      const double c2 = s_cost[x];
      const uint32_t i2 = s_idx[x];
      const bool better = (c2 < bc) | ((c2 == bc) & (i2 < bi));
      bc = better ? c2 : bc;
      bi = better ? i2 : bi;
    }
    const uint32_t bst = bi;
    if (g == pa.G) {
      if (b == 0 && live) {
#pragma unroll
        for (int j = 0; j < NA; ++j) {
          const int t = n_lo + j;
          if (t < n_hi) {
            pop_s[(size_t)t * P + r] = rows[(size_t)t * P + r];
            pop_s[(size_t)(SB + t) * P + r] = rows[(size_t)(SB + t) * P + r];
          }
        }
        if (h == 0) pa.cost[(size_t)s_prob * P + r] = cost_r;
      }
      if (b == 0 && threadIdx.x == 0) pa.best[s_prob] = bst;
      if (!pa.out_label) break;
      // one more pass counts the best tree alone (every lane holds it)
      bst_fin = bst;
      cost_fin = bc;
#pragma unroll
      for (int j = 0; j < NA; ++j) {
        const int t = n_lo + j;
        gt[j] = gt[NA + j] = 0.0;
        if (t < n_hi) {
          gt[j] = rows[(size_t)t * P + bst];
          gt[NA + j] = rows[(size_t)(SB + t) * P + bst];
        }
      }
      set_tree(gt);
      continue;
    }

    // ---- DE/best/1 mutation and binomial crossover of generation g + 1,
    // this half's nodes (the feature gene t and the threshold gene SB + t)
    if (live) {
      const double Fp1 = (double)F + 1.0;
#pragma unroll
      for (int j = 0; j < NA; ++j) {
        const int t = n_lo + j;
        if (t >= n_hi) continue;
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
          const int q = t + (hh ? SB : 0), jj = j + (hh ? NA : 0);
          const double a1 = rows[(size_t)q * P + r1];
          const double a2 = rows[(size_t)q * P + r2];
          const double a0 = rows[(size_t)q * P + r];
          const double d = __dsub_rn(a1, a2);
          double v = __dadd_rn(rows[(size_t)q * P + bst], __dmul_rn(Mr, d));
          const double hiq = hh ? 1.0 : Fp1;
          if (!(v >= 0.0)) v = 0.0;
          if (v > hiq) v = hiq;
          gt[jj] = ((cross >> q) & 1ull) ? v : a0;
        }
      }
    }
    set_tree(gt);
  }
}

// Blocks per CU: the per-generation exchange (count atomics, barrier, count
// reads) grows with the block count, the tile work shrinks with it.  Measured
// at depth 3 (F = 16, P = 128 and 256, n = 5e4 .. 4e6): about 4 waves per CU
// while a CU has up to 8 tiles, then 4 more waves per further 8 tiles, up to
// 16 waves.
uint32_t persist_bpc(uint32_t max_tiles, uint32_t num_cu, uint32_t waves) {
  const uint32_t per_cu = (max_tiles + num_cu - 1) / num_cu;
  uint32_t target = 4u * ((per_cu + 7u) / 8u);
  target = target < 4u ? 4u : (target > 16u ? 16u : target);
  const uint32_t bpc = target / waves;
  return bpc ? bpc : 1u;
}

// Problems of a multi-problem launch: tiles per problem (host) and the
// device buffers for the block map and the per-problem ranges.
struct Groups {
  const std::vector<uint32_t> *tiles;  // null: one problem
  uint16_t *prob_of_block;
  uint4 *ranges;
};

// Four wave groups exist only with resident tiles (staging every generation
// needs registers that four groups per block do not have).
template <int D, int WAVES, int H>
mh_status launch_w(Ctx *ctx, const PersistArgs &pa, uint32_t lds, uint32_t max_tiles,
                   const Groups &gr, bool *used) {
  const void *kres = reinterpret_cast<const void *>(k_deoct_persist<D, WAVES, H, true>);
  // staged tiles: the compact form trades bytes for the work of rebuilding
  // the masks, which pays from PERSIST_COMPACT_MIN_F features on (measured:
  // F = 20, n = 10^6, a level's launch 6.0 -> 4.9 ms; F = 8, n = 10^7, the
  // launches of a moving-horizon run 186 -> 237 ms)
  const void *kstage = nullptr;
  if constexpr (H < 4)
    kstage = pa.F >= PERSIST_COMPACT_MIN_F
                 ? reinterpret_cast<const void *>(k_deoct_persist<D, WAVES, H, false, true>)
                 : reinterpret_cast<const void *>(k_deoct_persist<D, WAVES, H, false, false>);
  const void *kern = kstage ? kstage : kres;
  const int per_cu = coop_per_cu(ctx, kern, H * WAVES * 64, lds);
  if (per_cu < 1)
    return MH_OK;  // not co-resident: the caller tries fewer groups, then the
                   // per-generation kernels
  const uint32_t want = persist_bpc(max_tiles, (uint32_t)ctx->num_cu, H * WAVES);
  // with many tiles per CU the tile work dominates, and the per-generation
  // kernels win where they keep more waves per CU busy than the whole-run
  // kernel can (measured at n = 1e6, P = 512, depth 4: one 8-wave block per
  // CU against two, 355 against 281 us per generation; at P = 128 and 256
  // the whole-run kernel wins or ties)
  {
    uint32_t fw = pad64(pa.P) / 64;
    fw = fw > 4 ? 8 : (fw > 2 ? 4 : fw);
    const uint32_t have = (want < (uint32_t)per_cu ? want : (uint32_t)per_cu) * H * WAVES;
    if (!ctx->persist_blocks_per_cu && max_tiles > 16u * (uint32_t)ctx->num_cu &&
        ctx->fit_blocks_per_cu * fw > have)
      return MH_OK;
  }
  uint32_t bpc = ctx->persist_blocks_per_cu ? ctx->persist_blocks_per_cu : want;
  bpc = bpc < (uint32_t)per_cu ? bpc : (uint32_t)per_cu;
  // at most four blocks per CU: a cooperative grid of about six blocks per CU
  // (of another kernel) was accepted by the launch but did not become
  // resident all at once
  bpc = bpc > 4u ? 4u : bpc;
  uint32_t grid = (uint32_t)ctx->num_cu * (bpc ? bpc : 1u);
  PersistArgs a = pa;
  a.tph = 0;
  uint32_t per_block = (max_tiles + grid - 1) / grid;  // tiles of one block, at most
  if (gr.tiles) {
    // blocks in proportion to each problem's tiles, at least one each
    const std::vector<uint32_t> &tl = *gr.tiles;
    const uint32_t np = (uint32_t)tl.size();
    uint64_t total = 0;
    for (uint32_t t : tl) total += t;
    std::vector<uint4> rg(np);
    std::vector<uint16_t> pob;
    uint32_t t0 = 0;
    for (uint32_t i = 0; i < np; ++i) {
      uint64_t nbk = total ? (uint64_t)grid * tl[i] / total : 1;
      nbk = nbk < 1 ? 1 : nbk;
      nbk = tl[i] && nbk > tl[i] ? tl[i] : nbk;
      rg[i] = make_uint4(t0, t0 + tl[i], (uint32_t)pob.size(), (uint32_t)nbk);
      pob.insert(pob.end(), (size_t)nbk, (uint16_t)i);
      t0 += tl[i];
    }
    if (pob.size() > (size_t)per_cu * (size_t)ctx->num_cu || pob.size() > (size_t)ctx->num_cu * 8u)
      return MH_OK;  // more blocks than can be co-resident
    grid = (uint32_t)pob.size();
    per_block = 0;
    for (uint32_t i = 0; i < np; ++i) {
      const uint32_t pb = (tl[i] + rg[i].w - 1) / rg[i].w;
      per_block = pb > per_block ? pb : per_block;
    }
    MH_HIP(ctx, hipMemcpyAsync(gr.ranges, rg.data(), np * sizeof(uint4), hipMemcpyHostToDevice,
                               ctx->stream));
    MH_HIP(ctx, hipMemcpyAsync(gr.prob_of_block, pob.data(), pob.size() * 2,
                               hipMemcpyHostToDevice, ctx->stream));
    MH_HIP(ctx, hipStreamSynchronize(ctx->stream));  // the host vectors go out of scope
    a.prob_of_block = gr.prob_of_block;
    a.ranges = gr.ranges;
  }
  // resident tiles when every block's tiles fit the LDS next to the DE rows
  uint32_t lds_use = lds;
  if (ctx->persist_resident) {
    const uint32_t SB = (1u << D) - 1u;
    const uint32_t tph = (per_block + H - 1) / H;
    const uint32_t tile = align16u(mask_region(pa.F) + pa.F * MCOL);
    const uint64_t need = (uint64_t)align16u(persist_exchange_bytes(SB, pa.P, H)) +
                          (uint64_t)H * tph * tile + align16u(2 * SB * pa.P * 8) +
                          align16u(pa.F * 4) + PERSIST_TAIL;
    if (tph >= 1 && tph <= MAX_TPH && need <= ctx->max_lds &&
        (uint64_t)coop_per_cu(ctx, kres, H * WAVES * 64, (size_t)need) * ctx->num_cu >= grid) {
      a.tph = tph;
      lds_use = (uint32_t)need;
      kern = kres;
    }
  }
  if (!a.tph && !kstage) return MH_OK;  // four groups need resident tiles
  if (!a.tph) kern = kstage;
  if (coop_is_bad(ctx, kern, grid)) return MH_OK;
  if (ctx->debug)
    std::fprintf(stderr,
                 "k_deoct_persist<%d,%d,%d,%s>: grid %u (per CU %d by occupancy), tiles %u "
                 "(per block %u), LDS %u bytes\n",
                 D, WAVES, H, a.tph ? "true" : "false", grid, per_cu, max_tiles, per_block,
                 lds_use);
  void *args[] = {&a};
  hipError_t e = launch_grid_sync(ctx, kern, dim3(grid), dim3(H * WAVES * 64), args, lds_use);
  if (e == hipErrorInvalidValue || e == hipErrorCooperativeLaunchTooLarge ||
      e == hipErrorInvalidConfiguration) {
    // a shape the launch refuses (LDS, block count): the per-generation
    // kernels take the run
    (void)hipGetLastError();
    return MH_OK;
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "k_deoct_persist");
  ctx->last_coop_kern = kern;
  ctx->last_coop_grid = grid;
  *used = true;
  return MH_OK;
}

template <int D, int H>
mh_status launch_d(Ctx *ctx, uint32_t waves, const PersistArgs &pa, uint32_t lds,
                   uint32_t max_tiles, const Groups &gr, bool *used) {
  switch (waves) {
    case 1: return launch_w<D, 1, H>(ctx, pa, lds, max_tiles, gr, used);
    case 2: return launch_w<D, 2, H>(ctx, pa, lds, max_tiles, gr, used);
    case 4: return launch_w<D, 4, H>(ctx, pa, lds, max_tiles, gr, used);
    default: return launch_w<D, (H == 1 ? 8 : 4), H>(ctx, pa, lds, max_tiles, gr, used);
  }
}

template <int D>
mh_status launch_dh(Ctx *ctx, uint32_t waves, uint32_t H, const PersistArgs &pa, uint32_t lds,
                    uint32_t max_tiles, const Groups &gr, bool *used) {
  if (H == 4) return launch_d<D, 4>(ctx, waves, pa, lds, max_tiles, gr, used);
  if (H == 2) return launch_d<D, 2>(ctx, waves, pa, lds, max_tiles, gr, used);
  return launch_d<D, 1>(ctx, waves, pa, lds, max_tiles, gr, used);
}

// One problem (ptiles == null) or the problems of a multi-problem tile set.
mh_status persist_run(Ctx *ctx, const void *tiles, uint32_t F, uint32_t K, uint32_t n_sub,
                      uint64_t n_eval, uint32_t n_problems, uint32_t D, const mh_de_params *prm,
                      uint64_t prob,
                      const uint64_t *prob_ids, const std::vector<uint32_t> *ptiles,
                      const uint32_t *n_unique, double *pop, double *cost, uint32_t *best,
                      uint32_t *err, const PersistFinal *fin, bool *used) {
  *used = false;
  const uint32_t P = prm->P, SB = (1u << D) - 1u, m = 2 * SB;
  if (!ctx->coop || D < 1 || D > 5 || P > 512 || F > 80 || n_problems == 0 ||
      n_problems > 65535)
    return MH_OK;
  // barrier targets (G + 2) * blocks must fit the 32-bit arrival counters
  if ((uint64_t)(prm->G + 2) * (uint64_t)ctx->num_cu * 8u >= (1ull << 31)) return MH_OK;
  uint32_t waves = pad64(P) / 64;
  waves = waves > 4 ? 8 : (waves > 2 ? 4 : waves);
  // up to persist_halves tile streams per block, as the LDS and the
  // 1024-thread limit allow
  const uint32_t max_lds = ctx->max_lds;
  uint32_t H = 1;
  for (uint32_t hh = 2; hh <= 4; hh *= 2)
    if (ctx->persist_halves >= hh && waves <= 4 && persist_lds_bytes(F, P, SB, hh) <= max_lds)
      H = hh;
  if (persist_lds_bytes(F, P, SB, H) > max_lds) return MH_OK;
  (void)m;
  const size_t cstride = (size_t)SB * K * pad64(P);
  const uint32_t bar_words = barrier_words((uint32_t)ctx->num_cu * 8u);
  uint32_t *cnt = (uint32_t *)arena_get(ctx, "ps_cnt", (size_t)n_problems * 3 * cstride * 4);
  uint32_t *bar = (uint32_t *)arena_get(ctx, "ps_bar", (size_t)n_problems * bar_words * 4);
  if (!cnt || !bar) return MH_ENOMEM;
  Groups gr{ptiles, nullptr, nullptr};
  if (ptiles) {
    gr.prob_of_block = (uint16_t *)arena_get(ctx, "ps_pob", (size_t)ctx->num_cu * 8u * 2);
    gr.ranges = (uint4 *)arena_get(ctx, "ps_ranges", (size_t)n_problems * sizeof(uint4));
    if (!gr.prob_of_block || !gr.ranges) return MH_ENOMEM;
  }
  hipStream_t st = ctx->stream;
  mh_status zs = launch_zero(ctx, {{cnt, (size_t)n_problems * 3 * cstride * 4},
                                   {bar, (size_t)n_problems * bar_words * 4},
                                   {err, 4}});
  if (zs) return zs;
  PersistArgs pa;
  pa.hdr = reinterpret_cast<const TileHdr *>(tiles);
  pa.n_unique = n_unique;
  pa.pop = pop;
  pa.cost = cost;
  pa.best = best;
  pa.cnt = cnt;
  pa.bar = bar;
  pa.err = err;
  pa.M = prm->M;
  pa.CR = prm->CR;
  pa.alpha = prm->alpha;
  pa.seed = prm->seed;
  pa.prob = prob;
  pa.P = P;
  pa.G = prm->G;
  pa.n_min = prm->n_min;
  pa.F = F;
  pa.K = K;
  pa.prob_of_block = nullptr;
  pa.ranges = nullptr;
  pa.prob_ids = prob_ids;
  pa.bar_stride = bar_words;
  pa.tph = 0;
  pa.out_feat = fin ? fin->feat : nullptr;
  pa.out_tau = fin ? fin->tau : nullptr;
  pa.out_label = fin ? fin->label : nullptr;
  pa.out_correct = fin ? fin->correct : nullptr;
  pa.out_cost = fin ? fin->cost : nullptr;
  pa.wait_ticks = ctx->wait_ticks;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const bool timed = prof_pair(ctx, &e0, &e1);
  if (timed) MH_HIP(ctx, hipEventRecord(e0, st));
  mh_status s = MH_OK;
  const uint32_t max_tiles = tile_layout(n_sub, F, K, n_problems).max_tiles;
  // the most wave groups that launch, down to one
  for (uint32_t hh = H; hh >= 1 && !*used; hh /= 2) {
    const uint32_t lds_h = persist_lds_bytes(F, P, SB, hh);
    switch (D) {
      case 1: s = launch_dh<1>(ctx, waves, hh, pa, lds_h, max_tiles, gr, used); break;
      case 2: s = launch_dh<2>(ctx, waves, hh, pa, lds_h, max_tiles, gr, used); break;
      case 3: s = launch_dh<3>(ctx, waves, hh, pa, lds_h, max_tiles, gr, used); break;
      case 4: s = launch_dh<4>(ctx, waves, hh, pa, lds_h, max_tiles, gr, used); break;
      default: s = launch_dh<5>(ctx, waves, hh, pa, lds_h, max_tiles, gr, used); break;
    }
    if (s) return s;
  }
  if (timed) {
    MH_HIP(ctx, hipEventRecord(e1, st));
    if (*used) ctx->prof_launches += 1;
  }
  if (*used) ctx->prof_evals += (uint64_t)(prm->G + 1) * n_eval * P;
  return MH_OK;
}

}  // namespace

mh_status launch_deoct_persist(Ctx *ctx, const void *tiles, uint32_t F, uint32_t K,
                               uint32_t n_sub, uint32_t D, const mh_de_params *prm, uint64_t prob,
                               const uint32_t *n_unique, double *pop, double *cost,
                               uint32_t *best, uint32_t *err, const PersistFinal *fin,
                               bool *used) {
  return persist_run(ctx, tiles, F, K, n_sub, n_sub, 1, D, prm, prob, nullptr, nullptr, n_unique,
                     pop, cost, best, err, fin, used);
}

mh_status launch_deoct_persist_multi(Ctx *ctx, const void *tiles, uint32_t F, uint32_t K,
                                     uint32_t n_sub, uint32_t n_problems,
                                     const uint32_t *class_counts, uint32_t D,
                                     const mh_de_params *prm, const uint64_t *prob_ids,
                                     const uint32_t *n_unique, double *pop, double *cost,
                                     uint32_t *best, uint32_t *err, bool *used) {
  // tiles per problem, in the layout's order (problem-major, then class)
  std::vector<uint32_t> tl(n_problems, 0);
  uint64_t n_eval = 0;
  for (uint32_t i = 0; i < n_problems; ++i)
    for (uint32_t k = 0; k < K; ++k) {
      tl[i] += (class_counts[(size_t)i * K + k] + TILE_CAP - 1) / TILE_CAP;
      n_eval += class_counts[(size_t)i * K + k];
    }
  return persist_run(ctx, tiles, F, K, n_sub, n_eval, n_problems, D, prm, 0, prob_ids, &tl,
                     n_unique, pop, cost, best, err, nullptr, used);
}

}  // namespace mh
