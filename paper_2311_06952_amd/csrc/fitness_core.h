// fitness_core.h -- device helpers of the tiled fitness evaluation (Algorithm 1
// in bitmask form): the LDS layout of a staged tile, the per-lane node state,
// the interleaved binary searches and the reach-mask update.  Shared by the
// per-generation fitness kernels and the persistent DEOCT kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mh {
namespace {

// LDS layout of one staged tile: sorted ranks [F][65] u32 (one pad word per
// column spreads columns over banks), then prefix masks [F][65] u64.
constexpr uint32_t SCOL = 65 * 4;
constexpr uint32_t MCOL = 65 * 8;
static_assert(MCOL == 2 * SCOL, "mask column offset is twice the rank column offset");
// Byte offset of the mask region (8-byte aligned for ds_read_b64).
__host__ __device__ __forceinline__ uint32_t mask_region(uint32_t F) {
  return (F * SCOL + 15u) & ~15u;
}

template <int D>
struct NodeState {
  static constexpr int SB = (1 << D) - 1;
  uint32_t col[SB];   // LDS address of the node feature's sorted column
  uint32_t thr[SB];   // tau
  uint32_t acc[SB];   // left counts since the last flush
};

// Nodes are evaluated in heap (BFS) order, in groups of up to ILP nodes: the
// binary searches of a group are independent and run interleaved (6 rounds of
// ILP independent LDS reads), then the group's masks update the reach masks
// R (R_2t = R_t & pm, R_2t+1 = R_t & ~pm) and the left counts.
constexpr int ILP = 16;

// LDS reads go through an address-space-3 pointer with base 0 and absolute
// byte addresses (the kernel's dynamic LDS base is folded into the column
// offsets once), so that each search step is one read, compare and select.
typedef __attribute__((address_space(3))) const uint32_t lds_u32_t;
typedef __attribute__((address_space(3))) const uint64_t lds_u64_t;

__device__ __forceinline__ uint32_t lds_rd32(uint32_t addr) {
  return *reinterpret_cast<lds_u32_t *>(static_cast<uintptr_t>(addr));
}
__device__ __forceinline__ uint64_t lds_rd64(uint32_t addr) {
  return *reinterpret_cast<lds_u64_t *>(static_cast<uintptr_t>(addr));
}

// One search step: a + (v < t ? 4 s : 0) for ranks and thresholds below
// 2^31 (the tile layout's unused entries are 0x7FFFFFFF), where the sign of
// v - t is v < t.  The shift and add are the one instruction they are
// written as, so that the compiler neither turns the sign test back into a
// compare and select through VCC (whose hazard costs a wait state per step)
// nor splits it into shift, mask and add.
__device__ __forceinline__ uint32_t step_if_less(uint32_t a, uint32_t v, uint32_t t, int s) {
  const uint32_t bit = (v - t) >> 31;
  const uint32_t sh = (uint32_t)__builtin_ctz((unsigned)s) + 2u;  // log2(4 s)
  uint32_t r;
  asm("v_lshl_add_u32 %0, %1, %2, %3" : "=v"(r) : "v"(bit), "s"(sh), "v"(a));
  return r;
}

// delta: byte offset of the staged tile from the one the node columns were
// set up for (kmask is that tile's), so that one node state serves several
// staged tiles.
template <int D, int T0, int T1>
__device__ __forceinline__ void eval_group(uint32_t kmask, NodeState<D> &ns,
                                           uint64_t (&R)[1 << D], uint32_t delta) {
  constexpr int NG = T1 - T0;
  uint32_t a[NG];
#pragma unroll
  for (int i = 0; i < NG; ++i) a[i] = ns.col[T0 - 1 + i] + delta;
  kmask -= delta;
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) {
    uint32_t v[NG];
#pragma unroll
    for (int i = 0; i < NG; ++i) v[i] = lds_rd32(a[i] + (s - 1) * 4);
#pragma unroll
    for (int i = 0; i < NG; ++i) a[i] = step_if_less(a[i], v[i], ns.thr[T0 - 1 + i], s);
  }
  uint64_t m[NG];
#pragma unroll
  for (int i = 0; i < NG; ++i) m[i] = lds_rd64(kmask + 2 * a[i]);
#pragma unroll
  for (int i = 0; i < NG; ++i) {
    constexpr int SL = 1 << D;
    const int t = T0 + i;
    const uint64_t A = R[t] & m[i];
    ns.acc[t - 1] += (uint32_t)__popcll(A);
    if (2 * t < SL) {
      R[2 * t + 1] = R[t] & ~m[i];
      R[2 * t] = A;
    }
  }
}

template <int D, int T0>
__device__ __forceinline__ void eval_nodes(uint32_t kmask, NodeState<D> &ns,
                                           uint64_t (&R)[1 << D], uint32_t delta = 0) {
  constexpr int SB = (1 << D) - 1;
  if constexpr (T0 <= SB) {
    constexpr int T1 = (T0 + ILP <= SB + 1) ? T0 + ILP : SB + 1;
    eval_group<D, T0, T1>(kmask, ns, R, delta);
    eval_nodes<D, T1>(kmask, ns, R, delta);
  }
}

// Two staged tiles of the same class at once (byte offsets da and db from
// the tile the node columns were set up for): the searches of both tiles run
// interleaved, so twice as many LDS reads are in flight, and both tiles' left
// counts go to the same counters.
template <int D, int T0, int T1>
__device__ __forceinline__ void eval_group2(uint32_t kmask, NodeState<D> &ns,
                                            uint64_t (&Ra)[1 << D], uint64_t (&Rb)[1 << D],
                                            uint32_t da, uint32_t db) {
  constexpr int NG = T1 - T0;
  uint32_t a[NG], c[NG];
#pragma unroll
  for (int i = 0; i < NG; ++i) {
    a[i] = ns.col[T0 - 1 + i] + da;
    c[i] = ns.col[T0 - 1 + i] + db;
  }
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) {
    uint32_t va[NG], vc[NG];
#pragma unroll
    for (int i = 0; i < NG; ++i) {
      va[i] = lds_rd32(a[i] + (s - 1) * 4);
      vc[i] = lds_rd32(c[i] + (s - 1) * 4);
    }
#pragma unroll
    for (int i = 0; i < NG; ++i) {
      a[i] = step_if_less(a[i], va[i], ns.thr[T0 - 1 + i], s);
      c[i] = step_if_less(c[i], vc[i], ns.thr[T0 - 1 + i], s);
    }
  }
  uint64_t ma[NG], mc[NG];
#pragma unroll
  for (int i = 0; i < NG; ++i) {
    ma[i] = lds_rd64(kmask - da + 2 * a[i]);
    mc[i] = lds_rd64(kmask - db + 2 * c[i]);
  }
#pragma unroll
  for (int i = 0; i < NG; ++i) {
    constexpr int SL = 1 << D;
    const int t = T0 + i;
    const uint64_t A = Ra[t] & ma[i], C = Rb[t] & mc[i];
    ns.acc[t - 1] += (uint32_t)__popcll(A) + (uint32_t)__popcll(C);
    if (2 * t < SL) {
      Ra[2 * t + 1] = Ra[t] & ~ma[i];
      Ra[2 * t] = A;
      Rb[2 * t + 1] = Rb[t] & ~mc[i];
      Rb[2 * t] = C;
    }
  }
}

template <int D, int T0>
__device__ __forceinline__ void eval_nodes2(uint32_t kmask, NodeState<D> &ns,
                                            uint64_t (&Ra)[1 << D], uint64_t (&Rb)[1 << D],
                                            uint32_t da, uint32_t db) {
  constexpr int SB = (1 << D) - 1;
  if constexpr (T0 <= SB) {
    constexpr int T1 = (T0 + ILP <= SB + 1) ? T0 + ILP : SB + 1;
    eval_group2<D, T0, T1>(kmask, ns, Ra, Rb, da, db);
    eval_nodes2<D, T1>(kmask, ns, Ra, Rb, da, db);
  }
}

// Staging: the tile record (sorted [F][64] u32, then masks [F][64] u64) moves
// as 16-byte chunks; chunk c < 16F is four ranks of column c / 16, the rest
// two masks each.  Up to PF chunks per thread are prefetched into registers
// one tile ahead so that the HBM latency hides behind the current tile.
constexpr int PF = 4;

__device__ __forceinline__ void stage_chunk(uint8_t *__restrict__ lds, uint32_t mregion,
                                            uint32_t F, uint32_t c, const uint4 &v) {
  if (c < 16u * F) {
    const uint32_t f = c >> 4, j0 = (c & 15u) * 4u;
    uint32_t *d = reinterpret_cast<uint32_t *>(lds + f * SCOL) + j0;
    d[0] = v.x;
    d[1] = v.y;
    d[2] = v.z;
    d[3] = v.w;
  } else {
    const uint32_t cc = c - 16u * F;
    const uint32_t f = cc >> 5, e0 = (cc & 31u) * 2u;
    uint64_t *d = reinterpret_cast<uint64_t *>(lds + mregion + f * MCOL) + e0;
    d[0] = ((uint64_t)v.y << 32) | v.x;
    d[1] = ((uint64_t)v.w << 32) | v.z;
  }
}

}  // namespace
}  // namespace mh
