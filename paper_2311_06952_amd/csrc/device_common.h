// device_common.h -- device-side helpers: the counter-based random stream,
// individual decoding, and wave64 primitives.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mh {

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): the k-th output of the
// generator seeded with s is fmix(s + k * 0x9E3779B97F4A7C15), where fmix is
// the variant-13 64-bit finaliser.  Being a function of (s, k) it serves as a
// counter-based generator.
__host__ __device__ __forceinline__ uint64_t sm64_fmix(uint64_t z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__host__ __device__ __forceinline__ uint64_t sm64_out(uint64_t s, uint64_t k) {
  return sm64_fmix(s + k * 0x9E3779B97F4A7C15ull);
}
// DE stream: problem key = output (problem + 1) of the seed's stream; the
// draw for (generation g, individual r, slot) is output
// ((g << 40 | r << 20 | slot) + 1) of the key's stream.
__host__ __device__ __forceinline__ uint64_t de_key(uint64_t seed, uint64_t prob) {
  return sm64_out(seed, prob + 1);
}
__host__ __device__ __forceinline__ uint64_t de_draw(uint64_t key, uint32_t g, uint32_t r,
                                                     uint32_t slot) {
  uint64_t c = ((uint64_t)g << 40) | ((uint64_t)r << 20) | (uint64_t)slot;
  return sm64_out(key, c + 1);
}
// [0, 1) from the top 53 bits.
__host__ __device__ __forceinline__ double to_unit(uint64_t u) {
  return (double)(u >> 11) * 0x1.0p-53;
}
// [0, m) by multiply-shift of the top 32 bits.
__host__ __device__ __forceinline__ uint32_t to_below(uint64_t u, uint32_t m) {
  return (uint32_t)(((u >> 32) * (uint64_t)m) >> 32);
}

// Decoding of one node (eq. aenc, eq. benc): feature gene a in [0, F+1]
// selects feature floor(a) (0 = no split, capped at F); threshold gene b in
// [0, 1] selects threshold index floor(b (n_f + 1)), capped at n_f.  Genes are
// clamped first (NaN counts as below range).  Exact IEEE f64 arithmetic.
__device__ __forceinline__ void decode_node(double a, double b, uint32_t F,
                                            const uint32_t *__restrict__ n_unique,
                                            uint32_t &feat, uint32_t &tau) {
  double Fp1 = (double)F + 1.0;
  if (!(a >= 0.0)) a = 0.0;
  if (a > Fp1) a = Fp1;
  if (!(b >= 0.0)) b = 0.0;
  if (b > 1.0) b = 1.0;
  double fa = floor(a);
  uint32_t f = (fa >= (double)F) ? F : (uint32_t)fa;
  uint32_t th = 0;
  if (f != 0) {
    uint32_t nf = n_unique[f - 1];
    double x = floor(__dmul_rn(b, (double)(nf + 1u)));
    th = (x >= (double)nf) ? nf : (uint32_t)x;
  }
  feat = f;
  tau = th;
}

// wave64 helpers
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

template <typename T>
__device__ __forceinline__ T shfl_xor64(T v, int m) {
  return __shfl_xor(v, m, 64);
}

}  // namespace mh
