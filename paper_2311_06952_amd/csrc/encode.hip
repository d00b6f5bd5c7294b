// encode.hip -- a tree written back into genes, the inverse of the decode of
// eq. aenc and eq. benc, so that a tree (from the moving horizon, a
// greedy split sequence, an earlier run) can seed a DEOCT population as a
// warm start (the warm-started variants of Section 4).
//
// Each gene is the centre of the interval that decodes to the node's value:
// a^ = a + 0.5 and b^ = (tau + 0.5) / (n_f + 1), in f64; a node with no
// split (a = 0, or a > F, which is no feature) gets (0.5, 0).  The decode
// returns the tree exactly for every tau in [0, n_f].
#include "internal.h"

namespace mh {
namespace {

__global__ __launch_bounds__(256) void k_tree_encode(const uint8_t *__restrict__ feat,
                                                     const uint32_t *__restrict__ tau,
                                                     uint32_t P, uint32_t SB, uint32_t F,
                                                     const uint32_t *__restrict__ n_unique,
                                                     double *__restrict__ genes) {
  const uint64_t k = (uint64_t)blockIdx.x * 256u + threadIdx.x;
  if (k >= (uint64_t)P * SB) return;
  const uint32_t r = (uint32_t)(k / SB), t = (uint32_t)(k % SB);
  const uint32_t f = feat[k];
  double a = 0.5, b = 0.0;
  if (f != 0 && f <= F) {
    a = __dadd_rn((double)f, 0.5);
    b = __ddiv_rn(__dadd_rn((double)tau[k], 0.5), __dadd_rn((double)n_unique[f - 1], 1.0));
  }
  double *g = genes + (size_t)r * 2u * SB;
  g[t] = a;
  g[SB + t] = b;
}

}  // namespace

mh_status launch_tree_encode(Ctx *ctx, const uint8_t *feat, const uint32_t *tau, uint32_t P,
                             uint32_t D, uint32_t F, const uint32_t *n_unique, double *genes) {
  const uint32_t SB = (1u << D) - 1u;
  const uint64_t total = (uint64_t)P * SB;
  if (total == 0) return MH_OK;
  k_tree_encode<<<(uint32_t)((total + 255) / 256), 256, 0, ctx->stream>>>(feat, tau, P, SB, F,
                                                                            n_unique, genes);
  MH_LAUNCHED(ctx, "k_tree_encode");
  return MH_OK;
}

}  // namespace mh

using namespace mh;

extern "C" mh_status tree_encode(mh_ctx *ctx, const uint8_t *feat, const uint32_t *tau,
                                 uint32_t P, uint32_t D, uint32_t F, const uint32_t *n_unique,
                                 double *genes) {
  if (!ctx) return fail(nullptr, MH_EINVAL, "context is null");
  Ctx *c = &ctx->c;
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  if (D < 1 || D > MH_MAX_DEPTH) return fail(c, MH_EINVAL, "D must be in 1..10");
  if (F == 0 || F > MH_MAX_FEATURES) return fail(c, MH_EINVAL, "F must be in 1..255");
  if (P == 0) return MH_OK;
  if (!feat || !tau || !n_unique || !genes) return fail(c, MH_EINVAL, "null pointer");
  const uint64_t total = (uint64_t)P * ((1u << D) - 1u);
  if (total > (1ull << 31)) return fail(c, MH_EINVAL, "P * (2^D - 1) must be <= 2^31");
  return launch_tree_encode(c, feat, tau, P, D, F, n_unique, genes);
}
