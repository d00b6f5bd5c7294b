// clear.hip -- zeroing of several small device buffers in one launch (the
// counters, barrier words and status flags that a run starts from).
#include "internal.h"

namespace mh {
namespace {

struct ZeroList {
  uint32_t *p[MAX_ZERO_RANGES];
  uint32_t words[MAX_ZERO_RANGES];
  uint32_t n;
};

__global__ __launch_bounds__(256) void k_zero(ZeroList z) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t r = 0; r < z.n; ++r)
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < z.words[r]; i += stride)
      z.p[r][i] = 0u;
}

}  // namespace

mh_status launch_zero(Ctx *ctx, std::initializer_list<ZeroRange> ranges) {
  ZeroList z{};
  uint32_t most = 0;
  for (const ZeroRange &r : ranges) {
    if (!r.ptr || r.bytes == 0) continue;
    if (z.n == MAX_ZERO_RANGES) return fail(ctx, MH_EINVAL, "launch_zero: too many ranges");
    if (r.bytes % 4 != 0 || r.bytes / 4 > 0xFFFFFFFFull)
      return fail(ctx, MH_EINVAL, "launch_zero: size not a multiple of 4 bytes");
    z.p[z.n] = static_cast<uint32_t *>(r.ptr);
    z.words[z.n] = (uint32_t)(r.bytes / 4);
    most = std::max(most, z.words[z.n]);
    ++z.n;
  }
  if (z.n == 0) return MH_OK;
  const uint32_t blocks = std::min<uint32_t>((most + 255) / 256, 1024u);
  k_zero<<<blocks, 256, 0, ctx->stream>>>(z);
  MH_LAUNCHED(ctx, "k_zero");
  return MH_OK;
}

}  // namespace mh
