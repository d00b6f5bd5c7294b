// grid_sync.h -- a grid barrier for cooperative launches.
//
// All blocks of the barrier's group must be resident at once: the launcher
// keeps the grid within what the device holds, with a margin, and a wait's
// time limit turns a grid that is not resident into an error, not a hang.
//
// Ordering.  Every datum that crosses blocks at a barrier is written with
// agent-scope atomic stores or read-modify-writes and read with agent-scope
// atomic loads, which the hardware performs at the point of coherence shared
// by all XCDs (they do not stop in a CU's or an XCD's cache).  Before a block
// arrives, each of its waves waits until its own memory operations have
// completed (s_waitcnt 0) and the block synchronises, so the arrival is
// issued after the block's atomics are done at that point; a waiter issues
// its loads only after it has seen the release word and the block has
// synchronised again, so they are served after the release.  The barrier
// words themselves are relaxed agent-scope atomics.  Release on the arrivals
// and an acquire fence after the wait, the language-level form of the same
// ordering, cost an L2 write-back and invalidate at every barrier: a whole
// DEOCT run at n = 10^5, F = 16, P = 256, depth 3 took 3.09 instead of
// 2.14 ms, rank encoding 0.42 instead of 0.37 ms, with identical results.
// Plain (non-atomic) memory written before a barrier must not be read by
// another block after it.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mh {

// A barrier wait gives up after `limit` ticks of the device wall clock (by
// default WAIT_LIMIT_TICKS: 2 s at its usual 100 MHz), or at once when
// another block already gave up.
constexpr uint64_t WAIT_LIMIT_TICKS = 200000000ull;

// Barrier words, each on its own 256-byte line: [0] arrivals of group
// leaders, [64] release (the number of completed barriers), [128 + 64 g]
// arrivals in group g of BAR_GROUP consecutive blocks.  A block arrives at its
// group; the last arrival of a group arrives at the top; the last top arrival
// publishes the release.  Spreading the arrivals over separate words avoids
// serialising every block on one address.
constexpr uint32_t BAR_GROUP = 16;
__host__ __device__ __forceinline__ uint32_t barrier_words(uint32_t blocks) {
  return 128 + 64 * ((blocks + BAR_GROUP - 1) / BAR_GROUP);
}

// Barrier number k (0-based) among the nb blocks of a problem (block b of
// them), in two parts
// so that a block can do independent work between arriving and waiting.
// Arrival: every wave's atomics are complete, then thread 0 arrives.
__device__ __forceinline__ void barrier_arrive(uint32_t *bar, uint32_t k, uint32_t b, uint32_t nb) {
  __builtin_amdgcn_s_waitcnt(0);  // vmcnt(0) expcnt(0) lgkmcnt(0): this wave's atomics are done
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t grp = b / BAR_GROUP;
    const uint32_t gsize = min(BAR_GROUP, nb - grp * BAR_GROUP);
    const uint32_t ngroups = (nb + BAR_GROUP - 1) / BAR_GROUP;
    const uint32_t old = __hip_atomic_fetch_add(bar + 128 + 64 * grp, 1u, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
    if (old == (k + 1) * gsize - 1) {
      const uint32_t o2 = __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (o2 == (k + 1) * ngroups - 1)
        __hip_atomic_store(bar + 64, k + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}
// Wait: thread 0 polls the release word, then the block proceeds together.
__device__ __forceinline__ void barrier_wait(uint32_t *bar, uint32_t k, uint32_t *err,
                                             uint64_t limit = WAIT_LIMIT_TICKS) {
  if (threadIdx.x == 0) {
    const uint64_t t0 = wall_clock64();
    while (__hip_atomic_load(bar + 64, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < k + 1) {
      if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
          wall_clock64() - t0 > limit) {
        __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
  }
  __syncthreads();
}

}  // namespace mh
