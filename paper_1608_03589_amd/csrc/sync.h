// Grid-wide arrival counting for the "last block finishes the iteration"
// pattern and for the grid barrier of the persistent batch driver.
//
// One counter hit by every block serialises all their atomics on one address
// (and, if it shares a cache line with a polled word, the polls as well).
// Blocks therefore arrive on one of kSyncGroups sub-counters (blockIdx mod 8,
// which is also the XCD the block was dispatched to) and only the last
// arrival of each group touches the top counter.  Every word lives on its own
// 256-byte line.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tvpd {

constexpr int kSyncGroups = 8;

struct alignas(256) SyncLine {
  uint32_t v;
  uint32_t pad[63];
};

struct SyncArea {
  SyncLine sub[kSyncGroups];
  SyncLine top;
  SyncLine gen;  // barrier generation (persistent driver only)
};
static_assert(sizeof(SyncArea) == 256 * (kSyncGroups + 2), "sync area");

constexpr size_t kSyncOffset = 512;  // byte offset of the SyncArea in a header

namespace dev {

// Called by one thread per block, after a release fence.  Returns true in
// the last block to arrive; counters are back at zero when it returns true.
__device__ __forceinline__ bool arrive_last(SyncArea* s, unsigned nblocks) {
  const unsigned grp = blockIdx.x % kSyncGroups;
  const unsigned in_grp =
      nblocks / kSyncGroups + (grp < nblocks % kSyncGroups ? 1u : 0u);
  const unsigned a = atomicAdd(&s->sub[grp].v, 1u);
  if (a != in_grp - 1) return false;
  __hip_atomic_store(&s->sub[grp].v, 0u, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
  const unsigned groups = nblocks < kSyncGroups ? nblocks : kSyncGroups;
  __threadfence();
  const unsigned t = atomicAdd(&s->top.v, 1u);
  if (t != groups - 1) return false;
  __hip_atomic_store(&s->top.v, 0u, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
  return true;
}

}  // namespace dev
}  // namespace tvpd
