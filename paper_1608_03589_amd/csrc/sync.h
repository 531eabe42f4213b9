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

// Ordering between blocks.  The L2 caches of the XCDs are not coherent with
// each other: data handed to blocks elsewhere is written back from L2 before
// the signal (an agent-scope release: an L2 writeback), and the receiver
// drops its stale L2 and L1 lines after seeing the signal (an agent-scope
// acquire: an invalidate).  A release orders only the releasing wave's own
// stores, so every wave of a block first waits until its stores have
// reached L2 (wait_vmem) and, after the block barrier, one release by
// thread 0 covers the whole block.  Neither is a full fence: a block that
// only signals needs no invalidate, and one that only waits no writeback.

// s_waitcnt with vmcnt 0 and the other counters at their maxima (expcnt 7,
// lgkmcnt 15): wait for this wave's vector memory operations only.
constexpr int kWaitVmem = 0x0F70;
__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(kWaitVmem); }
__device__ __forceinline__ void release_agent() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
}
__device__ __forceinline__ void acquire_agent() {
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// Called by one thread per block, after the block's release.  Returns true
// in the last block to arrive, which then acquires; counters are back at
// zero when it returns true.  The counter updates themselves are relaxed:
// every block's data is in memory before its first arrival, each arrival
// is ordered after the one it counted, and the last block's acquire comes
// after the final count.
__device__ __forceinline__ bool arrive_last(SyncArea* s, unsigned nblocks) {
  const unsigned grp = blockIdx.x % kSyncGroups;
  const unsigned in_grp =
      nblocks / kSyncGroups + (grp < nblocks % kSyncGroups ? 1u : 0u);
  const unsigned a = atomicAdd(&s->sub[grp].v, 1u);
  if (a != in_grp - 1) return false;
  __hip_atomic_store(&s->sub[grp].v, 0u, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
  const unsigned groups = nblocks < kSyncGroups ? nblocks : kSyncGroups;
  const unsigned t = atomicAdd(&s->top.v, 1u);
  if (t != groups - 1) return false;
  __hip_atomic_store(&s->top.v, 0u, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
  acquire_agent();
  return true;
}

}  // namespace dev
}  // namespace tvpd
