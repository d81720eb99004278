// strip_sync.h -- device helpers shared by the 32-bit and the packed 16-bit
// strip kernels: DPP lane shifts, border records through agent-scope
// atomics, the chunk counters that hand a border row from one strip to the
// next, and their bounded waits.
#pragma once

#include <hip/hip_runtime.h>

#include "engine.h"

namespace swh {
namespace strip_dev {

constexpr int kDppWaveShl1 = 0x130;   // lane i reads lane i+1 (lane 63: keeps old)
constexpr int kDppWaveShr1 = 0x138;   // lane i reads lane i-1 (lane 0: keeps old)

__device__ __forceinline__ int shr1(int old, int src)
{
    return __builtin_amdgcn_update_dpp(old, src, kDppWaveShr1, 0xF, 0xF, false);
}

__device__ __forceinline__ int shl1(int old, int src)
{
    return __builtin_amdgcn_update_dpp(old, src, kDppWaveShl1, 0xF, 0xF, false);
}

__device__ __forceinline__ int max3i(int a, int b, int c) { return max(max(a, b), c); }

template <bool V>
struct BoolC {
    static constexpr bool value = V;
};

// Border traffic goes through agent-scope relaxed atomics (coherent across
// the XCDs' L2s per location); ordering is explicit: stores are drained with
// s_waitcnt vmcnt(0) before the chunk counter is published.
__device__ __forceinline__ void store_border(Border *p, int h, int f)
{
    uint64_t v = (uint64_t)(uint32_t)h | ((uint64_t)(uint32_t)f << 32);
    __hip_atomic_store((uint64_t *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void load_border(const Border *p, int &h, int &f)
{
    uint64_t v = __hip_atomic_load((const uint64_t *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    h = (int)(uint32_t)v;
    f = (int)(uint32_t)(v >> 32);
}

__device__ __forceinline__ void drain_stores()
{
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0x0F70);     // vmcnt(0), expcnt/lgkmcnt untouched
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Wait until chunk counter >= need.  Every value that decides a branch is
// made wave-uniform (readfirstlane) so that no loop exit can diverge: the
// kernel's lane shifts assume all 64 lanes execute together.  Bounded: on
// expiry (or when another wave has given up) sets/observes abort and returns
// false.
__device__ __forceinline__ bool wait_chunk(const StripArgs &a, const int32_t *flags, int chunk, int need)
{
    const uint64_t t0 = wall_clock64();
    for (;;) {
        const int v = __builtin_amdgcn_readfirstlane(
            __hip_atomic_load(flags + chunk, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (v >= need) return true;
        const int ab = __builtin_amdgcn_readfirstlane(
            __hip_atomic_load(a.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (ab) return false;
        if (wall_clock64() - t0 > a.wait_ticks) {
            __hip_atomic_store(a.abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(2);
    }
}

// Chunk counter, read without waiting for it (the value is checked a whole
// block of steps later, when the load has long returned).
__device__ __forceinline__ int peek_chunk(const int32_t *flags, int chunk)
{
    return __hip_atomic_load(flags + chunk, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A lane-identity DPP move: its result is a plain register value, so the
// loads that produced v are waited for here, outside the step loop.
__device__ __forceinline__ int settled(int v) { return __builtin_amdgcn_update_dpp(0, v, 0xE4, 0xF, 0xF, false); }

}  // namespace strip_dev
}  // namespace swh
