// Wavefront-level helpers for device code (wave64, gfx950).
#pragma once

#include <hip/hip_runtime.h>

namespace em {

// Slot of this lane in a wave-wide push (lanes with want = true, in lane
// order); count (wave-uniform) grows by the number of pushing lanes.  Call in
// wave-uniform control flow.
__device__ __forceinline__ int wave_push(bool want, int &count)
{
    const unsigned long long m = __ballot(want);
    const int below = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
    const int slot = count + below;
    count += __popcll(m);
    return slot;
}

// Orders LDS writes of one wavefront before its later reads by other lanes.
__device__ __forceinline__ void lds_sync_wave()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Logical index of this workgroup in an XCD-aware order.  Workgroups are
// dispatched round-robin over the 8 XCDs (workgroup b to XCD b mod 8); this
// gives XCD x a contiguous run of logical indices (x * per + min(x, rem) ...,
// per = nb / 8, rem = nb mod 8), so neighbouring work shares one L2.  A
// bijection of [0, nb).
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb)
{
    const unsigned x = b & 7u, k = b >> 3, per = nb >> 3, rem = nb & 7u;
    return x * per + (x < rem ? x : rem) + k;
}

}  // namespace em
