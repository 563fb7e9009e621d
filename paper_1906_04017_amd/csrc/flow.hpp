// Device helpers of the dataflow schedules (single problem and batched):
// agent-scope counter access and the bounded wait of one wave on a range of
// done flags.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace dgsn {

__device__ __forceinline__ unsigned flow_load(const unsigned *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned flow_add(unsigned *p, unsigned v)
{
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void flow_store(unsigned *p, unsigned v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Whole wave: wait until done[lo..hi] all hold at least `target` (one flag per
// lane, 64 at a time; lo > hi waits for nothing).  Gives up after spin_limit
// polls of one group of flags, or as soon as the error word is set, and then
// sets the error word.
__device__ __forceinline__ void flow_wait_range(const unsigned *done, unsigned lo, unsigned hi,
                                                unsigned target, int lane, unsigned spin_limit,
                                                unsigned *err)
{
    for (unsigned base = lo; base <= hi; base += 64) {
        const unsigned idx = base + lane;
        bool ok = idx > hi;
        for (unsigned it = 0;; ++it) {
            if (!ok) ok = flow_load(done + idx) >= target;
            if (__all(ok)) break;
            if (it >= spin_limit || __any(flow_load(err) != 0u)) {
                if (lane == 0) flow_store(err, 1u);
                return;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
}

}  // namespace dgsn
