// Injected allocation failures, for tests of the library's error paths.
//
// While armed (RSF_FAULT=alloc_fail:N[:K] in the environment when the
// library loads, or rsf_set_fault), every device or pinned host allocation
// the library attempts is counted from 1, and attempts N .. N+K-1 (K = 1 by
// default) fail with hipErrorOutOfMemory without allocating, as a real
// out-of-memory would.  Disarmed, the wrappers are plain hipMalloc and
// hipHostMalloc.
#pragma once

#include <hip/hip_runtime.h>

namespace rsf {

// Counts one allocation attempt; true when the armed fault makes it fail.
bool fault_take_alloc();

template <class T>
hipError_t dev_alloc(T **p, size_t bytes)
{
    *p = nullptr;
    if (fault_take_alloc()) return hipErrorOutOfMemory;
    void *q = nullptr;
    const hipError_t e = hipMalloc(&q, bytes);
    if (e == hipSuccess) *p = static_cast<T *>(q);
    return e;
}

template <class T>
hipError_t pinned_alloc(T **p, size_t bytes)
{
    *p = nullptr;
    if (fault_take_alloc()) return hipErrorOutOfMemory;
    void *q = nullptr;
    const hipError_t e = hipHostMalloc(&q, bytes, hipHostMallocDefault);
    if (e == hipSuccess) *p = static_cast<T *>(q);
    return e;
}

}  // namespace rsf
