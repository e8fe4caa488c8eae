// Global-memory loads and stores through the global address space.  A
// pointer read from an LDS table, or passed into a non-inlined device
// function, is generic to the compiler, which then emits flat instructions;
// a flat load also counts on the LDS counter, so every wait for an LDS read
// waits for the flat loads in flight as well.
#pragma once

#include <hip/hip_runtime.h>

namespace pne {
namespace dev {

template <typename T>
__device__ __forceinline__ T gld(const T *p) {
    return *(const __attribute__((address_space(1))) T *)p;
}

template <typename T>
__device__ __forceinline__ void gst(T *p, T v) {
    *(__attribute__((address_space(1))) T *)p = v;
}

}  // namespace dev
}  // namespace pne
