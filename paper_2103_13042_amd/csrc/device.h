// Device-side types shared by the kernel sources of libspamm.so.
#pragma once

#include <hip/hip_runtime.h>

namespace spamm {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));

// p as a pointer into global memory.  A pointer read from memory (a
// descriptor array) carries no address space, so the compiler emits flat
// accesses through it, which also count against the LDS wait counter (an LDS
// wait then waits for every load in flight too); the integer round trip gives
// it the global address space, which the compiler keeps through inlining.
template <typename T>
__device__ __forceinline__ T* global_ptr(T* p) {
    return (T*)(__attribute__((address_space(1))) T*)reinterpret_cast<uintptr_t>(p);
}

// whether a launch gated on the plan's pair count runs (PairGate, internal.h)
template <typename Gate>
__device__ __forceinline__ bool gate_open(const Gate& g) {
    return g.pairs == nullptr || ((*g.pairs >= g.threshold) == (g.when_at_least != 0));
}

}  // namespace spamm
