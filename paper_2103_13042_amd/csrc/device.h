// Device-side types shared by the kernel sources of libspamm.so.
#pragma once

#include <hip/hip_runtime.h>

namespace spamm {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));

// whether a launch gated on the plan's pair count runs (PairGate, internal.h)
template <typename Gate>
__device__ __forceinline__ bool gate_open(const Gate& g) {
    return g.pairs == nullptr || ((*g.pairs >= g.threshold) == (g.when_at_least != 0));
}

}  // namespace spamm
