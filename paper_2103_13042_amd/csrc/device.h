// Device-side types shared by the kernel sources of libspamm.so.
#pragma once

#include <hip/hip_runtime.h>

namespace spamm {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));

}  // namespace spamm
