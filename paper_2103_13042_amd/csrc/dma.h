// Device-side pieces shared by the LDS-DMA multiply kernels (FP32 and
// reduced precision): cost weights of the macro-tile partition, hand-counted
// copy waits, and the check that such a kernel uses no scratch memory.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace spamm {

constexpr int kUnionCost = 4;   // partition cost per union k of a macro tile
constexpr int kMacroWrite = 2;  // partition cost per macro tile written

constexpr int kDmaThreads = 1024;
constexpr int kDmaStores = 16;  // per wave per macro tile
#ifndef SPAMM_DMA_KC
#define SPAMM_DMA_KC 64
#endif
#ifndef SPAMM_DMA_STAGES
#define SPAMM_DMA_STAGES 2
#endif
constexpr int kDmaKC = SPAMM_DMA_KC;          // k per item
constexpr int kDmaStages = SPAMM_DMA_STAGES;  // LDS stages (items in flight + 1)
constexpr int kDmaCopies = 2 * kDmaKC / 32;   // copies per wave per item
static_assert(kDmaStages * (2 * 64 * kDmaKC * 4 * 2) <= 160 * 1024, "LDS budget");

template <int N>
__device__ __forceinline__ void wait_vmcnt() {
    static_assert(N >= 0 && N <= 63, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 0xF) | (0x7 << 4) | (0xF << 8) | ((N >> 4) << 14));
}

// wait until at most `newer` vector memory operations are outstanding, where
// newer = BASE + kDmaStores * stores (above 63: wait for 63, which forces the
// awaited copies too because operations complete in issue order)
template <int BASE>
__device__ __forceinline__ void wait_copies(int stores) {
    switch (stores) {
        case 0: wait_vmcnt<BASE>(); break;
        case 1: wait_vmcnt<(BASE + kDmaStores > 63 ? 63 : BASE + kDmaStores)>(); break;
        case 2: wait_vmcnt<(BASE + 2 * kDmaStores > 63 ? 63 : BASE + 2 * kDmaStores)>(); break;
        case 3: wait_vmcnt<(BASE + 3 * kDmaStores > 63 ? 63 : BASE + 3 * kDmaStores)>(); break;
        default: wait_vmcnt<63>(); break;
    }
}

// The copy-completion waits above count this kernel's own memory operations;
// a register spill would add scratch accesses to that count.  Kernels that
// rely on the count are checked once per process to use no scratch memory.
template <typename K>
static hipError_t check_no_scratch(K kernel, int* state) {
    if (*state == 0) {
        hipFuncAttributes attr{};
        const hipError_t e = hipFuncGetAttributes(&attr, reinterpret_cast<const void*>(kernel));
        if (e != hipSuccess) return e;
        *state = attr.localSizeBytes == 0 ? 1 : 2;
    }
    return *state == 1 ? hipSuccess : hipErrorInvalidDeviceFunction;
}


}  // namespace spamm
