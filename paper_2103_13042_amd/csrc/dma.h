// Device-side pieces shared by the LDS-DMA multiply kernels (FP32 and
// reduced precision): cost weights of the macro-tile partition, hand-counted
// copy waits, and the check that such a kernel uses no scratch memory.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace spamm {

constexpr int kUnionCost = 4;   // partition cost per union k of a macro tile
constexpr int kMacroWrite = 2;  // partition cost per macro tile written

// Item-level partition of the FP32 multiply.  Measured per-workgroup times
// fit  t = a * items + b * kept + c * macro tiles  with a : b : c close to
// 5 : 4 : 5 (an item's fixed cost of copies and barrier, the MFMA work of each
// output tile that keeps the item's k, the store of a finished macro tile).
constexpr int kItemCost = 5;
constexpr int kKeptCost = 4;
constexpr int kStoreCost = 5;
// Workgroups of the split multiply and the per-workgroup partial slots of the
// macro tiles split between workgroups (two per workgroup: the first and the
// last macro tile it touches), 128 x 128 FP32 each.
constexpr int kSplitMaxGroups = 256;
constexpr int kSplitSlotFloats = 128 * 128;

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
// a register spill would add scratch accesses to that count, and in any
// multiply kernel it would put slow scratch traffic in the inner loop.  Every
// multiply kernel is checked once per process to use no scratch memory (a
// kernel that does is not launched: hipErrorInvalidDeviceFunction).
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


// Modelled cost of the macro tiles before m (row-major), bdim = 2 mb even:
// kStoreCost per tile + kItemCost per union k (uprefix) + kKeptCost per kept
// pair, the pairs of the tiles before m read off the plan's offsets (all tile
// rows above the macro row, and the first 2J tiles of its two tile rows).
// offsets == nullptr: every item feeds all four quarters (leaf-128 tiles).
__device__ inline int64_t macro_cost_before(int64_t m, int64_t mb, const int32_t* __restrict__ uprefix,
                                            const int32_t* __restrict__ offsets) {
    const int64_t bdim = 2 * mb;
    int64_t kept;
    if (offsets == nullptr) {
        kept = 4 * int64_t(uprefix[m]);
    } else if (m >= mb * mb) {
        kept = offsets[bdim * bdim];
    } else {
        const int64_t I = m / mb, J = m - (m / mb) * mb, r0 = 2 * I * bdim;
        kept = int64_t(offsets[r0 + 2 * J]) + offsets[r0 + bdim + 2 * J] - offsets[r0 + bdim];
    }
    return kStoreCost * m + kItemCost * int64_t(uprefix[m]) + kKeptCost * kept;
}

// Boundary gg of G in the item-level partition, wave-cooperative (every lane
// returns the same value): the first item whose modelled cost before it
// reaches gg * total / G (the store of a macro tile counted before its items),
// as (macro tile m, item index p) with uprefix[m] <= p < uprefix[m + 1], or
// (m, uprefix[m]) at a clean macro-tile start (the end is (nm, uprefix[nm])).
struct SplitBound {
    int64_t m, p;
};

__device__ inline SplitBound split_bound(int64_t gg, int64_t G, int64_t mb, const int32_t* __restrict__ uprefix,
                                         const int32_t* __restrict__ offsets, const uint32_t* __restrict__ items) {
    const int lane = threadIdx.x & 63;
    const int64_t nm = mb * mb;
    if (gg <= 0) return {0, 0};
    if (gg >= G) return {nm, int64_t(uprefix[nm])};
    const int64_t T = gg * macro_cost_before(nm, mb, uprefix, offsets) / G;
    // largest m < nm with cost_before(m) <= T: 64-ary search, invariant
    // cost_before(lo) <= T and the answer in [lo, hi)
    int64_t lo = 0, hi = nm;
    while (hi - lo > 1) {
        const int64_t step = (hi - lo + 63) / 64;
        const int64_t c = lo + step * (lane + 1);
        const bool le = lane < 63 && c < hi && macro_cost_before(c, mb, uprefix, offsets) <= T;
        const int cnt = __popcll(__ballot(le));  // monotone: lanes 0 .. cnt-1
        lo += step * cnt;
        hi = (lo + step < hi) ? lo + step : hi;
    }
    const int64_t m = lo, u0 = uprefix[m], u1 = uprefix[m + 1];
    int64_t c0 = macro_cost_before(m, mb, uprefix, offsets) + kStoreCost;  // cost before item u0
    if (c0 >= T) return {m, u0};
    for (int64_t base = u0; base < u1; base += 64) {
        const int64_t i = base + lane;
        const int cst = i < u1 ? kItemCost + kKeptCost * __popc(items[i] & 15u) : 0;
        int incl = cst;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int up = __shfl_up(incl, o);
            if (lane >= o) incl += up;
        }
        const uint64_t hit = __ballot(i < u1 && c0 + (incl - cst) >= T);
        if (hit) return {m, base + __ffsll(static_cast<unsigned long long>(hit)) - 1};
        c0 += __shfl(incl, 63);
    }
    return {m + 1, u1};
}

}  // namespace spamm
