// Multiply of the kept leaf pairs at leaf 16 (the smallest leaf, LoNum = 16 in
// the paper's notation, section 3).
//
// A 16 x 16 leaf product is 8 KFLOP against 2 KB of operands, so the kernel is
// bound by operand latency, not by the matrix cores: one wave per output tile,
// its A and B tiles read from global memory (L2) straight into MFMA operand
// registers, the next kept pair's loads issued before the current pair's
// MFMAs.  v_mfma_f32_16x16x4f32: lane l supplies row (or column) l & 15 and
// k-index g = l >> 4 of each step; in step s lane (r, g) holds A[r][4g + s]
// and B[4g + s][c], so the four steps cover the tile's 16 k in a fixed order
// and A is read as one 16-byte load per lane (four consecutive k of its row).
// Pairs are taken in ascending k; tiles with no kept pair are written as zero
// (beta = 0, section 2.1).  Loads outside the N x N matrix (ragged edge) read
// zero, stores there are skipped.
#include <hip/hip_runtime.h>

#include "device.h"
#include "dma.h"
#include "internal.h"

namespace spamm {

namespace {
constexpr int kL16 = 16;
constexpr int kL16Waves = 4;
}  // namespace

template <bool VEC>
__global__ __launch_bounds__(kL16Waves * 64) void multiply_leaf16_kernel(const float* __restrict__ A,
                                                                        const float* __restrict__ B,
                                                                        float* __restrict__ C, int64_t n,
                                                                        int64_t bdim, const int32_t* __restrict__ off,
                                                                        const int32_t* __restrict__ klist) {
    const int lane = threadIdx.x & 63;
    const int64_t t = int64_t(blockIdx.x) * kL16Waves + (threadIdx.x >> 6);
    if (t >= bdim * bdim) return;
    const int64_t ti = t / bdim, tj = t - (t / bdim) * bdim;
    const int r = lane & 15, g = lane >> 4;
    const int64_t arow = ti * kL16 + r, bcol = tj * kL16 + r;
    const bool arow_in = arow < n, bcol_in = bcol < n;
    const int32_t q0 = off[t], q1 = off[t + 1];

    auto load = [&](int32_t q, float (&ra)[4], float (&rb)[4]) __attribute__((always_inline)) {
        const int64_t k0 = int64_t(klist[q]) * kL16 + 4 * g;
        if (VEC && arow_in && k0 + 3 < n) {
            const f4 x = *reinterpret_cast<const f4*>(A + arow * n + k0);
#pragma unroll
            for (int s = 0; s < 4; ++s) ra[s] = x[s];
        } else {
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const bool in = arow_in && k0 + s < n;
                const float x = A[in ? arow * n + k0 + s : 0];
                ra[s] = in ? x : 0.0f;
            }
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const bool in = bcol_in && k0 + s < n;
            const float x = B[in ? (k0 + s) * n + bcol : 0];
            rb[s] = in ? x : 0.0f;
        }
    };
    f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    auto mma = [&](const float (&ra)[4], const float (&rb)[4]) __attribute__((always_inline)) {
#pragma unroll
        for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ra[s], rb[s], acc, 0, 0, 0);
    };
    float ra0[4], rb0[4], ra1[4], rb1[4];
    if (q0 < q1) {
        load(q0, ra0, rb0);
        for (int32_t q = q0; q < q1; q += 2) {
            if (q + 1 < q1) load(q + 1, ra1, rb1);
            mma(ra0, rb0);
            if (q + 1 >= q1) break;
            if (q + 2 < q1) load(q + 2, ra0, rb0);
            mma(ra1, rb1);
        }
    }
    // accumulator register v of lane l: row 4 (l >> 4) + v, column l & 15
    if (!bcol_in) return;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int64_t row = ti * kL16 + 4 * g + v;
        if (row < n) C[row * n + bcol] = acc[v];
    }
}

hipError_t launch_multiply_leaf16(const float* a, const float* b, float* c, int64_t n, int64_t bdim,
                                  const int32_t* offsets, const int32_t* klist, bool vec, hipStream_t s) {
    const int64_t nt = bdim * bdim;
    const unsigned blocks = unsigned((nt + kL16Waves - 1) / kL16Waves);
    static int scratch_state[2] = {0, 0};
    const hipError_t ce = vec ? check_no_scratch(multiply_leaf16_kernel<true>, &scratch_state[1])
                              : check_no_scratch(multiply_leaf16_kernel<false>, &scratch_state[0]);
    if (ce != hipSuccess) return ce;
    if (vec)
        multiply_leaf16_kernel<true><<<blocks, kL16Waves * 64, 0, s>>>(a, b, c, n, bdim, offsets, klist);
    else
        multiply_leaf16_kernel<false><<<blocks, kL16Waves * 64, 0, s>>>(a, b, c, n, bdim, offsets, klist);
    return hipGetLastError();
}

}  // namespace spamm
