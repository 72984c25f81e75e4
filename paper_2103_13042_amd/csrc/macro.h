// Device code of the register-staged macro-tile multiply (leaf 32 and 64, any
// N), shared by the single-product kernels (multiply_macro.hip) and the
// batched ones (kernels.hip): the schedule of a product's macro tiles (one
// wave per macro tile) and the multiply of a range of its macro tiles.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.h"

namespace spamm {

constexpr int kMacThreads = 256;

// One wave per macro tile m: k-bitmaps of its four tiles (zero for tiles
// outside the grid) and the size of their union.  sw: the wave's 4 x 16 words
// of LDS scratch.
__device__ __forceinline__ void macro_words_wave(const int32_t* __restrict__ off, const int32_t* __restrict__ klist,
                                                 int64_t bdim, int64_t mb, int nw, uint64_t* __restrict__ words,
                                                 int32_t* __restrict__ ucount, int64_t m,
                                                 unsigned long long (*sw)[16]) {
    const int lane = threadIdx.x & 63;
    const int64_t I = m / mb, J = m - (m / mb) * mb;
    sw[lane >> 4][lane & 15] = 0ull;
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): zeroing done before the ORs
    for (int ab = 0; ab < 4; ++ab) {
        const int64_t ti = 2 * I + (ab >> 1), tj = 2 * J + (ab & 1);
        if (ti >= bdim || tj >= bdim) continue;
        const int64_t t = ti * bdim + tj;
        const int32_t q0 = off[t], q1 = off[t + 1];
        for (int32_t q = q0 + lane; q < q1; q += 64) {
            const int32_t k = klist[q];
            atomicOr(&sw[ab][k >> 6], 1ull << (k & 63));
        }
    }
    __builtin_amdgcn_s_waitcnt(0xC07F);
    int cnt = 0;
    if (lane < nw) {
        const uint64_t u = sw[0][lane] | sw[1][lane] | sw[2][lane] | sw[3][lane];
        cnt = __popcll(u);
    }
    if (lane < 4 * nw) words[(m * 4 + lane / nw) * nw + lane % nw] = sw[lane / nw][lane % nw];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) cnt += __shfl_xor(cnt, o);
    if (lane == 0) ucount[m] = cnt;
}

// packed pair item: I << 23 | J << 14 | k << 4 | membership (bit a*2+b)
__device__ __forceinline__ uint32_t mi_pack(uint32_t I, uint32_t J, uint32_t k, uint32_t mem) {
    return (I << 23) | (J << 14) | (k << 4) | mem;
}

// One wave per macro tile m: its union k values in ascending order, as packed
// items at items[uprefix[m] ..].
__device__ __forceinline__ void macro_items_wave(const uint64_t* __restrict__ words,
                                                 const int32_t* __restrict__ uprefix, int64_t mb, int nw,
                                                 uint32_t* __restrict__ items, int64_t m) {
    const int lane = threadIdx.x & 63;
    const uint32_t I = uint32_t(m / mb), J = uint32_t(m - (m / mb) * mb);
    const uint64_t* wp = words + m * 4 * nw;
    int64_t base = uprefix[m];
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int w = 0; w < nw; ++w) {
        const uint64_t w0 = wp[w], w1 = wp[nw + w], w2 = wp[2 * nw + w], w3 = wp[3 * nw + w];
        const uint64_t u = w0 | w1 | w2 | w3;
        if ((u >> lane) & 1ull) {
            const uint32_t mem = uint32_t((w0 >> lane) & 1) | uint32_t(((w1 >> lane) & 1) << 1) |
                                 uint32_t(((w2 >> lane) & 1) << 2) | uint32_t(((w3 >> lane) & 1) << 3);
            items[base + __popcll(u & below)] = mi_pack(I, J, uint32_t(w) * 64 + lane, mem);
        }
        base += __popcll(u);
    }
}

// four floats read with one 16-byte load from a 4-byte aligned address
// (global loads accept it)
typedef float f4_dw __attribute__((ext_vector_type(4), aligned(4)));

template <int LEAF>
struct MacGeom {
    static constexpr int KC = 32;                 // k per pipeline stage
    static constexpr int NB = LEAF / 32;          // 32x32 MFMA blocks per wave-tile side
    static constexpr int SPC = KC / 2;            // MFMA steps per stage (two lane groups)
    static constexpr int NCH = LEAF / KC;         // stages per leaf pair
    static constexpr int ROWS = 2 * LEAF;         // A rows / B columns staged per item
    static constexpr int AST = KC + 4;            // A row stride (floats)
    static constexpr int BST = ROWS;              // B row stride (floats)
    static constexpr int ASZ = ROWS * AST;
    static constexpr int STAGE = ASZ + KC * BST;
    static constexpr int NV = ROWS * KC / 4 / kMacThreads;  // float4 per thread per operand
    static constexpr int OCC = LEAF == 64 ? 2 : 4;          // workgroups per CU
    static_assert(NV >= 1 && NV * 4 * kMacThreads == ROWS * KC, "stage split");
};

// Macro tiles [m_begin, m_end) of one product with register-staged operands
// (any N: loads outside the matrix read as zero, stores outside are skipped):
// every tile of the range is written.  lds: 2 * MacGeom<LEAF>::STAGE floats.
// All threads of the (kMacThreads) workgroup call it with the same range.
template <int LEAF, bool VEC>
__device__ __forceinline__ void macro_range(const float* __restrict__ A, const float* __restrict__ B,
                                            float* __restrict__ C, int64_t n, int64_t bdim, int64_t mb,
                                            const uint32_t* __restrict__ items, const int32_t* __restrict__ uprefix,
                                            int64_t m_begin, int64_t m_end, float* lds) {
    using Gm = MacGeom<LEAF>;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wa = wave >> 1, wb = wave & 1;
    const int ir = lane & 31, g = lane >> 5;

    if (m_begin >= m_end) return;
    const int64_t nitems = int64_t(uprefix[m_end] - uprefix[m_begin]) * Gm::NCH;

    // this group's slice of the item list (wave-uniform); past the end the
    // last item repeats (a harmless reload)
    const uint32_t* ip = items + uprefix[m_begin];
    const int64_t npairs = int64_t(uprefix[m_end] - uprefix[m_begin]);
    int64_t pp = 0;
    uint32_t last = 0;
    auto produce = [&]() -> uint32_t {
        if (pp < npairs) last = ip[pp];
        ++pp;
        return last;
    };

    typedef f16v acc_t;
    acc_t acc[Gm::NB][Gm::NB];
    auto zero_acc = [&]() {
#pragma unroll
        for (int a = 0; a < Gm::NB; ++a)
#pragma unroll
            for (int b = 0; b < Gm::NB; ++b)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;
    };
    auto store_macro = [&](int64_t m) {
        const int64_t ti = 2 * (m / mb) + wa, tj = 2 * (m - (m / mb) * mb) + wb;
        if (ti >= bdim || tj >= bdim) return;
#pragma unroll
        for (int a = 0; a < Gm::NB; ++a)
#pragma unroll
            for (int b = 0; b < Gm::NB; ++b)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int64_t row = ti * LEAF + a * 32 + 8 * (r >> 2) + 4 * g + (r & 3);
                    const int64_t col = tj * LEAF + b * 32 + ir;
                    if (row < n && col < n) C[row * n + col] = acc[a][b][r];
                }
    };

    // global -> registers for one item (pair item pi, chunk ch): A rows
    // [2I*L, 2I*L + 2L) x k-chunk, B k-chunk x columns [2J*L, 2J*L + 2L).  Every
    // lane issues every load (clamped) and zeroes what lies outside the matrix.
    // Rows that are not 16-byte aligned (VEC false) take 16-byte loads at
    // 4-byte alignment; chunks that cross the matrix's edge, one per element.
    auto fetch = [&](uint32_t pi, int ch, f4 (&ra)[Gm::NV], f4 (&rb)[Gm::NV]) {
        const int64_t I = pi >> 23, J = (pi >> 14) & 511, kt = (pi >> 4) & 1023;
        const int64_t arow0 = 2 * I * LEAF, acol0 = kt * LEAF + ch * Gm::KC;
        const int64_t brow0 = kt * LEAF + ch * Gm::KC, bcol0 = 2 * J * LEAF;
        const f4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int v = 0; v < Gm::NV; ++v) {
            const int e = tid + v * kMacThreads;
            {
                const int r = e / (Gm::KC / 4), c4 = e % (Gm::KC / 4);
                const int64_t row = arow0 + r, col = acol0 + 4 * c4;
                if (VEC) {
                    const bool in = row < n && col < n;
                    const f4 x = *reinterpret_cast<const f4*>(A + (in ? row * n + col : 0));
                    ra[v] = in ? x : zero;
                } else if (row < n && col + 3 < n) {  // 4-byte aligned: one 16-byte load
                    ra[v] = *reinterpret_cast<const f4_dw*>(A + row * n + col);
                } else {
#pragma unroll
                    for (int q4 = 0; q4 < 4; ++q4) {
                        const bool in = row < n && col + q4 < n;
                        const float x = A[in ? row * n + col + q4 : 0];
                        ra[v][q4] = in ? x : 0.0f;
                    }
                }
            }
            {
                const int r = e / (Gm::ROWS / 4), c4 = e % (Gm::ROWS / 4);
                const int64_t row = brow0 + r, col = bcol0 + 4 * c4;
                if (VEC) {
                    const bool in = row < n && col < n;
                    const f4 x = *reinterpret_cast<const f4*>(B + (in ? row * n + col : 0));
                    rb[v] = in ? x : zero;
                } else if (row < n && col + 3 < n) {  // 4-byte aligned: one 16-byte load
                    rb[v] = *reinterpret_cast<const f4_dw*>(B + row * n + col);
                } else {
#pragma unroll
                    for (int q4 = 0; q4 < 4; ++q4) {
                        const bool in = row < n && col + q4 < n;
                        const float x = B[in ? row * n + col + q4 : 0];
                        rb[v][q4] = in ? x : 0.0f;
                    }
                }
            }
        }
    };
    auto commit = [&](int stage, const f4 (&ra)[Gm::NV], const f4 (&rb)[Gm::NV]) {
        float* sa = lds + stage * Gm::STAGE;
        float* sb = sa + Gm::ASZ;
#pragma unroll
        for (int v = 0; v < Gm::NV; ++v) {
            const int e = tid + v * kMacThreads;
            {
                const int r = e / (Gm::KC / 4), c4 = e % (Gm::KC / 4);
                *reinterpret_cast<f4*>(sa + r * Gm::AST + 4 * c4) = ra[v];
            }
            {
                const int r = e / (Gm::ROWS / 4), c4 = e % (Gm::ROWS / 4);
                const int swz = ((r / Gm::SPC) & 1) * 32;
                *reinterpret_cast<f4*>(sb + r * Gm::BST + ((4 * c4) ^ swz)) = rb[v];
            }
        }
    };
    // wave (wa, wb): rows [wa*L, wa*L + L) of the A stage, columns [wb*L, ..) of B.
    // MFMA step s, lane group g: k = g*SPC + s.
    auto compute = [&](int stage) {
        const float* sa = lds + stage * Gm::STAGE + (wa * LEAF + ir) * Gm::AST + g * Gm::SPC;
        const float* sb = lds + stage * Gm::STAGE + Gm::ASZ + g * Gm::SPC * Gm::BST;
        const int swz = g * 32;
#pragma unroll
        for (int q = 0; q < Gm::SPC / 4; ++q) {
            f4 av[Gm::NB];
#pragma unroll
            for (int a = 0; a < Gm::NB; ++a) av[a] = *reinterpret_cast<const f4*>(sa + a * 32 * Gm::AST + 4 * q);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int s = 4 * q + u;
                float bv[Gm::NB];
#pragma unroll
                for (int b = 0; b < Gm::NB; ++b) bv[b] = sb[s * Gm::BST + ((wb * LEAF + b * 32 + ir) ^ swz)];
#pragma unroll
                for (int a = 0; a < Gm::NB; ++a)
#pragma unroll
                    for (int b = 0; b < Gm::NB; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[a][u], bv[b], acc[a][b], 0, 0, 0);
            }
        }
    };

    // pair items of the compute item (f0) and the next two pairs
    uint32_t f0 = produce();
    uint32_t f1 = produce();
    uint32_t f2 = produce();
    constexpr int AHEAD = 2 / Gm::NCH;  // pair distance of item it+2 from item it's pair
    int64_t out_m = m_begin;            // macro tile being accumulated; earlier ones are written
    f4 ra0[Gm::NV], rb0[Gm::NV], ra1[Gm::NV], rb1[Gm::NV];
    auto step = [&](int64_t it, f4 (&fa)[Gm::NV], f4 (&fb)[Gm::NV], const f4 (&na)[Gm::NV],
                    const f4 (&nb)[Gm::NV]) {
        const uint32_t pi = f0;
        const int64_t m_it = int64_t(pi >> 23) * mb + ((pi >> 14) & 511);
        while (out_m < m_it) {  // macro tile out_m is complete (or has no pairs)
            store_macro(out_m);
            zero_acc();
            ++out_m;
        }
        fetch(AHEAD == 1 ? f1 : f2, int((it + 2) % Gm::NCH), fa, fb);
        __syncthreads();
        if ((pi >> wave) & 1) compute(int(it & 1));
        if (it + 1 < nitems) commit(int((it + 1) & 1), na, nb);
        if ((it + 1) % Gm::NCH == 0) {
            f0 = f1;
            f1 = f2;
            f2 = produce();
        }
    };
    zero_acc();
    if (nitems > 0) {
        fetch(f0, 0, ra0, rb0);
        if (Gm::NCH == 1)
            fetch(f1, 0, ra1, rb1);
        else
            fetch(f0, 1, ra1, rb1);
        commit(0, ra0, rb0);
    }
    for (int64_t it = 0; it < nitems; it += 2) {
        step(it, ra0, rb0, ra1, rb1);
        if (it + 1 >= nitems) break;
        step(it + 1, ra1, rb1, ra0, rb0);
    }
    while (out_m < m_end) {
        store_macro(out_m);
        zero_acc();
        ++out_m;
    }
}

}  // namespace spamm
