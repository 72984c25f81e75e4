// Reduced-precision operands for the leaf products.
//
// bf16:  every element rounded to bfloat16 (round to nearest even).
// f16x3: per matrix one power-of-two scale s = 2^e, e = 15 - ceil(log2 M) with
//        M the largest leaf-tile Frobenius norm (so |s x| <= M s <= 2^15, inside
//        the FP16 range); hi = fp16(s x), lo = fp16(s x - hi), both round to
//        nearest even (s x and s x - hi are exact in FP32).
//
// A keeps its row-major layout; B is written transposed (Bt[j][k] = B[k][j])
// so that both MFMA operands read k-contiguous rows.  Both are HBM-bound
// streaming passes: 4 B read and 2 B (bf16) or 4 B (f16x3) written per element.
#include <hip/hip_runtime.h>

#include <cmath>

#include "device.h"
#include "internal.h"

namespace spamm {

// e per matrix from the leaf level of its pyramid: the largest leaf norm of A
// and of B (grid-wide maximum of non-negative doubles through their bit
// patterns, which order like unsigned integers), then e from it.
__global__ void split_scale_init_kernel(unsigned long long* __restrict__ mx) {
    if (threadIdx.x < 2) mx[threadIdx.x] = 0ull;
}

__global__ __launch_bounds__(256) void split_max_kernel(const double* __restrict__ pyr_a,
                                                        const double* __restrict__ pyr_b, int64_t bdim, int lv,
                                                        unsigned long long* __restrict__ mx) {
    const int64_t side = int64_t(1) << lv;
    const int m = blockIdx.y;
    const double* leaf = (m == 0 ? pyr_a : pyr_b) + level_offset(lv);
    double v = 0.0;
    for (int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x; t < bdim * bdim; t += int64_t(gridDim.x) * 256)
        v = fmax(v, leaf[(t / bdim) * side + t % bdim]);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    if ((threadIdx.x & 63) == 0) atomicMax(&mx[m], static_cast<unsigned long long>(__double_as_longlong(v)));
}

__global__ void split_scale_kernel(const unsigned long long* __restrict__ mx, int32_t* __restrict__ exps) {
    if (threadIdx.x < 2) {
        const double m = __longlong_as_double(static_cast<long long>(mx[threadIdx.x]));
        int e = 0;
        if (m > 0.0) {
            int x = 0;
            const double f = frexp(m, &x);  // m = f 2^x, f in [0.5, 1)
            e = 15 - (f == 0.5 ? x - 1 : x);
        }
        exps[threadIdx.x] = e;
    }
}

template <int MODE>
struct Conv;

template <>
struct Conv<kPrecBf16> {
    static __device__ __forceinline__ void run(float x, float, uint16_t* hi, uint16_t*) {
        const __bf16 h = static_cast<__bf16>(x);
        *hi = __builtin_bit_cast(uint16_t, h);
    }
};

template <>
struct Conv<kPrecF16x3> {
    static __device__ __forceinline__ void run(float x, float s, uint16_t* hi, uint16_t* lo) {
        const float y = x * s;  // exact: s is a power of two
        const _Float16 h = static_cast<_Float16>(y);
        const _Float16 l = static_cast<_Float16>(y - static_cast<float>(h));
        *hi = __builtin_bit_cast(uint16_t, h);
        *lo = __builtin_bit_cast(uint16_t, l);
    }
};

// A: row-major, 4 elements per thread per step (n % 4 == 0)
template <int MODE>
__global__ __launch_bounds__(256) void split_rows_kernel(const float* __restrict__ x, int64_t count,
                                                         const int32_t* __restrict__ exps, uint16_t* __restrict__ hi,
                                                         uint16_t* __restrict__ lo, PairGate gate) {
    if (!gate_open(gate)) return;
    const float s = MODE == kPrecF16x3 ? ldexpf(1.0f, exps[0]) : 1.0f;
    const int64_t n4 = count / 4;
    const f4* x4 = reinterpret_cast<const f4*>(x);
    for (int64_t q = int64_t(blockIdx.x) * 256 + threadIdx.x; q < n4; q += int64_t(gridDim.x) * 256) {
        const f4 v = x4[q];
        uint16_t h[4], l[4] = {0, 0, 0, 0};
#pragma unroll
        for (int i = 0; i < 4; ++i) Conv<MODE>::run(v[i], s, &h[i], &l[i]);
        const uint64_t hp = uint64_t(h[0]) | uint64_t(h[1]) << 16 | uint64_t(h[2]) << 32 | uint64_t(h[3]) << 48;
        reinterpret_cast<uint64_t*>(hi)[q] = hp;
        if (MODE == kPrecF16x3) {
            const uint64_t lp = uint64_t(l[0]) | uint64_t(l[1]) << 16 | uint64_t(l[2]) << 32 | uint64_t(l[3]) << 48;
            reinterpret_cast<uint64_t*>(lo)[q] = lp;
        }
    }
}

// B transposed, one 64 x 64 tile per block through LDS (n % 64 == 0):
// read rows of B coalesced, write rows of Bt (= columns of B) coalesced.
template <int MODE>
__global__ __launch_bounds__(256) void split_transpose_kernel(const float* __restrict__ x, int64_t n,
                                                              const int32_t* __restrict__ exps,
                                                              uint16_t* __restrict__ hi, uint16_t* __restrict__ lo,
                                                              PairGate gate) {
    if (!gate_open(gate)) return;
    __shared__ float t[64][65];
    const float s = MODE == kPrecF16x3 ? ldexpf(1.0f, exps[1]) : 1.0f;
    const int64_t r0 = int64_t(blockIdx.y) * 64, c0 = int64_t(blockIdx.x) * 64;
    const int tid = threadIdx.x;
#pragma unroll
    for (int u = 0; u < 4; ++u) {  // 64 rows x 16 float4
        const int e = tid + 256 * u, r = e >> 4, c4 = e & 15;
        const f4 v = *reinterpret_cast<const f4*>(x + (r0 + r) * n + c0 + 4 * c4);
#pragma unroll
        for (int i = 0; i < 4; ++i) t[r][4 * c4 + i] = v[i];
    }
    __syncthreads();
    // Bt row j = c0 + jj holds B[r0 .. r0+63][c0 + jj]: 64 halves = 8 chunks of 8
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int e = tid + 256 * u, jj = e >> 3, ch = e & 7;
        uint16_t h[8], l[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            l[i] = 0;
            Conv<MODE>::run(t[8 * ch + i][jj], s, &h[i], &l[i]);
        }
        uint4 hp, lp;
        hp.x = h[0] | uint32_t(h[1]) << 16;
        hp.y = h[2] | uint32_t(h[3]) << 16;
        hp.z = h[4] | uint32_t(h[5]) << 16;
        hp.w = h[6] | uint32_t(h[7]) << 16;
        const int64_t off = (c0 + jj) * n + r0 + 8 * ch;
        *reinterpret_cast<uint4*>(hi + off) = hp;
        if (MODE == kPrecF16x3) {
            lp.x = l[0] | uint32_t(l[1]) << 16;
            lp.y = l[2] | uint32_t(l[3]) << 16;
            lp.z = l[4] | uint32_t(l[5]) << 16;
            lp.w = l[6] | uint32_t(l[7]) << 16;
            *reinterpret_cast<uint4*>(lo + off) = lp;
        }
    }
}

hipError_t launch_split_scales(int64_t bdim, int lv, const double* pyr_a, const double* pyr_b, int32_t* header,
                               hipStream_t s) {
    // the header holds exps[2] (bytes 0..7) and the two maxima (bytes 8..23)
    unsigned long long* mx = reinterpret_cast<unsigned long long*>(header + 2);
    split_scale_init_kernel<<<1, 64, 0, s>>>(mx);
    const int64_t tiles = bdim * bdim;
    const unsigned blocks = unsigned(tiles < 64 * 256 ? (tiles + 255) / 256 : 64);
    split_max_kernel<<<dim3{blocks, 2u, 1u}, 256, 0, s>>>(pyr_a, pyr_b, bdim, lv, mx);
    split_scale_kernel<<<1, 64, 0, s>>>(mx, header);
    return hipGetLastError();
}

hipError_t launch_split_planes(const float* a, const float* b, int64_t n, int precision, const SplitLayout& L,
                               const PairGate& gate, hipStream_t s) {
    const int64_t n4 = n * n / 4;
    const unsigned rows_grid = unsigned(n4 < 2048 * 256 ? (n4 + 255) / 256 : 2048);
    const dim3 tgrid{unsigned(n / 64), unsigned(n / 64), 1u};
    if (precision == kPrecBf16) {
        split_rows_kernel<kPrecBf16><<<rows_grid, 256, 0, s>>>(a, n * n, L.exps, L.a_hi, nullptr, gate);
        split_transpose_kernel<kPrecBf16><<<tgrid, 256, 0, s>>>(b, n, L.exps, L.bt_hi, nullptr, gate);
    } else {
        split_rows_kernel<kPrecF16x3><<<rows_grid, 256, 0, s>>>(a, n * n, L.exps, L.a_hi, L.a_lo, gate);
        split_transpose_kernel<kPrecF16x3><<<tgrid, 256, 0, s>>>(b, n, L.exps, L.bt_hi, L.bt_lo, gate);
    }
    return hipGetLastError();
}

hipError_t launch_split(const float* a, const float* b, int64_t n, int64_t bdim, int lv, const double* pyr_a,
                        const double* pyr_b, int precision, const SplitLayout& L, hipStream_t s) {
    hipError_t e = launch_split_scales(bdim, lv, pyr_a, pyr_b, L.exps, s);
    if (e != hipSuccess) return e;
    return launch_split_planes(a, b, n, precision, L, PairGate{}, s);
}

}  // namespace spamm
