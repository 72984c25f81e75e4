// gfx950 kernels of the SpAMM hot path.
//
//   leaf_sumsq_*      Frobenius norms of every leaf tile (Eq. 2), FP64 sums
//   pyramid_kernel    quadtree of node norms (Eq. 1), bottom-up, FP64
//   plan_*            norm-product tests (Algorithm 1 / Algorithm 2's bitmap),
//                     ballot bitmaps, scan, compaction into ascending k-lists
//   (in multiply)     cost-balanced static partition of output tiles
//   multiply_kernel   FP32 MFMA products of the kept leaf pairs into C
//
// Wave size is 64 throughout.
#include <hip/hip_runtime.h>

#include "device.h"
#include "dma.h"
#include "internal.h"
#include "macro.h"

namespace spamm {

// --------------------------------------------------------------------------
// Leaf norms.  A block of 256 threads reads a strip of `leaf` rows by 1024
// columns; each thread owns 4 adjacent columns and sums their squares down the
// strip in FP64 (an FP32 square is exact in FP64), then the leaf/4 threads of
// one tile combine their sums with an xor butterfly.  Rows are read as whole
// 4 KiB segments per block, so the pass streams HBM at full coalescing.

constexpr int kNormThreads = 256;
constexpr int kNormCols = kNormThreads * 4;

// strip `strip` (tile row) x column chunk `chunk` of x; tile (strip, tj) goes to
// sumsq / norms[strip * ld + tj] (either may be null)
// NT: nontemporal loads, for a pass whose input is larger than the
// infinity cache: A and B are read once here, and keeping them out of the
// caches leaves room for the multiply's tiles (measured on the N = 8192 step:
// norm pass 112 -> 90 us, multiply unchanged).  Below that size the multiply
// profits from what the pass leaves in the cache (batch of small products:
// 2 % slower with NT).
template <bool NT, typename T>
__device__ __forceinline__ T load_nt(const T* p) {
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

template <int LEAF, bool VEC, bool NT = false>
__device__ __forceinline__ void leaf_sumsq_strip(const float* __restrict__ x, int64_t n, int64_t bdim, int64_t strip,
                                                 int64_t chunk, double* sumsq, double* norms, int64_t ld) {
    constexpr int G = LEAF / 4;  // threads per tile
    const int64_t r0 = strip * LEAF;
    const int64_t r1 = r0 + LEAF < n ? r0 + LEAF : n;
    const int t = threadIdx.x;
    if (VEC) {  // rows 16-byte aligned (n % 4 == 0): columns 4t .. 4t+3 of the chunk
        const int64_t col = chunk * kNormCols + 4 * t;
        double acc0 = 0.0, acc1 = 0.0;
        if (col < n) {
            const float* p = x + r0 * n + col;
            int64_t r = r0;
#pragma unroll 4
            for (; r + 1 < r1; r += 2) {
                f4 v = load_nt<NT>(reinterpret_cast<const f4*>(p));
                f4 w = load_nt<NT>(reinterpret_cast<const f4*>(p + n));
                p += 2 * n;
                acc0 += double(v.x) * double(v.x) + double(v.y) * double(v.y);
                acc1 += double(v.z) * double(v.z) + double(v.w) * double(v.w);
                acc0 += double(w.x) * double(w.x) + double(w.y) * double(w.y);
                acc1 += double(w.z) * double(w.z) + double(w.w) * double(w.w);
            }
            if (r < r1) {
                f4 v = load_nt<NT>(reinterpret_cast<const f4*>(p));
                acc0 += double(v.x) * double(v.x) + double(v.y) * double(v.y);
                acc1 += double(v.z) * double(v.z) + double(v.w) * double(v.w);
            }
        }
        double s = acc0 + acc1;
#pragma unroll
        for (int off = 1; off < G; off <<= 1) s += __shfl_xor(s, off);
        const int64_t tj = col / LEAF;
        if ((t % G) == 0 && tj < bdim) {
            const int64_t i = strip * ld + tj;
            if (sumsq) sumsq[i] = s;
            if (norms) norms[i] = sqrt(s);
        }
        return;
    }
    // Rows not 16-byte aligned (n % 4 != 0, or x itself only 4-byte aligned):
    // 16-byte loads at aligned positions, counted from xa, the 16-byte
    // boundary at or below x (xoff floats before it, inside the same
    // allocation since allocations are at least 16-byte aligned).  In row r
    // the chunk starts s = (xoff + r n + cb) mod 4 elements past such a
    // position, so thread t's load holds columns 4t - s .. 4t - s + 3 of the
    // chunk: those below the thread's own tile (first thread of a tile, s > 0)
    // belong to the tile before it, those below 0 to the previous chunk (which
    // loads them with its last thread's second load, below).  A load that
    // would reach past the end of the matrix is done element-wise.
    const int xoff = int((reinterpret_cast<uintptr_t>(x) >> 2) & 3);
    const float* xa = x - xoff;
    const int64_t cb = chunk * kNormCols, nn = n * n, end = nn + xoff;  // end: counted from xa
    const int lim = int(n - cb < kNormCols ? n - cb : kNormCols);  // columns of this chunk
    const int home = (4 * t) / LEAF * LEAF;  // first column of the thread's tile
    double acc_home = 0.0, acc_prev = 0.0;
    auto add = [&](int64_t q, int c0) {  // the 4 elements at xa[q ..] = columns c0 .. c0+3
        if (c0 + 3 < 0 || c0 >= lim) return;
        float v[4];
        if (q + 4 <= end) {
            const f4 w = *reinterpret_cast<const f4*>(xa + q);
            v[0] = w.x;
            v[1] = w.y;
            v[2] = w.z;
            v[3] = w.w;
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = (q + e < end) ? xa[q + e] : 0.0f;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int c = c0 + e;
            if (c >= 0 && c < lim) {
                const double d = double(v[e]);
                if (c < home)
                    acc_prev += d * d;
                else
                    acc_home += d * d;
            }
        }
    };
    // rows whose loads all end inside the matrix (r n + cb + kNormCols + 4 <=
    // n^2): unconditional loads, the chunk's columns picked by a select
    const int64_t room = nn - cb - kNormCols - 4;
    int64_t r_fast = room < 0 ? r0 : room / n + 1;
    r_fast = r_fast < r0 ? r0 : (r_fast > r1 ? r1 : r_fast);
    auto take = [&](const f4& w, int c0) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int c = c0 + e;
            const double d = (c >= 0 && c < lim) ? double(w[e]) : 0.0;
            if (c < home)
                acc_prev += d * d;
            else
                acc_home += d * d;
        }
    };
#pragma unroll 4
    for (int64_t r = r0; r < r_fast; ++r) {
        const int64_t base = xoff + r * n + cb;
        const int s = int(base & 3);
        take(load_nt<NT>(reinterpret_cast<const f4*>(xa + base - s + 4 * t)), 4 * t - s);
    }
    if (t == kNormThreads - 1) {  // the chunk's last s columns of those rows
        for (int64_t r = r0; r < r_fast; ++r) {
            const int64_t base = xoff + r * n + cb;
            const int s = int(base & 3);
            if (s > 0) take(*reinterpret_cast<const f4*>(xa + base - s + kNormCols), kNormCols - s);
        }
    }
    for (int64_t r = r_fast; r < r1; ++r) {  // the matrix's last rows: guarded loads
        const int64_t base = xoff + r * n + cb;
        const int s = int(base & 3);
        const int64_t a0 = base - s;
        add(a0 + 4 * t, 4 * t - s);
        if (t == kNormThreads - 1 && s > 0) add(a0 + kNormCols, kNormCols - s);
    }
    double s = acc_home;
#pragma unroll
    for (int off = 1; off < G; off <<= 1) s += __shfl_xor(s, off);
    __shared__ double prev[kNormThreads];  // per tile of the chunk: its part held by the next tile's first thread
    if ((t % G) == 0) prev[t / G] = acc_prev;
    __syncthreads();
    if ((t % G) == 0) {
        const int g = t / G;
        if (g + 1 < kNormThreads / G) s += prev[g + 1];
        const int64_t tj = cb / LEAF + g;
        if (tj < bdim) {
            const int64_t i = strip * ld + tj;
            if (sumsq) sumsq[i] = s;
            if (norms) norms[i] = sqrt(s);
        }
    }
    __syncthreads();  // prev is reused by the block's next strip
}

// words the first block of a norm pass sets to zero (a pair counter, the
// look-back state of the plan that follows)
__device__ __forceinline__ void clear_words(const NormJob& job) {
    if (job.clear && (blockIdx.x | blockIdx.y | blockIdx.z) == 0) {
        const int64_t cnt = job.clear_count > 0 ? job.clear_count : 1;
        for (int64_t e = threadIdx.x; e < cnt; e += blockDim.x) job.clear[e] = 0;
    }
}

// Grid (strip, column chunk, matrix), strips fastest: blocks dispatched
// together read 4 KiB row segments of different strips (2 MiB apart at
// N = 8192), which streams faster than neighbouring chunks of one strip
// (N = 8192, A and B: 83 against 92 us).
template <int LEAF, bool VEC, bool NT>
__global__ __launch_bounds__(kNormThreads) void leaf_sumsq_kernel(NormJob job, int64_t n, int64_t bdim) {
    const int m = blockIdx.z;
    clear_words(job);
    leaf_sumsq_strip<LEAF, VEC, NT>(job.x[m], n, bdim, blockIdx.x, blockIdx.y, job.sumsq[m], job.norms[m], job.ld);
}

// Small matrices (too few strips to fill the GPU with the kernel above): 1024
// threads per strip x 1024-column chunk, four row groups of LEAF/4 rows whose
// loads are all in flight at once; the four partial sums of a column group
// are added in row-group order through LDS, then across the tile's threads.
// Rows 16-byte aligned (n % 4 == 0, x 16-byte aligned).
constexpr int kNormSmallThreads = 1024;

template <int LEAF>
__global__ __launch_bounds__(kNormSmallThreads) void leaf_sumsq_small_kernel(NormJob job, int64_t n, int64_t bdim) {
    constexpr int G = LEAF / 4;           // threads per tile (4 columns each)
    constexpr int RPG = LEAF / 4;         // rows per row group
    __shared__ double part[3][kNormCols / 4];
    const int m = blockIdx.z;
    clear_words(job);
    const float* __restrict__ x = job.x[m];
    const int t = threadIdx.x, cg = t & 255, rg = t >> 8;
    const int64_t strip = blockIdx.y, col = int64_t(blockIdx.x) * kNormCols + 4 * cg;
    const int64_t r0 = strip * LEAF + rg * RPG;
    double acc = 0.0;
    if (col < n) {
        f4 v[RPG];
#pragma unroll
        for (int r = 0; r < RPG; ++r) {
            const int64_t row = r0 + r;
            v[r] = row < n ? *reinterpret_cast<const f4*>(x + row * n + col) : f4{0.0f, 0.0f, 0.0f, 0.0f};
        }
        double a0 = 0.0, a1 = 0.0;
#pragma unroll
        for (int r = 0; r < RPG; ++r) {
            a0 += double(v[r].x) * double(v[r].x) + double(v[r].y) * double(v[r].y);
            a1 += double(v[r].z) * double(v[r].z) + double(v[r].w) * double(v[r].w);
        }
        acc = a0 + a1;
    }
    if (rg > 0) part[rg - 1][cg] = acc;
    __syncthreads();
    if (rg != 0) return;
    double s = ((acc + part[0][cg]) + part[1][cg]) + part[2][cg];
#pragma unroll
    for (int off = 1; off < G; off <<= 1) s += __shfl_xor(s, off);
    const int64_t tj = col / LEAF;
    if ((cg % G) == 0 && col < n && tj < bdim) {
        const int64_t i = strip * job.ld + tj;
        if (job.sumsq[m]) job.sumsq[m][i] = s;
        if (job.norms[m]) job.norms[m][i] = sqrt(s);
    }
}

// Any other leaf size: one block per tile, strided over its elements.
__global__ __launch_bounds__(kNormThreads) void leaf_sumsq_generic_kernel(NormJob job, int64_t n, int64_t bdim,
                                                                          int32_t leaf) {
    __shared__ double partial[kNormThreads / 64];
    const int m = blockIdx.z;
    clear_words(job);
    const float* __restrict__ x = job.x[m];
    const int64_t ti = blockIdx.y, tj = blockIdx.x;
    const int64_t rows = (ti * leaf + leaf < n ? leaf : n - ti * leaf);
    const int64_t cols = (tj * leaf + leaf < n ? leaf : n - tj * leaf);
    double acc = 0.0;
    for (int64_t e = threadIdx.x; e < rows * cols; e += kNormThreads) {
        const int64_t r = ti * leaf + e / cols, c = tj * leaf + e % cols;
        const double v = double(x[r * n + c]);
        acc += v * v;
    }
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0) partial[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kNormThreads / 64; ++w) s += partial[w];
        const int64_t t = ti * job.ld + tj;
        if (job.sumsq[m]) job.sumsq[m][t] = s;
        if (job.norms[m]) job.norms[m][t] = sqrt(s);
    }
}

constexpr double kInfinityCacheBytes = 256.0 * 1024 * 1024;  // MI355X's last-level cache
constexpr int64_t kSmallNormBlocks = 256;                      // one block per CU

template <int LEAF>
static hipError_t launch_leaf_fixed(const NormJob& job, int nmat, int64_t n, int64_t bdim, bool vec,
                                    hipStream_t s) {
    dim3 grid(unsigned((n + kNormCols - 1) / kNormCols), unsigned(bdim), unsigned(nmat));
    const bool nt = 4.0 * double(n) * double(n) * nmat > kInfinityCacheBytes;
    if constexpr (LEAF == 16 || LEAF == 32 || LEAF == 64) {
        // fewer blocks than CUs: the four-row-group form keeps more loads in flight
        if (vec && int64_t(grid.x) * grid.y * grid.z < kSmallNormBlocks) {
            leaf_sumsq_small_kernel<LEAF><<<grid, kNormSmallThreads, 0, s>>>(job, n, bdim);
            return hipGetLastError();
        }
    }
    const dim3 sgrid(grid.y, grid.x, grid.z);  // strips fastest
    if (vec && nt)
        leaf_sumsq_kernel<LEAF, true, true><<<sgrid, kNormThreads, 0, s>>>(job, n, bdim);
    else if (vec)
        leaf_sumsq_kernel<LEAF, true, false><<<sgrid, kNormThreads, 0, s>>>(job, n, bdim);
    else if (nt)
        leaf_sumsq_kernel<LEAF, false, true><<<sgrid, kNormThreads, 0, s>>>(job, n, bdim);
    else
        leaf_sumsq_kernel<LEAF, false, false><<<sgrid, kNormThreads, 0, s>>>(job, n, bdim);
    return hipGetLastError();
}

hipError_t launch_leaf_norms(const NormJob& job, int nmat, int64_t n, int32_t leaf, bool vec, hipStream_t s) {
    const int64_t bdim = (n + leaf - 1) / leaf;
    switch (leaf) {
        case 16: return launch_leaf_fixed<16>(job, nmat, n, bdim, vec, s);
        case 32: return launch_leaf_fixed<32>(job, nmat, n, bdim, vec, s);
        case 64: return launch_leaf_fixed<64>(job, nmat, n, bdim, vec, s);
        case 128: return launch_leaf_fixed<128>(job, nmat, n, bdim, vec, s);
        case 256: return launch_leaf_fixed<256>(job, nmat, n, bdim, vec, s);
        default: break;
    }
    dim3 grid{unsigned(bdim), unsigned(bdim), unsigned(nmat)};
    leaf_sumsq_generic_kernel<<<grid, kNormThreads, 0, s>>>(job, n, bdim, leaf);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// Pyramid.  One block per matrix walks the levels bottom-up.  A parent's
// sum of squares is (s00 + s01) + (s10 + s11) of its children: sums of
// non-negative FP64 values round monotonically, so a parent is never below any
// child, and neither is its square root.  That is what lets the plan drop a
// whole range of k on a parent's test without ever dropping a pair that the
// leaf test keeps.

constexpr int kPyrThreads = 1024;
constexpr int kPyrLdsTop = 6;                        // highest level kept in LDS
constexpr int kPyrLdsLevel = 1 << (2 * kPyrLdsTop);  // its node count

__device__ __forceinline__ void pyramid_build(double* __restrict__ sp, double* __restrict__ np, int64_t bdim,
                                              int lv) {
    const int64_t side = int64_t(1) << lv;
    if (bdim < side) {  // padding tiles of the leaf level: norm 0
        const int64_t base = level_offset(lv);
        for (int64_t idx = threadIdx.x; idx < side * side; idx += kPyrThreads) {
            const int64_t i = idx >> lv, j = idx & (side - 1);
            if (i >= bdim || j >= bdim) {
                sp[base + idx] = 0.0;
                np[base + idx] = 0.0;
            }
        }
    }
    // levels of at most kPyrLdsLevel nodes (l <= 6) are also kept in LDS, in
    // buffer l & 1, so the levels above the first such one read their children
    // there instead of waiting on the global writes of the level below
    __shared__ double lvl0[kPyrLdsLevel];      // levels 6, 4, 2, 0
    __shared__ double lvl1[kPyrLdsLevel / 4];  // levels 5, 3, 1
    for (int l = lv - 1; l >= 0; --l) {
        __syncthreads();
        const int64_t w = int64_t(1) << l, cw = 2 * w;
        const int64_t base = level_offset(l), cbase = level_offset(l + 1);
        // the leaf level (l + 1 == lv) is only in global memory
        const bool from_lds = l + 1 <= kPyrLdsTop && l + 1 < lv, to_lds = l <= kPyrLdsTop;
        const double* src = from_lds ? ((l + 1) & 1 ? lvl1 : lvl0) : sp + cbase;
        double* dst = (l & 1) ? lvl1 : lvl0;
#pragma unroll 4
        for (int64_t idx = threadIdx.x; idx < w * w; idx += kPyrThreads) {
            const int64_t i = idx >> l, j = idx & (w - 1);
            const double* c0 = src + (2 * i) * cw + 2 * j;
            const double* c1 = c0 + cw;
            const double v = (c0[0] + c0[1]) + (c1[0] + c1[1]);
            sp[base + idx] = v;
            np[base + idx] = sqrt(v);
            if (to_lds) dst[idx] = v;
        }
    }
}

__global__ __launch_bounds__(kPyrThreads) void pyramid_kernel(PyramidJob job, int64_t bdim, int lv) {
    pyramid_build(job.spyr[blockIdx.x], job.pyr[blockIdx.x], bdim, lv);
}

hipError_t launch_pyramid(const PyramidJob& job, int nmat, int64_t bdim, int lv, hipStream_t s) {
    pyramid_kernel<<<nmat, kPyrThreads, 0, s>>>(job, bdim, lv);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// Plan.  Block (jb, i) owns the 64 output tiles (i, 64*jb .. 64*jb+63) and
// walks k in chunks of 64.  A chunk is one pyramid node of 64 x 64 leaf tiles
// (level Lv-6) on each side; when that node product is below tau every leaf
// product in the chunk is too (a node norm bounds the norms below it), so the
// chunk is settled for all 64 tiles at once (uniform branch).  Otherwise the
// chunk's 64 x 64 block of B leaf norms is staged in LDS, each lane takes one
// k, and one ballot per tile gives the 64-bit bitmap of selected k.
//
// SKIPPED selects the complement: the triples whose product is below tau, the
// pairs SpAMM drops (their product sum is the error matrix AB - SpAMM).

constexpr int kPlanThreads = 256;

template <bool MASKS, bool SKIPPED>
__device__ __forceinline__ void plan_mask_block(const double* __restrict__ pyr_a, const double* __restrict__ pyr_b,
                                                int64_t bdim, int lv, double tau, uint64_t* __restrict__ masks,
                                                int32_t* __restrict__ counts, int32_t* __restrict__ block_sums,
                                                int64_t jb, int64_t i) {
    __shared__ double sb[64][65];
    __shared__ int wsum[kPlanThreads / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t j0 = jb * 64;
    const int64_t side = int64_t(1) << lv;
    const int nw = int((bdim + 63) / 64);
    const double* la = pyr_a + level_offset(lv);
    const double* lb = pyr_b + level_offset(lv);
    int cnt[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) cnt[u] = 0;
    for (int c = 0; c < nw; ++c) {
        bool below;
        if (lv >= 6) {
            const int lc = lv - 6;
            const int64_t w = int64_t(1) << lc;
            below = !(pyr_a[level_offset(lc) + (i >> 6) * w + c] * pyr_b[level_offset(lc) + int64_t(c) * w + (j0 >> 6)] >=
                      tau);
        } else {
            below = !(pyr_a[0] * pyr_b[0] >= tau);
        }
        if (below) {
            // every real triple of the chunk is dropped: none selected, or all
            // of them in the complement
            const int64_t k = int64_t(c) * 64 + lane;
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int64_t j = j0 + wave + 4 * u;
                const uint64_t mk = SKIPPED ? __ballot(k < bdim && j < bdim) : 0ull;
                if (MASKS && lane == 0 && j < bdim) masks[(i * bdim + j) * nw + c] = mk;
                cnt[u] += __popcll(mk);
            }
            continue;
        }
        // stage the chunk's 64 x 64 B norms: all loads first, then the LDS writes
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = threadIdx.x + u * kPlanThreads;
            const int64_t k = int64_t(c) * 64 + (e >> 6), j = j0 + (e & 63);
            v[u] = (k < side && j < side) ? lb[k * side + j] : 0.0;
        }
        const int64_t k = int64_t(c) * 64 + lane;
        const double a = k < side ? la[i * side + k] : 0.0;
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = threadIdx.x + u * kPlanThreads;
            sb[e >> 6][e & 63] = v[u];
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int jj = wave + 4 * u;
            const int64_t j = j0 + jj;
            const double p = a * sb[lane][jj];
            const bool bit = (SKIPPED ? !(p >= tau) : (p >= tau)) && (k < bdim) && (j < bdim);
            const uint64_t mk = __ballot(bit);
            if (MASKS && lane == 0 && j < bdim) masks[(i * bdim + j) * nw + c] = mk;
            cnt[u] += __popcll(mk);
        }
    }
    int tot = 0;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int64_t j = j0 + wave + 4 * u;
        if (j < bdim) {
            if (MASKS && lane == 0) counts[i * bdim + j] = cnt[u];
            tot += cnt[u];
        }
    }
    if (lane == 0) wsum[wave] = tot;
    __syncthreads();
    if (threadIdx.x == 0) block_sums[i * nw + jb] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

template <bool MASKS, bool SKIPPED>
__global__ __launch_bounds__(kPlanThreads) void plan_mask_kernel(const double* __restrict__ pyr_a,
                                                                 const double* __restrict__ pyr_b, int64_t bdim,
                                                                 int lv, double tau, uint64_t* __restrict__ masks,
                                                                 int32_t* __restrict__ counts,
                                                                 int32_t* __restrict__ block_sums) {
    plan_mask_block<MASKS, SKIPPED>(pyr_a, pyr_b, bdim, lv, tau, masks, counts, block_sums, blockIdx.x, blockIdx.y);
}

hipError_t launch_plan_mask(const double* pyr_a, const double* pyr_b, int64_t bdim, int lv, double tau, bool skipped,
                            uint64_t* masks, int32_t* counts, int32_t* block_sums, hipStream_t s) {
    dim3 grid{unsigned((bdim + 63) / 64), unsigned(bdim), 1u};
    if (skipped)
        plan_mask_kernel<true, true><<<grid, kPlanThreads, 0, s>>>(pyr_a, pyr_b, bdim, lv, tau, masks, counts,
                                                                   block_sums);
    else
        plan_mask_kernel<true, false><<<grid, kPlanThreads, 0, s>>>(pyr_a, pyr_b, bdim, lv, tau, masks, counts,
                                                                    block_sums);
    return hipGetLastError();
}

hipError_t launch_plan_count(const double* pyr_a, const double* pyr_b, int64_t bdim, int lv, double tau,
                             int32_t* block_sums, hipStream_t s) {
    dim3 grid{unsigned((bdim + 63) / 64), unsigned(bdim), 1u};
    plan_mask_kernel<false, false><<<grid, kPlanThreads, 0, s>>>(pyr_a, pyr_b, bdim, lv, tau, nullptr, nullptr,
                                                                 block_sums);
    return hipGetLastError();
}

// Mean of nA[i,k] * nB[k,j] over all leaf triples of the bdim^3 grid, as
// sum_k (sum_i nA[i,k]) (sum_j nB[k,j]) / bdim^3 (one block; FP64; fixed order).
constexpr int kAveThreads = 1024;

__global__ __launch_bounds__(kAveThreads) void mean_norm_product_kernel(const double* __restrict__ pyr_a,
                                                                        const double* __restrict__ pyr_b,
                                                                        int64_t bdim, int lv, double* __restrict__ out) {
    __shared__ double wsum[kAveThreads / 64];
    const int64_t side = int64_t(1) << lv;
    const double* la = pyr_a + level_offset(lv);
    const double* lb = pyr_b + level_offset(lv);
    double part = 0.0;
    for (int64_t k = threadIdx.x; k < bdim; k += kAveThreads) {
        double ca = 0.0, rb = 0.0;
        for (int64_t i = 0; i < bdim; ++i) ca += la[i * side + k];
        for (int64_t j = 0; j < bdim; ++j) rb += lb[k * side + j];
        part += ca * rb;
    }
    for (int o = 32; o >= 1; o >>= 1) part += __shfl_xor(part, o);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int w = 0; w < kAveThreads / 64; ++w) tot += wsum[w];
        *out = tot / (double(bdim) * double(bdim) * double(bdim));
    }
}

hipError_t launch_mean_norm_product(const double* pyr_a, const double* pyr_b, int64_t bdim, int lv, double* out,
                                    hipStream_t s) {
    mean_norm_product_kernel<<<1, kAveThreads, 0, s>>>(pyr_a, pyr_b, bdim, lv, out);
    return hipGetLastError();
}

// Exclusive scan of the block sums (one per 64 output tiles): one block, each
// thread a contiguous segment, wave scans with shuffles, then across waves.
constexpr int kScanThreads = 256;

__device__ __forceinline__ void plan_scan_block(const int32_t* __restrict__ block_sums, int64_t nb,
                                                int32_t* block_offsets, int32_t* offsets, int64_t nt,
                                                int64_t* __restrict__ pairs) {
    __shared__ int64_t wsum[kScanThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t seg = (nb + kScanThreads - 1) / kScanThreads;
    const int64_t b = tid * seg, e = (b + seg < nb ? b + seg : nb);
    int64_t local = 0;
    for (int64_t t = b; t < e; ++t) local += block_sums[t];
    int64_t incl = local;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int64_t up = __shfl_up(incl, off);
        if (lane >= off) incl += up;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int64_t run = incl - local;
    for (int w = 0; w < wave; ++w) run += wsum[w];
    if (block_offsets) {
        for (int64_t t = b; t < e; ++t) {
            block_offsets[t] = int32_t(run);
            run += block_sums[t];
        }
    }
    if (tid == kScanThreads - 1) {
        int64_t total = 0;
        for (int w = 0; w < kScanThreads / 64; ++w) total += wsum[w];
        if (offsets) offsets[nt] = int32_t(total);
        if (pairs) *pairs = total;
    }
}

__global__ __launch_bounds__(kScanThreads) void plan_scan_kernel(const int32_t* __restrict__ block_sums,
                                                                 int64_t nb, int32_t* block_offsets,
                                                                 int32_t* offsets, int64_t nt,
                                                                 int64_t* __restrict__ pairs) {
    plan_scan_block(block_sums, nb, block_offsets, offsets, nt, pairs);
}

hipError_t launch_plan_scan(const int32_t* block_sums, int64_t nblocks, int32_t* block_offsets, int32_t* offsets,
                            int64_t ntiles, int64_t* pairs, hipStream_t s) {
    plan_scan_kernel<<<1, kScanThreads, 0, s>>>(block_sums, nblocks, block_offsets, offsets, ntiles, pairs);
    return hipGetLastError();
}

// One wave per output tile t = (i, j): its offset is the offset of its block
// of 64 tiles plus the counts of the tiles before it in the block (a masked
// wave sum); then every lane whose bit is set writes its k at the offset plus
// the number of set bits below it (ascending k).
__device__ __forceinline__ void plan_fill_wave(const uint64_t* __restrict__ masks, const int32_t* __restrict__ counts,
                                               const int32_t* __restrict__ block_offsets, int64_t bdim,
                                               int32_t* __restrict__ offsets, int32_t* __restrict__ klist,
                                               int64_t t) {
    const int lane = threadIdx.x & 63;
    const int nw = int((bdim + 63) / 64);
    const int64_t i = t / bdim, j = t % bdim, jb = j >> 6;
    const int64_t jl = (jb * 64 + lane < bdim) ? jb * 64 + lane : -1;  // the block's tile for this lane
    int before = (jl >= 0 && (jl & 63) < (j & 63)) ? counts[i * bdim + jl] : 0;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) before += __shfl_xor(before, off);
    int64_t base = int64_t(block_offsets[i * nw + jb]) + before;
    if (lane == 0) offsets[t] = int32_t(base);
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int w = 0; w < nw; ++w) {
        const uint64_t m = masks[t * nw + w];
        if ((m >> lane) & 1ull) klist[base + __popcll(m & below)] = w * 64 + lane;
        base += __popcll(m);
    }
}

__global__ __launch_bounds__(256) void plan_fill_kernel(const uint64_t* __restrict__ masks,
                                                        const int32_t* __restrict__ counts,
                                                        const int32_t* __restrict__ block_offsets, int64_t bdim,
                                                        int32_t* __restrict__ offsets, int32_t* __restrict__ klist) {
    const int64_t t = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (t >= bdim * bdim) return;
    plan_fill_wave(masks, counts, block_offsets, bdim, offsets, klist, t);
}

hipError_t launch_plan_fill(const uint64_t* masks, const int32_t* counts, const int32_t* block_offsets,
                            int64_t bdim, int32_t* offsets, int32_t* klist, hipStream_t s) {
    const int64_t nt = bdim * bdim;
    plan_fill_kernel<<<unsigned((nt + 3) / 4), 256, 0, s>>>(masks, counts, block_offsets, bdim, offsets, klist);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// Multiply.
//
// A persistent grid of G workgroups (4 waves each).  Output tiles t = i*bdim+j
// are split into G contiguous row-major ranges of equal cost, where a tile
// costs kPairCost per kept pair plus one for writing it; the cost prefix is
// kPairCost*offsets[t] + t, so each group finds its range by binary search in
// the plan offsets.  Block ids are remapped so the groups on one XCD (ids
// congruent mod 8) own neighbouring ranges and share A/B tiles in that XCD's
// L2.
//
// A group first writes its pairs as packed (ti << 20 | tj << 10 | k) words into
// pair_scratch and streams them through a 128-entry LDS ring, refilled 64 at a
// time right after a stage commit (when no tile load is in flight), so the
// tile-load prefetch never waits on an index load.  The flat stream of (pair, k-chunk)
// items then runs through two register sets and two LDS stages: while the four
// waves multiply item it out of LDS, item it+1 sits in registers waiting to be
// stored to the other stage and the global loads of item it+2 are in flight.
// Tile loads are unconditional (out-of-range lanes read a valid address and
// select zero) so the wait before storing item it+1 leaves item it+2's loads
// outstanding.  Wave w computes
// the (w>>1, w&1) quadrant of the output tile with FP32 MFMA: 32x32x2 for
// quadrants of 32 or 64, 16x16x4 for quadrants of 16.  In MFMA step s, lane
// group g takes k = g*(KC/G) + s, so a lane reads 4 consecutive A operands
// with one 16-byte LDS load; B rows are XOR-swizzled by lane group so the G
// groups read disjoint LDS banks.  Tiles are finished in ascending k and written
// from the accumulators; tiles without pairs are written as zeros.

constexpr int kMulThreads = 256;
constexpr int kPairCost = 4;
constexpr int kIdxBits = 10;  // packed pair = ti << 20 | tj << 10 | k  (all < 1024)
constexpr int32_t kIdxMask = (1 << kIdxBits) - 1;
constexpr int kRing = 512;  // packed pairs held in LDS (a power of two)

// Tile shapes per leaf: MFMA edge, k per pipeline stage, workgroups per CU.
#ifndef SPAMM_KC64
#define SPAMM_KC64 64
#endif
#ifndef SPAMM_OCC64
#define SPAMM_OCC64 2
#endif
#ifndef SPAMM_OCC32
#define SPAMM_OCC32 2
#endif
#ifndef SPAMM_OCC128
#define SPAMM_OCC128 1
#endif
template <int LEAF>
struct MulCfg;
template <>
struct MulCfg<32> {
    static constexpr int MF = 16, KC = 32, OCC = SPAMM_OCC32;
};
template <>
struct MulCfg<64> {
    static constexpr int MF = 32, KC = SPAMM_KC64, OCC = SPAMM_OCC64;
};
template <>
struct MulCfg<128> {
    // one workgroup per CU: at two (256 registers per lane) the kernel spilled
    // to scratch, also with 16 k per stage
    static constexpr int MF = 32, KC = 32, OCC = SPAMM_OCC128;
};

template <int LEAF>
struct MulGeom {
    static constexpr int MF = MulCfg<LEAF>::MF;   // MFMA output edge
    static constexpr int KC = MulCfg<LEAF>::KC;   // k per pipeline stage
    static constexpr int QM = LEAF / 2;           // quadrant edge per wave
    static constexpr int NB = QM / MF;            // MFMA blocks per quadrant side
    static constexpr int G = 64 / MF;             // lane groups along k
    static constexpr int SPC = KC / G;            // MFMA steps per stage
    static constexpr int NCH = LEAF / KC;         // stages per leaf pair
    static constexpr int AST = KC + 4;            // A stage row stride (floats)
    static constexpr int BST = LEAF < 64 ? 64 : LEAF;  // B stage row stride (room for the swizzle)
    static constexpr int SWZ = 64 / G;            // B column swizzle unit
    static constexpr int ASZ = LEAF * AST;
    static constexpr int BSZ = KC * BST;
    static constexpr int STAGE = ASZ + BSZ;
    static constexpr int NV = LEAF * KC / 4 / kMulThreads;  // float4 per thread per operand
    static constexpr int ACC = (MF == 32 ? 16 : 4);         // accumulator floats per MFMA block
    static_assert(SPC % 4 == 0, "A reads are 4 steps wide");
    static_assert(NV >= 1 && NV * 4 * kMulThreads == LEAF * KC, "stage split");
};

template <int MF>
struct Mfma;
template <>
struct Mfma<32> {
    typedef f16v acc_t;
    static __device__ __forceinline__ acc_t step(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
    }
    // output element of accumulator register r for lane l: row, col in block
    static __device__ __forceinline__ int row(int r, int l) { return 8 * (r >> 2) + 4 * (l >> 5) + (r & 3); }
    static __device__ __forceinline__ int col(int, int l) { return l & 31; }
};
template <>
struct Mfma<16> {
    typedef f4 acc_t;
    static __device__ __forceinline__ acc_t step(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int r, int l) { return 4 * (l >> 4) + r; }
    static __device__ __forceinline__ int col(int, int l) { return l & 15; }
};

// First tile of logical group g: smallest t with (kPairCost*off[t] + t) * G >= g * total.
__device__ __forceinline__ int64_t partition_start(const int32_t* __restrict__ off, int64_t nt, int64_t g,
                                                   int64_t groups, int64_t total) {
    const int64_t target = g * total;
    int64_t lo = 0, hi = nt;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t(kPairCost) * off[mid] + mid) * groups >= target)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

// The multiply of the output tiles [t_begin, t_end) of one product, by one
// workgroup: lds holds the two staging buffers, ring the pair ring.
template <int LEAF, bool VEC>
__device__ __forceinline__ void mul_range(const float* __restrict__ A, const float* __restrict__ B,
                                          float* __restrict__ C, int64_t n, int64_t bdim,
                                          const int32_t* __restrict__ off, const int32_t* __restrict__ klist,
                                          int32_t* pairs, int64_t t_begin, int64_t t_end, float* lds,
                                          int32_t* ring) {
    using Gm = MulGeom<LEAF>;
    using M = Mfma<Gm::MF>;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int ir = lane % Gm::MF, g = lane / Gm::MF;
    const int64_t q_begin = off[t_begin], q_end = off[t_end];
    const int64_t nitems = (q_end - q_begin) * Gm::NCH;

    // packed (ti, tj, k) of every pair of the range
    for (int64_t q = q_begin + tid; q < q_end; q += kMulThreads) {
        int64_t lo = t_begin, hi = t_end - 1;  // tile of q: last t with off[t] <= q
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (off[mid] <= q)
                lo = mid;
            else
                hi = mid - 1;
        }
        const int32_t ti = int32_t(lo / bdim), tj = int32_t(lo - int64_t(ti) * bdim);
        pairs[q] = (ti << (2 * kIdxBits)) | (tj << kIdxBits) | klist[q];
    }
    __syncthreads();
    const int64_t npairs = q_end - q_begin;
    for (int e = tid; e < kRing; e += kMulThreads) ring[e] = e < npairs ? pairs[q_begin + e] : 0;
    __syncthreads();
    int64_t rbase = 0;  // ring holds pairs [rbase, rbase + kRing)
    auto pk_of_item = [&](int64_t it) -> int32_t { return ring[(it / Gm::NCH) & (kRing - 1)]; };

    typename M::acc_t acc[Gm::NB][Gm::NB];
    auto zero_acc = [&]() {
#pragma unroll
        for (int a = 0; a < Gm::NB; ++a)
#pragma unroll
            for (int b = 0; b < Gm::NB; ++b)
#pragma unroll
                for (int r = 0; r < Gm::ACC; ++r) acc[a][b][r] = 0.0f;
    };
    auto store_tile = [&](int32_t ti, int32_t tj) {
#pragma unroll
        for (int a = 0; a < Gm::NB; ++a)
#pragma unroll
            for (int b = 0; b < Gm::NB; ++b)
#pragma unroll
                for (int r = 0; r < Gm::ACC; ++r) {
                    const int64_t row = int64_t(ti) * LEAF + wr * Gm::QM + a * Gm::MF + M::row(r, lane);
                    const int64_t col = int64_t(tj) * LEAF + wc * Gm::QM + b * Gm::MF + M::col(r, lane);
                    if (row < n && col < n) C[row * n + col] = acc[a][b][r];
                }
    };

    // global -> register staging of one (pair, chunk) item; every lane issues
    // every load (clamped to a valid address) and zeroes what lies outside C.
    // Rows that are not 16-byte aligned (VEC false) are read with 16-byte
    // loads at 4-byte alignment, which global loads accept; only chunks that
    // cross the matrix's edge are read element by element
    auto fetch = [&](int32_t pk, int ch, f4 (&ra)[Gm::NV], f4 (&rb)[Gm::NV]) {
        const int64_t ti = (uint32_t(pk) >> (2 * kIdxBits)) & kIdxMask, tj = (uint32_t(pk) >> kIdxBits) & kIdxMask,
                      kt = uint32_t(pk) & kIdxMask;
        const int64_t arow0 = ti * LEAF, acol0 = kt * LEAF + ch * Gm::KC;
        const int64_t brow0 = kt * LEAF + ch * Gm::KC, bcol0 = tj * LEAF;
        const f4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int v = 0; v < Gm::NV; ++v) {
            const int e = tid + v * kMulThreads;
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
                const int r = e / (LEAF / 4), c4 = e % (LEAF / 4);
                const int64_t row = brow0 + r, col = bcol0 + 4 * c4;
                if (VEC) {
                    const bool in = row < n && col < n;
                    const f4 x = *reinterpret_cast<const f4*>(B + (in ? row * n + col : 0));
                    rb[v] = in ? x : zero;
                } else if (row < n && col + 3 < n) {
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
            const int e = tid + v * kMulThreads;
            {
                const int r = e / (Gm::KC / 4), c4 = e % (Gm::KC / 4);
                *reinterpret_cast<f4*>(sa + r * Gm::AST + 4 * c4) = ra[v];
            }
            {
                const int r = e / (LEAF / 4), c4 = e % (LEAF / 4);
                const int swz = ((r / Gm::SPC) % Gm::G) * Gm::SWZ;
                *reinterpret_cast<f4*>(sb + r * Gm::BST + ((4 * c4) ^ swz)) = rb[v];
            }
        }
    };
    auto compute = [&](int stage) {
        const float* sa = lds + stage * Gm::STAGE;
        const float* sb = sa + Gm::ASZ + g * Gm::SPC * Gm::BST;
        const int swz = g * Gm::SWZ;
#pragma unroll
        for (int q = 0; q < Gm::SPC / 4; ++q) {
            f4 av[Gm::NB];
#pragma unroll
            for (int a = 0; a < Gm::NB; ++a)
                av[a] = *reinterpret_cast<const f4*>(sa + (wr * Gm::QM + a * Gm::MF + ir) * Gm::AST + g * Gm::SPC +
                                                     4 * q);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int s = 4 * q + u;
                float bv[Gm::NB];
#pragma unroll
                for (int b = 0; b < Gm::NB; ++b)
                    bv[b] = sb[s * Gm::BST + ((wc * Gm::QM + b * Gm::MF + ir) ^ swz)];
#pragma unroll
                for (int a = 0; a < Gm::NB; ++a)
#pragma unroll
                    for (int b = 0; b < Gm::NB; ++b) acc[a][b] = M::step(av[a][u], bv[b], acc[a][b]);
            }
        }
    };

    // output tile being accumulated: linear index t, coordinates (ti, tj);
    // tiles before it are written
    int64_t t = t_begin;
    int32_t ti = int32_t(t_begin / bdim), tj = int32_t(t_begin - int64_t(ti) * bdim);
    auto advance_tile = [&]() {
        store_tile(ti, tj);
        zero_acc();
        ++t;
        if (++tj == bdim) {
            tj = 0;
            ++ti;
        }
    };
    // one item of the stream: R_free receives item it+2, R_next (item it+1)
    // goes to LDS after the multiply of item it
    f4 ra0[Gm::NV], rb0[Gm::NV], ra1[Gm::NV], rb1[Gm::NV];
    auto step = [&](int64_t it, f4 (&fa)[Gm::NV], f4 (&fb)[Gm::NV], const f4 (&na)[Gm::NV],
                    const f4 (&nb)[Gm::NV]) {
        const int32_t pk = pk_of_item(it);
        const int64_t t_it =
            int64_t((uint32_t(pk) >> (2 * kIdxBits)) & kIdxMask) * bdim + ((uint32_t(pk) >> kIdxBits) & kIdxMask);
        while (t < t_it) advance_tile();  // tile t is complete (or has no pairs)
        const int64_t i2 = it + 2 < nitems ? it + 2 : nitems - 1;  // past the end: a harmless reload
        fetch(pk_of_item(i2), int(i2 % Gm::NCH), fa, fb);
        __syncthreads();
        compute(int(it & 1));
        if (it + 1 < nitems) commit(int((it + 1) & 1), na, nb);
        // every wave is past pair (it+1)/NCH - 1: recycle the older half of the ring
        if ((it + 1) / Gm::NCH >= rbase + kRing / 2) {
            for (int e = tid; e < kRing / 2; e += kMulThreads) {
                const int64_t p = rbase + kRing + e;
                ring[(rbase + e) & (kRing - 1)] = p < npairs ? pairs[q_begin + p] : 0;
            }
            rbase += kRing / 2;
        }
    };
    zero_acc();
    if (nitems > 0) {
        fetch(pk_of_item(0), 0, ra0, rb0);
        const int64_t i1 = nitems > 1 ? 1 : 0;
        fetch(pk_of_item(i1), int(i1 % Gm::NCH), ra1, rb1);
        commit(0, ra0, rb0);
    }
    for (int64_t it = 0; it < nitems; it += 2) {
        step(it, ra0, rb0, ra1, rb1);
        if (it + 1 >= nitems) break;
        step(it + 1, ra1, rb1, ra0, rb0);
    }
    while (t < t_end) advance_tile();
}


template <int LEAF, bool VEC>
__global__ __launch_bounds__(kMulThreads, MulCfg<LEAF>::OCC) void multiply_kernel(const float* __restrict__ A,
                                                                  const float* __restrict__ B, float* __restrict__ C,
                                                                  int64_t n, int64_t bdim,
                                                                  const int32_t* __restrict__ off,
                                                                  const int32_t* __restrict__ klist,
                                                                  int32_t* pairs) {
    __shared__ __attribute__((aligned(16))) float lds[2 * MulGeom<LEAF>::STAGE];
    __shared__ int32_t ring[kRing];
    // this group's range of output tiles
    const int64_t groups = gridDim.x;
    const int64_t bid = blockIdx.x;
    const int64_t lg = (bid & 7) * (groups >> 3) + (bid >> 3);
    const int64_t nt = bdim * bdim;
    const int64_t total = int64_t(kPairCost) * off[nt] + nt;
    const int64_t t_begin = partition_start(off, nt, lg, groups, total);
    const int64_t t_end = partition_start(off, nt, lg + 1, groups, total);
    if (t_begin >= t_end) return;
    mul_range<LEAF, VEC>(A, B, C, n, bdim, off, klist, pairs, t_begin, t_end, lds, ring);
}

template <int LEAF>
static hipError_t launch_mul(const float* a, const float* b, float* c, int64_t n, int64_t bdim,
                             const int32_t* offsets, const int32_t* klist, int32_t* pair_scratch, bool vec,
                             int num_cus, hipStream_t s) {
    const int64_t nt = bdim * bdim;
    int64_t groups = int64_t(num_cus) * MulCfg<LEAF>::OCC;
    const int64_t cap = ((nt + 7) / 8) * 8;
    if (groups > cap) groups = cap;
    groups = ((groups + 7) / 8) * 8;
    static int scratch_state[2] = {0, 0};
    const hipError_t ce = vec ? check_no_scratch(multiply_kernel<LEAF, true>, &scratch_state[1])
                              : check_no_scratch(multiply_kernel<LEAF, false>, &scratch_state[0]);
    if (ce != hipSuccess) return ce;
    if (vec)
        multiply_kernel<LEAF, true>
            <<<unsigned(groups), kMulThreads, 0, s>>>(a, b, c, n, bdim, offsets, klist, pair_scratch);
    else
        multiply_kernel<LEAF, false>
            <<<unsigned(groups), kMulThreads, 0, s>>>(a, b, c, n, bdim, offsets, klist, pair_scratch);
    return hipGetLastError();
}

hipError_t launch_multiply(const float* a, const float* b, float* c, int64_t n, int32_t leaf, int64_t bdim,
                           const int32_t* offsets, const int32_t* klist, int32_t* pair_scratch, bool vec,
                           int num_cus, hipStream_t s) {
    switch (leaf) {
        case 16: return launch_multiply_leaf16(a, b, c, n, bdim, offsets, klist, vec, s);
        case 32: return launch_mul<32>(a, b, c, n, bdim, offsets, klist, pair_scratch, vec, num_cus, s);
        case 64: return launch_mul<64>(a, b, c, n, bdim, offsets, klist, pair_scratch, vec, num_cus, s);
        case 128: return launch_mul<128>(a, b, c, n, bdim, offsets, klist, pair_scratch, vec, num_cus, s);
        default: return hipErrorInvalidValue;
    }
}

// --------------------------------------------------------------------------
// Batched products.  Every stage of the path runs as one launch over all
// products (the multiply as one persistent launch per leaf class present): a
// block finds its product by binary search over the prefix of its work in the
// descriptor array, then runs the single-product code on it.

// product i's descriptor with every pointer in it marked as global memory
__device__ __forceinline__ BatchProduct product_at(const BatchProduct* __restrict__ P, int64_t i) {
    BatchProduct q = P[i];
    q.a = global_ptr(q.a);
    q.b = global_ptr(q.b);
    q.c = global_ptr(q.c);
    for (int m = 0; m < 2; ++m) {
        q.spyr[m] = global_ptr(q.spyr[m]);
        q.pyr[m] = global_ptr(q.pyr[m]);
    }
    q.masks = global_ptr(q.masks);
    q.counts = global_ptr(q.counts);
    q.bsums = global_ptr(q.bsums);
    q.boffs = global_ptr(q.boffs);
    q.offsets = global_ptr(q.offsets);
    q.klist = global_ptr(q.klist);
    q.pair_scratch = global_ptr(q.pair_scratch);
    q.pairs = global_ptr(q.pairs);
    q.mwords = global_ptr(q.mwords);
    q.mcount = global_ptr(q.mcount);
    q.mprefix = global_ptr(q.mprefix);
    q.mitems = global_ptr(q.mitems);
    return q;
}

constexpr int kFindTile = 0, kFindMask = 1, kFindNorm = 2;

__device__ __forceinline__ int32_t batch_find(const BatchProduct* __restrict__ P, int32_t count, int64_t x,
                                              int which) {
    int32_t lo = 0, hi = count - 1;  // last p with base(p) <= x
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        const int64_t base = which == kFindMask ? P[mid].mask_base
                             : which == kFindNorm ? P[mid].norm_base
                                                  : P[mid].tile_base;
        if (base <= x)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// leaf norms: one block per (tile row, 1024-column chunk) of A (blockIdx.y = 0)
// or B (1), as in the single-product pass
template <int LEAF>
__device__ __forceinline__ void batch_strip(const BatchProduct& q, int m, int64_t b) {
    const int64_t chunks = (q.n + kNormCols - 1) / kNormCols;
    const int64_t side = int64_t(1) << q.lv, at = level_offset(q.lv);
    const float* x = m == 0 ? q.a : q.b;
    double* sp = (m == 0 ? q.spyr[0] : q.spyr[1]) + at;  // selected, not indexed: q stays in registers
    double* np = (m == 0 ? q.pyr[0] : q.pyr[1]) + at;
    // chunks fastest here: with the products' strips in strips-fastest order
    // the batch's pass took 1134 against 1086 us
    if (q.vec)
        leaf_sumsq_strip<LEAF, true>(x, q.n, q.bdim, b / chunks, b % chunks, sp, np, side);
    else
        leaf_sumsq_strip<LEAF, false>(x, q.n, q.bdim, b / chunks, b % chunks, sp, np, side);
}

__global__ __launch_bounds__(kNormThreads) void batch_norms_kernel(const BatchProduct* __restrict__ P, int32_t count,
                                                                   int64_t total_strips) {
    const int m = blockIdx.y;
    for (int64_t bg = blockIdx.x; bg < total_strips; bg += gridDim.x) {
        const BatchProduct q = product_at(P, batch_find(P, count, bg, kFindNorm));
        const int64_t b = bg - q.norm_base;
        switch (q.leaf) {
            case 32: batch_strip<32>(q, m, b); break;
            case 64: batch_strip<64>(q, m, b); break;
            default: batch_strip<128>(q, m, b); break;
        }
    }
}

// The pyramid, mask, scan and fill launches plan the products with more than
// 64 tiles per side (the others have no mask blocks and no tiles in the
// prefixes; the two small-plan launches below plan them).
__global__ __launch_bounds__(kPyrThreads) void batch_pyramid_kernel(const BatchProduct* __restrict__ P) {
    const BatchProduct q = product_at(P, blockIdx.x);
    if (q.nw == 1) return;
    const bool b = blockIdx.y != 0;
    pyramid_build(b ? q.spyr[1] : q.spyr[0], b ? q.pyr[1] : q.pyr[0], q.bdim, q.lv);
}

__global__ __launch_bounds__(kPlanThreads) void batch_plan_mask_kernel(const BatchProduct* __restrict__ P,
                                                                       int32_t count, int64_t total_blocks) {
    for (int64_t bg = blockIdx.x; bg < total_blocks; bg += gridDim.x) {
        const BatchProduct q = product_at(P, batch_find(P, count, bg, kFindMask));
        const int64_t b = bg - q.mask_base;
        plan_mask_block<true, false>(q.pyr[0], q.pyr[1], q.bdim, q.lv, q.tau, q.masks, q.counts, q.bsums, b % q.nw,
                                     b / q.nw);
        __syncthreads();
    }
}

__global__ __launch_bounds__(kScanThreads) void batch_plan_scan_kernel(const BatchProduct* __restrict__ P) {
    const BatchProduct q = product_at(P, blockIdx.x);
    if (q.nw == 1) return;
    plan_scan_block(q.bsums, q.bdim * q.nw, q.boffs, q.offsets, q.bdim * q.bdim, q.pairs);
}

// Each wave takes kFillRun consecutive tiles of the batch: one search for the
// product of the first, then a forward walk over the products (in base order;
// the last of several products with the same base is the one owning the work).
constexpr int kFillRun = 8;
__global__ __launch_bounds__(256) void batch_plan_fill_kernel(const BatchProduct* __restrict__ P, int32_t count,
                                                              int64_t total_tiles) {
    for (int64_t t0 = (int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6)) * kFillRun; t0 < total_tiles;
         t0 += int64_t(gridDim.x) * 4 * kFillRun) {
        int32_t p = batch_find(P, count, t0, kFindTile);
        const int64_t t1 = t0 + kFillRun < total_tiles ? t0 + kFillRun : total_tiles;
        for (int64_t tg = t0; tg < t1; ++tg) {
            while (p + 1 < count && P[p + 1].tile_base <= tg) ++p;
            const BatchProduct q = product_at(P, p);
            plan_fill_wave(q.masks, q.counts, q.boffs, q.bdim, q.offsets, q.klist, tg - q.tile_base);
        }
    }
}

// Products with at most 64 tiles per side (one k word per tile) are planned
// by two launches over (product, group of 16 tile rows), in place of the
// pyramid, mask, scan and fill launches above, which then cover only the
// larger products.  The node tests there only skip work (a node norm bounds
// every leaf norm below it, and rounding is monotone), so the kept set is the
// same.  The test launch: wave w of group g takes tile row i = 16 g + w, B's
// leaf norms staged in LDS transposed (one tile's k column is a contiguous
// read), one ballot per tile, and writes the row's bitmaps and its pair count.
// The fill launch: each row's offset is the sum of the counts of the rows
// above it; then the row's tiles write their k in ascending order.
constexpr int kSmallPlanThreads = 1024;
constexpr int kSmallPlanRows = kSmallPlanThreads / 64;  // tile rows per workgroup
constexpr int kSmallPlanGroups = 64 / kSmallPlanRows;    // workgroups per product
constexpr int kSmallPlanPitch = 65;                      // doubles per row of the transposed B norms

__global__ __launch_bounds__(kSmallPlanThreads) void batch_plan_small_test_kernel(const BatchProduct* __restrict__ P) {
    __shared__ double sbt[64 * kSmallPlanPitch];
    const BatchProduct q = product_at(P, blockIdx.x);
    const int bdim = int(q.bdim);
    if (q.nw != 1 || int(blockIdx.y) * kSmallPlanRows >= bdim) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lv = q.lv, side = 1 << lv;
    const double tau = q.tau;
    const double* la = q.pyr[0] + level_offset(lv);
    const double* lb = q.pyr[1] + level_offset(lv);
    for (int e = tid; e < side * side; e += kSmallPlanThreads)
        sbt[(e & (side - 1)) * kSmallPlanPitch + (e >> lv)] = lb[e];
    __syncthreads();
    const int i = int(blockIdx.y) * kSmallPlanRows + wave;
    if (i >= bdim) return;
    const double a = lane < bdim ? la[i * side + lane] : 0.0;
    const bool live = lane < bdim;
    uint64_t mask = 0;
    for (int j0 = 0; j0 < bdim; j0 += 8) {
        double bv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) bv[u] = sbt[((j0 + u) & 63) * kSmallPlanPitch + lane];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (j0 + u < bdim) {
                const double p = a * bv[u];
                const uint64_t m = __ballot(live && p >= tau);
                if (lane == j0 + u) mask = m;
            }
        }
    }
    int32_t c = __popcll(mask);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o);
    if (live) q.masks[i * bdim + lane] = mask;
    if (lane == 0) q.bsums[i] = c;
}

__global__ __launch_bounds__(kSmallPlanThreads) void batch_plan_small_fill_kernel(const BatchProduct* __restrict__ P) {
    const BatchProduct q = product_at(P, blockIdx.x);
    const int bdim = int(q.bdim);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = int(blockIdx.y) * kSmallPlanRows + wave;
    if (q.nw != 1 || i >= bdim) return;
    const int32_t rs = lane < bdim ? q.bsums[lane] : 0;
    int32_t before = lane < i ? rs : 0;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) before += __shfl_xor(before, o);
    const bool live = lane < bdim;
    const uint64_t mask = live ? q.masks[i * bdim + lane] : 0ull;
    const int32_t c = __popcll(mask);
    int32_t incl = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t up = __shfl_up(incl, o);
        if (lane >= o) incl += up;
    }
    const int32_t base = before + incl - c;
    if (live) q.offsets[i * bdim + lane] = base;
    if (i == 0) {
        int32_t total = rs;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) total += __shfl_xor(total, o);
        if (lane == 0) {
            q.offsets[bdim * bdim] = total;
            *q.pairs = total;
        }
    }
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const uint32_t mlo = uint32_t(mask), mhi = uint32_t(mask >> 32);
    for (int j = 0; j < bdim; ++j) {
        const uint64_t m = uint64_t(uint32_t(__builtin_amdgcn_readlane(int(mlo), j))) |
                           (uint64_t(uint32_t(__builtin_amdgcn_readlane(int(mhi), j))) << 32);
        const int32_t at = __builtin_amdgcn_readlane(base, j);
        if ((m >> lane) & 1ull) q.klist[at + __popcll(m & below)] = lane;
    }
}

// per class, the prefix of multiply cost (kPairCost per kept pair + 1 per
// tile, as in the single-product partition) over its members, in order
// Macro-tile schedule of the leaf-32 and leaf-64 products: one wave per macro
// tile of the batch (prefix macro_base), as macro_words_kernel /
// macro_items_kernel do for one product, and one block per product for the
// prefix of union sizes.
__device__ __forceinline__ int32_t batch_find_macro(const BatchProduct* __restrict__ P, int32_t count, int64_t x) {
    int32_t lo = 0, hi = count - 1;  // last p with macro_base(p) <= x
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (P[mid].macro_base <= x)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

constexpr int kMacroRun = 4;  // consecutive macro tiles per wave (one search, then a walk)
__global__ __launch_bounds__(256) void batch_macro_words_kernel(const BatchProduct* __restrict__ P, int32_t count,
                                                                int64_t total_macros) {
    __shared__ unsigned long long sw[4][4][16];  // [wave][tile][word]
    const int wave = threadIdx.x >> 6;
    for (int64_t m0 = (int64_t(blockIdx.x) * 4 + wave) * kMacroRun; m0 < total_macros;
         m0 += int64_t(gridDim.x) * 4 * kMacroRun) {
        int32_t p = batch_find_macro(P, count, m0);
        const int64_t m1 = m0 + kMacroRun < total_macros ? m0 + kMacroRun : total_macros;
        for (int64_t gm = m0; gm < m1; ++gm) {
            while (p + 1 < count && P[p + 1].macro_base <= gm) ++p;
            const BatchProduct q = product_at(P, p);
            macro_words_wave(q.offsets, q.klist, q.bdim, q.mb, q.nw, q.mwords, q.mcount, gm - q.macro_base,
                             sw[wave]);
        }
    }
}

__global__ __launch_bounds__(kScanThreads) void batch_macro_scan_kernel(const BatchProduct* __restrict__ P) {
    const BatchProduct q = product_at(P, blockIdx.x);
    if (q.mb == 0) return;
    const int64_t nm = q.mb * q.mb;
    plan_scan_block(q.mcount, nm, q.mprefix, q.mprefix, nm, nullptr);
}

__global__ __launch_bounds__(256) void batch_macro_items_kernel(const BatchProduct* __restrict__ P, int32_t count,
                                                                int64_t total_macros) {
    const int wave = threadIdx.x >> 6;
    for (int64_t m0 = (int64_t(blockIdx.x) * 4 + wave) * kMacroRun; m0 < total_macros;
         m0 += int64_t(gridDim.x) * 4 * kMacroRun) {
        int32_t p = batch_find_macro(P, count, m0);
        const int64_t m1 = m0 + kMacroRun < total_macros ? m0 + kMacroRun : total_macros;
        for (int64_t gm = m0; gm < m1; ++gm) {
            while (p + 1 < count && P[p + 1].macro_base <= gm) ++p;
            const BatchProduct q = product_at(P, p);
            macro_items_wave(q.mwords, q.mprefix, q.mb, q.nw, q.mitems, gm - q.macro_base);
        }
    }
}

// Cost prefix of each leaf class over its products: leaf 32 runs on macro
// tiles (kUnionCost per union k + kMacroWrite per macro tile, as the
// single-product macro kernel), leaf 64 and 128 on single tiles (kPairCost
// per pair + 1 per tile).  One workgroup; each class's members (contiguous in
// `members`) are scanned in chunks of kCostThreads.
constexpr int kCostThreads = 1024;
__global__ __launch_bounds__(kCostThreads) void batch_cost_kernel(BatchProduct* __restrict__ P,
                                                                  const int32_t* __restrict__ members, int32_t c0,
                                                                  int32_t c1, int32_t c2,
                                                                  int64_t* __restrict__ class_total) {
    __shared__ int64_t wsum[kCostThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int32_t cnt[kBatchClasses] = {c0, c1, c2};
    int32_t first = 0;
    for (int c = 0; c < kBatchClasses; ++c) {
        int64_t carry = 0;
        for (int32_t start = 0; start < cnt[c]; start += kCostThreads) {
            const int32_t k = start + tid;
            int64_t cost = 0;
            const int32_t idx = k < cnt[c] ? members[first + k] : -1;
            if (idx >= 0) {
                const BatchProduct q = product_at(P, idx);
                if (q.mb > 0) {
                    const int64_t nm = q.mb * q.mb;
                    cost = int64_t(kUnionCost) * q.mprefix[nm] + int64_t(kMacroWrite) * nm;
                } else {
                    cost = int64_t(kPairCost) * (*q.pairs) + q.bdim * q.bdim;
                }
            }
            int64_t incl = cost;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int64_t up = __shfl_up(incl, o);
                if (lane >= o) incl += up;
            }
            if (lane == 63) wsum[wave] = incl;
            __syncthreads();
            int64_t before = carry;
            for (int w = 0; w < wave; ++w) before += wsum[w];
            if (idx >= 0) P[idx].cost_base = before + incl - cost;
            int64_t chunk = 0;
            for (int w = 0; w < kCostThreads / 64; ++w) chunk += wsum[w];
            __syncthreads();
            carry += chunk;
        }
        if (tid == 0) class_total[c] = carry;
        first += cnt[c];
    }
}

// first macro tile m of product q whose cost position reaches g * total / groups
__device__ __forceinline__ int64_t batch_macro_partition(const BatchProduct& q, int64_t g, int64_t groups,
                                                         int64_t total) {
    const int64_t target = g * total, nm = q.mb * q.mb;
    int64_t lo = 0, hi = nm;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((q.cost_base + int64_t(kUnionCost) * q.mprefix[mid] + int64_t(kMacroWrite) * mid) * groups >= target)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

// Leaf 32 and 64: a persistent grid over the class's macro tiles (all its
// products in turn), each workgroup a contiguous range of equal cost.  Three
// workgroups per CU: the kernel holds both the aligned and the unaligned form
// of the macro-tile multiply, and at four per CU (128 registers per lane) it
// spilled to scratch.
constexpr int kBatchMacOcc = 3;

template <int LEAF>
__global__ __launch_bounds__(kMacThreads, kBatchMacOcc) void multiply_batch_macro_kernel(
    const BatchProduct* __restrict__ P, const int32_t* __restrict__ members, int32_t nmem,
    const int64_t* __restrict__ class_total, int cls) {
    __shared__ __attribute__((aligned(16))) float lds[2 * MacGeom<LEAF>::STAGE];
    const int64_t groups = gridDim.x;
    const int64_t bid = blockIdx.x;
    const int64_t lg = (bid & 7) * (groups >> 3) + (bid >> 3);
    const int64_t total = class_total[cls];
    int32_t lo = 0, hi = nmem - 1;  // last member with cost_base * groups <= lg * total
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (P[members[mid]].cost_base * groups <= lg * total)
            lo = mid;
        else
            hi = mid - 1;
    }
    for (int32_t k = lo; k < nmem; ++k) {
        const BatchProduct q = product_at(P, members[k]);
        if (q.cost_base * groups >= (lg + 1) * total) break;
        const int64_t m0 = batch_macro_partition(q, lg, groups, total);
        const int64_t m1 = batch_macro_partition(q, lg + 1, groups, total);
        if (m0 >= m1) continue;
        if (q.vec)
            macro_range<LEAF, true>(q.a, q.b, q.c, q.n, q.bdim, q.mb, q.mitems, q.mprefix, m0, m1, lds);
        else
            macro_range<LEAF, false>(q.a, q.b, q.c, q.n, q.bdim, q.mb, q.mitems, q.mprefix, m0, m1, lds);
        __syncthreads();
    }
}

// first tile t of product q whose cost position reaches target / groups
__device__ __forceinline__ int64_t batch_partition(const BatchProduct& q, int64_t g, int64_t groups, int64_t total) {
    const int64_t target = g * total, nt = q.bdim * q.bdim;
    int64_t lo = 0, hi = nt;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((q.cost_base + int64_t(kPairCost) * q.offsets[mid] + mid) * groups >= target)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

template <int LEAF>
__global__ __launch_bounds__(kMulThreads, MulCfg<LEAF>::OCC) void multiply_batch_kernel(
    const BatchProduct* __restrict__ P, const int32_t* __restrict__ members, int32_t nmem,
    const int64_t* __restrict__ class_total, int cls) {
    __shared__ __attribute__((aligned(16))) float lds[2 * MulGeom<LEAF>::STAGE];
    __shared__ int32_t ring[kRing];
    const int64_t groups = gridDim.x;
    const int64_t bid = blockIdx.x;
    const int64_t lg = (bid & 7) * (groups >> 3) + (bid >> 3);
    const int64_t total = class_total[cls];
    // members whose cost range meets [lg, lg + 1) * total / groups
    int32_t lo = 0, hi = nmem - 1;  // last member with cost_base * groups <= lg * total
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (P[members[mid]].cost_base * groups <= lg * total)
            lo = mid;
        else
            hi = mid - 1;
    }
    for (int32_t k = lo; k < nmem; ++k) {
        const BatchProduct q = product_at(P, members[k]);
        if (q.cost_base * groups >= (lg + 1) * total) break;
        const int64_t t0 = batch_partition(q, lg, groups, total), t1 = batch_partition(q, lg + 1, groups, total);
        if (t0 >= t1) continue;
        if (q.vec)
            mul_range<LEAF, true>(q.a, q.b, q.c, q.n, q.bdim, q.offsets, q.klist, q.pair_scratch, t0, t1, lds, ring);
        else
            mul_range<LEAF, false>(q.a, q.b, q.c, q.n, q.bdim, q.offsets, q.klist, q.pair_scratch, t0, t1, lds,
                                   ring);
        __syncthreads();
    }
}

hipError_t launch_batch(const BatchProduct* prods, int32_t count, const int32_t* members,
                        const int32_t* class_count_host, int64_t* class_total, int64_t total_tiles,
                        int64_t total_mask_blocks, int64_t total_strips, int64_t total_macros, int32_t small_count,
                        int num_cus, hipStream_t s) {
    auto blocks = [](int64_t work, int64_t cap) { return unsigned(work < cap ? (work > 0 ? work : 1) : cap); };
    batch_norms_kernel<<<dim3{blocks(total_strips, 1 << 20), 2u, 1u}, kNormThreads, 0, s>>>(prods, count,
                                                                                           total_strips);
    if (total_mask_blocks > 0) {
        batch_pyramid_kernel<<<dim3{unsigned(count), 2u, 1u}, kPyrThreads, 0, s>>>(prods);
        batch_plan_mask_kernel<<<blocks(total_mask_blocks, 1 << 20), kPlanThreads, 0, s>>>(prods, count,
                                                                                           total_mask_blocks);
        batch_plan_scan_kernel<<<unsigned(count), kScanThreads, 0, s>>>(prods);
        batch_plan_fill_kernel<<<blocks((total_tiles + 4 * kFillRun - 1) / (4 * kFillRun), 1 << 20), 256, 0, s>>>(
            prods, count, total_tiles);
    }
    if (small_count > 0) {
        const dim3 grid{unsigned(count), unsigned(kSmallPlanGroups), 1u};
        batch_plan_small_test_kernel<<<grid, kSmallPlanThreads, 0, s>>>(prods);
        batch_plan_small_fill_kernel<<<grid, kSmallPlanThreads, 0, s>>>(prods);
    }
    if (total_macros > 0) {
        const unsigned mblocks = blocks((total_macros + 4 * kMacroRun - 1) / (4 * kMacroRun), 1 << 20);
        batch_macro_words_kernel<<<mblocks, 256, 0, s>>>(prods, count, total_macros);
        batch_macro_scan_kernel<<<unsigned(count), kScanThreads, 0, s>>>(prods);
        batch_macro_items_kernel<<<mblocks, 256, 0, s>>>(prods, count, total_macros);
    }
    batch_cost_kernel<<<1, kCostThreads, 0, s>>>(const_cast<BatchProduct*>(prods), members, class_count_host[0],
                                       class_count_host[1], class_count_host[2], class_total);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    static int scratch_state[3] = {0, 0, 0};
    if ((e = check_no_scratch(multiply_batch_macro_kernel<32>, &scratch_state[0])) != hipSuccess ||
        (e = check_no_scratch(multiply_batch_kernel<64>, &scratch_state[1])) != hipSuccess ||
        (e = check_no_scratch(multiply_batch_kernel<128>, &scratch_state[2])) != hipSuccess)
        return e;
    int32_t first = 0;
    for (int c = 0; c < kBatchClasses; ++c) {
        const int32_t nmem = class_count_host[c];
        if (nmem > 0) {
            const unsigned groups = unsigned(num_cus * (c == 1 ? MulCfg<64>::OCC : MulCfg<128>::OCC));
            switch (c) {
                case 0:
                    multiply_batch_macro_kernel<32><<<unsigned(num_cus * kBatchMacOcc), kMacThreads, 0, s>>>(
                        prods, members + first, nmem, class_total, c);
                    break;
                case 1:
                    multiply_batch_kernel<64><<<groups, kMulThreads, 0, s>>>(prods, members + first, nmem,
                                                                             class_total, c);
                    break;
                default:
                    multiply_batch_kernel<128><<<groups, kMulThreads, 0, s>>>(prods, members + first, nmem,
                                                                              class_total, c);
                    break;
            }
        }
        first += nmem;
    }
    return hipGetLastError();
}

}  // namespace spamm
