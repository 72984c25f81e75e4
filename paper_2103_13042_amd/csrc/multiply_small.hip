// Small products (leaf 32, at most 64 tiles per side): the threshold test of
// Algorithm 1 and the multiply of the kept pairs in one launch after the leaf
// norm pass, instead of the pyramid, plan, schedule and multiply launches of
// the general path.  At these sizes every launch of the general path is a few
// microseconds of ramp and drain for well under a microsecond of work, and
// the multiply has too few macro tiles to give every SIMD more than one wave.
//
// One workgroup per 2x2 block of output tiles (macro tile (I, J)), sixteen
// waves in four k-groups of four (wave w: k-group g = w >> 2, output tile
// q = 2a+b = (w + g) & 3, so the four waves w, w+4, w+8, w+12 that share a
// SIMD hold the four different tiles and every SIMD gets a quarter of each
// tile's entries, whichever tiles keep more k):
//  * every wave tests, lane k for every k < bdim, the four products
//    nA[2I+a][k] * nB[k][2J+b] >= tau (the comparison of the plan kernel, on the
//    same leaf norms, so the kept pairs are the same; the pyramid only skips
//    subtrees whose leaf products all fail); the k kept by any of the four
//    tiles, in ascending order, form the union list, and k-group g takes its
//    entries g, g+4, g+8, ...; wave 0 adds the number of kept pairs to the
//    pair counter;
//  * wave 4g+q multiplies the entries of its k-group that tile q keeps, with
//    operands read from global memory (L2) straight into MFMA operand
//    registers, the next entry's loads issued before the current entry's MFMAs;
//  * the four k-groups' partial tiles are added in group order through LDS, so
//    the result does not depend on timing, and group 0 writes C (zero for a
//    tile with no kept pair).
#include <hip/hip_runtime.h>

#include "device.h"
#include "dma.h"
#include "internal.h"

namespace spamm {

namespace {
constexpr int kSmallLeaf = 32;
constexpr int kSmallWaves = 16;
constexpr int kSmallGroups = kSmallWaves / 4;
}  // namespace

__global__ __launch_bounds__(kSmallWaves * 64, 1) void multiply_small_kernel(
    const float* __restrict__ A, const float* __restrict__ B, float* __restrict__ C, int64_t n, int64_t bdim,
    int64_t mb, const double* __restrict__ na, const double* __restrict__ nb, int64_t ld, double tau,
    unsigned long long* __restrict__ pairs) {
    constexpr int L = kSmallLeaf;
    __shared__ float red[kSmallGroups - 1][4][16][64];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int grp = wave >> 2, q = (wave + grp) & 3, wa = q >> 1, wb = q & 1;
    const int ir = lane & 31, g = lane >> 5;
    const int64_t m = blockIdx.x;
    const int64_t I = m / mb, J = m - (m / mb) * mb;

    // Every wave tests lane k's four products itself (the same few norms for
    // all waves of the block, read from L2), so no barrier separates the test
    // from the multiply.  u = the position of k in the union k-list; the wave
    // takes the k its tile keeps whose position is grp modulo the group count.
    uint64_t todo;
    {
        const int k = lane;
        const int64_t kc = k < bdim ? k : bdim - 1;
        double nav[2], nbv[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int64_t ti = 2 * I + h < bdim ? 2 * I + h : bdim - 1;
            const int64_t tj = 2 * J + h < bdim ? 2 * J + h : bdim - 1;
            nav[h] = na[ti * ld + kc];
            nbv[h] = nb[kc * ld + tj];
        }
        uint32_t mem = 0;
#pragma unroll
        for (int ab = 0; ab < 4; ++ab) {
            const bool in = k < bdim && 2 * I + (ab >> 1) < bdim && 2 * J + (ab & 1) < bdim;
            if (in && nav[ab >> 1] * nbv[ab & 1] >= tau) mem |= 1u << ab;
        }
        const uint64_t bal = __ballot(mem != 0);
        const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
        const int u = __popcll(bal & below);
        todo = __ballot(((mem >> q) & 1) && (u % kSmallGroups) == grp);
        if (wave == 0) {
            int cnt = __popc(mem);
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) cnt += __shfl_xor(cnt, o);
            if (lane == 0 && cnt) atomicAdd(pairs, static_cast<unsigned long long>(cnt));
        }
    }

    // this wave's operands: A rows of output tile row 2I+wa, B columns of tile
    // column 2J+wb; lane (ir, g) holds k = 16g + s of MFMA step s
    const int64_t arow = (2 * I + wa) * L + ir, bcol = (2 * J + wb) * L + ir;
    const bool arow_in = arow < n, bcol_in = bcol < n;
    const f4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
    auto load = [&](int kt, f4 (&ra)[4], float (&rb)[16]) __attribute__((always_inline)) {
        const int64_t k0 = int64_t(kt) * L + 16 * g;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t col = k0 + 4 * v;
            const bool in = arow_in && col < n;
            const f4 x = *reinterpret_cast<const f4*>(A + (in ? arow * n + col : 0));
            ra[v] = in ? x : zero;
        }
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const int64_t row = k0 + s;
            const bool in = bcol_in && row < n;
            const float x = B[in ? row * n + bcol : 0];
            rb[s] = in ? x : 0.0f;
        }
    };
    f16v acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    auto mma = [&](const f4 (&ra)[4], const float (&rb)[16]) __attribute__((always_inline)) {
#pragma unroll
        for (int s = 0; s < 16; ++s) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(ra[s >> 2][s & 3], rb[s], acc, 0, 0, 0);
    };

    f4 ra0[4], ra1[4];
    float rb0[16], rb1[16];
    // the wave's k values in ascending order (bits of todo), one ahead
    auto pop = [&]() __attribute__((always_inline)) {
        const int kt = __builtin_ctzll(todo);
        todo &= todo - 1;
        return kt;
    };
    if (todo) {
        load(pop(), ra0, rb0);
        while (true) {
            const bool more1 = todo != 0;
            if (more1) load(pop(), ra1, rb1);
            mma(ra0, rb0);
            if (!more1) break;
            const bool more2 = todo != 0;
            if (more2) load(pop(), ra0, rb0);
            mma(ra1, rb1);
            if (!more2) break;
        }
    }

    // partial tiles of groups 1.. through LDS, added in group order
    if (grp > 0) {
#pragma unroll
        for (int r = 0; r < 16; ++r) red[grp - 1][q][r][lane] = acc[r];
    }
    __syncthreads();
    if (grp != 0) return;
#pragma unroll
    for (int h = 0; h < kSmallGroups - 1; ++h)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] += red[h][q][r][lane];
    const int64_t ti = 2 * I + wa, tj = 2 * J + wb;
    if (ti >= bdim || tj >= bdim || !bcol_in) return;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int64_t row = ti * L + 8 * (r >> 2) + 4 * g + (r & 3);
        if (row < n) C[row * n + bcol] = acc[r];
    }
}

hipError_t launch_small_multiply(const float* a, const float* b, float* c, int64_t n, int64_t bdim,
                                 const double* na, const double* nb, int64_t ld, double tau, int64_t* pairs,
                                 hipStream_t s) {
    if (bdim < 1 || bdim > kSmallMaxBdim || n > bdim * kSmallLeaf || n % 4 != 0) return hipErrorInvalidValue;
    const int64_t mb = (bdim + 1) / 2;
    static int scratch_state = 0;
    const hipError_t ce = check_no_scratch(multiply_small_kernel, &scratch_state);
    if (ce != hipSuccess) return ce;
    multiply_small_kernel<<<unsigned(mb * mb), kSmallWaves * 64, 0, s>>>(
        a, b, c, n, bdim, mb, na, nb, ld, tau, reinterpret_cast<unsigned long long*>(pairs));
    return hipGetLastError();
}

}  // namespace spamm
