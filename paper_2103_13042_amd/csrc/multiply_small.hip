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
//    tiles, in ascending order, form the union list, whose entry u goes to
//    k-group u mod 4; wave 0 adds the number of kept pairs to the pair counter;
//  * step s stages in LDS, for every k-group, the four operand tiles of the
//    group's s-th entry (A rows of tile rows 2I, 2I+1 and B columns of tile
//    columns 2J, 2J+1 at that k), each of the group's waves loading one tile
//    (one no kept product reads is skipped), the next step's loads in flight
//    during this step's MFMAs; wave (g, q) multiplies tile q's product from
//    LDS when tile q keeps the entry's k, so each wave accumulates its entries
//    in ascending k;
//  * the four k-groups' partial tiles are added in group order through LDS, so
//    the result does not depend on timing, and group 0 writes C (zero for a
//    tile with no kept pair).
// Staging each operand tile once per block and reading it from LDS, instead
// of every wave reading its own operands from global memory into registers,
// took the kernel at N = 1024 from 21.3 to 18.6 us: the operand loads, not the
// MFMAs, bound it.
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

// LDS staging: per k-group and step, the four operand tiles of the group's
// entry (A rows 2I, 2I+1 and B columns 2J, 2J+1 at that k), one tile loaded
// by each of the group's four waves; two steps in flight.  A tiles: rows of
// 32 floats, 16-byte chunks XOR-swizzled by the row; B tiles: rows of 32
// floats with rows 16..31 moved 32 floats on, so the two lane halves of an
// MFMA operand read fall in different banks.
constexpr int kSmallTileFloats = 32 * 32 + 32;

__global__ __launch_bounds__(kSmallWaves * 64, 1) void multiply_small_kernel(
    const float* __restrict__ A, const float* __restrict__ B, float* __restrict__ C, int64_t n, int64_t bdim,
    int64_t mb, const double* __restrict__ na, const double* __restrict__ nb, int64_t ld, double tau,
    unsigned long long* __restrict__ pairs) {
    constexpr int L = kSmallLeaf;
    __shared__ __attribute__((aligned(16))) float stage[2][kSmallGroups][4][kSmallTileFloats];
    static_assert(sizeof(stage) >= sizeof(float) * (kSmallGroups - 1) * 4 * 16 * 64, "reduction area");
    float (*red)[4][16][64] = reinterpret_cast<float (*)[4][16][64]>(&stage[0][0][0][0]);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int grp = wave >> 2, q = (wave + grp) & 3, wa = q >> 1, wb = q & 1, role = wave & 3;
    const int ir = lane & 31, g = lane >> 5;
    const int64_t m = blockIdx.x;
    const int64_t I = m / mb, J = m - (m / mb) * mb;

    // the threshold test, lane k, by every wave (no barrier between the test
    // and the staging): mem = the tiles of the block that keep k; the union
    // k-list in ascending order is dealt to the k-groups round-robin
    uint32_t mem = 0;
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
#pragma unroll
        for (int ab = 0; ab < 4; ++ab) {
            const bool in = k < bdim && 2 * I + (ab >> 1) < bdim && 2 * J + (ab & 1) < bdim;
            if (in && nav[ab >> 1] * nbv[ab & 1] >= tau) mem |= 1u << ab;
        }
        if (wave == 0) {
            int cnt = __popc(mem);
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) cnt += __shfl_xor(cnt, o);
            if (lane == 0 && cnt) atomicAdd(pairs, static_cast<unsigned long long>(cnt));
        }
    }
    const uint64_t bal = __ballot(mem != 0);
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const int rank = __popcll(bal & below);
    const int nunion = __popcll(bal);
    const int steps = (nunion + kSmallGroups - 1) / kSmallGroups;
    // entry of k-group grp at step s: the union entry of rank kSmallGroups*s + grp
    auto entry_k = [&](int s) -> int {
        const uint64_t sel = __ballot(((bal >> lane) & 1) && rank == kSmallGroups * s + grp);
        return sel ? __builtin_ctzll(sel) : -1;
    };

    // this wave's operand tile of a step: role 0, 1: A rows of tile row
    // 2I + role; role 2, 3: B columns of tile column 2J + role - 2; chunk
    // e = lane + 64 v holds row e >> 3, columns 4 (e & 7) .. + 3
    const f4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
    f4 stg[4];
    auto fetch = [&](int s) {
        const int k = entry_k(s);
        const uint32_t mk = k >= 0 ? uint32_t(__shfl(int(mem), k)) : 0u;
        const uint32_t need = role == 0 ? 3u : role == 1 ? 12u : role == 2 ? 5u : 10u;
        const bool any = (mk & need) != 0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int e = lane + 64 * v, r = e >> 3, c4 = e & 7;
            int64_t row, col;
            if (role < 2) {
                row = (2 * I + role) * L + r;
                col = int64_t(k) * L + 4 * c4;
            } else {
                row = int64_t(k) * L + r;
                col = (2 * J + role - 2) * L + 4 * c4;
            }
            const bool in = any && row < n && col < n;
            const f4 x = *reinterpret_cast<const f4*>((role < 2 ? A : B) + (in ? row * n + col : 0));
            stg[v] = in ? x : zero;
        }
    };
    auto commit = [&](int s) {
        float* t = stage[s & 1][grp][role];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int e = lane + 64 * v, r = e >> 3, c4 = e & 7;
            const int at = role < 2 ? r * 32 + 4 * (c4 ^ (r & 7)) : r * 32 + (r >= 16 ? 32 : 0) + 4 * c4;
            *reinterpret_cast<f4*>(t + at) = stg[v];
        }
    };
    f16v acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    // lane (ir, g) supplies k = 16 g + u of MFMA step u: A[ir][16g + u], B[16g + u][ir]
    auto compute = [&](int s) {
        const int k = entry_k(s);
        if (k < 0) return;
        const uint32_t mk = uint32_t(__shfl(int(mem), k));
        if (!((mk >> q) & 1)) return;
        const float* ta = stage[s & 1][grp][wa];
        const float* tb = stage[s & 1][grp][2 + wb] + 16 * g * 32 + (g ? 32 : 0) + ir;
        f4 av[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) av[v] = *reinterpret_cast<const f4*>(ta + ir * 32 + 4 * ((4 * g + v) ^ (ir & 7)));
#pragma unroll
        for (int u = 0; u < 16; ++u) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[u >> 2][u & 3], tb[u * 32], acc, 0, 0, 0);
    };

    if (steps > 0) {
        fetch(0);
        commit(0);
    }
    __syncthreads();
    for (int s = 0; s < steps; ++s) {
        if (s + 1 < steps) fetch(s + 1);  // in flight during this step's MFMAs
        compute(s);
        if (s + 1 < steps) commit(s + 1);  // the stage step s-1 used; every wave is past it
        __syncthreads();
    }

    // partial tiles of groups 1.. through LDS (the stages are free), added in group order
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
    const int64_t bcol = tj * L + ir;
    if (ti >= bdim || tj >= bdim || bcol >= n) return;
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
