// The pruning plan and the macro-tile schedule of the multiply in one launch
// (leaf 32 and 64): the work of plan_mask, plan_scan, plan_fill (the bitmap,
// map_offset and validNum of Algorithm 2, and Algorithm 1's norm tests) and of
// macro_words, its scan and macro_items (the union k-lists of 2x2 blocks of
// output tiles that the multiply streams, section 3.5.1's balanced work
// split reads their prefix), with identical outputs.  Every triple is tested
// on the leaf norms: the plan kernel's node tests on the pyramid only skip
// work (a node norm bounds every leaf norm below it, and rounding is
// monotone), and at these grid sizes building the pyramid for them cost more
// than they saved, so the pyramid above the leaf level is not needed here.
//
// One workgroup of sixteen waves per macro-tile row I (output tile rows 2I
// and 2I+1), taken in order of a ticket so that every lower row's workgroup
// has started; grids of up to 256 tiles per side, so that the row pair's
// bitmaps stay in LDS:
//  1. the tests: per (64-column block, k-chunk of 64), B's leaf norms staged
//     in LDS, one ballot per (tile, chunk)
//     gives the bitmap of kept k (kept in LDS); per tile the count V, per
//     macro tile the size of the union of its four bitmaps;
//  2. the row's two sums (kept pairs, union entries) are combined with those
//     of the rows before it by a decoupled look-back: each row publishes its
//     sums, then its inclusive prefix, in one 64-bit word per row written and
//     read with device-scope atomics (the payload is the word itself, so no
//     other memory needs to be made visible across XCDs); one wave reads 64
//     predecessors' words at a time;
//  3. offsets and the ascending k-lists of the row's tiles, the union prefix
//     and packed items of its macro tiles.
// The look-back words and the ticket must be zero before the launch (the
// leaf norm pass clears them).
#include <hip/hip_runtime.h>

#include "device.h"
#include "internal.h"
#include "macro.h"

namespace spamm {

namespace {
constexpr int kPmThreads = 1024;
constexpr int kPmWaves = kPmThreads / 64;
constexpr int64_t kPmMaxBdim = kPlanMacroMaxBdim;
constexpr int kPmMaxNw = int(kPmMaxBdim / 64);
constexpr uint32_t kPmMaxSpins = 1u << 22;

// look-back word: state in bits 62-63 (1: the row's own sums, 2: inclusive
// prefix), kept pairs in bits 31-61, union entries in bits 0-30
constexpr unsigned long long kStAgg = 1ull << 62, kStIncl = 2ull << 62;
constexpr unsigned long long kField = (1ull << 31) - 1;

__device__ __forceinline__ unsigned long long pack_sums(unsigned long long pairs, unsigned long long uni) {
    return (pairs << 31) | uni;
}

__device__ __forceinline__ unsigned long long atomic_load_agent(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void atomic_store_agent(unsigned long long* p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A workgroup barrier that orders LDS accesses only: unlike __syncthreads it
// does not wait for this wave's global loads, so a prefetch stays in flight.
__device__ __forceinline__ void lds_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}
}  // namespace

// la, lb: leaf norms of A and B, row stride `side`
__global__ __launch_bounds__(kPmThreads) void plan_macro_kernel(const double* __restrict__ la,
                                                                const double* __restrict__ lb, int64_t side,
                                                                int64_t bdim, double tau, PlanMacroOut o) {
    __shared__ double sb[64][65];                         // B leaf norms of a chunk: [k][j]
    __shared__ uint64_t smask[2][kPmMaxBdim][kPmMaxNw];   // bitmaps of the row pair's tiles
    __shared__ int32_t tcount[2][kPmMaxBdim];             // V of the row pair's tiles
    __shared__ int32_t ucnt[kPmMaxBdim / 2];              // union sizes of the row's macro tiles
    __shared__ int64_t wsum[2][kPmWaves];
    __shared__ unsigned long long s_excl;
    __shared__ int64_t s_row;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) s_row = atomicAdd(o.ticket, 1u);
    const int64_t mb = (bdim + 1) / 2, nm = mb * mb;
    const int nw = int((bdim + 63) / 64);
    __syncthreads();
    const int64_t I = s_row;
    if (I >= mb) return;       // only if the ticket was not cleared before the launch
    const int64_t r0 = 2 * I;  // tile rows r0 and r0 + 1 (the latter may lie outside the grid)

    // ---- 1. tests, bitmaps, counts: every (column block jb, k-chunk c), the
    // norms of the next one loaded while this one is tested
    const int nit = nw * nw;
    // this thread's four entries of a chunk's B norms, and the A norms of
    // rows r0 and r0 + 1 at lane's k
    double vb[4], va[2];
    auto fetch = [&](int it) {
        const int64_t jb = it / nw, c = it - (it / nw) * nw;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = tid + u * kPmThreads;
            const int64_t k = c * 64 + (e >> 6), j = jb * 64 + (e & 63);
            vb[u] = (k < side && j < side) ? lb[k * side + j] : 0.0;
        }
        const int64_t k = c * 64 + lane;
        va[0] = k < side ? la[r0 * side + k] : 0.0;
        va[1] = (k < side && r0 + 1 < side) ? la[(r0 + 1) * side + k] : 0.0;
    };
    fetch(0);
    for (int64_t jb = 0; jb < nw; ++jb) {
        // wave w: macro columns J = 32 jb + w + 16 u (u = 0, 1) of this column block
        int cnt[2][4], uc[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            uc[u] = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) cnt[u][q] = 0;
        }
        for (int c = 0; c < nw; ++c) {
            const int it = int(jb) * nw + c;
            const double a0 = va[0], a1 = va[1];
            lds_barrier();  // every wave is done with the previous chunk's norms
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = tid + u * kPmThreads;
                sb[e >> 6][e & 63] = vb[u];
            }
            lds_barrier();
            if (it + 1 < nit) fetch(it + 1);  // in flight during this chunk's tests
            const int64_t k = int64_t(c) * 64 + lane;
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int jj = 2 * (wave + 16 * u);  // first tile column of the macro column, in the block
                uint64_t uni = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int h = q >> 1, bcol = q & 1;
                    const int64_t r = r0 + h, j = jb * 64 + jj + bcol;
                    const double p = (h ? a1 : a0) * sb[lane][jj + bcol];
                    const uint64_t mk = __ballot(p >= tau && k < bdim && r < bdim && j < bdim);
                    if (lane == 0 && j < bdim) smask[h][j][c] = mk;
                    cnt[u][q] += __popcll(mk);
                    uni |= mk;
                }
                uc[u] += __popcll(uni);
            }
        }
        if (lane == 0) {
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int64_t J = jb * 32 + wave + 16 * u;
                if (J < mb) ucnt[J] = uc[u];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t j = 2 * J + (q & 1);
                    if (j < bdim) tcount[q >> 1][j] = cnt[u][q];
                }
            }
        }
    }
    __syncthreads();

    // ---- 2. the row's sums, then the look-back over the rows before it
    {
        int64_t sp = 0, su = 0;
        for (int64_t e = tid; e < 2 * bdim; e += kPmThreads) {
            const int h = int(e / bdim);
            if (r0 + h < bdim) sp += tcount[h][e - h * bdim];
        }
        for (int64_t e = tid; e < mb; e += kPmThreads) su += ucnt[e];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            sp += __shfl_xor(sp, off);
            su += __shfl_xor(su, off);
        }
        if (lane == 0) {
            wsum[0][wave] = sp;
            wsum[1][wave] = su;
        }
    }
    __syncthreads();
    if (wave == 0) {
        unsigned long long own_p = 0, own_u = 0;
#pragma unroll
        for (int w = 0; w < kPmWaves; ++w) {
            own_p += (unsigned long long)wsum[0][w];
            own_u += (unsigned long long)wsum[1][w];
        }
        const unsigned long long own = pack_sums(own_p, own_u);
        if (lane == 0) atomic_store_agent(o.flags + I, (I == 0 ? kStIncl : kStAgg) | own);
        // exclusive prefix: walk back in windows of 64 rows; lane l reads row
        // top - l; the window ends at the nearest inclusive prefix, and every
        // row after it must have published its sums
        unsigned long long ex_p = 0, ex_u = 0;
        int64_t top = I - 1;
        // every wait ends: rows below I have all started (ticket order) and
        // publish without waiting on later rows; the spin is still bounded
        // (seconds), after which the plan is marked invalid (pairs = -1)
        uint32_t spins = 0;
        bool timed_out = false;
        while (top >= 0) {
            const int64_t p = top - lane;
            const unsigned long long wv = p >= 0 ? atomic_load_agent(o.flags + p) : kStIncl;
            const uint64_t incl = __ballot((wv >> 62) == 2);
            const uint64_t ready = __ballot((wv >> 62) != 0);
            // lanes up to and including the first inclusive one must all be ready
            const int first = incl ? __ffsll((unsigned long long)incl) - 1 : 63;
            const uint64_t need = first == 63 ? ~0ull : ((2ull << first) - 1);
            if ((ready & need) != need) {
                if (++spins > kPmMaxSpins) {
                    timed_out = true;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
                continue;  // re-read the same window
            }
            unsigned long long cp = 0, cu = 0;
            if (lane <= first && p >= 0) {
                cp = (wv >> 31) & kField;
                cu = wv & kField;
            }
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                cp += __shfl_xor(cp, off);
                cu += __shfl_xor(cu, off);
            }
            ex_p += cp;
            ex_u += cu;
            if (incl) break;
            top -= 64;
        }
        if (lane == 0) {
            if (I > 0) atomic_store_agent(o.flags + I, kStIncl | pack_sums(ex_p + own_p, ex_u + own_u));
            s_excl = pack_sums(ex_p, ex_u);
            if (I == mb - 1) {  // the last row: totals
                o.offsets[bdim * bdim] = int32_t(ex_p + own_p);
                o.uprefix[nm] = int32_t(ex_u + own_u);
                if (o.pairs) *o.pairs = int64_t(ex_p + own_p);
            }
            if (timed_out && o.pairs) *o.pairs = -1;
        }
    }
    __syncthreads();

    // ---- 3. offsets, k-lists, union prefix, items
    const int64_t base_p = int64_t((s_excl >> 31) & kField), base_u = int64_t(s_excl & kField);
    // in-row exclusive prefixes of the counts, in place (one wave per array)
    if (wave < 3) {
        int32_t* arr = wave < 2 ? tcount[wave] : ucnt;
        const int64_t len = wave < 2 ? (r0 + wave < bdim ? bdim : 0) : mb;
        int32_t run = 0;
        for (int64_t b0 = 0; b0 < len; b0 += 64) {
            const int64_t e = b0 + lane;
            const int32_t v = e < len ? arr[e] : 0;
            int32_t incl = v;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int32_t up = __shfl_up(incl, off);
                if (lane >= off) incl += up;
            }
            if (e < len) arr[e] = run + incl - v;
            run += __shfl(incl, 63);
        }
        if (wave < 2 && lane == 0) wsum[0][wave] = run;  // the tile row's total
    }
    __syncthreads();
    // tiles: one thread per (tile of rows r0, r0 + 1, k-chunk); its kept k
    // in ascending order, after the k of the tile's earlier chunks
    const int64_t row0_total = wsum[0][0];
    for (int64_t x = tid; x < 2 * bdim * nw; x += kPmThreads) {
        const int c = int(x % nw);
        const int64_t e = x / nw;
        const int h = int(e / bdim);
        const int64_t j = e - h * bdim, r = r0 + h;
        if (r >= bdim) continue;
        int64_t base = base_p + (h ? row0_total : 0) + tcount[h][j];
        for (int cc = 0; cc < c; ++cc) base += __popcll(smask[h][j][cc]);
        if (c == 0) o.offsets[r * bdim + j] = int32_t(base);
        for (uint64_t m = smask[h][j][c]; m; m &= m - 1) o.klist[base++] = c * 64 + __builtin_ctzll(m);
    }
    // macro tiles: one thread per (macro tile of row I, k-chunk); the union of
    // the four bitmaps in ascending k, packed as macro_items_wave packs them
    for (int64_t x = tid; x < mb * nw; x += kPmThreads) {
        const int c = int(x % nw);
        const int64_t J = x / nw, m = I * mb + J;
        auto word = [&](int q, int cc) -> uint64_t {
            const int64_t r = r0 + (q >> 1), j = 2 * J + (q & 1);
            return (r < bdim && j < bdim) ? smask[q >> 1][j][cc] : 0ull;
        };
        int64_t base = base_u + ucnt[J];
        for (int cc = 0; cc < c; ++cc) base += __popcll(word(0, cc) | word(1, cc) | word(2, cc) | word(3, cc));
        if (c == 0) o.uprefix[m] = int32_t(base);
        const uint64_t w0 = word(0, c), w1 = word(1, c), w2 = word(2, c), w3 = word(3, c);
        for (uint64_t u = w0 | w1 | w2 | w3; u; u &= u - 1) {
            const int b = __builtin_ctzll(u);
            const uint32_t mem = uint32_t((w0 >> b) & 1) | uint32_t(((w1 >> b) & 1) << 1) |
                                 uint32_t(((w2 >> b) & 1) << 2) | uint32_t(((w3 >> b) & 1) << 3);
            o.items[base++] = mi_pack(uint32_t(I), uint32_t(J), uint32_t(c * 64 + b), mem);
        }
    }
}

hipError_t launch_plan_macro(const double* norms_a, const double* norms_b, int64_t side, int64_t bdim, double tau,
                             const PlanMacroOut& o, hipStream_t s) {
    if (bdim < 1 || bdim > kPmMaxBdim || side < bdim) return hipErrorInvalidValue;
    const int64_t mb = (bdim + 1) / 2;
    plan_macro_kernel<<<unsigned(mb), kPmThreads, 0, s>>>(norms_a, norms_b, side, bdim, tau, o);
    return hipGetLastError();
}

}  // namespace spamm
