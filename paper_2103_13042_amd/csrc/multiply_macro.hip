// Multiply of the kept leaf pairs on 2x2 blocks of output tiles ("macro
// tiles"), for leaf 32 and 64.
//
// A macro tile (I, J) covers output tiles (2I+a, 2J+b), a, b in {0, 1}.  Its
// k-stream is the union of the four tiles' k-lists in ascending order; for each
// k the workgroup stages A[2I..2I+1, k] and B[k, 2J..2J+1] once and every wave
// (a, b) whose own tile keeps that k multiplies its 64x64 (or 32x32) part.  One
// staged A/B pair thus feeds up to four leaf products, which halves the bytes
// per flop against one tile per workgroup for banded pair patterns, and every
// barrier is amortised over twice the MFMA work.
//
// Work units: a persistent grid of G workgroups splits the macro tiles into
// contiguous row-major ranges of equal cost (kUnionCost per union k plus
// kMacroWrite per macro tile, from the prefix of union sizes), XCD-aware as in
// the single-tile kernel; the leaf-64 LDS-DMA kernel below splits at item
// granularity instead (see its comment).  The schedule step lists, for every
// macro tile in order, its union k values with the 4-bit membership of the
// four tiles (packed items); a workgroup streams its contiguous slice of that
// list with scalar loads, a few items ahead of the one it multiplies.
#include <hip/hip_runtime.h>

#include "device.h"
#include "dma.h"
#include "internal.h"
#include "macro.h"

namespace spamm {

// One wave per macro tile: k-bitmaps and union size (macro_words_wave).
__global__ __launch_bounds__(256) void macro_words_kernel(const int32_t* __restrict__ off,
                                                          const int32_t* __restrict__ klist, int64_t bdim, int64_t mb,
                                                          int nw, uint64_t* __restrict__ words,
                                                          int32_t* __restrict__ ucount) {
    __shared__ unsigned long long sw[4][4][16];  // [wave][tile][word]
    const int wave = threadIdx.x >> 6;
    const int64_t m = int64_t(blockIdx.x) * 4 + wave;
    if (m >= mb * mb) return;
    macro_words_wave(off, klist, bdim, mb, nw, words, ucount, m, sw[wave]);
}

// One wave per macro tile: its packed items (macro_items_wave).
__global__ __launch_bounds__(256) void macro_items_kernel(const uint64_t* __restrict__ words,
                                                          const int32_t* __restrict__ uprefix, int64_t mb, int nw,
                                                          uint32_t* __restrict__ items) {
    const int64_t m = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (m >= mb * mb) return;
    macro_items_wave(words, uprefix, mb, nw, items, m);
}

// A persistent grid over the macro tiles, split into contiguous ranges of
// equal cost (kUnionCost per union k, kMacroWrite per macro tile).
template <int LEAF, bool VEC>
__global__ __launch_bounds__(kMacThreads, MacGeom<LEAF>::OCC) void multiply_macro_kernel(
    const float* __restrict__ A, const float* __restrict__ B, float* __restrict__ C, int64_t n, int64_t bdim,
    int64_t mb, const uint32_t* __restrict__ items, const int32_t* __restrict__ uprefix) {
    __shared__ __attribute__((aligned(16))) float lds[2 * MacGeom<LEAF>::STAGE];
    const int64_t groups = gridDim.x;
    const int64_t bid = blockIdx.x;
    const int64_t lg = (bid & 7) * (groups >> 3) + (bid >> 3);
    const int64_t nm = mb * mb;
    const int64_t total = int64_t(kUnionCost) * uprefix[nm] + int64_t(kMacroWrite) * nm;
    auto start_of = [&](int64_t gg) {
        const int64_t target = gg * total;
        int64_t lo = 0, hi = nm;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if ((int64_t(kUnionCost) * uprefix[mid] + int64_t(kMacroWrite) * mid) * groups >= target)
                hi = mid;
            else
                lo = mid + 1;
        }
        return lo;
    };
    macro_range<LEAF, VEC>(A, B, C, n, bdim, mb, items, uprefix, start_of(lg), start_of(lg + 1), lds);
}

// ---------------------------------------------------------------------------
// Leaf 64 with N a multiple of 128 (whole macro tiles, every access inside
// the matrix): the same macro-tile stream, but tiles move from global memory
// straight into LDS (global_load_lds_dwordx4) through kDmaStages LDS stages of
// one item (kDmaKC k) each, so the copies of the next items are in flight
// while one is multiplied and no registers stage the data.
//
// Sixteen waves: wave w computes the 32x32 quadrant (w >> 3 & 1, w >> 2 & 1)
// of output tile (w + (w >> 2)) & 3 of the macro tile.  Waves are dealt to the
// four SIMDs round-robin (w, w+4, w+8, w+12 on one SIMD), so each output tile
// has one wave on every SIMD and the MFMA load of an item is the same on all
// SIMDs whichever of the four tiles keep its k.
//
// LDS rows are stored without padding; 16-byte chunks are XOR-swizzled so the
// MFMA operand reads are free of bank conflicts.
//
// Completion of the copies is tracked by hand with s_waitcnt vmcnt: with two
// stages, a wave's vector-memory operations issued after its copies of item
// it are exactly the kDmaStores stores of each macro tile it finished since
// (shared tiles included: their partial sums are stored the same way), so
// the wait counts those stores whatever number of copies the item needed.
// Empty asm statements with a memory clobber keep the compiler from moving
// LDS or global accesses across the hand-placed waits and the barrier.
//
// Work split: workgroup g takes the items between boundaries g and g+1 of the
// item-level cost partition (split_bound), so a macro tile may be shared by
// consecutive workgroups.  Each sharer writes its partial sums to its own
// slot instead of C; macro_fixup_kernel, launched next on the stream, adds the
// partials of every shared tile in workgroup order and writes C.
__global__ __launch_bounds__(kDmaThreads, 1) void multiply_macro_dma_kernel(
    const float* __restrict__ A, const float* __restrict__ B, float* __restrict__ C, int64_t n, int64_t bdim,
    int64_t mb, const uint32_t* __restrict__ items, const int32_t* __restrict__ uprefix,
    const int32_t* __restrict__ offsets, int64_t* __restrict__ bounds, float* __restrict__ fix_slots) {
    constexpr int LEAF = 64, KC = kDmaKC, NCH = LEAF / KC, SPC = KC / 2;
    constexpr int ABYTES = 2 * LEAF * KC * 4, BBYTES = KC * 2 * LEAF * 4;
    constexpr int STAGE_BYTES = ABYTES + BBYTES;
    // one LDS object (the stages, then the two partition boundaries): a second
    // __shared__ array makes the compiler wait for every outstanding copy
    // before each LDS read
    __shared__ __attribute__((aligned(1024))) char lds[kDmaStages * STAGE_BYTES + 6 * sizeof(int64_t)];
    int64_t(*sbound)[2] = reinterpret_cast<int64_t(*)[2]>(lds + kDmaStages * STAGE_BYTES);

    // the wave index as a scalar, so that what derives from it (the tile, the
    // copy half and its membership tests) stays in scalar registers
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    // waves w, w+4, w+8, w+12 share a SIMD: give them different output tiles
    // (and each tile one wave per quadrant), so every SIMD holds one wave of
    // each tile and the MFMA work of an item is spread evenly whichever tiles
    // keep its k
    const int tile = (wave + (wave >> 2)) & 3, wa = tile >> 1, wb = tile & 1, qr = (wave >> 3) & 1,
              qc = (wave >> 2) & 1;
    const int ir = lane & 31, g = lane >> 5;

    const int64_t groups = gridDim.x;
    const int64_t bid = blockIdx.x;
    const int64_t lg = (bid & 7) * (groups >> 3) + (bid >> 3);
    const int64_t nm = mb * mb;
    // boundaries lg, lg+1 and lg-1, one wave each
    if (wave < 3) {
        const SplitBound sbd = split_bound(wave < 2 ? lg + wave : lg - 1, groups, mb, uprefix, offsets, items);
        if (lane == 0) {
            sbound[wave][0] = sbd.m;
            sbound[wave][1] = sbd.p;
        }
    }
    __syncthreads();
    const int64_t m_first = sbound[0][0], p_begin = sbound[0][1];
    const int64_t m_next = sbound[1][0], p_end = sbound[1][1];
    const bool has_items = p_begin < p_end;
    const bool head_split = has_items && p_begin > uprefix[m_first];
    const bool tail_split = has_items && m_next < nm && p_end > uprefix[m_next];
    // record for macro_fixup_kernel: boundary lg; the macro tile it opens
    // for sharing (boundary lg lies inside it and boundary lg-1 does not), or
    // -1; and lg if this workgroup then holds the rest of that tile (it is
    // the last of the two contributors), else -1
    if (tid < 4) {
        const bool inside = m_first < nm && p_begin > uprefix[m_first];
        const bool opens = inside && !(sbound[2][0] == m_first && sbound[2][1] > uprefix[m_first]);
        const int64_t v = tid < 2    ? sbound[0][tid]
                          : tid == 2 ? (opens ? m_first : int64_t(-1))
                                     : (opens && has_items && p_end >= uprefix[m_first + 1] ? lg : int64_t(-1));
        bounds[4 * lg + tid] = v;
    }
    const int64_t m_begin = m_first, m_end = m_next + (tail_split ? 1 : 0);
    if (m_begin >= m_end) return;

    // this group's slice of the item list (wave-uniform); past the end the
    // last item repeats (a harmless reload)
    const uint32_t* ip = items + p_begin;
    const int64_t npairs = p_end - p_begin;
    const int64_t nitems = npairs * NCH;
    int64_t pp = 0;
    uint32_t last = 0;
    auto produce = [&]() -> uint32_t {
        if (pp < npairs) last = ip[pp];
        ++pp;
        return last;
    };

    f16v acc;
    auto zero_acc = [&]() {
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    };
    // exactly kDmaStores stores per wave: the accumulators of finished macro
    // tile m to C, or for a tile shared with other workgroups to this
    // workgroup's slot (a 128 x 128 row-major tile; side 1 if this workgroup
    // holds the tile's first item, the tile being its last, side 0 otherwise,
    // the tile being its first)
    auto store_macro = [&](int64_t m, bool shared) {
        const int64_t I = m / mb, J = m - (m / mb) * mb;
        float* base;
        int64_t ld;
        if (shared) {
            const int side = p_begin <= int64_t(uprefix[m]) ? 1 : 0;
            base = fix_slots + (lg * 2 + side) * int64_t(kSplitSlotFloats);
            ld = 2 * LEAF;
        } else {
            base = C + 2 * I * LEAF * n + 2 * J * LEAF;
            ld = n;
        }
        float* dst = base + (wa * LEAF + qr * 32 + 4 * g) * ld + wb * LEAF + qc * 32 + ir;
#pragma unroll
        for (int r = 0; r < 16; ++r) dst[(8 * (r >> 2) + (r & 3)) * ld] = acc[r];
    };

    // copies of item (pair item pi, chunk ch) into stage st: KC/32 A and KC/32
    // B instructions of 1 KiB per wave.  A is staged as 128 rows of KC; B as
    // two column halves (one per output tile column), each KC rows of 64.
    // Waves 0-7 copy the first half of each operand (A rows of output tile row
    // 0, B columns of tile column 0), waves 8-15 the second; a half that no
    // tile keeping the item's k reads is not copied (the membership bits tell),
    // so an item kept by one tile moves half the bytes.  The copy waits count
    // only the stores issued after a wave's copies, which holds for any number
    // of copies per wave with two stages.
    static_assert(kDmaStages == 2, "copies per wave vary with the item");
    constexpr int ACH = KC / 4;  // 16-byte chunks per A row
    constexpr int BHALF = KC * LEAF * 4;  // bytes of one B column half
    auto aswz = [](int r) { return KC == 32 ? ((r >> 1) & 7) : (r & 15); };
    const int half = wave >> 3;
    const uint32_t need_a = half ? 12u : 3u, need_b = half ? 10u : 5u;
    // each copy's address: the item's part (uniform: a scalar base) plus the
    // lane's part, the same for every item (a 32-bit byte offset computed
    // once: row r of the copy's block times n, plus its swizzled chunk), so
    // the copies of an item cost no per-lane address arithmetic
    uint32_t a_off[KC / 32], b_off[KC / 32];
#pragma unroll
    for (int j = 0; j < KC / 32; ++j) {
        {  // A: 1024 / (4 KC) rows per instruction
            const int blk = wave * (KC / 32) + j;
            const int r = blk * (256 / KC) + lane / ACH, p = lane % ACH;
            a_off[j] = uint32_t((int64_t(r) * n + 4 * (p ^ aswz(r))) * 4);
        }
        {  // B: 4 rows of 16 chunks of one half per instruction
            const int blk = (wave & 7) * (KC / 32) + j;
            const int r = blk * 4 + (lane >> 4), p = lane & 15;
            b_off[j] = uint32_t((int64_t(r) * n + half * LEAF + 4 * (p ^ (8 * ((r / SPC) & 1)))) * 4);
        }
    }
    auto copy_item = [&](uint32_t pi, int ch, int st) {
        const int64_t I = pi >> 23, J = (pi >> 14) & 511, kt = (pi >> 4) & 1023;
        char* sbase = lds + st * STAGE_BYTES;
        if (pi & need_a) {
            const char* base = reinterpret_cast<const char*>(A + 2 * I * LEAF * n + kt * LEAF + ch * KC);
#pragma unroll
            for (int j = 0; j < KC / 32; ++j) {
                const int blk = wave * (KC / 32) + j;
                __builtin_amdgcn_global_load_lds(reinterpret_cast<const float*>(base + a_off[j]),
                                                 (__attribute__((address_space(3))) void*)(sbase + blk * 1024), 16, 0,
                                                 0);
            }
        }
        if (pi & need_b) {
            const char* base = reinterpret_cast<const char*>(B + (kt * LEAF + ch * KC) * n + 2 * J * LEAF);
#pragma unroll
            for (int j = 0; j < KC / 32; ++j) {
                const int blk = (wave & 7) * (KC / 32) + j;
                __builtin_amdgcn_global_load_lds(
                    reinterpret_cast<const float*>(base + b_off[j]),
                    (__attribute__((address_space(3))) void*)(sbase + ABYTES + half * BHALF + blk * 1024), 16, 0, 0);
            }
        }
    };
    // operands are read in groups of GRP MFMA steps, one group ahead of the
    // MFMAs that use them, so the LDS latency hides behind MFMA work
    constexpr int GRP = 8, NGRP = SPC / GRP;
    static_assert(SPC % GRP == 0, "operand groups");
    auto compute = [&](int st) {
        const char* sa = lds + st * STAGE_BYTES;
        const char* sb = sa + ABYTES;
        const int r = wa * 64 + qr * 32 + ir;
        const int cc = qc * 32 + ir;  // column within tile column wb's half of B
        const char* brow = sb + wb * BHALF + ((cc >> 2) ^ (8 * g)) * 16 + (cc & 3) * 4;
        f4 av[2][GRP / 4];
        float bv[2][GRP];
        auto load = [&](int grp, int buf) {
#pragma unroll
            for (int q = 0; q < GRP / 4; ++q) {
                const int c = (g * (SPC / 4) + grp * (GRP / 4) + q) ^ aswz(r);
                av[buf][q] = *reinterpret_cast<const f4*>(sa + r * (KC * 4) + c * 16);
            }
#pragma unroll
            for (int u = 0; u < GRP; ++u) {
                const int kr = g * SPC + grp * GRP + u;
                bv[buf][u] = *reinterpret_cast<const float*>(brow + kr * (LEAF * 4));
            }
        };
        // a wave in its MFMA block goes first in its SIMD's issue arbitration,
        // ahead of the waves that issue their copies or wait at the barrier,
        // so the matrix unit is not left idle while copies are issued
        __builtin_amdgcn_s_setprio(1);
        load(0, 0);
#pragma unroll
        for (int grp = 0; grp < NGRP; ++grp) {
            if (grp + 1 < NGRP) load(grp + 1, (grp + 1) & 1);
            __builtin_amdgcn_sched_barrier(0);  // keep the next group's reads ahead of these MFMAs
#pragma unroll
            for (int u = 0; u < GRP; ++u)
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[grp & 1][u >> 2][u & 3], bv[grp & 1][u], acc, 0, 0, 0);
        }
        __builtin_amdgcn_s_setprio(0);
    };

    // pair items of item it (f[0]) and of the next pairs; item it + S - 1 lies
    // at most S - 1 pairs ahead
    constexpr int S = kDmaStages;
    uint32_t f[S];
#pragma unroll
    for (int i = 0; i < S; ++i) f[i] = produce();
#pragma unroll
    for (int i = 0; i < S - 1; ++i) copy_item(f[i / NCH], i % NCH, i);
    int64_t out_m = m_begin;
    int ns[S];  // macro tiles stored in the last S-1 steps (ns[0]: this step)
#pragma unroll
    for (int i = 0; i < S; ++i) ns[i] = 0;
    // finish macro tile out_m: its C tile, or this workgroup's partial sums of
    // a shared tile (kDmaStores stores per wave either way)
    auto finish = [&]() {
        store_macro(out_m, (out_m == m_first && head_split) || (out_m == m_next && tail_split));
        ++ns[0];
        zero_acc();
        ++out_m;
    };
    zero_acc();
    for (int64_t it = 0; it < nitems; ++it) {
        const uint32_t pi = f[0];
        const int64_t m_it = int64_t(pi >> 23) * mb + ((pi >> 14) & 511);
#pragma unroll
        for (int i = S - 1; i > 0; --i) ns[i] = ns[i - 1];
        ns[0] = 0;
        while (out_m < m_it) finish();
        int stores = 0;
#pragma unroll
        for (int i = 0; i < S - 1; ++i) stores += ns[i];
        // this wave's copies of item it are complete once at most the copies
        // of items it+1 .. it+S-2 and the stores issued since are outstanding
        asm volatile("" ::: "memory");
        wait_copies<(S - 2) * kDmaCopies>(stores);
        __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): this wave's LDS reads of item it-1 are done
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        {   // item it+S-1 -> the stage item it-1 used
            const int64_t il = it + S - 1;
            const int ahead = int((it % NCH + S - 1) / NCH);  // pairs ahead of item it's pair
            uint32_t pl = f[0];
#pragma unroll
            for (int i = 1; i < S; ++i)
                if (ahead == i) pl = f[i];
            copy_item(pl, int(il % NCH), int(il % S));
        }
        if ((pi >> tile) & 1) compute(int(it % S));
        if ((it + 1) % NCH == 0) {
#pragma unroll
            for (int i = 0; i < S - 1; ++i) f[i] = f[i + 1];
            f[S - 1] = produce();
        }
    }
    while (out_m < m_end) finish();
    __builtin_amdgcn_s_waitcnt(0);  // no copy into LDS may outlive the workgroup
}

// One workgroup per interior boundary g = 1 .. G-1 of the split multiply,
// from the records the multiply kernel left in bounds[4g ..]: (macro tile,
// item position) of boundary g, the shared macro tile M boundary g opens (or
// -1) and M's last contributor (or -1: found here from the later
// boundaries).  M's contributors are workgroups g-1 (slot side 1), g, g+1, ...
// (side 0; those with empty ranges skipped); their partial sums are added in
// that order and written to C.
__global__ __launch_bounds__(kDmaThreads) void macro_fixup_kernel(float* __restrict__ C, int64_t n, int64_t mb,
                                                                  const int32_t* __restrict__ uprefix,
                                                                  const int64_t* __restrict__ bounds,
                                                                  const float* __restrict__ fix_slots,
                                                                  int64_t groups) {
    constexpr int LEAF = 64;
    // element e = tid + 1024 j of the 128 x 128 tile: row e / 128, column e % 128
    constexpr int EL = (2 * LEAF * 2 * LEAF) / kDmaThreads;
    const int tid = threadIdx.x;
    const int64_t nm = mb * mb, gb = int64_t(blockIdx.x) + 1;
    const int64_t m = bounds[4 * gb + 2], last = bounds[4 * gb + 3];
    if (m < 0) return;
    auto slot = [&](int64_t c, int side) { return fix_slots + (c * 2 + side) * int64_t(kSplitSlotFloats); };
    float sum[EL];
    if (last >= 0) {  // two contributors, gb-1 and gb
        const float* s0 = slot(gb - 1, 1);
        const float* s1 = slot(gb, 0);
#pragma unroll
        for (int j = 0; j < EL; ++j) sum[j] = s0[tid + j * kDmaThreads] + s1[tid + j * kDmaThreads];
    } else {  // gb-1, then the non-empty ones of gb .. the one holding the tile's last item
        const float* s0 = slot(gb - 1, 1);
#pragma unroll
        for (int j = 0; j < EL; ++j) sum[j] = s0[tid + j * kDmaThreads];
        auto pos = [&](int64_t c) { return c >= groups ? int64_t(uprefix[nm]) : bounds[4 * c + 1]; };
        const int64_t u1 = uprefix[m + 1];
        for (int64_t c = gb, pc = pos(gb); pc < u1; ++c) {
            const int64_t pn = pos(c + 1);
            if (pc < pn) {
                const float* sc = slot(c, 0);
#pragma unroll
                for (int j = 0; j < EL; ++j) sum[j] += sc[tid + j * kDmaThreads];
            }
            pc = pn;
        }
    }
    const int64_t I = m / mb, J = m - (m / mb) * mb;
    float* dst = C + 2 * I * LEAF * n + 2 * J * LEAF;
#pragma unroll
    for (int j = 0; j < EL; ++j) {
        const int e = tid + j * kDmaThreads;
        dst[(e / (2 * LEAF)) * n + e % (2 * LEAF)] = sum[j];
    }
}

// Leaf 128 with N a multiple of 128 on the same kernel: a 128x128 output tile
// is a macro tile of four 64x64 quarters that all keep every k, so each kept
// pair (i, k, j) becomes two items (one per 64-wide half of k) with all four
// membership bits set.  One wave per output tile t: its items at
// 2 offsets[t] .., and uprefix[t] = 2 offsets[t].
__global__ __launch_bounds__(256) void leaf128_items_kernel(const int32_t* __restrict__ off,
                                                            const int32_t* __restrict__ klist, int64_t bdim,
                                                            int32_t* __restrict__ uprefix,
                                                            uint32_t* __restrict__ items) {
    const int lane = threadIdx.x & 63;
    const int64_t t = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (t > bdim * bdim) return;
    if (lane == 0) uprefix[t] = 2 * off[t];
    if (t == bdim * bdim) return;
    const uint32_t i = uint32_t(t / bdim), j = uint32_t(t - (t / bdim) * bdim);
    for (int32_t q = off[t] + lane; q < off[t + 1]; q += 64) {
        const uint32_t k = uint32_t(klist[q]);
        items[2 * int64_t(q)] = mi_pack(i, j, 2 * k, 15u);
        items[2 * int64_t(q) + 1] = mi_pack(i, j, 2 * k + 1, 15u);
    }
}

hipError_t launch_leaf128_schedule(const int32_t* offsets, const int32_t* klist, int64_t bdim, int32_t* uprefix,
                                   uint32_t* items, hipStream_t s) {
    leaf128_items_kernel<<<unsigned((bdim * bdim + 1 + 3) / 4), 256, 0, s>>>(offsets, klist, bdim, uprefix, items);
    return hipGetLastError();
}

hipError_t launch_leaf128_multiply(const float* a, const float* b, float* c, int64_t n, int64_t bdim,
                                   const int32_t* uprefix, const uint32_t* items, int64_t* bounds, float* fix_slots,
                                   int num_cus, hipStream_t s) {
    const int64_t mb = bdim, nm = mb * mb;  // one macro tile per 128x128 output tile
    const int64_t cap = ((nm + 7) / 8) * 8;
    static int scratch_state = 0;
    const hipError_t ce = check_no_scratch(multiply_macro_dma_kernel, &scratch_state);
    if (ce != hipSuccess) return ce;
    int64_t groups = int64_t(num_cus);
    if (groups > cap) groups = cap;
    groups = ((groups + 7) / 8) * 8;
    if (groups > kSplitMaxGroups) groups = kSplitMaxGroups;
    multiply_macro_dma_kernel<<<unsigned(groups), kDmaThreads, 0, s>>>(a, b, c, n, 2 * mb, mb, items, uprefix,
                                                                      nullptr, bounds, fix_slots);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess || groups < 2) return e;
    macro_fixup_kernel<<<unsigned(groups - 1), kDmaThreads, 0, s>>>(c, n, mb, uprefix, bounds, fix_slots, groups);
    return hipGetLastError();
}

hipError_t launch_macro_schedule(const int32_t* offsets, const int32_t* klist, int64_t bdim, const MacroSchedule& ms,
                                 hipStream_t s) {
    const int64_t mb = (bdim + 1) / 2, nm = mb * mb;
    const int nw = int((bdim + 63) / 64);
    macro_words_kernel<<<unsigned((nm + 3) / 4), 256, 0, s>>>(offsets, klist, bdim, mb, nw, ms.words, ms.ucount);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_plan_scan(ms.ucount, nm, ms.uprefix, ms.uprefix, nm, nullptr, s);
    if (e != hipSuccess) return e;
    macro_items_kernel<<<unsigned((nm + 3) / 4), 256, 0, s>>>(ms.words, ms.uprefix, mb, nw, ms.items);
    return hipGetLastError();
}

template <int LEAF>
static hipError_t launch_macro_run(const float* a, const float* b, float* c, int64_t n, int64_t bdim,
                                   const int32_t* offsets, const MacroSchedule& ms, bool vec, int num_cus,
                                   hipStream_t s) {
    const int64_t mb = (bdim + 1) / 2, nm = mb * mb;
    const int64_t cap = ((nm + 7) / 8) * 8;
    if (LEAF == 64 && vec && n % 128 == 0) {
        if (!ms.bounds || !ms.fix_slots) return hipErrorInvalidValue;
        static int scratch_state = 0;
        const hipError_t ce = check_no_scratch(multiply_macro_dma_kernel, &scratch_state);
        if (ce != hipSuccess) return ce;
        int64_t groups = int64_t(num_cus);
        if (groups > cap) groups = cap;
        groups = ((groups + 7) / 8) * 8;
        if (groups > kSplitMaxGroups) groups = kSplitMaxGroups;
        multiply_macro_dma_kernel<<<unsigned(groups), kDmaThreads, 0, s>>>(a, b, c, n, bdim, mb, ms.items, ms.uprefix,
                                                                          offsets, ms.bounds, ms.fix_slots);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess || groups < 2) return e;
        macro_fixup_kernel<<<unsigned(groups - 1), kDmaThreads, 0, s>>>(c, n, mb, ms.uprefix, ms.bounds,
                                                                        ms.fix_slots, groups);
        return hipGetLastError();
    }
    int64_t groups = int64_t(num_cus) * MacGeom<LEAF>::OCC;
    if (groups > cap) groups = cap;
    groups = ((groups + 7) / 8) * 8;
    static int scratch_state[2] = {0, 0};
    const hipError_t ce = vec ? check_no_scratch(multiply_macro_kernel<LEAF, true>, &scratch_state[1])
                              : check_no_scratch(multiply_macro_kernel<LEAF, false>, &scratch_state[0]);
    if (ce != hipSuccess) return ce;
    if (vec)
        multiply_macro_kernel<LEAF, true>
            <<<unsigned(groups), kMacThreads, 0, s>>>(a, b, c, n, bdim, mb, ms.items, ms.uprefix);
    else
        multiply_macro_kernel<LEAF, false>
            <<<unsigned(groups), kMacThreads, 0, s>>>(a, b, c, n, bdim, mb, ms.items, ms.uprefix);
    return hipGetLastError();
}

hipError_t launch_macro_multiply(const float* a, const float* b, float* c, int64_t n, int32_t leaf, int64_t bdim,
                                 const int32_t* offsets, const MacroSchedule& ms, bool vec, int num_cus,
                                 hipStream_t s) {
    switch (leaf) {
        case 32: return launch_macro_run<32>(a, b, c, n, bdim, offsets, ms, vec, num_cus, s);
        case 64: return launch_macro_run<64>(a, b, c, n, bdim, offsets, ms, vec, num_cus, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace spamm
