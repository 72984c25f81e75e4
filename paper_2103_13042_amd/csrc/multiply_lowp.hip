// Reduced-precision leaf products (leaf 64, N a multiple of 128) from the split
// operands of split.hip, on the macro-tile schedule of multiply_macro.hip.
#include <hip/hip_runtime.h>

#include "device.h"
#include "dma.h"
#include "internal.h"

namespace spamm {

// ---------------------------------------------------------------------------
// Work split of the reduced-precision multiplies.  XCD x (the blocks congruent
// to x mod 8) takes the macro tiles between the cost boundaries x W and
// (x+1) W of the G-way partition (kUnionCost per union k, kMacroWrite per
// macro tile; W = G / 8).  Its W workgroups share the range's tiles that have
// items in snake order of their rank (rank r goes to workgroup r mod W in even
// rounds, W-1 - (r mod W) in odd ones, as tile costs change slowly along the
// band), so the workgroups of one XCD work at the same time on neighbouring
// band tiles, which share A rows and B columns in that XCD's L2; the tiles
// without items (most of a banded range) are written as zeros by position,
// workgroup w taking slice w of W.  Without dealing (xcd_deal false) each
// workgroup takes the contiguous range between its own cost boundaries (the
// blocks of an XCD neighbouring ranges), the same code with W = 1.  Every
// macro tile is computed whole by one workgroup in ascending k, so C does not
// depend on the split.  (Macro tiles number at most 512 x 512 and item
// positions fit the int32 prefix.)
constexpr int kDealList = 3072;  // tiles per window of a workgroup's list
constexpr int kDealBytes = kDealList * 2 * 4 + (kDmaThreads / 64) * 4;

struct Deal {
    int32_t a, b, W, w;  // the XCD's range [a, b), workgroups per XCD, this one's index
};

__device__ __forceinline__ Deal deal_of(const int32_t* __restrict__ uprefix, int64_t mb, bool xcd_deal) {
    const int64_t groups = gridDim.x, bid = blockIdx.x, nm = mb * mb;
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
    Deal d;
    if (xcd_deal) {
        d.W = int32_t(groups >> 3);
        d.w = int32_t(bid >> 3);
        d.a = int32_t(start_of((bid & 7) * d.W));
        d.b = int32_t(start_of(((bid & 7) + 1) * d.W));
    } else {
        const int64_t lg = (bid & 7) * (groups >> 3) + (bid >> 3);
        d.W = 1;
        d.w = 0;
        d.a = int32_t(start_of(lg));
        d.b = int32_t(start_of(lg + 1));
    }
    return d;
}

// One scan of the XCD's range by the whole block: the item ranges (first,
// end) of this workgroup's tiles with items of list positions q0 .. q0 +
// kDealList - 1 go to lst; returns how many such tiles the workgroup has.
__device__ __forceinline__ int32_t deal_list(const Deal& d, const int32_t* __restrict__ uprefix, int32_t q0,
                                             int32_t* lst, int32_t* wcount) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    int32_t carry = 0;
    for (int32_t c0 = d.a; c0 < d.b; c0 += kDmaThreads) {
        const int32_t m = c0 + tid;
        int32_t lo = 0, hi = 0;
        if (m < d.b) {
            lo = uprefix[m];
            hi = uprefix[m + 1];
        }
        const bool has = hi > lo;
        const uint64_t bal = __ballot(has);
        if (lane == 0) wcount[wave] = __popcll(bal);
        __syncthreads();
        int32_t before = carry, chunk = 0;
        for (int v = 0; v < kDmaThreads / 64; ++v) {
            const int32_t c = wcount[v];
            if (v < wave) before += c;
            chunk += c;
        }
        const int32_t r = before + __popcll(bal & below);
        const int32_t round = r / d.W, owner = (round & 1) ? d.W - 1 - r % d.W : r % d.W;
        if (has && owner == d.w) {
            const int32_t q = round - q0;
            if (q >= 0 && q < kDealList) {
                lst[2 * q] = lo;
                lst[2 * q + 1] = hi;
            }
        }
        carry += chunk;
        __syncthreads();
    }
    const int32_t full = carry / d.W, rem = carry % d.W;
    return full + (rem > 0 && ((full & 1) ? d.w >= d.W - rem : d.w < rem) ? 1 : 0);
}

// The workgroup's multiply: for each window of its list, the items of the
// listed tiles through S LDS stages (copy(item, stage) issues COPIES copies
// per wave, compute(stage) multiplies the wave's part if its tile keeps the
// item's k, store(m) writes macro tile m from the accumulators with exactly
// kDmaStores stores per wave, zero() clears them); then the tiles without
// items of its slice, written as zeros.  lst and wcount lie in the same LDS
// object as the stages.
template <int S, int COPIES, typename Copy, typename Compute, typename Store, typename Zero>
__device__ __forceinline__ void deal_run(const Deal& d, const uint32_t* __restrict__ items,
                                         const int32_t* __restrict__ uprefix, int64_t mb, int32_t* lst,
                                         int32_t* wcount, int tile, Copy copy_item, Compute compute,
                                         Store store_macro, Zero zero_acc) {
    const int lane = threadIdx.x & 63;
    // the items of the listed tiles in turn; past the end the last item
    // repeats (a harmless reload)
    int32_t nlist = 0, ci = -1, pp = 0, pend = 0;
    uint32_t last = 0;
    auto produce = [&]() -> uint32_t {
        while (pp >= pend && ci + 1 < nlist) {
            ++ci;
            pp = __builtin_amdgcn_readfirstlane(lst[2 * ci]);
            pend = __builtin_amdgcn_readfirstlane(lst[2 * ci + 1]);
        }
        if (pp < pend) last = items[pp++];
        return last;
    };
    zero_acc();
    const int32_t mine = deal_list(d, uprefix, 0, lst, wcount);
    for (int32_t q0 = 0; q0 < mine; q0 += kDealList) {
        if (q0 > 0) deal_list(d, uprefix, q0, lst, wcount);
        nlist = mine - q0 < kDealList ? mine - q0 : kDealList;
        ci = -1;
        pp = pend = 0;
        int32_t nitems = 0;
        for (int e = lane; e < nlist; e += 64) nitems += lst[2 * e + 1] - lst[2 * e];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) nitems += __shfl_xor(nitems, o);
        nitems = __builtin_amdgcn_readfirstlane(nitems);
        uint32_t f[S];
#pragma unroll
        for (int i = 0; i < S; ++i) f[i] = produce();
#pragma unroll
        for (int i = 0; i < S - 1; ++i) copy_item(f[i], i);
        int32_t cur_m = -1;  // macro tile being accumulated
        int ns[S];           // macro tiles stored in the last S-1 steps (ns[0]: this step)
#pragma unroll
        for (int i = 0; i < S; ++i) ns[i] = 0;
        for (int32_t it = 0; it < nitems; ++it) {
            const uint32_t pi = f[0];
            const int32_t m_it = int32_t(pi >> 23) * int32_t(mb) + int32_t((pi >> 14) & 511);
#pragma unroll
            for (int i = S - 1; i > 0; --i) ns[i] = ns[i - 1];
            ns[0] = 0;
            if (m_it != cur_m) {  // listed tiles all have items: one store per change
                if (cur_m >= 0) {
                    store_macro(cur_m);
                    zero_acc();
                    ++ns[0];
                }
                cur_m = m_it;
            }
            int stores = 0;
#pragma unroll
            for (int i = 0; i < S - 1; ++i) stores += ns[i];
            asm volatile("" ::: "memory");
            wait_copies<(S - 2) * COPIES>(stores);
            __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
            __builtin_amdgcn_s_barrier();
            asm volatile("" ::: "memory");
            copy_item(f[S - 1], int((it + S - 1) % S));  // item it+S-1 -> the stage item it-1 used
            if ((pi >> tile) & 1) compute(int(it % S));
#pragma unroll
            for (int i = 0; i < S - 1; ++i) f[i] = f[i + 1];
            f[S - 1] = produce();
        }
        if (cur_m >= 0) {
            store_macro(cur_m);
            zero_acc();
        }
        __builtin_amdgcn_s_waitcnt(0);  // the stages are free before the list is rebuilt
        __syncthreads();
    }
    const int32_t len = d.b - d.a;
    for (int32_t m = d.a + len * d.w / d.W; m < d.a + len * (d.w + 1) / d.W; ++m)
        if (uprefix[m + 1] == uprefix[m]) store_macro(m);
    __builtin_amdgcn_s_waitcnt(0);  // no copy into LDS may outlive the workgroup
}

// ---------------------------------------------------------------------------
// Reduced-precision leaf products (leaf 64, N a multiple of 128): the macro-tile
// stream of the FP32 DMA kernel (multiply_macro.hip), with operands from the split pass: A rows
// and Bt rows (columns of B) of 64 halves per leaf k-range, so an item is one
// union k and a stage holds A rows [2I*64, 2I*64+128) and Bt rows
// [2J*64, 2J*64+128), one plane (bf16) or two (FP16 hi and lo) each.
//
// Each wave computes the same 32x32 quadrant as in the FP32 kernel with
// v_mfma_f32_32x32x16 (lane l takes k = 16 s + 8 (l >> 5) + 0..7 of row l & 31
// of both operands: one 16-byte LDS read each).  FP16: per k-step the three
// products hi*hi, hi*lo, lo*hi accumulate into one FP32 accumulator; the
// result is scaled by 2^-(eA + eB) when stored.  Rows are 128 bytes in LDS;
// 16-byte chunk c of row r sits at position c ^ (r & 7), which spreads the 8
// rows a group of 8 lanes reads over all banks.
template <int MODE>
struct LowpGeom {
    static constexpr int NP = MODE == kPrecF16x3 ? 2 : 1;  // planes per operand
    static constexpr int PLANE = 128 * 64 * 2;             // 128 rows x 64 halves
    static constexpr int STAGE = 2 * NP * PLANE;
    static constexpr int S = MODE == kPrecF16x3 ? 2 : 3;   // stages
    static constexpr int COPIES = 2 * NP;                  // per wave per item
    static_assert(S * STAGE <= 160 * 1024, "LDS budget");
};

// the wave's index in its workgroup as a scalar, so that what derives from
// it (its tile and copy rows) stays in scalar registers
__device__ __forceinline__ int wave_index() { return __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6); }

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef _Float16 h2 __attribute__((ext_vector_type(2)));
typedef float f2 __attribute__((ext_vector_type(2)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));

template <int MODE>
__global__ __launch_bounds__(kDmaThreads, 1) void multiply_lowp_kernel(
    const uint16_t* __restrict__ Ah, const uint16_t* __restrict__ Al, const uint16_t* __restrict__ Bh,
    const uint16_t* __restrict__ Bl, const int32_t* __restrict__ exps, float* __restrict__ C, int64_t n,
    int64_t bdim, int64_t mb, const uint32_t* __restrict__ items, const int32_t* __restrict__ uprefix, PairGate gate) {
    if (!gate_open(gate)) return;
    using G = LowpGeom<MODE>;
    constexpr int LEAF = 64, S = G::S;
    static_assert(S * G::STAGE + kDealBytes <= 160 * 1024, "LDS budget");
    __shared__ __attribute__((aligned(1024))) char lds[S * G::STAGE + kDealBytes];  // stages, then the deal's list

    const int tid = threadIdx.x, lane = tid & 63, wave = wave_index();
    const int tile = (wave + (wave >> 2)) & 3, wa = tile >> 1, wb = tile & 1, qr = (wave >> 3) & 1,
              qc = (wave >> 2) & 1;
    const int ir = lane & 31, g = lane >> 5;

    // dealt within each XCD for BF16; FP16 hi+lo (three products per k-step)
    // measured slower dealt on a dense pair pattern (27.2 -> 32.7 ms at
    // N = 16384), BF16 faster (16.2 -> 14.5 ms)
    const Deal d = deal_of(uprefix, mb, MODE == kPrecBf16);
    const float inv = MODE == kPrecF16x3 ? ldexpf(1.0f, -(exps[0] + exps[1])) : 1.0f;

    f16v acc;
    auto zero_acc = [&]() {
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    };
    auto store_macro = [&](int64_t m) {  // exactly kDmaStores stores per wave
        const int64_t ti = 2 * (m / mb) + wa, tj = 2 * (m - (m / mb) * mb) + wb;
        float* dst = C + (ti * LEAF + qr * 32 + 4 * g) * n + tj * LEAF + qc * 32 + ir;
#pragma unroll
        for (int r = 0; r < 16; ++r) dst[(8 * (r >> 2) + (r & 3)) * n] = acc[r] * inv;
    };
    // one 1 KiB copy per plane per wave: rows wave*8 .. wave*8+7 of the stage
    // the lane's part of each copy's address (row rr of its block, swizzled
    // chunk) is the same for every item: a byte offset computed once; the
    // item's part is a scalar base
    const int lrow = wave * 8 + (lane >> 3), lchunk = (lane & 7) ^ (lrow & 7);
    const uint32_t lane_off = uint32_t((int64_t(lrow) * n + 8 * lchunk) * 2);
    auto copy_item = [&](uint32_t pi, int st) {
        const int64_t I = pi >> 23, J = (pi >> 14) & 511, kt = (pi >> 4) & 1023;
        char* sbase = lds + st * G::STAGE + wave * 1024;
        const int64_t aoff = 2 * I * LEAF * n + kt * LEAF, boff = 2 * J * LEAF * n + kt * LEAF;  // item's part
        const uint16_t* ah = reinterpret_cast<const uint16_t*>(reinterpret_cast<const char*>(Ah + aoff) + lane_off);
        const uint16_t* bh = reinterpret_cast<const uint16_t*>(reinterpret_cast<const char*>(Bh + boff) + lane_off);
        __builtin_amdgcn_global_load_lds(ah, (__attribute__((address_space(3))) void*)(sbase), 16, 0, 0);
        if (G::NP == 2) {
            const uint16_t* al = reinterpret_cast<const uint16_t*>(reinterpret_cast<const char*>(Al + aoff) + lane_off);
            __builtin_amdgcn_global_load_lds(al, (__attribute__((address_space(3))) void*)(sbase + G::PLANE), 16, 0,
                                             0);
        }
        __builtin_amdgcn_global_load_lds(bh, (__attribute__((address_space(3))) void*)(sbase + G::NP * G::PLANE), 16,
                                         0, 0);
        if (G::NP == 2) {
            const uint16_t* bl = reinterpret_cast<const uint16_t*>(reinterpret_cast<const char*>(Bl + boff) + lane_off);
            __builtin_amdgcn_global_load_lds(bl, (__attribute__((address_space(3))) void*)(sbase + 3 * G::PLANE), 16,
                                             0, 0);
        }
    };
    auto compute = [&](int st) {
        const char* sa = lds + st * G::STAGE;
        const char* sb = sa + G::NP * G::PLANE;
        const int ra = wa * 64 + qr * 32 + ir, rb = wb * 64 + qc * 32 + ir;
        const char* arow = sa + ra * 128;
        const char* brow = sb + rb * 128;
        if (MODE == kPrecF16x3) {
            // two k-steps of operands at a time (32 registers): the second
            // pair's reads issue while the first pair's MFMAs execute
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                h8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int s4 = 2 * h + u;
                    const int pa = ((2 * s4 + g) ^ (ra & 7)) * 16, pb = ((2 * s4 + g) ^ (rb & 7)) * 16;
                    ah[u] = *reinterpret_cast<const h8*>(arow + pa);
                    al[u] = *reinterpret_cast<const h8*>(arow + G::PLANE + pa);
                    bh[u] = *reinterpret_cast<const h8*>(brow + pb);
                    bl[u] = *reinterpret_cast<const h8*>(brow + G::PLANE + pb);
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah[u], bh[u], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah[u], bl[u], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(al[u], bh[u], acc, 0, 0, 0);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        } else {
            b8 av[4], bv[4];
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
                const int pa = ((2 * s4 + g) ^ (ra & 7)) * 16, pb = ((2 * s4 + g) ^ (rb & 7)) * 16;
                av[s4] = *reinterpret_cast<const b8*>(arow + pa);
                bv[s4] = *reinterpret_cast<const b8*>(brow + pb);
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[s4], bv[s4], acc, 0, 0, 0);
        }
    };

    deal_run<S, G::COPIES>(d, items, uprefix, mb, reinterpret_cast<int32_t*>(lds + S * G::STAGE),
                           reinterpret_cast<int32_t*>(lds + S * G::STAGE + kDealList * 2 * 4), tile, copy_item,
                           compute, store_macro, zero_acc);
}

// ---------------------------------------------------------------------------
// Reduced-precision products straight from the FP32 inputs: the copies, LDS
// stages and swizzles of the FP32 DMA kernel (multiply_macro.hip: A rows of 64
// floats, chunk c of row r at c ^ (r & 15); B rows of 128 floats, chunk p of
// row r at p ^ (8 ((r >> 5) & 1))), and at the operand reads the conversion of
// split.hip in registers, then the MFMA sequence of multiply_lowp_kernel<MODE>
// (k-step s4 = 0..3, k = 16 s4 + 8 (lane >> 5) + 0..7):
//   FP16 hi+lo: y = s x, hi = fp16(y), lo = fp16(y - hi), nearest-even; per
//     k-step hi*hi, hi*lo, lo*hi;
//   BF16: bf16(x), nearest-even; one product per k-step.
// The same operand values and the same products in the same order as the
// split path, and every macro tile computed whole by one workgroup as there,
// so C is bitwise the same, without the split pass's read and write of A and
// B.
template <int MODE>
__global__ __launch_bounds__(kDmaThreads, 1) void multiply_fused_kernel(
    const float* __restrict__ A, const float* __restrict__ B, const int32_t* __restrict__ exps, float* __restrict__ C,
    int64_t n, int64_t bdim, int64_t mb, const uint32_t* __restrict__ items, const int32_t* __restrict__ uprefix,
    PairGate gate) {
    if (!gate_open(gate)) return;
    constexpr int LEAF = 64, KC = 64, S = 2;
    constexpr int ABYTES = 2 * LEAF * KC * 4, BBYTES = KC * 2 * LEAF * 4;
    constexpr int STAGE_BYTES = ABYTES + BBYTES;
    constexpr int COPIES = 2 * KC / 32;  // per wave per item
    static_assert(S * STAGE_BYTES + kDealBytes <= 160 * 1024, "LDS budget");
    __shared__ __attribute__((aligned(1024))) char lds[S * STAGE_BYTES + kDealBytes];  // stages, then the deal's list

    const int tid = threadIdx.x, lane = tid & 63, wave = wave_index();
    const int tile = (wave + (wave >> 2)) & 3, wa = tile >> 1, wb = tile & 1, qr = (wave >> 3) & 1,
              qc = (wave >> 2) & 1;
    const int ir = lane & 31, g = lane >> 5;

    const Deal d = deal_of(uprefix, mb, true);
    constexpr bool F16 = MODE == kPrecF16x3;  // else BF16: no scales (exps may be null)
    const float sa_scale = F16 ? ldexpf(1.0f, exps[0]) : 1.0f, sb_scale = F16 ? ldexpf(1.0f, exps[1]) : 1.0f;
    const float inv = F16 ? ldexpf(1.0f, -(exps[0] + exps[1])) : 1.0f;

    f16v acc;
    auto zero_acc = [&]() {
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    };
    auto store_macro = [&](int64_t m) {  // exactly kDmaStores stores per wave
        const int64_t ti = 2 * (m / mb) + wa, tj = 2 * (m - (m / mb) * mb) + wb;
        float* dst = C + (ti * LEAF + qr * 32 + 4 * g) * n + tj * LEAF + qc * 32 + ir;
#pragma unroll
        for (int r = 0; r < 16; ++r) dst[(8 * (r >> 2) + (r & 3)) * n] = acc[r] * inv;
    };
    // copies of item pi into stage st: 2 A and 2 B instructions of 1 KiB per wave
    constexpr int ACH = KC / 4;  // 16-byte chunks per A row
    // the lane's part of each copy's address (row of its block and swizzled
    // chunk) is the same for every item: byte offsets computed once; the
    // item's part is a scalar base
    uint32_t a_off[KC / 32], b_off[KC / 32];
#pragma unroll
    for (int j = 0; j < KC / 32; ++j) {
        const int blk = wave * (KC / 32) + j;
        {  // A: 4 rows of 16 chunks per instruction
            const int r = blk * (256 / KC) + lane / ACH, p = lane % ACH;
            a_off[j] = uint32_t((int64_t(r) * n + 4 * (p ^ (r & 15))) * 4);
        }
        {  // B: 2 rows of 32 chunks per instruction
            const int r = blk * 2 + (lane >> 5), p = lane & 31;
            b_off[j] = uint32_t((int64_t(r) * n + 4 * (p ^ (8 * ((r >> 5) & 1)))) * 4);
        }
    }
    auto copy_item = [&](uint32_t pi, int st) {
        const int64_t I = pi >> 23, J = (pi >> 14) & 511, kt = (pi >> 4) & 1023;
        char* sbase = lds + st * STAGE_BYTES;
        const char* abase = reinterpret_cast<const char*>(A + 2 * I * LEAF * n + kt * LEAF);
        const char* bbase = reinterpret_cast<const char*>(B + kt * LEAF * n + 2 * J * LEAF);
#pragma unroll
        for (int j = 0; j < KC / 32; ++j) {
            const int blk = wave * (KC / 32) + j;
            __builtin_amdgcn_global_load_lds(reinterpret_cast<const float*>(abase + a_off[j]),
                                             (__attribute__((address_space(3))) void*)(sbase + blk * 1024), 16, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < KC / 32; ++j) {
            const int blk = wave * (KC / 32) + j;
            __builtin_amdgcn_global_load_lds(reinterpret_cast<const float*>(bbase + b_off[j]),
                                             (__attribute__((address_space(3))) void*)(sbase + ABYTES + blk * 1024),
                                             16, 0, 0);
        }
    };
    // two elements at a time, as split.hip's Conv<kPrecF16x3>: y = s x (exact),
    // hi = fp16(y), lo = fp16(y - hi) (y - hi exact), nearest-even; then four
    // pairs make one 8-half MFMA operand
    auto split2 = [](float x0, float x1, float s, h2& hi, h2& lo) {
        const f2 y = {x0 * s, x1 * s};
        hi = __builtin_convertvector(y, h2);
        lo = __builtin_convertvector(y - __builtin_convertvector(hi, f2), h2);
    };
    auto cat8 = [](h2 p0, h2 p1, h2 p2, h2 p3) {
        const h4 q0 = __builtin_shufflevector(p0, p1, 0, 1, 2, 3), q1 = __builtin_shufflevector(p2, p3, 0, 1, 2, 3);
        return h8(__builtin_shufflevector(q0, q1, 0, 1, 2, 3, 4, 5, 6, 7));
    };
    auto compute = [&](int st) {
        const char* sa = lds + st * STAGE_BYTES;
        const char* sb = sa + ABYTES;
        const int ra = wa * 64 + qr * 32 + ir;
        const int cc = wb * 64 + qc * 32 + ir;
        // k-step s4 covers k = 16 s4 + 8 g .. + 7 of this lane's A row and B column
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            const int q0 = 4 * s4 + 2 * g;
            const f4 a0 = *reinterpret_cast<const f4*>(sa + ra * (KC * 4) + ((q0 ^ (ra & 15)) * 16));
            const f4 a1 = *reinterpret_cast<const f4*>(sa + ra * (KC * 4) + (((q0 + 1) ^ (ra & 15)) * 16));
            const char* bcol = sb + ((cc >> 2) ^ (8 * (s4 >> 1))) * 16 + (cc & 3) * 4;
            float bv[8];
#pragma unroll
            for (int i = 0; i < 8; ++i)
                bv[i] = *reinterpret_cast<const float*>(bcol + (16 * s4 + 8 * g + i) * (2 * LEAF * 4));
            if constexpr (F16) {
                h2 ph[4], pl[4];
                split2(a0[0], a0[1], sa_scale, ph[0], pl[0]);
                split2(a0[2], a0[3], sa_scale, ph[1], pl[1]);
                split2(a1[0], a1[1], sa_scale, ph[2], pl[2]);
                split2(a1[2], a1[3], sa_scale, ph[3], pl[3]);
                const h8 ah = cat8(ph[0], ph[1], ph[2], ph[3]), al = cat8(pl[0], pl[1], pl[2], pl[3]);
#pragma unroll
                for (int i = 0; i < 4; ++i) split2(bv[2 * i], bv[2 * i + 1], sb_scale, ph[i], pl[i]);
                const h8 bh = cat8(ph[0], ph[1], ph[2], ph[3]), bl = cat8(pl[0], pl[1], pl[2], pl[3]);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, bh, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, bl, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(al, bh, acc, 0, 0, 0);
            } else {
                const b8 ab = {__bf16(a0[0]), __bf16(a0[1]), __bf16(a0[2]), __bf16(a0[3]),
                               __bf16(a1[0]), __bf16(a1[1]), __bf16(a1[2]), __bf16(a1[3])};
                const b8 bb = {__bf16(bv[0]), __bf16(bv[1]), __bf16(bv[2]), __bf16(bv[3]),
                               __bf16(bv[4]), __bf16(bv[5]), __bf16(bv[6]), __bf16(bv[7])};
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ab, bb, acc, 0, 0, 0);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    };

    deal_run<S, COPIES>(d, items, uprefix, mb, reinterpret_cast<int32_t*>(lds + S * STAGE_BYTES),
                        reinterpret_cast<int32_t*>(lds + S * STAGE_BYTES + kDealList * 2 * 4), tile, copy_item,
                        compute, store_macro, zero_acc);
}

hipError_t launch_fused_multiply(const float* a, const float* b, int precision, const int32_t* exps, float* c,
                                 int64_t n, int64_t bdim, const uint32_t* items, const int32_t* uprefix, int num_cus,
                                 const PairGate& gate, hipStream_t s) {
    const int64_t mb = (bdim + 1) / 2, nm = mb * mb;
    const int64_t cap = ((nm + 7) / 8) * 8;
    int64_t groups = int64_t(num_cus);
    if (groups > cap) groups = cap;
    groups = ((groups + 7) / 8) * 8;
    static int scratch_bf16 = 0, scratch_f16 = 0;
    if (precision == kPrecBf16) {
        const hipError_t ce = check_no_scratch(multiply_fused_kernel<kPrecBf16>, &scratch_bf16);
        if (ce != hipSuccess) return ce;
        multiply_fused_kernel<kPrecBf16><<<unsigned(groups), kDmaThreads, 0, s>>>(a, b, exps, c, n, bdim, mb, items,
                                                                                 uprefix, gate);
    } else {
        const hipError_t ce = check_no_scratch(multiply_fused_kernel<kPrecF16x3>, &scratch_f16);
        if (ce != hipSuccess) return ce;
        multiply_fused_kernel<kPrecF16x3><<<unsigned(groups), kDmaThreads, 0, s>>>(a, b, exps, c, n, bdim, mb, items,
                                                                                  uprefix, gate);
    }
    return hipGetLastError();
}

hipError_t launch_lowp_multiply(const SplitLayout& L, float* c, int64_t n, int64_t bdim, int precision,
                                const uint32_t* items, const int32_t* uprefix, int num_cus, const PairGate& gate,
                                hipStream_t s) {
    const int64_t mb = (bdim + 1) / 2, nm = mb * mb;
    const int64_t cap = ((nm + 7) / 8) * 8;
    int64_t groups = int64_t(num_cus);
    if (groups > cap) groups = cap;
    groups = ((groups + 7) / 8) * 8;
    static int scratch_bf16 = 0, scratch_f16 = 0;
    if (precision == kPrecBf16) {
        const hipError_t ce = check_no_scratch(multiply_lowp_kernel<kPrecBf16>, &scratch_bf16);
        if (ce != hipSuccess) return ce;
        multiply_lowp_kernel<kPrecBf16><<<unsigned(groups), kDmaThreads, 0, s>>>(
            L.a_hi, L.a_lo, L.bt_hi, L.bt_lo, L.exps, c, n, bdim, mb, items, uprefix, gate);
    } else {
        const hipError_t ce = check_no_scratch(multiply_lowp_kernel<kPrecF16x3>, &scratch_f16);
        if (ce != hipSuccess) return ce;
        multiply_lowp_kernel<kPrecF16x3><<<unsigned(groups), kDmaThreads, 0, s>>>(
            L.a_hi, L.a_lo, L.bt_hi, L.bt_lo, L.exps, c, n, bdim, mb, items, uprefix, gate);
    }
    return hipGetLastError();
}

}  // namespace spamm
