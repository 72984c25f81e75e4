// Internal interface between the host C-ABI (api.hip) and the gfx950 kernels
// (kernels.hip).  Not installed; the public interface is include/spamm.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace spamm {

// Level l of a norm pyramid starts at entry (4^l - 1) / 3 (levels 0..Lv).
__host__ __device__ inline int64_t level_offset(int l) { return ((int64_t(1) << (2 * l)) - 1) / 3; }

// Up to two matrices are processed by one launch of the norm and pyramid
// kernels (A and B of one product).
struct NormJob {
    const float* x[2];
    double* sumsq[2];     // leaf sums of squares, row stride ld, or null
    double* norms[2];     // leaf norms, row stride ld, or null
    int64_t ld;           // row stride of the outputs (bdim, or the padded pyramid side)
    int64_t* clear;       // device int64 words set to zero by the launch, or null
    int64_t clear_count;  // how many (1 when clear is set and this is 0)
};

// The leaf level of both pyramids is written by the norm pass (stride = side);
// the pyramid kernel zeroes its padding tiles and builds the levels above.
struct PyramidJob {
    double* spyr[2];  // [pyramid] sums of squares at every level (scratch)
    double* pyr[2];   // [pyramid] norms at every level (output)
};

// Norm pass: leaf sums of squares / norms of nmat matrices.
hipError_t launch_leaf_norms(const NormJob& job, int nmat, int64_t n, int32_t leaf, bool vec, hipStream_t s);

// Pyramid: bottom-up quadtree of sums of squares and norms for nmat matrices.
hipError_t launch_pyramid(const PyramidJob& job, int nmat, int64_t bdim, int lv, hipStream_t s);

// Plan: per output tile, the ballot bitmap of kept k (words of 64) and its
// count V; per block of 64 tiles (i, 64*jb ..) the sum of V (block b = i*nw + jb).
// With `skipped` the bitmaps select the dropped triples instead.
hipError_t launch_plan_mask(const double* pyr_a, const double* pyr_b, int64_t bdim, int lv, double tau, bool skipped,
                            uint64_t* masks, int32_t* counts, int32_t* block_sums, hipStream_t s);
// Plan counts only (no bitmaps): per block of 64 tiles the number of kept triples.
hipError_t launch_plan_count(const double* pyr_a, const double* pyr_b, int64_t bdim, int lv, double tau,
                             int32_t* block_sums, hipStream_t s);
// Mean norm product over the bdim^3 leaf triples, into one device double.
hipError_t launch_mean_norm_product(const double* pyr_a, const double* pyr_b, int64_t bdim, int lv, double* out,
                                    hipStream_t s);
// Plan: exclusive scan of the block sums into block_offsets; the total goes to
// offsets[T] and *pairs.  Each of the three outputs may be null; block_offsets
// and offsets may be the same array (they are written at disjoint indices).
hipError_t launch_plan_scan(const int32_t* block_sums, int64_t nblocks, int32_t* block_offsets, int32_t* offsets,
                            int64_t ntiles, int64_t* pairs, hipStream_t s);
// Plan: per tile offset (block offset + prefix inside the block) and the
// compaction of its bitmap into an ascending k-list.
hipError_t launch_plan_fill(const uint64_t* masks, const int32_t* counts, const int32_t* block_offsets,
                            int64_t bdim, int32_t* offsets, int32_t* klist, hipStream_t s);

// Plan and macro-tile schedule in one launch (plan_macro.hip; leaf 32 and 64,
// bdim <= kPlanMacroMaxBdim): the outputs of launch_plan_mask +
// launch_plan_scan + launch_plan_fill (offsets, klist, pairs) and of
// launch_macro_schedule (uprefix, items); flags (mb words, mb = ceil(bdim /
// 2)) and the ticket after them must be zero before the launch
// (plan_macro_clear_words(bdim) words from flags).
constexpr int64_t kPlanMacroMaxBdim = 256;
struct PlanMacroOut {
    int32_t* offsets;
    int32_t* klist;
    int64_t* pairs;  // may be null
    int32_t* uprefix;
    uint32_t* items;
    unsigned long long* flags;
    unsigned int* ticket;
};
inline int64_t plan_macro_clear_words(int64_t bdim) { return (bdim + 1) / 2 + 1; }
// norms_a, norms_b: the leaf norms (row stride side); the pyramid above the
// leaf level is not used
hipError_t launch_plan_macro(const double* norms_a, const double* norms_b, int64_t side, int64_t bdim, double tau,
                             const PlanMacroOut& o, hipStream_t s);

// Small products (leaf 32, bdim <= kSmallMaxBdim, n % 4 == 0, a and b 16-byte
// aligned): the threshold test on the leaf norms na / nb (row stride ld) and
// the multiply of the kept pairs in one launch; adds the number of kept pairs
// to *pairs, which must be zero before (the norm pass clears it).
constexpr int64_t kSmallMaxBdim = 64;
hipError_t launch_small_multiply(const float* a, const float* b, float* c, int64_t n, int64_t bdim,
                                 const double* na, const double* nb, int64_t ld, double tau, int64_t* pairs,
                                 hipStream_t s);

// Multiply: persistent, cost-balanced multiply of the kept pairs into C
// (leaf 32, 64, 128; leaf 16 goes to launch_multiply_leaf16).
// pair_scratch holds bdim^3 int32 (each group's packed (tile, k) pairs).
hipError_t launch_multiply(const float* a, const float* b, float* c, int64_t n, int32_t leaf, int64_t bdim,
                           const int32_t* offsets, const int32_t* klist, int32_t* pair_scratch, bool vec,
                           int num_cus, hipStream_t s);

// Leaf 16: one wave per output tile, operands straight from global memory
// into MFMA registers (multiply_leaf16.hip); every tile of c is written.
hipError_t launch_multiply_leaf16(const float* a, const float* b, float* c, int64_t n, int64_t bdim,
                                  const int32_t* offsets, const int32_t* klist, bool vec, hipStream_t s);

// Multiply on 2x2 macro tiles (leaf 32 and 64), in two steps.  Schedule:
// per-macro-tile k bitmaps into words [mb*mb*4*nwords], union sizes into
// ucount [mb*mb], their exclusive prefix into uprefix [mb*mb + 1], and the
// union k lists as packed items into items [<= mb*mb*bdim].  Multiply: the
// persistent kernel over that schedule; the leaf-64 LDS-DMA kernel (which
// also reads the plan's offsets for its cost model) writes four records per
// workgroup to bounds [4 * kSplitMaxGroups] and the partial sums of macro
// tiles shared between workgroups to fix_slots [kSplitMaxGroups * 2 * 128 *
// 128], which a second kernel adds into C.
struct MacroSchedule {
    uint64_t* words;
    int32_t *ucount, *uprefix;
    uint32_t* items;
    int64_t* bounds;
    float* fix_slots;
};
hipError_t launch_macro_schedule(const int32_t* offsets, const int32_t* klist, int64_t bdim, const MacroSchedule& ms,
                                 hipStream_t s);
hipError_t launch_macro_multiply(const float* a, const float* b, float* c, int64_t n, int32_t leaf, int64_t bdim,
                                 const int32_t* offsets, const MacroSchedule& ms, bool vec, int num_cus,
                                 hipStream_t s);
// Leaf 128 with N a multiple of 128 (bdim <= kLeaf128MaxBdim) on the LDS-DMA
// kernel: two items per kept pair (uprefix [bdim*bdim + 1], items
// [2 * pairs]), then the multiply and fixup kernels with one macro tile per
// output tile.
constexpr int64_t kLeaf128MaxBdim = 512;  // item fields: tile index < 512, k half < 1024
hipError_t launch_leaf128_schedule(const int32_t* offsets, const int32_t* klist, int64_t bdim, int32_t* uprefix,
                                   uint32_t* items, hipStream_t s);
hipError_t launch_leaf128_multiply(const float* a, const float* b, float* c, int64_t n, int64_t bdim,
                                   const int32_t* uprefix, const uint32_t* items, int64_t* bounds, float* fix_slots,
                                   int num_cus, hipStream_t s);

// --------------------------------------------------------------------------
// Learned threshold (learned.hip).

constexpr int kSumBlocks = 1024;  // partials of launch_sumsq
constexpr int kMlpIn = 129, kMlpHid = 128;

// Offsets into the flat parameter array and into the activation scratch of
// a batch (in floats).
struct MlpLayout {
    int64_t w1 = 0;
    int64_t b1 = w1 + int64_t(kMlpHid) * kMlpIn;
    int64_t w2 = b1 + kMlpHid;
    int64_t b2 = w2 + int64_t(kMlpHid) * kMlpHid;
    int64_t w3 = b2 + kMlpHid;
    int64_t b3 = w3 + kMlpHid;
    int64_t count = b3 + 1;
    // activations: Z1 H1 Z2 H2 D1 D2 [B][128] each, then y, dy [B]
    int64_t z1 = 0, h1 = 0, z2 = 0, h2 = 0, d1 = 0, d2 = 0, y = 0, dy = 0, acts_total = 0;
    static MlpLayout acts(int batch) {
        MlpLayout L{};
        const int64_t bh = int64_t(batch) * kMlpHid;
        L.z1 = 0;
        L.h1 = bh;
        L.z2 = 2 * bh;
        L.h2 = 3 * bh;
        L.d1 = 4 * bh;
        L.d2 = 5 * bh;
        L.y = 6 * bh;
        L.dy = L.y + batch;
        L.acts_total = L.dy + batch;
        return L;
    }
};

hipError_t launch_tau_features(const double* pyr_a, const double* pyr_b, int64_t bdim, int lv, float log_target,
                               float* out, hipStream_t s);
// out[0] = smallest norm product >= lo (+inf bits if none), out[1] = largest
// product, as double bit patterns.
hipError_t launch_product_bounds(const double* pyr_a, const double* pyr_b, int64_t bdim, int lv, double lo,
                                 unsigned long long* out, hipStream_t s);
// *out = sum of x[q]^2 in FP64; partials holds kSumBlocks doubles.
hipError_t launch_sumsq(const float* x, int64_t count, double* partials, double* out, hipStream_t s);
hipError_t launch_mlp_forward(const float* params, const float* x, int batch, float* acts, float* y, hipStream_t s);
hipError_t launch_mlp_loss_grad(const float* params, const float* x, const float* t, int batch, float* acts,
                                float* grad, float* loss, hipStream_t s);
hipError_t launch_adam(float* params, const float* grad, float* m, float* v, int64_t count, float lr, float b1,
                       float b2, float eps, float c1, float c2, hipStream_t s);

// --------------------------------------------------------------------------
// Reduced-precision leaf products (split.hip, multiply_macro.hip).

constexpr int kPrecFp32 = 0, kPrecBf16 = 1, kPrecF16x3 = 2;

// Device pointers into a split buffer: scale exponents [2] (A, B), A planes
// (row-major, n x n halves), Bt planes (B transposed, n x n halves); the lo
// planes are used by f16x3 only.
struct SplitLayout {
    int32_t* exps;
    uint16_t *a_hi, *a_lo, *bt_hi, *bt_lo;
};

// A launch that runs only when the pair count the plan left on the device is
// at least (when_at_least = 1) or below (0) a threshold; pairs == nullptr:
// always.  Lets one stream hold both forms of a step and the device pick.
struct PairGate {
    const int64_t* pairs = nullptr;
    int64_t threshold = 0;
    int when_at_least = 1;
};

hipError_t launch_split(const float* a, const float* b, int64_t n, int64_t bdim, int lv, const double* pyr_a,
                        const double* pyr_b, int precision, const SplitLayout& L, hipStream_t s);
// The planes alone, after the exponents (launch_split_scales) are in L.exps.
hipError_t launch_split_planes(const float* a, const float* b, int64_t n, int precision, const SplitLayout& L,
                               const PairGate& gate, hipStream_t s);
// The f16x3 scale exponents alone (int32 exps at header[0..1], the two
// largest leaf norms at header + 8 bytes).
hipError_t launch_split_scales(int64_t bdim, int lv, const double* pyr_a, const double* pyr_b, int32_t* header,
                               hipStream_t s);
// Reduced-precision products (kPrecBf16 or kPrecF16x3) straight from the FP32
// inputs (the conversion done in registers), bitwise the same C as
// launch_split + launch_lowp_multiply.  exps: the split scale exponents
// (F16X3 only; may be null for BF16).
hipError_t launch_fused_multiply(const float* a, const float* b, int precision, const int32_t* exps, float* c,
                                 int64_t n, int64_t bdim, const uint32_t* items, const int32_t* uprefix, int num_cus,
                                 const PairGate& gate, hipStream_t s);
hipError_t launch_lowp_multiply(const SplitLayout& L, float* c, int64_t n, int64_t bdim, int precision,
                                const uint32_t* items, const int32_t* uprefix, int num_cus, const PairGate& gate,
                                hipStream_t s);

// --------------------------------------------------------------------------
// Batched products (kernels.hip): one descriptor per product in device memory.

struct BatchProduct {
    const float* a;
    const float* b;
    float* c;
    double* spyr[2];  // sums of squares (scratch) of A, B
    double* pyr[2];   // norm pyramids of A, B
    uint64_t* masks;
    int32_t* counts;
    int32_t* bsums;
    int32_t* boffs;
    int32_t* offsets;
    int32_t* klist;
    int32_t* pair_scratch;
    int64_t* pairs;  // this product's slot of the caller's pairs array
    int64_t n, bdim;
    int32_t leaf, lv, nw, vec;
    double tau;
    int64_t tile_base;  // prefix of bdim^2 over the batch's products with nw > 1
    int64_t mask_base;  // prefix of nw * bdim over the batch's products with nw > 1
    int64_t norm_base;  // prefix of bdim * ceil(n / 1024) (norm-pass strips) over the batch
    int64_t cost_base;  // written on the device: prefix of multiply cost within its leaf class
    // macro-tile schedule (leaf 32 and 64; mb = 0 for leaf 128): k bitmaps,
    // union sizes, their prefix, packed items, as in the single-product path
    uint64_t* mwords;
    int32_t* mcount;
    int32_t* mprefix;
    uint32_t* mitems;
    int64_t mb;          // macro tiles per side
    int64_t macro_base;  // prefix of mb^2 over the batch
};

// leaf classes of the batched multiply: 32, 64, 128
constexpr int kBatchClasses = 3;

// members: product indices grouped by class (class_count[c] entries each, in
// class order); class_total receives each class's total multiply cost.
// total_tiles and total_mask_blocks count the products with nw > 1 only;
// small_count is the number of products with nw = 1.
hipError_t launch_batch(const BatchProduct* prods, int32_t count, const int32_t* members,
                        const int32_t* class_count_host, int64_t* class_total, int64_t total_tiles,
                        int64_t total_mask_blocks, int64_t total_strips, int64_t total_macros, int32_t small_count,
                        int num_cus, hipStream_t s);

}  // namespace spamm
