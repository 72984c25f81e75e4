/*
 * spamm.h - C ABI of libspamm.so, Sparse Approximate Matrix Multiplication
 * (SpAMM) on AMD Instinct MI355X (gfx950).
 *
 * The method is the one of Liu et al., "Accelerating Sparse Approximate Matrix
 * Multiplication on GPUs" (arXiv 2103.13042), section 2.1 and section 3:
 * C = A*B restricted to the leaf-tile products A[i,k]*B[k,j] whose Frobenius
 * norm product ||A[i,k]||_F * ||B[k,j]||_F is at least tau (Algorithm 1,
 * Eq. 1, Eq. 2), with alpha = 1 and beta = 0 (C is overwritten), square N x N.
 *
 * Conventions shared by every entry point:
 *  - Matrices are FP32, row-major, contiguous, leading dimension N, and live in
 *    DEVICE memory.  Norms and pyramids are FP64 device arrays.
 *  - leaf is the edge of a leaf tile (the paper's LoNum); bdim = ceil(N/leaf)
 *    tiles per side.  The matrix is treated as zero padded to bdim*leaf (and,
 *    for the quadtree, to leaf*2^Lv with Lv = ceil(log2(bdim))).
 *  - stream is a hipStream_t (NULL: the default stream).  Every call only
 *    enqueues work on that stream and returns; nothing synchronises the host.
 *    Outputs are valid once the stream reaches that point.
 *  - Callers pass every output buffer.  The workspace is either the caller's
 *    (at least spamm_workspace_bytes(N, leaf) bytes of device memory; the
 *    library then allocates nothing) or NULL: the library then uses one
 *    workspace per device that it allocates on first use, grows when a call
 *    needs more (after synchronising the device, so the first call at a new
 *    largest size must not be under graph capture), and frees in
 *    spamm_release(); workspace_bytes is ignored.  The library never frees or
 *    retains caller memory.  Calls that share a workspace, including the
 *    cached one of a device, must be ordered (same stream, or synchronised),
 *    and a pair of calls that passes state through it (spamm_prepare, then
 *    spamm_execute) must not be separated by a call that grows it.
 *  - Errors: argument checks happen on the host before anything is enqueued;
 *    on a failure nothing is written and a status code is returned.
 *    SPAMM_EDEVICE reports a failed HIP call; spamm_last_error() gives the
 *    detail (per thread).
 */
#ifndef SPAMM_H
#define SPAMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum spamm_status {
    SPAMM_OK = 0,
    SPAMM_EINVAL = 1,       /* invalid argument: size, pointer, tau, aliasing */
    SPAMM_ENOSPACE = 2,     /* workspace or output capacity too small, or the cached
                               workspace could not be allocated */
    SPAMM_EDEVICE = 3,      /* a HIP runtime call or kernel launch failed */
    SPAMM_EUNSUPPORTED = 4  /* leaf size or problem size not handled by the GPU path */
} spamm_status;

/* Largest tile grid the GPU path accepts (bdim <= SPAMM_MAX_BDIM keeps every
 * pair index of the worst case bdim^3 inside int32). */
#define SPAMM_MAX_BDIM 1024

/* ceil(n / leaf), or 0 when n <= 0 or leaf <= 0.  Host only. */
int64_t spamm_bdim(int64_t n, int32_t leaf);

/* Lv = ceil(log2(bdim)): quadtree depth above the leaf tiles (Eq. 1).  Host only. */
int32_t spamm_levels(int64_t n, int32_t leaf);

/* Number of FP64 entries of a norm pyramid: sum over l = 0..Lv of 4^l.  Host only. */
int64_t spamm_pyramid_size(int64_t n, int32_t leaf);

/* 1 when the GPU path has multiply kernels for this leaf size (LoNum of
 * section 3: 16, 32, 64, 128), else 0. */
int32_t spamm_leaf_supported(int32_t leaf);

/* Free the workspaces the library allocated for calls with a NULL workspace
 * (one per device that ran such a call), after synchronising each of those
 * devices.  Later calls with a NULL workspace allocate again.  Host only;
 * SPAMM_EDEVICE when a HIP call fails. */
spamm_status spamm_release(void);

/* Workspace size that every entry point below accepts for (n, leaf); 0 when the
 * arguments are invalid.  Host only. */
size_t spamm_workspace_bytes(int64_t n, int32_t leaf);

/* Leaf-tile Frobenius norms (Eq. 2; the get-norm kernel of section 3.2).
 *   x      [n*n] FP32 device matrix.
 *   norms  [bdim*bdim] FP64 device output, row-major: norms[i*bdim + j] =
 *          ||X[i,j]||_F over the tile's elements inside the matrix.
 * Squares are summed in FP64 (every FP32 square is exact in FP64).  Any leaf
 * in 1..1024 is accepted.  EINVAL: null pointer, n <= 0, bad leaf. */
spamm_status spamm_norms(const float* x, int64_t n, int32_t leaf, double* norms, void* stream);

/* Quadtree norm pyramid (Eq. 1 and Eq. 2 at every level, the norms Algorithm 1
 * tests at each recursion level).
 *   pyramid [spamm_pyramid_size(n, leaf)] FP64 device output.  Level l (0 = root,
 *           Lv = leaf tiles) holds 2^l x 2^l node norms, row-major, starting at
 *           entry (4^l - 1)/3.  Tiles outside the bdim x bdim grid have norm 0.
 * Each parent's sum of squares is the FP64 sum of its four children's, so a
 * parent norm is never below a child norm.
 *   workspace: at least spamm_workspace_bytes(n, leaf) bytes of device memory.
 * EINVAL as spamm_norms; ENOSPACE when workspace_bytes is too small. */
spamm_status spamm_pyramid(const float* x, int64_t n, int32_t leaf, double* pyramid, void* workspace,
                           size_t workspace_bytes, void* stream);

/* Pruning plan (Algorithm 1's norm tests flattened as in section 3.1, and the
 * bitmap / offset list of the multiplication kernel, Algorithm 2).
 *   pyr_a, pyr_b  pyramids of A and B from spamm_pyramid (same n, leaf).
 *   tau           threshold, 0 <= tau <= +inf.  Triple (i,k,j) is kept when
 *                 the FP64 product pyr_a[leaf](i,k) * pyr_b[leaf](k,j) >= tau;
 *                 pyramid levels above the leaves only skip ranges of k whose
 *                 node product is already below tau.
 *   offsets       [bdim*bdim + 1] int32 device output: the kept k of output
 *                 tile t = i*bdim + j are klist[offsets[t] .. offsets[t+1]),
 *                 ascending.  offsets[bdim*bdim] is the total.
 *   klist         int32 device output, capacity klist_capacity entries, which
 *                 must be >= bdim^3 (ENOSPACE otherwise).
 *   pairs         one int64 in device memory: number of kept triples.
 * EINVAL: null pointer, bad n/leaf, tau NaN or negative. */
spamm_status spamm_plan(const double* pyr_a, const double* pyr_b, int64_t n, int32_t leaf, double tau,
                        int32_t* offsets, int32_t* klist, int64_t klist_capacity, int64_t* pairs,
                        void* workspace, size_t workspace_bytes, void* stream);

/* Multiply the kept leaf pairs of a plan (the multiplication kernel, section 3.3,
 * with the load balancing of section 3.5.1 done by a cost-balanced static
 * partition of the output tiles).
 *   a, b      [n*n] FP32 device inputs; c [n*n] FP32 device output, overwritten
 *             (beta = 0): tiles with no kept pair become zero.
 *   offsets, klist: a plan from spamm_plan for the same n and leaf.
 * Products use FP32 matrix-core instructions with FP32 accumulation, k in
 * ascending order per output tile.  The leaf must be supported
 * (spamm_leaf_supported), else EUNSUPPORTED.  EINVAL: null pointer, c
 * overlapping a or b. */
spamm_status spamm_execute(const float* a, const float* b, int64_t n, int32_t leaf, const int32_t* offsets,
                           const int32_t* klist, float* c, void* workspace, size_t workspace_bytes, void* stream);

/* spamm_execute in its two launch steps, for callers that time the multiply
 * kernel on its own.  spamm_schedule derives from a plan what the multiply
 * kernel streams (for leaf 32 and 64: per 2x2 block of output tiles the four
 * k-bitmaps and the size of their union, and the prefix of those sizes; for
 * leaf 128 nothing) and keeps it in the workspace; spamm_execute_scheduled
 * then launches the multiply kernel alone.  The pair equals spamm_execute when
 * both get the same plan and workspace with no other call on that workspace
 * in between.  Arguments and errors as spamm_execute (section 3.3, 3.5.1). */
spamm_status spamm_schedule(const int32_t* offsets, const int32_t* klist, int64_t n, int32_t leaf, void* workspace,
                            size_t workspace_bytes, void* stream);
spamm_status spamm_execute_scheduled(const float* a, const float* b, int64_t n, int32_t leaf, const int32_t* offsets,
                                     const int32_t* klist, float* c, void* workspace, size_t workspace_bytes,
                                     void* stream);

/* The first half of the hot path for one product: leaf norms and pyramids of A
 * and B (one launch each for both matrices) and the plan for tau, as
 * spamm_pyramid and spamm_plan would produce them.  The pyramids stay in the
 * workspace; offsets, klist and pairs are as in spamm_plan.  Followed by
 * spamm_execute this enqueues the kernels of spamm_multiply, except for the
 * small products that spamm_multiply runs in two launches (below).
 * Errors as spamm_plan, plus EINVAL for null a or b. */
spamm_status spamm_prepare(const float* a, const float* b, int64_t n, double tau, int32_t leaf, int32_t* offsets,
                           int32_t* klist, int64_t klist_capacity, int64_t* pairs, void* workspace,
                           size_t workspace_bytes, void* stream);

/* spamm_prepare followed by spamm_schedule on the plan it writes (the first
 * half of spamm_multiply): the same offsets, klist and pairs, and a workspace
 * from which spamm_execute_scheduled may follow.  For leaf 32 and 64 the
 * plan and the multiply schedule come from one launch (the norm tests,
 * bitmaps, map_offset and validNum of Algorithm 2 and the union k-lists of
 * section 3.5.1's work split, with the prefix over tile rows by a
 * single-pass look-back) instead of six; that launch (up to 256 tiles per
 * side) tests every triple on the leaf norms, and the pyramid above the leaf
 * level is not built.  Errors as spamm_prepare and spamm_schedule. */
spamm_status spamm_prepare_schedule(const float* a, const float* b, int64_t n, double tau, int32_t leaf,
                                    int32_t* offsets, int32_t* klist, int64_t klist_capacity, int64_t* pairs,
                                    void* workspace, size_t workspace_bytes, void* stream);

/* The whole SpAMM hot path: pyramids of A and B, the plan for tau, and the
 * multiplication of the kept pairs, enqueued back to back on one stream.
 *   c      [n*n] FP32 device output, overwritten.
 *   pairs  one int64 in device memory (may be NULL): number of multiplied
 *          leaf-tile pairs, i.e. the valid ratio of section 3.5.2 times bdim^3.
 * Small products (leaf 32, at most 64 tiles per side, n a multiple of 4, a and
 * b 16-byte aligned) take two launches instead: the leaf norm pass, then one
 * kernel that applies the threshold test of Algorithm 1 to the leaf norms and
 * multiplies the kept pairs.  The pairs are those of the plan; C differs from
 * spamm_prepare + spamm_execute only in the order of the FP32 additions (the
 * k-range of an output tile is split four ways and the parts are added in a
 * fixed order, so repeated calls agree bitwise); the workspace then holds the
 * leaf norms but no pyramid or plan.
 * Errors as spamm_pyramid, spamm_plan and spamm_execute. */
spamm_status spamm_multiply(const float* a, const float* b, int64_t n, double tau, int32_t leaf, float* c,
                            int64_t* pairs, void* workspace, size_t workspace_bytes, void* stream);

/* Reduced-precision leaf products.  The skip mask is that of the FP32 inputs
 * (norms, pyramid and plan as above); only the leaf products change, as the
 * paper's FP16 tensor-core variant does (Algorithm 3, section 3.3):
 *   SPAMM_PREC_BF16   every element of A and B rounded to bfloat16 (nearest,
 *                     ties to even); FP32 accumulation of the exact products.
 *   SPAMM_PREC_F16X3  per matrix a power-of-two scale s = 2^(15 - ceil(log2 M)),
 *                     M its largest leaf-tile norm; hi = fp16(s x),
 *                     lo = fp16(s x - hi); per leaf product hi*hi + hi*lo +
 *                     lo*hi accumulated in FP32, scaled by 1/(sA sB) when stored.
 * Supported for leaf 64 and n a multiple of 128 (EUNSUPPORTED otherwise). */
#define SPAMM_PREC_FP32 0
#define SPAMM_PREC_BF16 1
#define SPAMM_PREC_F16X3 2

/* Bytes of the split operands of A and B for a precision (0 for FP32 or bad
 * arguments): a 256-byte header (int32 scale exponents of A and B at byte 0,
 * the largest leaf norms as doubles at byte 8), then n*n halves per
 * plane: A (row-major), [A lo], B transposed, [B lo transposed]. */
size_t spamm_split_bytes(int64_t n, int32_t precision);

/* Write the split operands of A and B into `split` (device, 256-byte aligned,
 * spamm_split_bytes bytes).  pyr_a, pyr_b: their pyramids (spamm_pyramid or
 * spamm_prepare's workspace copies), used for the f16x3 scales.  EINVAL: null
 * pointer, misalignment (a and b 16 bytes), overlap with a or b, precision not
 * BF16/F16X3; ENOSPACE: split too small. */
spamm_status spamm_split(const float* a, const float* b, int64_t n, int32_t leaf, int32_t precision,
                         const double* pyr_a, const double* pyr_b, void* split, size_t split_bytes, void* stream);

/* spamm_execute with reduced-precision products from split operands:
 * spamm_execute_split = spamm_schedule + spamm_execute_split_scheduled (the
 * multiply kernel alone, after spamm_schedule on the same plan and workspace). */
spamm_status spamm_execute_split(const void* split, int64_t n, int32_t leaf, int32_t precision,
                                 const int32_t* offsets, const int32_t* klist, float* c, void* workspace,
                                 size_t workspace_bytes, void* stream);
spamm_status spamm_execute_split_scheduled(const void* split, int64_t n, int32_t leaf, int32_t precision,
                                           const int32_t* offsets, const int32_t* klist, float* c, void* workspace,
                                           size_t workspace_bytes, void* stream);

/* The F16X3 scale exponents alone, as spamm_split writes them into the first
 * 256 bytes of its buffer (int32 exponents of A and B at byte 0, their
 * largest leaf norms as doubles at byte 8), from the pyramids of A and B.
 * header: device, 256-byte aligned, header_bytes >= 256.  EINVAL: null
 * pointer, misalignment, bad size; ENOSPACE: header_bytes < 256;
 * EUNSUPPORTED: leaf or n outside the reduced-precision shapes. */
spamm_status spamm_split_scales(const double* pyr_a, const double* pyr_b, int64_t n, int32_t leaf, void* header,
                                size_t header_bytes, void* stream);

/* F16X3 products straight from the FP32 inputs, after spamm_schedule on the
 * same plan and workspace: one kernel stages FP32 tiles of A and B and splits
 * them into hi and lo in registers with the exponents of `header`
 * (spamm_split_scales), so C is bitwise the C of spamm_split +
 * spamm_execute_split_scheduled without the split pass over A and B.  a, b:
 * device, 16-byte aligned.  Errors as spamm_execute_split_scheduled (EINVAL
 * also for c overlapping the header). */
spamm_status spamm_execute_f16x3_scheduled(const float* a, const float* b, int64_t n, int32_t leaf,
                                           const void* header, const int32_t* offsets, const int32_t* klist,
                                           float* c, void* workspace, size_t workspace_bytes, void* stream);

/* BF16 products (section 3.3's reduced-precision leaf products, FP32
 * accumulation) straight from the FP32 inputs, after spamm_prepare and
 * spamm_schedule on the same plan and workspace: one kernel stages FP32 tiles
 * of A and B and rounds them to BF16 (nearest-even) in registers, so C is
 * bitwise the C of spamm_split + spamm_execute_split_scheduled with
 * SPAMM_PREC_BF16, without the split pass over A and B.  a, b: device, 16-byte
 * aligned; c overwritten.  Errors as spamm_execute_split_scheduled. */
spamm_status spamm_execute_bf16_scheduled(const float* a, const float* b, int64_t n, int32_t leaf,
                                          const int32_t* offsets, const int32_t* klist, float* c, void* workspace,
                                          size_t workspace_bytes, void* stream);

/* spamm_prepare followed by spamm_split_scales on the pyramids it leaves in
 * the workspace (the first stage of the F16X3 path of
 * spamm_multiply_precision).  Errors as spamm_prepare and spamm_split_scales
 * (EINVAL also for a header overlapping a or b). */
spamm_status spamm_prepare_scales(const float* a, const float* b, int64_t n, double tau, int32_t leaf,
                                  int32_t* offsets, int32_t* klist, int64_t klist_capacity, int64_t* pairs,
                                  void* header, size_t header_bytes, void* workspace, size_t workspace_bytes,
                                  void* stream);

/* spamm_prepare_schedule followed by spamm_split_scales on the leaf norms it
 * leaves in the workspace: the plan, the multiply schedule and the FP16 hi+lo
 * scale exponents, so that spamm_execute_f16x3_scheduled can follow directly
 * (the first stage of the in-register F16X3 path of spamm_multiply_precision,
 * which uses the one-launch plan and schedule where spamm_prepare_schedule
 * does).  Arguments as spamm_prepare_scales; the same offsets, k-lists, pairs
 * and header.  The header (256-byte aligned, at least 256 bytes, not
 * overlapping a or b: else EINVAL or ENOSPACE) is checked before anything is
 * enqueued.  Other errors as spamm_prepare_schedule. */
spamm_status spamm_prepare_schedule_scales(const float* a, const float* b, int64_t n, double tau, int32_t leaf,
                                           int32_t* offsets, int32_t* klist, int64_t klist_capacity,
                                           int64_t* pairs, void* header, size_t header_bytes, void* workspace,
                                           size_t workspace_bytes, void* stream);

/* spamm_prepare followed by spamm_split on the pyramids it leaves in the
 * workspace (the first half of spamm_multiply_precision).  Errors as
 * spamm_prepare and spamm_split. */
spamm_status spamm_prepare_split(const float* a, const float* b, int64_t n, double tau, int32_t leaf,
                                 int32_t precision, int32_t* offsets, int32_t* klist, int64_t klist_capacity,
                                 int64_t* pairs, void* split, size_t split_bytes, void* workspace,
                                 size_t workspace_bytes, void* stream);

/* The whole path with reduced-precision products.  F16X3:
 * spamm_prepare_schedule_scales into the first 256 bytes of `split`, then
 * either the planes and the split multiply (spamm_split's planes,
 * spamm_execute_split_scheduled) or the in-register split
 * (spamm_execute_f16x3_scheduled), picked on the device from the plan's pair
 * count: the planes when it keeps at least 45 pairs per output tile on
 * average.  With split_bytes below spamm_split_bytes (at least 256), always
 * in registers and the planes are not written.  BF16: the same with
 * spamm_prepare_schedule (no scales) and spamm_execute_bf16_scheduled, the planes from
 * 16 pairs per tile; split may be NULL (then always in registers).  Either
 * way C is bitwise the C of the split path.  SPAMM_PREC_FP32 is
 * spamm_multiply (split unused, may be NULL).  Errors as spamm_multiply and
 * spamm_split (F16X3: EINVAL for a header that is null, not 256-byte aligned
 * or overlapping a, b or c; ENOSPACE below 256 bytes). */
spamm_status spamm_multiply_precision(const float* a, const float* b, int64_t n, double tau, int32_t leaf,
                                      int32_t precision, float* c, int64_t* pairs, void* split, size_t split_bytes,
                                      void* workspace, size_t workspace_bytes, void* stream);

/* Batches of independent products (each its own n, leaf and tau; the same
 * result as spamm_multiply on each, up to FP32 accumulation order).  Every
 * stage of the path is one launch over the whole batch: leaf norms, pyramids,
 * plan (mask, scan, fill), the per-class cost prefix, and one persistent
 * multiply launch per leaf class present (32, 64, 128) whose workgroups split
 * the class's total cost (section 3.5.1's balance, across products).
 *
 * spamm_batch_workspace_bytes: device bytes for a batch (0 on bad arguments).
 * spamm_batch_setup: binds the batch to its matrices.  a, b, c: HOST arrays of
 *   `count` device pointers (n[p] x n[p] FP32 row-major, c overwritten); n,
 *   leaf, tau: HOST arrays; pairs: DEVICE int64[count], receives each
 *   product's kept pairs.  Lays out the workspace and uploads per-product
 *   descriptors (synchronous).  EINVAL/EUNSUPPORTED per product as
 *   spamm_multiply (leaf 32, 64 or 128); ENOSPACE: workspace too small.
 * spamm_batch_run: runs a set-up batch (same count, n, leaf, workspace):
 *   kernel launches only, no host synchronisation, no allocation and no
 *   copies, so it can be captured in a graph and replayed. */
size_t spamm_batch_workspace_bytes(int32_t count, const int64_t* n, const int32_t* leaf);
spamm_status spamm_batch_setup(int32_t count, const float* const* a, const float* const* b, float* const* c,
                               const int64_t* n, const int32_t* leaf, const double* tau, int64_t* pairs,
                               void* workspace, size_t workspace_bytes, void* stream);
spamm_status spamm_batch_run(int32_t count, const int64_t* n, const int32_t* leaf, void* workspace,
                             size_t workspace_bytes, void* stream);

/* The valid-ratio search of section 3.5.2: the threshold tau whose valid
 * ratio (kept leaf triples / bdim^3) is within tol of target.  ave is the
 * mean of the norm products over all bdim^3 triples; tau starts at ave; while
 * the ratio at the upper bound k*ave exceeds target + tol, k grows by one (at
 * most 1024 times); then tau is bisected in [0, k*ave] until the ratio is
 * within tol of target or max_iters bisections ran.
 *   pyr_a, pyr_b  pyramids from spamm_pyramid (device).
 *   tau_out       HOST double: the threshold found (the last one tried).
 *   pairs_out     HOST int64 (may be NULL): kept triples at tau_out.
 *   iters_out     HOST int32 (may be NULL): bisection steps taken.
 * Synchronous: reads each count back to the host (the stream is synchronised
 * once per tried tau).  EINVAL: target outside (0, 1], tol < 0,
 * max_iters < 0, null pointer. */
spamm_status spamm_search_valid_ratio(const double* pyr_a, const double* pyr_b, int64_t n, int32_t leaf,
                                      double target, double tol, int32_t max_iters, double* tau_out,
                                      int64_t* pairs_out, int32_t* iters_out, void* workspace, size_t workspace_bytes,
                                      void* stream);

/* Static description of a status code. */
const char* spamm_strerror(spamm_status status);

/* Detail of the last failure on the calling thread ("" if none). */
const char* spamm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SPAMM_H */
