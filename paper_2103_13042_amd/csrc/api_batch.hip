// Host side of the batched entry points: many independent SpAMM products, each
// stage of the path one launch over all of them.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "host.h"
#include "internal.h"
#include "spamm.h"

using namespace spamm_host;

namespace {

constexpr size_t kAlignB = 256;
constexpr int64_t kNormCols = 1024;  // columns per block of the norm pass
size_t up(size_t v) { return (v + kAlignB - 1) / kAlignB * kAlignB; }

int leaf_class(int32_t leaf) { return leaf == 32 ? 0 : leaf == 64 ? 1 : leaf == 128 ? 2 : -1; }

struct BatchPlan {
    size_t header = 0, total = 0;
    std::vector<size_t> base;  // per product region offset
    std::vector<Geom> geom;
    int64_t tiles = 0, mask_blocks = 0, strips = 0, macros = 0;  // tiles, mask_blocks: products with nwords > 1
    int32_t small_count = 0;                                     // products with nwords = 1
    int32_t class_count[spamm::kBatchClasses] = {0, 0, 0};
};

// macro tiles per side of a product's multiply schedule (leaf 32; 0 for leaf
// 64 and 128, which run on single tiles: the register-staged macro kernel is
// slower than the single-tile one for the ragged leaf-64 products of a batch)
int64_t macro_side(const Geom& g) { return g.leaf == 32 ? (g.bdim + 1) / 2 : 0; }

size_t product_bytes(const Geom& g) {
    const size_t pyr = up(sizeof(double) * size_t(g.pyr));
    const size_t nt = size_t(g.ntiles), b = size_t(g.bdim), nw = size_t(g.nwords);
    const size_t nm = size_t(macro_side(g)) * size_t(macro_side(g));
    const size_t macro = nm ? up(sizeof(uint64_t) * nm * 4 * nw) + up(sizeof(int32_t) * nm) +
                                  up(sizeof(int32_t) * (nm + 1)) + up(sizeof(uint32_t) * nm * b)
                            : 0;
    return 4 * pyr + up(sizeof(uint64_t) * nt * nw) + up(sizeof(int32_t) * nt) + 2 * up(sizeof(int32_t) * b * nw) +
           up(sizeof(int32_t) * (nt + 1)) + 2 * up(sizeof(int32_t) * nt * b) + macro;
}

spamm_status plan_batch(int32_t count, const int64_t* n, const int32_t* leaf, BatchPlan* bp) {
    if (count < 1 || !n || !leaf) return fail(SPAMM_EINVAL, "empty batch or null size arrays");
    bp->geom.resize(size_t(count));
    bp->base.resize(size_t(count));
    bp->header = up(sizeof(spamm::BatchProduct) * size_t(count)) + up(sizeof(int32_t) * size_t(count)) +
                 up(sizeof(int64_t) * spamm::kBatchClasses);
    size_t o = bp->header;
    for (int32_t p = 0; p < count; ++p) {
        Geom& g = bp->geom[size_t(p)];
        if (!make_geom(n[p], leaf[p], &g)) return fail(SPAMM_EINVAL, "product %d: bad size n=%lld leaf=%d", p,
                                                       (long long)n[p], leaf[p]);
        if (leaf_class(leaf[p]) < 0) return fail(SPAMM_EUNSUPPORTED, "product %d: leaf %d (32, 64, 128)", p, leaf[p]);
        if (g.bdim > SPAMM_MAX_BDIM)
            return fail(SPAMM_EUNSUPPORTED, "product %d: tile grid %lld exceeds %d", p, (long long)g.bdim,
                        SPAMM_MAX_BDIM);
        bp->base[size_t(p)] = o;
        o += product_bytes(g);
        if (g.nwords > 1) {
            bp->tiles += g.ntiles;
            bp->mask_blocks += g.bdim * g.nwords;
        } else {
            ++bp->small_count;
        }
        bp->strips += g.bdim * ((g.n + kNormCols - 1) / kNormCols);
        bp->macros += macro_side(g) * macro_side(g);
        ++bp->class_count[leaf_class(leaf[p])];
    }
    bp->total = o;
    return SPAMM_OK;
}

}  // namespace

extern "C" {

size_t spamm_batch_workspace_bytes(int32_t count, const int64_t* n, const int32_t* leaf) {
    BatchPlan bp;
    return plan_batch(count, n, leaf, &bp) == SPAMM_OK ? bp.total : 0;
}

spamm_status spamm_batch_setup(int32_t count, const float* const* a, const float* const* b, float* const* c,
                               const int64_t* n, const int32_t* leaf, const double* tau, int64_t* pairs,
                               void* workspace, size_t workspace_bytes, void* stream) {
    g_last_error[0] = '\0';
    BatchPlan bp;
    spamm_status st = plan_batch(count, n, leaf, &bp);
    if (st != SPAMM_OK) return st;
    if (!a || !b || !c || !tau || !pairs || !workspace) return fail(SPAMM_EINVAL, "null pointer");
    if (workspace_bytes < bp.total)
        return fail(SPAMM_ENOSPACE, "batch workspace of %zu bytes, %zu needed", workspace_bytes, bp.total);
    if ((reinterpret_cast<uintptr_t>(workspace) & (kAlignB - 1)) != 0)
        return fail(SPAMM_EINVAL, "workspace must be 256-byte aligned");
    std::vector<spamm::BatchProduct> prods(static_cast<size_t>(count));
    std::vector<int32_t> members;
    members.reserve(size_t(count));
    char* ws = static_cast<char*>(workspace);
    int64_t tile_base = 0, mask_base = 0, norm_base = 0, macro_base = 0;
    for (int32_t p = 0; p < count; ++p) {
        const Geom& g = bp.geom[size_t(p)];
        if ((st = check_mul_args(g, a[p], b[p], c[p])) != SPAMM_OK || (st = check_tau(tau[p])) != SPAMM_OK) {
            char why[sizeof(g_last_error)];
            std::memcpy(why, g_last_error, sizeof(why));
            return fail(st, "product %d: %s", p, why);
        }
        spamm::BatchProduct& q = prods[size_t(p)];
        std::memset(&q, 0, sizeof(q));
        char* r = ws + bp.base[size_t(p)];
        auto take = [&](size_t bytes) {
            char* at = r;
            r += up(bytes);
            return at;
        };
        const size_t nt = size_t(g.ntiles), bd = size_t(g.bdim), nw = size_t(g.nwords);
        for (int m = 0; m < 2; ++m) q.spyr[m] = reinterpret_cast<double*>(take(sizeof(double) * size_t(g.pyr)));
        for (int m = 0; m < 2; ++m) q.pyr[m] = reinterpret_cast<double*>(take(sizeof(double) * size_t(g.pyr)));
        q.masks = reinterpret_cast<uint64_t*>(take(sizeof(uint64_t) * nt * nw));
        q.counts = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * nt));
        q.bsums = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * bd * nw));
        q.boffs = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * bd * nw));
        q.offsets = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * (nt + 1)));
        q.klist = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * nt * bd));
        q.pair_scratch = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * nt * bd));
        q.mb = macro_side(g);
        const size_t nm = size_t(q.mb) * size_t(q.mb);
        if (nm) {
            q.mwords = reinterpret_cast<uint64_t*>(take(sizeof(uint64_t) * nm * 4 * nw));
            q.mcount = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * nm));
            q.mprefix = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * (nm + 1)));
            q.mitems = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * nm * bd));
        }
        q.a = a[p];
        q.b = b[p];
        q.c = c[p];
        q.pairs = pairs + p;
        q.n = g.n;
        q.bdim = g.bdim;
        q.leaf = g.leaf;
        q.lv = g.lv;
        q.nw = g.nwords;
        q.vec = (g.n % 4) == 0 && aligned16(a[p]) && aligned16(b[p]);
        q.tau = tau[p];
        q.tile_base = tile_base;
        q.mask_base = mask_base;
        q.norm_base = norm_base;
        q.macro_base = macro_base;
        macro_base += q.mb * q.mb;
        if (g.nwords > 1) {
            tile_base += g.ntiles;
            mask_base += g.bdim * g.nwords;
        }
        norm_base += g.bdim * ((g.n + kNormCols - 1) / kNormCols);
    }
    for (int cls = 0; cls < spamm::kBatchClasses; ++cls)
        for (int32_t p = 0; p < count; ++p)
            if (leaf_class(leaf[p]) == cls) members.push_back(p);
    hipStream_t s = static_cast<hipStream_t>(stream);
    st = hip_check(hipMemcpyAsync(ws, prods.data(), sizeof(spamm::BatchProduct) * size_t(count),
                                  hipMemcpyHostToDevice, s),
                   "descriptor upload");
    if (st != SPAMM_OK) return st;
    st = hip_check(hipMemcpyAsync(ws + up(sizeof(spamm::BatchProduct) * size_t(count)), members.data(),
                                  sizeof(int32_t) * members.size(), hipMemcpyHostToDevice, s),
                   "descriptor upload");
    if (st != SPAMM_OK) return st;
    return hip_check(hipStreamSynchronize(s), "synchronize");
}

spamm_status spamm_batch_run(int32_t count, const int64_t* n, const int32_t* leaf, void* workspace,
                             size_t workspace_bytes, void* stream) {
    g_last_error[0] = '\0';
    BatchPlan bp;
    spamm_status st = plan_batch(count, n, leaf, &bp);
    if (st != SPAMM_OK) return st;
    if (!workspace) return fail(SPAMM_EINVAL, "null workspace");
    if (workspace_bytes < bp.total)
        return fail(SPAMM_ENOSPACE, "batch workspace of %zu bytes, %zu needed", workspace_bytes, bp.total);
    char* ws = static_cast<char*>(workspace);
    const auto* prods = reinterpret_cast<const spamm::BatchProduct*>(ws);
    const auto* members = reinterpret_cast<const int32_t*>(ws + up(sizeof(spamm::BatchProduct) * size_t(count)));
    auto* class_total = reinterpret_cast<int64_t*>(ws + up(sizeof(spamm::BatchProduct) * size_t(count)) +
                                                   up(sizeof(int32_t) * size_t(count)));
    int cus = device_cus();
    cus = (cus + 3) / 4 * 4;  // two groups per CU, a multiple of 8 in all
    return hip_check(spamm::launch_batch(prods, count, members, bp.class_count, class_total, bp.tiles,
                                         bp.mask_blocks, bp.strips, bp.macros, bp.small_count, cus,
                                         static_cast<hipStream_t>(stream)),
                     "batch kernels");
}

}  // extern "C"
