// Host side of libspamm.so: argument checks, workspace layout, and the
// enqueueing of the kernels of the SpAMM hot path on the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "spamm.h"
#include "dma.h"
#include "host.h"
#include "internal.h"

namespace spamm_host {


thread_local char g_last_error[512] = "";

spamm_status fail(spamm_status st, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
    return st;
}

spamm_status hip_check(hipError_t e, const char* what) {
    if (e == hipSuccess) return SPAMM_OK;
    return fail(SPAMM_EDEVICE, "%s: %s (%d)", what, hipGetErrorString(e), int(e));
}

bool make_geom(int64_t n, int32_t leaf, Geom* g) {
    if (n <= 0 || leaf <= 0 || leaf > 1024) return false;
    g->n = n;
    g->leaf = leaf;
    g->bdim = (n + leaf - 1) / leaf;
    int32_t lv = 0;
    while ((int64_t(1) << lv) < g->bdim) ++lv;
    g->lv = lv;
    g->side = int64_t(1) << lv;
    g->ntiles = g->bdim * g->bdim;
    g->pyr = spamm::level_offset(lv + 1);
    g->nwords = int32_t((g->bdim + 63) / 64);
    return true;
}

namespace {
constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
}  // namespace

Layout make_layout(const Geom& g) {
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    for (int m = 0; m < 2; ++m) L.spyr[m] = take(sizeof(double) * size_t(g.pyr));
    for (int m = 0; m < 2; ++m) L.pyr[m] = take(sizeof(double) * size_t(g.pyr));
    L.counts = take(sizeof(int32_t) * size_t(g.ntiles));
    L.bsums = take(sizeof(int32_t) * size_t(g.bdim) * size_t(g.nwords));
    L.boffs = take(sizeof(int32_t) * size_t(g.bdim) * size_t(g.nwords));
    L.masks = take(sizeof(uint64_t) * size_t(g.ntiles) * size_t(g.nwords));
    L.offsets = take(sizeof(int32_t) * size_t(g.ntiles + 1));
    L.klist = take(sizeof(int32_t) * size_t(g.ntiles) * size_t(g.bdim));
    L.pair_scratch = take(sizeof(int32_t) * size_t(g.ntiles) * size_t(g.bdim));
    const size_t nm = size_t((g.bdim + 1) / 2) * size_t((g.bdim + 1) / 2);
    L.mwords = take(sizeof(uint64_t) * nm * 4 * size_t(g.nwords));
    L.mcount = take(sizeof(int32_t) * nm);
    L.mprefix = take(sizeof(int32_t) * (nm + 1));
    L.mitems = take(sizeof(uint32_t) * nm * size_t(g.bdim));
    // leaf 128 on the LDS-DMA kernel: two items per kept pair, their prefix
    const bool l128 = g.leaf == 128 && g.n % 128 == 0 && g.bdim <= spamm::kLeaf128MaxBdim;
    L.leaf128_dma = l128;
    L.items128 = take(l128 ? sizeof(uint32_t) * 2 * size_t(g.ntiles) * size_t(g.bdim) : 0);
    L.uprefix128 = take(l128 ? sizeof(int32_t) * size_t(g.ntiles + 1) : 0);
    L.bounds = take(sizeof(int64_t) * 4 * spamm::kSplitMaxGroups);
    // partial sums of shared macro tiles (LDS-DMA kernel: leaf 64 or 128, N a
    // multiple of 128), two slots per workgroup, at most one workgroup per
    // macro tile
    const bool dma = (g.leaf == 64 && g.n % 128 == 0) || l128;
    const size_t macros = l128 ? size_t(g.ntiles) : nm;
    const size_t groups =
        macros < size_t(spamm::kSplitMaxGroups) ? (macros + 7) / 8 * 8 : size_t(spamm::kSplitMaxGroups);
    L.fix_slot_bytes = dma ? sizeof(float) * groups * 2 * spamm::kSplitSlotFloats : 0;
    L.fix_slots = take(L.fix_slot_bytes);
    L.pm_state = take(sizeof(int64_t) * size_t(spamm::plan_macro_clear_words(g.bdim)));
    L.pairs = take(sizeof(int64_t));
    L.scalars = take(4 * sizeof(double));
    L.partials = take(sizeof(double) * 1024);
    L.total = o;
    return L;
}

bool overlaps(const void* p, size_t pbytes, const void* q, size_t qbytes) {
    const char* a = static_cast<const char*>(p);
    const char* b = static_cast<const char*>(q);
    return a < b + qbytes && b < a + pbytes;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

int device_cus() {
    static std::mutex mu;
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    std::lock_guard<std::mutex> lock(mu);
    if (cached[dev] == 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        cached[dev] = cus;
    }
    return cached[dev];
}

spamm_status check_grid(const Geom& g) {
    if (g.bdim > SPAMM_MAX_BDIM)
        return fail(SPAMM_EUNSUPPORTED, "tile grid %lld exceeds %d per side", (long long)g.bdim, SPAMM_MAX_BDIM);
    return SPAMM_OK;
}

// Workspaces the library keeps for callers that pass none: one per device,
// grown to the largest size asked for, freed by spamm_release.
namespace {
constexpr int kMaxDevices = 64;
std::mutex g_cache_mu;
void* g_cache_ptr[kMaxDevices] = {};
size_t g_cache_bytes[kMaxDevices] = {};
}  // namespace

spamm_status cached_workspace(size_t need, void** ws, size_t* bytes) {
    int dev = 0;
    spamm_status st = hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (st != SPAMM_OK) return st;
    if (dev < 0 || dev >= kMaxDevices) return fail(SPAMM_EUNSUPPORTED, "device %d beyond the workspace cache", dev);
    std::lock_guard<std::mutex> lock(g_cache_mu);
    if (g_cache_bytes[dev] < need) {
        if (g_cache_ptr[dev]) {
            // the old buffer may still be in use by enqueued work
            if ((st = hip_check(hipDeviceSynchronize(), "synchronize before growing the cached workspace")) !=
                SPAMM_OK)
                return st;
            if ((st = hip_check(hipFree(g_cache_ptr[dev]), "hipFree of the cached workspace")) != SPAMM_OK)
                return st;
            g_cache_ptr[dev] = nullptr;
            g_cache_bytes[dev] = 0;
        }
        void* p = nullptr;
        if (hipMalloc(&p, need) != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(SPAMM_ENOSPACE, "cannot allocate a cached workspace of %zu bytes on device %d", need, dev);
        }
        g_cache_ptr[dev] = p;
        g_cache_bytes[dev] = need;
    }
    *ws = g_cache_ptr[dev];
    *bytes = g_cache_bytes[dev];
    return SPAMM_OK;
}

spamm_status release_cached_workspaces() {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    int cur = 0;
    spamm_status st = hip_check(hipGetDevice(&cur), "hipGetDevice");
    if (st != SPAMM_OK) return st;
    for (int d = 0; d < kMaxDevices; ++d) {
        if (!g_cache_ptr[d]) continue;
        if ((st = hip_check(hipSetDevice(d), "hipSetDevice")) != SPAMM_OK) break;
        if ((st = hip_check(hipDeviceSynchronize(), "synchronize before releasing the cached workspace")) != SPAMM_OK)
            break;
        if ((st = hip_check(hipFree(g_cache_ptr[d]), "hipFree of the cached workspace")) != SPAMM_OK) break;
        g_cache_ptr[d] = nullptr;
        g_cache_bytes[d] = 0;
    }
    const spamm_status st2 = hip_check(hipSetDevice(cur), "hipSetDevice");
    return st != SPAMM_OK ? st : st2;
}

spamm_status check_workspace(const Geom& g, void*& ws, size_t& bytes) {
    const size_t need = make_layout(g).total;
    if (!ws) return cached_workspace(need, &ws, &bytes);
    if (bytes < need)
        return fail(SPAMM_ENOSPACE, "workspace of %zu bytes, %zu needed", bytes, need);
    return SPAMM_OK;
}

spamm_status check_tau(double tau) {
    if (std::isnan(tau) || tau < 0.0) return fail(SPAMM_EINVAL, "tau must be >= 0 (got %g)", tau);
    return SPAMM_OK;
}

spamm_status enqueue_pyramids(const Geom& g, const float* const* x, int nmat, double* const* pyr_out, void* ws,
                              hipStream_t s, int64_t* clear, int64_t clear_count, bool levels) {
    const Layout L = make_layout(g);
    const int64_t leaf_level = spamm::level_offset(g.lv);
    spamm::NormJob nj{};
    spamm::PyramidJob pj{};
    nj.ld = g.side;  // the norm pass writes the padded leaf level of both pyramids
    nj.clear = clear;
    nj.clear_count = clear_count;
    bool vec = (g.n % 4) == 0;
    for (int m = 0; m < nmat; ++m) {
        nj.x[m] = x[m];
        pj.spyr[m] = at<double>(ws, L.spyr[m]);
        pj.pyr[m] = pyr_out[m];
        nj.sumsq[m] = pj.spyr[m] + leaf_level;
        nj.norms[m] = pj.pyr[m] + leaf_level;
        vec = vec && aligned16(x[m]);
    }
    spamm_status st = hip_check(spamm::launch_leaf_norms(nj, nmat, g.n, g.leaf, vec, s), "leaf norm kernel");
    if (st != SPAMM_OK || !levels) return st;
    return hip_check(spamm::launch_pyramid(pj, nmat, g.bdim, g.lv, s), "pyramid kernel");
}

spamm_status enqueue_plan(const Geom& g, const double* pa, const double* pb, double tau, bool skipped,
                          int32_t* offsets, int32_t* klist, int64_t* pairs, void* ws, hipStream_t s) {
    const Layout L = make_layout(g);
    uint64_t* masks = at<uint64_t>(ws, L.masks);
    int32_t* counts = at<int32_t>(ws, L.counts);
    int32_t* bsums = at<int32_t>(ws, L.bsums);
    int32_t* boffs = at<int32_t>(ws, L.boffs);
    spamm_status st = hip_check(spamm::launch_plan_mask(pa, pb, g.bdim, g.lv, tau, skipped, masks, counts, bsums, s),
                                "plan mask kernel");
    if (st != SPAMM_OK) return st;
    st = hip_check(spamm::launch_plan_scan(bsums, g.bdim * g.nwords, boffs, offsets, g.ntiles, pairs, s),
                   "plan scan kernel");
    if (st != SPAMM_OK) return st;
    return hip_check(spamm::launch_plan_fill(masks, counts, boffs, g.bdim, offsets, klist, s), "plan fill kernel");
}

spamm_status enqueue_prepare(const Geom& g, const float* a, const float* b, double tau, int32_t* offsets,
                             int32_t* klist, int64_t* pairs, void* ws, hipStream_t s, bool schedule) {
    const Layout L = make_layout(g);
    double* pa = at<double>(ws, L.pyr[0]);
    double* pb = at<double>(ws, L.pyr[1]);
    const float* xs[2] = {a, b};
    double* ps[2] = {pa, pb};
    const bool fused = schedule && (g.leaf == 32 || g.leaf == 64) && g.bdim <= spamm::kPlanMacroMaxBdim;
    // the fused plan tests on the leaf norms alone: no pyramid levels above
    int64_t* state = at<int64_t>(ws, L.pm_state);
    spamm_status st = enqueue_pyramids(g, xs, 2, ps, ws, s, fused ? state : nullptr,
                                       fused ? spamm::plan_macro_clear_words(g.bdim) : 0, !fused);
    if (st != SPAMM_OK) return st;
    if (!fused) {
        if ((st = enqueue_plan(g, pa, pb, tau, false, offsets, klist, pairs, ws, s)) != SPAMM_OK) return st;
        return schedule ? enqueue_schedule(g, offsets, klist, ws, s) : SPAMM_OK;
    }
    const spamm::MacroSchedule ms = macro_schedule(L, ws);
    spamm::PlanMacroOut o{};
    o.offsets = offsets;
    o.klist = klist;
    o.pairs = pairs;
    o.uprefix = ms.uprefix;
    o.items = ms.items;
    o.flags = reinterpret_cast<unsigned long long*>(state);
    o.ticket = reinterpret_cast<unsigned int*>(state + (g.bdim + 1) / 2);
    const int64_t leaf_level = spamm::level_offset(g.lv);
    return hip_check(spamm::launch_plan_macro(pa + leaf_level, pb + leaf_level, g.side, g.bdim, tau, o, s),
                     "plan and schedule kernel");
}

spamm_status check_mul_args(const Geom& g, const float* a, const float* b, const float* c) {
    if (!a || !b || !c) return fail(SPAMM_EINVAL, "null matrix pointer");
    const size_t bytes = sizeof(float) * size_t(g.n) * size_t(g.n);
    if (overlaps(c, bytes, a, bytes) || overlaps(c, bytes, b, bytes))
        return fail(SPAMM_EINVAL, "C overlaps A or B");
    if (!spamm_leaf_supported(g.leaf))
        return fail(SPAMM_EUNSUPPORTED, "leaf %d has no multiply kernel (16, 32, 64, 128)", g.leaf);
    return SPAMM_OK;
}


spamm::MacroSchedule macro_schedule(const Layout& L, void* ws) {
    spamm::MacroSchedule ms{};
    ms.words = at<uint64_t>(ws, L.mwords);
    ms.ucount = at<int32_t>(ws, L.mcount);
    ms.uprefix = at<int32_t>(ws, L.mprefix);
    ms.items = at<uint32_t>(ws, L.mitems);
    ms.bounds = at<int64_t>(ws, L.bounds);
    ms.fix_slots = L.fix_slot_bytes ? at<float>(ws, L.fix_slots) : nullptr;
    return ms;
}

spamm_status enqueue_schedule(const Geom& g, const int32_t* offsets, const int32_t* klist, void* ws, hipStream_t s) {
    const Layout L = make_layout(g);
    if (g.leaf == 128) {
        if (!L.leaf128_dma) return SPAMM_OK;  // the single-tile kernel reads the plan directly
        return hip_check(spamm::launch_leaf128_schedule(offsets, klist, g.bdim, at<int32_t>(ws, L.uprefix128),
                                                        at<uint32_t>(ws, L.items128), s),
                         "leaf-128 schedule kernel");
    }
    if (g.leaf != 32 && g.leaf != 64) return SPAMM_OK;
    return hip_check(spamm::launch_macro_schedule(offsets, klist, g.bdim, macro_schedule(L, ws), s),
                     "macro schedule kernels");
}

spamm_status enqueue_multiply(const Geom& g, const float* a, const float* b, const int32_t* offsets,
                              const int32_t* klist, float* c, void* ws, hipStream_t s) {
    const bool vec = (g.n % 4) == 0 && aligned16(a) && aligned16(b);
    const Layout L = make_layout(g);
    if (L.leaf128_dma && vec)
        return hip_check(spamm::launch_leaf128_multiply(a, b, c, g.n, g.bdim, at<int32_t>(ws, L.uprefix128),
                                                        at<uint32_t>(ws, L.items128), at<int64_t>(ws, L.bounds),
                                                        at<float>(ws, L.fix_slots), device_cus(), s),
                         "leaf-128 multiply kernels");
    if (g.leaf == 32 || g.leaf == 64)
        return hip_check(spamm::launch_macro_multiply(a, b, c, g.n, g.leaf, g.bdim, offsets, macro_schedule(L, ws),
                                                      vec, device_cus(), s),
                         "macro multiply kernel");
    return hip_check(spamm::launch_multiply(a, b, c, g.n, g.leaf, g.bdim, offsets, klist,
                                            at<int32_t>(ws, L.pair_scratch), vec, device_cus(), s),
                     "multiply kernel");
}

spamm_status enqueue_execute(const Geom& g, const float* a, const float* b, const int32_t* offsets,
                             const int32_t* klist, float* c, void* ws, hipStream_t s) {
    spamm_status st = enqueue_schedule(g, offsets, klist, ws, s);
    if (st != SPAMM_OK) return st;
    return enqueue_multiply(g, a, b, offsets, klist, c, ws, s);
}

namespace {
constexpr size_t kSplitHeaderBytes = 256;  // scale exponents and largest leaf norms
// F16X3 whole path: split A and B once when the plan keeps at least this many
// pairs per output tile on average, else split in registers.  The split pass
// reads and writes A and B once more (1 ms at N = 16384); the in-register
// split redoes the conversions in every wave that reads an operand, work that
// grows with the kept pairs.  Whole steps measured at N = 16384 on
// exponential decay cross near 50 pairs per tile (in registers 5.84 against
// 6.26 ms at 30 pairs per tile, planes 13.40 against 13.74 ms at 74).
constexpr int64_t kF16x3StagedPairsPerTile = 45;
// BF16: the in-register rounding reads the FP32 tiles (twice the bytes of the
// planes); the same measurement crosses near 19 pairs per tile (in registers
// 1.46 against 1.91 ms at 8 pairs per tile, planes 3.30 against 3.77 ms at 30).
constexpr int64_t kBf16StagedPairsPerTile = 16;
size_t plane_bytes(int64_t n) { return (size_t(n) * size_t(n) * 2 + 255) / 256 * 256; }
int split_planes(int32_t precision) { return precision == spamm::kPrecF16x3 ? 4 : 2; }

spamm::SplitLayout split_layout(void* split, int64_t n, int32_t precision) {
    char* base = static_cast<char*>(split);
    const size_t pb = plane_bytes(n);
    spamm::SplitLayout L{};
    L.exps = reinterpret_cast<int32_t*>(base);
    char* p = base + kSplitHeaderBytes;
    auto next = [&]() {
        uint16_t* q = reinterpret_cast<uint16_t*>(p);
        p += pb;
        return q;
    };
    L.a_hi = next();
    L.a_lo = precision == spamm::kPrecF16x3 ? next() : nullptr;
    L.bt_hi = next();
    L.bt_lo = precision == spamm::kPrecF16x3 ? next() : nullptr;
    return L;
}
}  // namespace

spamm_status check_lowp(const Geom& g, int32_t precision) {
    if (precision != spamm::kPrecBf16 && precision != spamm::kPrecF16x3)
        return fail(SPAMM_EINVAL, "precision %d is not a reduced-precision form (1: bf16, 2: f16x3)", precision);
    if (g.leaf != 64 || g.n % 128 != 0)
        return fail(SPAMM_EUNSUPPORTED, "reduced-precision products need leaf 64 and n a multiple of 128 (n=%lld "
                    "leaf=%d)", (long long)g.n, g.leaf);
    return check_grid(g);
}

}  // namespace spamm_host

using namespace spamm_host;

extern "C" {

int64_t spamm_bdim(int64_t n, int32_t leaf) {
    Geom g;
    return make_geom(n, leaf, &g) ? g.bdim : 0;
}

int32_t spamm_levels(int64_t n, int32_t leaf) {
    Geom g;
    return make_geom(n, leaf, &g) ? g.lv : 0;
}

int64_t spamm_pyramid_size(int64_t n, int32_t leaf) {
    Geom g;
    return make_geom(n, leaf, &g) ? g.pyr : 0;
}

int32_t spamm_leaf_supported(int32_t leaf) { return (leaf == 16 || leaf == 32 || leaf == 64 || leaf == 128) ? 1 : 0; }

spamm_status spamm_release(void) {
    g_last_error[0] = '\0';
    return release_cached_workspaces();
}

size_t spamm_workspace_bytes(int64_t n, int32_t leaf) {
    Geom g;
    if (!make_geom(n, leaf, &g) || g.bdim > SPAMM_MAX_BDIM) return 0;
    return make_layout(g).total;
}

spamm_status spamm_norms(const float* x, int64_t n, int32_t leaf, double* norms, void* stream) {
    g_last_error[0] = '\0';
    Geom g;
    if (!make_geom(n, leaf, &g)) return fail(SPAMM_EINVAL, "bad size n=%lld leaf=%d", (long long)n, leaf);
    if (!x || !norms) return fail(SPAMM_EINVAL, "null pointer");
    spamm::NormJob nj{};
    nj.x[0] = x;
    nj.sumsq[0] = nullptr;
    nj.norms[0] = norms;
    nj.ld = g.bdim;
    const bool vec = (n % 4) == 0 && aligned16(x);
    return hip_check(spamm::launch_leaf_norms(nj, 1, n, leaf, vec, static_cast<hipStream_t>(stream)),
                     "leaf norm kernel");
}

spamm_status spamm_pyramid(const float* x, int64_t n, int32_t leaf, double* pyramid, void* workspace,
                           size_t workspace_bytes, void* stream) {
    g_last_error[0] = '\0';
    Geom g;
    if (!make_geom(n, leaf, &g)) return fail(SPAMM_EINVAL, "bad size n=%lld leaf=%d", (long long)n, leaf);
    if (!x || !pyramid) return fail(SPAMM_EINVAL, "null pointer");
    spamm_status st = check_grid(g);
    if (st != SPAMM_OK) return st;
    if ((st = check_workspace(g, workspace, workspace_bytes)) != SPAMM_OK) return st;
    const float* xs[1] = {x};
    double* ps[1] = {pyramid};
    return enqueue_pyramids(g, xs, 1, ps, workspace, static_cast<hipStream_t>(stream));
}

spamm_status spamm_plan(const double* pyr_a, const double* pyr_b, int64_t n, int32_t leaf, double tau,
                        int32_t* offsets, int32_t* klist, int64_t klist_capacity, int64_t* pairs, void* workspace,
                        size_t workspace_bytes, void* stream) {
    g_last_error[0] = '\0';
    Geom g;
    if (!make_geom(n, leaf, &g)) return fail(SPAMM_EINVAL, "bad size n=%lld leaf=%d", (long long)n, leaf);
    if (!pyr_a || !pyr_b || !offsets || !klist || !pairs) return fail(SPAMM_EINVAL, "null pointer");
    spamm_status st = check_tau(tau);
    if (st != SPAMM_OK) return st;
    if ((st = check_grid(g)) != SPAMM_OK) return st;
    if ((st = check_workspace(g, workspace, workspace_bytes)) != SPAMM_OK) return st;
    if (klist_capacity < g.ntiles * g.bdim)
        return fail(SPAMM_ENOSPACE, "klist capacity %lld < bdim^3 = %lld", (long long)klist_capacity,
                    (long long)(g.ntiles * g.bdim));
    return enqueue_plan(g, pyr_a, pyr_b, tau, false, offsets, klist, pairs, workspace, static_cast<hipStream_t>(stream));
}

spamm_status spamm_execute(const float* a, const float* b, int64_t n, int32_t leaf, const int32_t* offsets,
                           const int32_t* klist, float* c, void* workspace, size_t workspace_bytes, void* stream) {
    g_last_error[0] = '\0';
    Geom g;
    if (!make_geom(n, leaf, &g)) return fail(SPAMM_EINVAL, "bad size n=%lld leaf=%d", (long long)n, leaf);
    spamm_status st = check_mul_args(g, a, b, c);
    if (st != SPAMM_OK) return st;
    if (!offsets || !klist) return fail(SPAMM_EINVAL, "null plan pointer");
    if ((st = check_grid(g)) != SPAMM_OK) return st;
    if ((st = check_workspace(g, workspace, workspace_bytes)) != SPAMM_OK) return st;
    return enqueue_execute(g, a, b, offsets, klist, c, workspace, static_cast<hipStream_t>(stream));
}

spamm_status spamm_schedule(const int32_t* offsets, const int32_t* klist, int64_t n, int32_t leaf, void* workspace,
                            size_t workspace_bytes, void* stream) {
    g_last_error[0] = '\0';
    Geom g;
    if (!make_geom(n, leaf, &g)) return fail(SPAMM_EINVAL, "bad size n=%lld leaf=%d", (long long)n, leaf);
    if (!offsets || !klist) return fail(SPAMM_EINVAL, "null plan pointer");
    if (!spamm_leaf_supported(leaf))
        return fail(SPAMM_EUNSUPPORTED, "leaf %d has no multiply kernel (16, 32, 64, 128)", leaf);
    spamm_status st = check_grid(g);
    if (st != SPAMM_OK) return st;
    if ((st = check_workspace(g, workspace, workspace_bytes)) != SPAMM_OK) return st;
    return enqueue_schedule(g, offsets, klist, workspace, static_cast<hipStream_t>(stream));
}

spamm_status spamm_execute_scheduled(const float* a, const float* b, int64_t n, int32_t leaf, const int32_t* offsets,
                                     const int32_t* klist, float* c, void* workspace, size_t workspace_bytes,
                                     void* stream) {
    g_last_error[0] = '\0';
    Geom g;
    if (!make_geom(n, leaf, &g)) return fail(SPAMM_EINVAL, "bad size n=%lld leaf=%d", (long long)n, leaf);
    spamm_status st = check_mul_args(g, a, b, c);
    if (st != SPAMM_OK) return st;
    if (!offsets || !klist) return fail(SPAMM_EINVAL, "null plan pointer");
    if ((st = check_grid(g)) != SPAMM_OK) return st;
    if ((st = check_workspace(g, workspace, workspace_bytes)) != SPAMM_OK) return st;
    return enqueue_multiply(g, a, b, offsets, klist, c, workspace, static_cast<hipStream_t>(stream));
}

spamm_status spamm_prepare(const float* a, const float* b, int64_t n, double tau, int32_t leaf, int32_t* offsets,
                           int32_t* klist, int64_t klist_capacity, int64_t* pairs, void* workspace,
                           size_t workspace_bytes, void* stream) {
    g_last_error[0] = '\0';
    Geom g;
    if (!make_geom(n, leaf, &g)) return fail(SPAMM_EINVAL, "bad size n=%lld leaf=%d", (long long)n, leaf);
    if (!a || !b || !offsets || !klist || !pairs) return fail(SPAMM_EINVAL, "null pointer");
    spamm_status st = check_tau(tau);
    if (st != SPAMM_OK) return st;
    if ((st = check_grid(g)) != SPAMM_OK) return st;
    if ((st = check_workspace(g, workspace, workspace_bytes)) != SPAMM_OK) return st;
    if (klist_capacity < g.ntiles * g.bdim)
        return fail(SPAMM_ENOSPACE, "klist capacity %lld < bdim^3 = %lld", (long long)klist_capacity,
                    (long long)(g.ntiles * g.bdim));
    return enqueue_prepare(g, a, b, tau, offsets, klist, pairs, workspace, static_cast<hipStream_t>(stream), false);
}

spamm_status spamm_prepare_schedule(const float* a, const float* b, int64_t n, double tau, int32_t leaf,
                                    int32_t* offsets, int32_t* klist, int64_t klist_capacity, int64_t* pairs,
                                    void* workspace, size_t workspace_bytes, void* stream) {
    g_last_error[0] = '\0';
    Geom g;
    if (!make_geom(n, leaf, &g)) return fail(SPAMM_EINVAL, "bad size n=%lld leaf=%d", (long long)n, leaf);
    if (!a || !b || !offsets || !klist || !pairs) return fail(SPAMM_EINVAL, "null pointer");
    if (!spamm_leaf_supported(leaf))
        return fail(SPAMM_EUNSUPPORTED, "leaf %d has no multiply kernel (16, 32, 64, 128)", leaf);
    spamm_status st = check_tau(tau);
    if (st != SPAMM_OK) return st;
    if ((st = check_grid(g)) != SPAMM_OK) return st;
    if ((st = check_workspace(g, workspace, workspace_bytes)) != SPAMM_OK) return st;
    if (klist_capacity < g.ntiles * g.bdim)
        return fail(SPAMM_ENOSPACE, "klist capacity %lld < bdim^3 = %lld", (long long)klist_capacity,
                    (long long)(g.ntiles * g.bdim));
    return enqueue_prepare(g, a, b, tau, offsets, klist, pairs, workspace, static_cast<hipStream_t>(stream), true);
}

namespace {
// Small products: the leaf norm pass (which also clears the pair counter),
// then the threshold test and the multiply in one launch.
spamm_status enqueue_small(const Geom& g, const float* a, const float* b, double tau, float* c, int64_t* pairs,
                           void* ws, hipStream_t s) {
    const Layout L = make_layout(g);
    const int64_t leaf_level = spamm::level_offset(g.lv);
    spamm::NormJob nj{};
    nj.ld = g.side;
    nj.clear = pairs;
    const float* xs[2] = {a, b};
    for (int m = 0; m < 2; ++m) {
        nj.x[m] = xs[m];
        nj.sumsq[m] = at<double>(ws, L.spyr[m]) + leaf_level;
        nj.norms[m] = at<double>(ws, L.pyr[m]) + leaf_level;
    }
    spamm_status st = hip_check(spamm::launch_leaf_norms(nj, 2, g.n, g.leaf, true, s), "leaf norm kernel");
    if (st != SPAMM_OK) return st;
    return hip_check(spamm::launch_small_multiply(a, b, c, g.n, g.bdim, nj.norms[0], nj.norms[1], g.side, tau, pairs,
                                                  s),
                     "small multiply kernel");
}
}  // namespace

spamm_status spamm_multiply(const float* a, const float* b, int64_t n, double tau, int32_t leaf, float* c,
                            int64_t* pairs, void* workspace, size_t workspace_bytes, void* stream) {
    g_last_error[0] = '\0';
    Geom g;
    if (!make_geom(n, leaf, &g)) return fail(SPAMM_EINVAL, "bad size n=%lld leaf=%d", (long long)n, leaf);
    spamm_status st = check_mul_args(g, a, b, c);
    if (st != SPAMM_OK) return st;
    if ((st = check_tau(tau)) != SPAMM_OK) return st;
    if ((st = check_grid(g)) != SPAMM_OK) return st;
    if ((st = check_workspace(g, workspace, workspace_bytes)) != SPAMM_OK) return st;
    const Layout L = make_layout(g);
    int64_t* np = pairs ? pairs : at<int64_t>(workspace, L.pairs);
    if (g.leaf == 32 && g.bdim <= spamm::kSmallMaxBdim && g.n % 4 == 0 && aligned16(a) && aligned16(b))
        return enqueue_small(g, a, b, tau, c, np, workspace, static_cast<hipStream_t>(stream));
    int32_t* offsets = at<int32_t>(workspace, L.offsets);
    int32_t* klist = at<int32_t>(workspace, L.klist);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((st = enqueue_prepare(g, a, b, tau, offsets, klist, np, workspace, s, true)) != SPAMM_OK) return st;
    return enqueue_multiply(g, a, b, offsets, klist, c, workspace, s);
}

size_t spamm_split_bytes(int64_t n, int32_t precision) {
    if (n <= 0 || (precision != spamm::kPrecBf16 && precision != spamm::kPrecF16x3)) return 0;
    return kSplitHeaderBytes + size_t(split_planes(precision)) * plane_bytes(n);
}

spamm_status spamm_split(const float* a, const float* b, int64_t n, int32_t leaf, int32_t precision,
                         const double* pyr_a, const double* pyr_b, void* split, size_t split_bytes, void* stream) {
    g_last_error[0] = '\0';
    Geom g;
    if (!make_geom(n, leaf, &g)) return fail(SPAMM_EINVAL, "bad size n=%lld leaf=%d", (long long)n, leaf);
    if (!a || !b || !pyr_a || !pyr_b || !split) return fail(SPAMM_EINVAL, "null pointer");
    spamm_status st = check_lowp(g, precision);
    if (st != SPAMM_OK) return st;
    if (!aligned16(a) || !aligned16(b) || (reinterpret_cast<uintptr_t>(split) & 255u) != 0)
        return fail(SPAMM_EINVAL, "a, b need 16-byte and split 256-byte alignment");
    if (split_bytes < spamm_split_bytes(n, precision))
        return fail(SPAMM_ENOSPACE, "split buffer of %zu bytes, %zu needed", split_bytes,
                    spamm_split_bytes(n, precision));
    const size_t sb = spamm_split_bytes(n, precision);
    const size_t mb = sizeof(float) * size_t(n) * size_t(n);
    if (overlaps(split, sb, a, mb) || overlaps(split, sb, b, mb))
        return fail(SPAMM_EINVAL, "split buffer overlaps a or b");
    return hip_check(spamm::launch_split(a, b, n, g.bdim, g.lv, pyr_a, pyr_b, precision,
                                         split_layout(split, n, precision), static_cast<hipStream_t>(stream)),
                     "split kernels");
}

spamm_status spamm_execute_split_scheduled(const void* split, int64_t n, int32_t leaf, int32_t precision,
                                           const int32_t* offsets, const int32_t* klist, float* c, void* workspace,
                                           size_t workspace_bytes, void* stream) {
    g_last_error[0] = '\0';
    Geom g;
    if (!make_geom(n, leaf, &g)) return fail(SPAMM_EINVAL, "bad size n=%lld leaf=%d", (long long)n, leaf);
    if (!split || !offsets || !klist || !c) return fail(SPAMM_EINVAL, "null pointer");
    spamm_status st = check_lowp(g, precision);
    if (st != SPAMM_OK) return st;
    if ((st = check_workspace(g, workspace, workspace_bytes)) != SPAMM_OK) return st;
    if (overlaps(c, sizeof(float) * size_t(n) * size_t(n), split, spamm_split_bytes(n, precision)))
        return fail(SPAMM_EINVAL, "c overlaps the split buffer");
    const Layout L = make_layout(g);
    return hip_check(spamm::launch_lowp_multiply(split_layout(const_cast<void*>(split), n, precision), c, n, g.bdim,
                                                 precision, at<uint32_t>(workspace, L.mitems),
                                                 at<int32_t>(workspace, L.mprefix), device_cus(), spamm::PairGate{},
                                                 static_cast<hipStream_t>(stream)),
                     "reduced-precision multiply kernel");
}

spamm_status spamm_execute_split(const void* split, int64_t n, int32_t leaf, int32_t precision,
                                 const int32_t* offsets, const int32_t* klist, float* c, void* workspace,
                                 size_t workspace_bytes, void* stream) {
    spamm_status st = spamm_schedule(offsets, klist, n, leaf, workspace, workspace_bytes, stream);
    if (st != SPAMM_OK) return st;
    return spamm_execute_split_scheduled(split, n, leaf, precision, offsets, klist, c, workspace, workspace_bytes,
                                         stream);
}

spamm_status spamm_split_scales(const double* pyr_a, const double* pyr_b, int64_t n, int32_t leaf, void* header,
                                size_t header_bytes, void* stream) {
    g_last_error[0] = '\0';
    Geom g;
    if (!make_geom(n, leaf, &g)) return fail(SPAMM_EINVAL, "bad size n=%lld leaf=%d", (long long)n, leaf);
    if (!pyr_a || !pyr_b || !header) return fail(SPAMM_EINVAL, "null pointer");
    spamm_status st = check_lowp(g, spamm::kPrecF16x3);
    if (st != SPAMM_OK) return st;
    if ((reinterpret_cast<uintptr_t>(header) & 255u) != 0) return fail(SPAMM_EINVAL, "header must be 256-byte aligned");
    if (header_bytes < kSplitHeaderBytes)
        return fail(SPAMM_ENOSPACE, "header of %zu bytes, %zu needed", header_bytes, kSplitHeaderBytes);
    return hip_check(spamm::launch_split_scales(g.bdim, g.lv, pyr_a, pyr_b, static_cast<int32_t*>(header),
                                                static_cast<hipStream_t>(stream)),
                     "scale kernels");
}

spamm_status spamm_execute_f16x3_scheduled(const float* a, const float* b, int64_t n, int32_t leaf,
                                           const void* header, const int32_t* offsets, const int32_t* klist,
                                           float* c, void* workspace, size_t workspace_bytes, void* stream) {
    g_last_error[0] = '\0';
    Geom g;
    if (!make_geom(n, leaf, &g)) return fail(SPAMM_EINVAL, "bad size n=%lld leaf=%d", (long long)n, leaf);
    if (!header || !offsets || !klist) return fail(SPAMM_EINVAL, "null pointer");
    spamm_status st = check_mul_args(g, a, b, c);
    if (st != SPAMM_OK) return st;
    if ((st = check_lowp(g, spamm::kPrecF16x3)) != SPAMM_OK) return st;
    if ((st = check_workspace(g, workspace, workspace_bytes)) != SPAMM_OK) return st;
    if (!aligned16(a) || !aligned16(b)) return fail(SPAMM_EINVAL, "a and b need 16-byte alignment");
    if (overlaps(c, sizeof(float) * size_t(n) * size_t(n), header, kSplitHeaderBytes))
        return fail(SPAMM_EINVAL, "c overlaps the header");
    const Layout L = make_layout(g);
    return hip_check(spamm::launch_fused_multiply(a, b, spamm::kPrecF16x3, static_cast<const int32_t*>(header), c, n,
                                                  g.bdim, at<uint32_t>(workspace, L.mitems),
                                                  at<int32_t>(workspace, L.mprefix), device_cus(), spamm::PairGate{},
                                                  static_cast<hipStream_t>(stream)),
                     "fused f16x3 multiply kernel");
}

spamm_status spamm_execute_bf16_scheduled(const float* a, const float* b, int64_t n, int32_t leaf,
                                          const int32_t* offsets, const int32_t* klist, float* c, void* workspace,
                                          size_t workspace_bytes, void* stream) {
    g_last_error[0] = '\0';
    Geom g;
    if (!make_geom(n, leaf, &g)) return fail(SPAMM_EINVAL, "bad size n=%lld leaf=%d", (long long)n, leaf);
    if (!offsets || !klist) return fail(SPAMM_EINVAL, "null pointer");
    spamm_status st = check_mul_args(g, a, b, c);
    if (st != SPAMM_OK) return st;
    if ((st = check_lowp(g, spamm::kPrecBf16)) != SPAMM_OK) return st;
    if ((st = check_workspace(g, workspace, workspace_bytes)) != SPAMM_OK) return st;
    if (!aligned16(a) || !aligned16(b)) return fail(SPAMM_EINVAL, "a and b need 16-byte alignment");
    const Layout L = make_layout(g);
    return hip_check(spamm::launch_fused_multiply(a, b, spamm::kPrecBf16, nullptr, c, n, g.bdim,
                                                  at<uint32_t>(workspace, L.mitems),
                                                  at<int32_t>(workspace, L.mprefix), device_cus(), spamm::PairGate{},
                                                  static_cast<hipStream_t>(stream)),
                     "fused bf16 multiply kernel");
}

spamm_status spamm_prepare_scales(const float* a, const float* b, int64_t n, double tau, int32_t leaf,
                                  int32_t* offsets, int32_t* klist, int64_t klist_capacity, int64_t* pairs,
                                  void* header, size_t header_bytes, void* workspace, size_t workspace_bytes,
                                  void* stream) {
    g_last_error[0] = '\0';
    Geom g;
    if (!make_geom(n, leaf, &g)) return fail(SPAMM_EINVAL, "bad size n=%lld leaf=%d", (long long)n, leaf);
    spamm_status st = check_lowp(g, spamm::kPrecF16x3);
    if (st != SPAMM_OK) return st;
    const size_t mbytes = sizeof(float) * size_t(n) * size_t(n);
    if (header && (overlaps(header, kSplitHeaderBytes, a, mbytes) || overlaps(header, kSplitHeaderBytes, b, mbytes)))
        return fail(SPAMM_EINVAL, "header overlaps a or b");
    st = spamm_prepare(a, b, n, tau, leaf, offsets, klist, klist_capacity, pairs, workspace, workspace_bytes, stream);
    if (st != SPAMM_OK) return st;
    const Layout L = make_layout(g);
    return spamm_split_scales(at<double>(workspace, L.pyr[0]), at<double>(workspace, L.pyr[1]), n, leaf, header,
                              header_bytes, stream);
}

spamm_status spamm_prepare_schedule_scales(const float* a, const float* b, int64_t n, double tau, int32_t leaf,
                                           int32_t* offsets, int32_t* klist, int64_t klist_capacity,
                                           int64_t* pairs, void* header, size_t header_bytes, void* workspace,
                                           size_t workspace_bytes, void* stream) {
    g_last_error[0] = '\0';
    Geom g;
    if (!make_geom(n, leaf, &g)) return fail(SPAMM_EINVAL, "bad size n=%lld leaf=%d", (long long)n, leaf);
    spamm_status st = check_lowp(g, spamm::kPrecF16x3);
    if (st != SPAMM_OK) return st;
    // the header is checked before anything is enqueued
    if (!header || (reinterpret_cast<uintptr_t>(header) & 255u) != 0)
        return fail(SPAMM_EINVAL, "the header must be non-null and 256-byte aligned");
    if (header_bytes < kSplitHeaderBytes)
        return fail(SPAMM_ENOSPACE, "header of %zu bytes, %zu needed", header_bytes, kSplitHeaderBytes);
    const size_t mbytes = sizeof(float) * size_t(n) * size_t(n);
    if (overlaps(header, kSplitHeaderBytes, a, mbytes) || overlaps(header, kSplitHeaderBytes, b, mbytes))
        return fail(SPAMM_EINVAL, "header overlaps a or b");
    st = spamm_prepare_schedule(a, b, n, tau, leaf, offsets, klist, klist_capacity, pairs, workspace,
                                workspace_bytes, stream);
    if (st != SPAMM_OK) return st;
    // the scale kernels read the leaf level, which either form of the plan leaves
    const Layout L = make_layout(g);
    return spamm_split_scales(at<double>(workspace, L.pyr[0]), at<double>(workspace, L.pyr[1]), n, leaf, header,
                              header_bytes, stream);
}

spamm_status spamm_prepare_split(const float* a, const float* b, int64_t n, double tau, int32_t leaf,
                                 int32_t precision, int32_t* offsets, int32_t* klist, int64_t klist_capacity,
                                 int64_t* pairs, void* split, size_t split_bytes, void* workspace,
                                 size_t workspace_bytes, void* stream) {
    g_last_error[0] = '\0';
    Geom g;
    if (!make_geom(n, leaf, &g)) return fail(SPAMM_EINVAL, "bad size n=%lld leaf=%d", (long long)n, leaf);
    spamm_status st = check_lowp(g, precision);
    if (st != SPAMM_OK) return st;
    st = spamm_prepare(a, b, n, tau, leaf, offsets, klist, klist_capacity, pairs, workspace, workspace_bytes, stream);
    if (st != SPAMM_OK) return st;
    const Layout L = make_layout(g);
    return spamm_split(a, b, n, leaf, precision, at<double>(workspace, L.pyr[0]), at<double>(workspace, L.pyr[1]),
                       split, split_bytes, stream);
}

spamm_status spamm_multiply_precision(const float* a, const float* b, int64_t n, double tau, int32_t leaf,
                                      int32_t precision, float* c, int64_t* pairs, void* split, size_t split_bytes,
                                      void* workspace, size_t workspace_bytes, void* stream) {
    g_last_error[0] = '\0';
    if (precision == spamm::kPrecFp32)
        return spamm_multiply(a, b, n, tau, leaf, c, pairs, workspace, workspace_bytes, stream);
    Geom g;
    if (!make_geom(n, leaf, &g)) return fail(SPAMM_EINVAL, "bad size n=%lld leaf=%d", (long long)n, leaf);
    spamm_status st = check_mul_args(g, a, b, c);
    if (st != SPAMM_OK) return st;
    if ((st = check_lowp(g, precision)) != SPAMM_OK) return st;
    if ((st = check_tau(tau)) != SPAMM_OK) return st;
    if ((st = check_workspace(g, workspace, workspace_bytes)) != SPAMM_OK) return st;
    const Layout L = make_layout(g);
    int32_t* offsets = at<int32_t>(workspace, L.offsets);
    int32_t* klist = at<int32_t>(workspace, L.klist);
    int64_t* np = pairs ? pairs : at<int64_t>(workspace, L.pairs);
    // With room for the planes the device picks, from the plan's pair count,
    // between converting A and B once and multiplying the planes (many pairs:
    // each tile feeds many products) and converting the FP32 tiles in
    // registers inside the multiply (few pairs: the split pass would cost more
    // than the conversions).  With less room (F16X3: only the 256-byte header
    // of scale exponents), always in registers.  Both give bitwise the same C.
    const bool f16 = precision == spamm::kPrecF16x3;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!aligned16(a) || !aligned16(b)) return fail(SPAMM_EINVAL, "a and b need 16-byte alignment");
    const bool planes = split_bytes >= spamm_split_bytes(n, precision);
    if (planes) {
        const size_t sb = spamm_split_bytes(n, precision), mbytes = sizeof(float) * size_t(n) * size_t(n);
        if (!split || overlaps(split, sb, a, mbytes) || overlaps(split, sb, b, mbytes) ||
            overlaps(split, sb, c, mbytes))
            return fail(SPAMM_EINVAL, "split buffer null or overlapping a, b or c");
    }
    if (f16) {  // the scale exponents go to the split buffer's 256-byte header
        const size_t mbytes = sizeof(float) * size_t(n) * size_t(n);
        if (!split || (reinterpret_cast<uintptr_t>(split) & 255u) != 0)
            return fail(SPAMM_EINVAL, "the split header must be non-null and 256-byte aligned");
        if (split_bytes < kSplitHeaderBytes)
            return fail(SPAMM_ENOSPACE, "header of %zu bytes, %zu needed", split_bytes, kSplitHeaderBytes);
        if (overlaps(split, kSplitHeaderBytes, a, mbytes) || overlaps(split, kSplitHeaderBytes, b, mbytes) ||
            overlaps(split, kSplitHeaderBytes, c, mbytes))
            return fail(SPAMM_EINVAL, "header overlaps a, b or c");
    }
    // norms, pyramids, then the plan and the multiply schedule in one launch
    if ((st = enqueue_prepare(g, a, b, tau, offsets, klist, np, workspace, s, true)) != SPAMM_OK) return st;
    const spamm::SplitLayout SL = split_layout(split, n, precision);
    if (f16 && (st = hip_check(spamm::launch_split_scales(g.bdim, g.lv, at<double>(workspace, L.pyr[0]),
                                                          at<double>(workspace, L.pyr[1]), SL.exps, s),
                               "scale kernels")) != SPAMM_OK)
        return st;
    const int64_t per_tile = f16 ? kF16x3StagedPairsPerTile : kBf16StagedPairsPerTile;
    spamm::PairGate staged{np, per_tile * g.bdim * g.bdim, 1}, fused{};
    if (planes) {
        fused = staged;
        fused.when_at_least = 0;
        if ((st = hip_check(spamm::launch_split_planes(a, b, n, precision, SL, staged, s), "split kernels")) !=
            SPAMM_OK)
            return st;
    }
    if (planes &&
        (st = hip_check(spamm::launch_lowp_multiply(SL, c, n, g.bdim, precision, at<uint32_t>(workspace, L.mitems),
                                                    at<int32_t>(workspace, L.mprefix), device_cus(), staged, s),
                        "reduced-precision multiply kernel")) != SPAMM_OK)
        return st;
    return hip_check(spamm::launch_fused_multiply(a, b, precision, f16 ? SL.exps : nullptr, c, n, g.bdim,
                                                  at<uint32_t>(workspace, L.mitems),
                                                  at<int32_t>(workspace, L.mprefix), device_cus(), fused, s),
                     "reduced-precision multiply kernel (in-register conversion)");
}

spamm_status spamm_search_valid_ratio(const double* pyr_a, const double* pyr_b, int64_t n, int32_t leaf,
                                      double target, double tol, int32_t max_iters, double* tau_out,
                                      int64_t* pairs_out, int32_t* iters_out, void* workspace, size_t workspace_bytes,
                                      void* stream) {
    g_last_error[0] = '\0';
    Geom g;
    if (!make_geom(n, leaf, &g)) return fail(SPAMM_EINVAL, "bad size n=%lld leaf=%d", (long long)n, leaf);
    if (!pyr_a || !pyr_b || !tau_out) return fail(SPAMM_EINVAL, "null pointer");
    if (!(target > 0.0 && target <= 1.0)) return fail(SPAMM_EINVAL, "target valid ratio must be in (0, 1]");
    if (!(tol >= 0.0) || max_iters < 0) return fail(SPAMM_EINVAL, "tol must be >= 0 and max_iters >= 0");
    spamm_status st = check_grid(g);
    if (st != SPAMM_OK) return st;
    if ((st = check_workspace(g, workspace, workspace_bytes)) != SPAMM_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Layout L = make_layout(g);
    double* d_ave = at<double>(workspace, L.scalars);
    int32_t* bsums = at<int32_t>(workspace, L.bsums);
    int64_t* d_pairs = at<int64_t>(workspace, L.pairs);
    const int64_t nb = g.bdim * g.nwords;
    const double triples = double(g.bdim) * double(g.bdim) * double(g.bdim);

    if ((st = hip_check(spamm::launch_mean_norm_product(pyr_a, pyr_b, g.bdim, g.lv, d_ave, s), "mean kernel")) !=
        SPAMM_OK)
        return st;
    double ave = 0.0;
    if ((st = hip_check(hipMemcpyAsync(&ave, d_ave, sizeof(double), hipMemcpyDeviceToHost, s), "copy")) != SPAMM_OK)
        return st;
    if ((st = hip_check(hipStreamSynchronize(s), "synchronize")) != SPAMM_OK) return st;

    int64_t cnt = 0;
    auto ratio = [&](double t, double* r) -> spamm_status {
        spamm_status e = hip_check(spamm::launch_plan_count(pyr_a, pyr_b, g.bdim, g.lv, t, bsums, s), "count kernel");
        if (e != SPAMM_OK) return e;
        e = hip_check(spamm::launch_plan_scan(bsums, nb, nullptr, nullptr, nb, d_pairs, s), "scan kernel");
        if (e != SPAMM_OK) return e;
        e = hip_check(hipMemcpyAsync(&cnt, d_pairs, sizeof(int64_t), hipMemcpyDeviceToHost, s), "copy");
        if (e != SPAMM_OK) return e;
        e = hip_check(hipStreamSynchronize(s), "synchronize");
        *r = double(cnt) / triples;
        return e;
    };
    // section 3.5.2: tau starts at ave; the upper bound k*ave grows by ave
    // while the ratio there is still above the target; then bisection in
    // [0, k*ave] until the ratio is within tol or max_iters bisections ran
    constexpr int kMaxExpand = 1024;
    int k = 1;
    double hi = ave, r = 0.0;
    if ((st = ratio(hi, &r)) != SPAMM_OK) return st;
    while (r > target + tol && k < kMaxExpand) {
        ++k;
        hi = k * ave;
        if ((st = ratio(hi, &r)) != SPAMM_OK) return st;
    }
    double tau = hi, lo = 0.0;
    int it = 0;
    while (std::fabs(r - target) > tol && it < max_iters) {
        const double mid = 0.5 * (lo + hi);
        if ((st = ratio(mid, &r)) != SPAMM_OK) return st;
        tau = mid;
        ++it;
        if (r > target)
            lo = mid;
        else
            hi = mid;
    }
    *tau_out = tau;
    if (pairs_out) *pairs_out = cnt;
    if (iters_out) *iters_out = it;
    return SPAMM_OK;
}

const char* spamm_strerror(spamm_status status) {
    switch (status) {
        case SPAMM_OK: return "success";
        case SPAMM_EINVAL: return "invalid argument";
        case SPAMM_ENOSPACE: return "workspace or output capacity too small";
        case SPAMM_EDEVICE: return "HIP runtime or kernel launch failure";
        case SPAMM_EUNSUPPORTED: return "unsupported leaf or problem size";
    }
    return "unknown status";
}

const char* spamm_last_error(void) { return g_last_error; }

}  // extern "C"
