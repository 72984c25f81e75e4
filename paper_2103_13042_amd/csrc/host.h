// Host-side helpers shared by the entry points of libspamm.so: error
// reporting, tile geometry, the workspace layout, argument checks, and the
// enqueueing of the pyramid, plan and multiply kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "internal.h"
#include "spamm.h"

namespace spamm_host {

extern thread_local char g_last_error[512];

spamm_status fail(spamm_status st, const char* fmt, ...);
spamm_status hip_check(hipError_t e, const char* what);

// Tile geometry of an n x n problem with leaf tiles of edge `leaf`.
struct Geom {
    int64_t n = 0, bdim = 0, side = 0, ntiles = 0, pyr = 0;
    int32_t leaf = 0, lv = 0, nwords = 0;
};

bool make_geom(int64_t n, int32_t leaf, Geom* g);

// Workspace regions, in order.  Every entry point uses a subset.
struct Layout {
    size_t spyr[2], pyr[2], counts, bsums, boffs, masks, offsets, klist, pair_scratch, mwords, mcount, mprefix,
        mitems, items128, uprefix128, bounds, fix_slots, fix_slot_bytes, pm_state, pairs, scalars, partials, total;
    bool leaf128_dma;  // leaf 128 runs on the LDS-DMA kernel (items128, uprefix128 in use)
};

Layout make_layout(const Geom& g);

template <typename T>
T* at(void* ws, size_t off) {
    return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

bool overlaps(const void* p, size_t pbytes, const void* q, size_t qbytes);
bool aligned16(const void* p);
int device_cus();

spamm_status check_grid(const Geom& g);
// A null ws is replaced by the calling device's cached workspace (allocated
// or grown here); otherwise bytes must cover the layout of g.
spamm_status check_workspace(const Geom& g, void*& ws, size_t& bytes);
spamm_status check_tau(double tau);
spamm_status check_mul_args(const Geom& g, const float* a, const float* b, const float* c);

// Norm pass and pyramid for nmat matrices whose pyramids go to pyr_out[m];
// the norm pass also zeroes clear_count int64 words at clear (if not null).
// levels = false: the leaf level only (the norm pass; no pyramid launch).
spamm_status enqueue_pyramids(const Geom& g, const float* const* x, int nmat, double* const* pyr_out, void* ws,
                              hipStream_t s, int64_t* clear = nullptr, int64_t clear_count = 0, bool levels = true);
// Norms, pyramids and plan of A and B into the workspace pyramids and the
// caller's offsets, klist, pairs; with `schedule` (leaf 32 or 64) also the
// multiply schedule, the plan and schedule then coming from one launch.
spamm_status enqueue_prepare(const Geom& g, const float* a, const float* b, double tau, int32_t* offsets,
                             int32_t* klist, int64_t* pairs, void* ws, hipStream_t s, bool schedule);
// Plan of the kept triples (norm product >= tau), or with `skipped` of the
// triples SpAMM drops (norm product < tau).
spamm_status enqueue_plan(const Geom& g, const double* pa, const double* pb, double tau, bool skipped,
                          int32_t* offsets, int32_t* klist, int64_t* pairs, void* ws, hipStream_t s);
// Multiply of the pairs of a plan into c (every tile of c is written): the
// schedule the multiply kernel streams (workspace), then the multiply kernel.
// The macro-tile schedule arrays of the workspace at ws.
spamm::MacroSchedule macro_schedule(const Layout& L, void* ws);
spamm_status enqueue_schedule(const Geom& g, const int32_t* offsets, const int32_t* klist, void* ws, hipStream_t s);
spamm_status enqueue_multiply(const Geom& g, const float* a, const float* b, const int32_t* offsets,
                              const int32_t* klist, float* c, void* ws, hipStream_t s);
spamm_status enqueue_execute(const Geom& g, const float* a, const float* b, const int32_t* offsets,
                             const int32_t* klist, float* c, void* ws, hipStream_t s);

}  // namespace spamm_host
