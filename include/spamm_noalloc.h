/*
 * spamm_noalloc.h - the SpAMM hot path of libspamm.so for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Conventions as in spamm.h.
 */
#ifndef SPAMM_NOALLOC_H
#define SPAMM_NOALLOC_H

#include <stdint.h>

#include "spamm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Bytes of the static per-device scratch (64 MiB). */
#define SPAMM_NOALLOC_SCRATCH_BYTES (64u << 20)

/* spamm_multiply with its workspace in a static device array of
 * SPAMM_NOALLOC_SCRATCH_BYTES that the library holds, one copy per device,
 * until the process ends: the call allocates and frees nothing.  a, b, c,
 * pairs, n, tau, leaf, stream, results and errors as spamm_multiply, plus
 * ENOSPACE (nothing enqueued) when spamm_workspace_bytes(n, leaf) exceeds the
 * scratch: n up to 8192 at leaf 64 or 128, 4096 at leaf 32, 2048 at leaf 16
 * fit.  Every call on a device shares that device's scratch and leaves its
 * contents behind: calls that overlap on one device (other streams or host
 * threads) race, so the caller orders them.  No call relies on the scratch
 * starting at zero; each writes what it later reads (the pair counter is
 * cleared by a kernel). */
spamm_status spamm_multiply_noalloc(const float* a, const float* b, int64_t n, double tau, int32_t leaf, float* c,
                                    int64_t* pairs, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SPAMM_NOALLOC_H */
