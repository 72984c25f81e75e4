/* spamm_tau.h: choosing the SpAMM threshold tau for a requested accuracy.
 *
 * The paper picks tau by a search on the valid ratio (section 3.5.2;
 * spamm_search_valid_ratio in spamm.h) and measures accuracy by the error
 * matrix AB - SpAMM(A, B, tau) (Eq. 5, section 4).  This part of libspamm.so
 * targets that error directly:
 *
 *   - spamm_error_for_tau measures ||AB - SpAMM(A, B, tau)||_F / ||AB||_F by
 *     multiplying exactly the leaf pairs SpAMM drops;
 *   - spamm_search_tau_for_error finds the largest leaf norm product tau whose
 *     relative error is <= target (optionally starting from a guess);
 *   - a small network (129 -> 128 -> 128 -> 1, GELU in erf form) maps the
 *     histograms of log10 leaf norms of A and B and log10(target) to a
 *     predicted log10(tau); its forward, loss gradient and Adam kernels are
 *     here, so it is trained and run on the GPU.
 *
 * Conventions are those of spamm.h: device pointers unless stated, a
 * workspace of spamm_workspace_bytes(n, leaf) bytes where one is taken,
 * asynchronous on `stream` unless stated, status codes and
 * spamm_last_error(). */
#ifndef SPAMM_TAU_H
#define SPAMM_TAU_H

#include "spamm.h"

#ifdef __cplusplus
extern "C" {
#endif

#define SPAMM_TAU_FEATURES 129 /* 64 + 64 histogram bins + log10(target) */
#define SPAMM_TAU_HIDDEN 128
#define SPAMM_TAU_HIST_LO (-46.0) /* log10 range of the histogram bins */
#define SPAMM_TAU_HIST_HI 3.0

/* Number of network parameters (33281), flat FP32 in the order W1 [128][129]
 * (row = output unit), b1 [128], W2 [128][128], b2 [128], w3 [128], b3 [1]. */
int64_t spamm_mlp_param_count(void);

/* Floats of activation scratch that a batch of `batch` rows needs. */
int64_t spamm_mlp_acts_floats(int32_t batch);

/* Features of one (A, B, target) problem, FP32 [129]: for A then B, 64 bins
 * of log10(leaf norm) over [-46, 3) in steps of 49/64, each the number of
 * leaf tiles with a positive norm in it per tile row (count / bdim, so that a
 * band of the same decay gives the same features at any N), capped at 4 (the
 * bins of tiny far-off-diagonal norms grow with N); a norm below or above the
 * range counts in the first or last bin, a zero norm in none; then
 * log10(target).
 *   pyr_a, pyr_b  pyramids from spamm_pyramid (device).
 *   features      device FP32 [129].
 * EINVAL: null pointer, bad size, target not > 0. */
spamm_status spamm_tau_features(const double* pyr_a, const double* pyr_b, int64_t n, int32_t leaf, double target,
                                float* features, void* stream);

/* Predicted log10(tau) for `batch` feature rows x [batch][129] into y [batch].
 * acts: device FP32 scratch of spamm_mlp_acts_floats(batch) floats.
 * EINVAL: null pointer, batch < 1. */
spamm_status spamm_mlp_forward(const float* params, const float* x, int32_t batch, float* y, float* acts,
                               void* stream);

/* Mean squared error of the predictions for x against targets t [batch]
 * (log10 tau) into *loss (device float), and its gradient with respect to the
 * parameters into grad (same layout as params).  Sums over the batch run in
 * ascending order (results are reproducible).  acts as above. */
spamm_status spamm_mlp_loss_grad(const float* params, const float* x, const float* t, int32_t batch, float* acts,
                                 float* grad, float* loss, void* stream);

/* One Adam step (Kingma and Ba, 2015) with bias correction, step >= 1:
 * m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * p -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps).
 * m and v start as zeros.  EINVAL: null pointer, step < 1. */
spamm_status spamm_mlp_adam(float* params, const float* grad, float* m, float* v, int32_t step, float lr,
                            float beta1, float beta2, float eps, void* stream);

/* *out (device double) = sum of x[q]^2 over count FP32 values, in FP64 with a
 * fixed reduction order (x may be NULL when count is 0).  scratch: device
 * memory of at least spamm_sumsq_scratch_bytes() bytes. */
size_t spamm_sumsq_scratch_bytes(void);
spamm_status spamm_sumsq(const float* x, int64_t count, double* out, void* scratch, size_t scratch_bytes,
                         void* stream);

/* Relative error of SpAMM at tau against the exact product:
 * ||E||_F / sqrt(ab_sumsq) with E = AB - SpAMM(A, B, tau) formed as the FP32
 * multiply of exactly the leaf pairs SpAMM drops (norm product < tau), so that
 * small errors are not lost to cancellation.
 *   pyr_a, pyr_b  pyramids of A and B (spamm_pyramid).
 *   ab_sumsq      ||AB||_F^2 as a HOST double (e.g. spamm_multiply at tau = 0
 *                 followed by spamm_sumsq).
 *   e_scratch     device FP32 [n*n]: receives E.
 *   err_out       HOST double; dropped_out (may be NULL) HOST int64: number of
 *                 dropped triples.
 * Synchronous (one stream synchronisation).  Uses the workspace's plan
 * regions, so it must not overlap other calls on the same workspace. */
spamm_status spamm_error_for_tau(const float* a, const float* b, int64_t n, int32_t leaf, double tau,
                                 const double* pyr_a, const double* pyr_b, double ab_sumsq, float* e_scratch,
                                 double* err_out, int64_t* dropped_out, void* workspace, size_t workspace_bytes,
                                 void* stream);

/* The largest leaf norm product tau with relative error <= target (the error
 * of spamm_error_for_tau), found by bisection on log(tau) over the norm
 * products: the bounds are the smallest positive product (every nonzero pair
 * kept, error 0) and the largest; each probe is rounded up to the next
 * product, and the search ends when no product lies between the largest
 * passing product and the smallest failing threshold.  With tau_guess > 0 the
 * bracket is first grown geometrically (factor 4) from the guess.  This is
 * the largest such product whenever the error grows with tau, which holds for
 * matrices with non-negative entries.
 *   target        relative error, > 0.
 *   max_evals     cap on error evaluations (>= 1); when reached the best
 *                 passing product so far is returned.
 *   tau_out, err_out (error at tau_out), pairs_out (kept triples at tau_out),
 *   evals_out     HOST outputs (all but tau_out may be NULL).
 * Synchronous.  Other arguments as spamm_error_for_tau. */
spamm_status spamm_search_tau_for_error(const float* a, const float* b, int64_t n, int32_t leaf, double target,
                                        double tau_guess, int32_t max_evals, const double* pyr_a,
                                        const double* pyr_b, double ab_sumsq, float* e_scratch, double* tau_out,
                                        double* err_out, int64_t* pairs_out, int32_t* evals_out, void* workspace,
                                        size_t workspace_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SPAMM_TAU_H */
