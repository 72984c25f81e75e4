// Host side of the threshold-selection entry points (spamm_tau.h): error of
// SpAMM at a given tau, the search for the largest tau meeting an error
// target, and the network kernels' launchers.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstring>
#include <limits>

#include "host.h"
#include "internal.h"
#include "spamm_tau.h"

using namespace spamm_host;

namespace {

constexpr double kInf = std::numeric_limits<double>::infinity();

double bits_to_double(unsigned long long u) {
    double d;
    static_assert(sizeof(d) == sizeof(u), "64-bit double");
    std::memcpy(&d, &u, sizeof(d));
    return d;
}

// The device-side pieces of one (A, B) problem that the search uses.
struct Probe {
    Geom g;
    const float *a, *b;
    const double *pa, *pb;
    double ab_sumsq;
    float* e;
    void* ws;
    hipStream_t s;

    // (smallest norm product >= lo, or +inf; largest norm product)
    spamm_status bounds(double lo, double* snap, double* pmax) const {
        const Layout L = make_layout(g);
        auto* d = at<unsigned long long>(ws, L.scalars) + 1;
        spamm_status st = hip_check(spamm::launch_product_bounds(pa, pb, g.bdim, g.lv, lo, d, s), "bounds kernel");
        if (st != SPAMM_OK) return st;
        unsigned long long h[2];
        if ((st = hip_check(hipMemcpyAsync(h, d, sizeof(h), hipMemcpyDeviceToHost, s), "copy")) != SPAMM_OK) return st;
        if ((st = hip_check(hipStreamSynchronize(s), "synchronize")) != SPAMM_OK) return st;
        *snap = bits_to_double(h[0]);
        if (pmax) *pmax = bits_to_double(h[1]);
        return SPAMM_OK;
    }

    // relative error at tau, and the number of dropped triples
    spamm_status error(double tau, double* err, int64_t* dropped) const {
        const Layout L = make_layout(g);
        int32_t* offsets = at<int32_t>(ws, L.offsets);
        int32_t* klist = at<int32_t>(ws, L.klist);
        int64_t* d_pairs = at<int64_t>(ws, L.pairs);
        double* d_sum = at<double>(ws, L.scalars);
        spamm_status st = enqueue_plan(g, pa, pb, tau, true, offsets, klist, d_pairs, ws, s);
        if (st != SPAMM_OK) return st;
        if ((st = enqueue_execute(g, a, b, offsets, klist, e, ws, s)) != SPAMM_OK) return st;
        st = hip_check(spamm::launch_sumsq(e, g.n * g.n, at<double>(ws, L.partials), d_sum, s), "sumsq kernels");
        if (st != SPAMM_OK) return st;
        double esq = 0.0;
        int64_t cnt = 0;
        if ((st = hip_check(hipMemcpyAsync(&esq, d_sum, sizeof(esq), hipMemcpyDeviceToHost, s), "copy")) != SPAMM_OK)
            return st;
        if ((st = hip_check(hipMemcpyAsync(&cnt, d_pairs, sizeof(cnt), hipMemcpyDeviceToHost, s), "copy")) !=
            SPAMM_OK)
            return st;
        if ((st = hip_check(hipStreamSynchronize(s), "synchronize")) != SPAMM_OK) return st;
        *err = std::sqrt(esq / ab_sumsq);
        if (dropped) *dropped = cnt;
        return SPAMM_OK;
    }

    // kept triples at tau (count-only plan)
    spamm_status kept(double tau, int64_t* out) const {
        const Layout L = make_layout(g);
        int32_t* bsums = at<int32_t>(ws, L.bsums);
        int64_t* d_pairs = at<int64_t>(ws, L.pairs);
        spamm_status st =
            hip_check(spamm::launch_plan_count(pa, pb, g.bdim, g.lv, tau, bsums, s), "count kernel");
        if (st != SPAMM_OK) return st;
        st = hip_check(spamm::launch_plan_scan(bsums, g.bdim * g.nwords, nullptr, nullptr, 0, d_pairs, s),
                       "scan kernel");
        if (st != SPAMM_OK) return st;
        if ((st = hip_check(hipMemcpyAsync(out, d_pairs, sizeof(int64_t), hipMemcpyDeviceToHost, s), "copy")) !=
            SPAMM_OK)
            return st;
        return hip_check(hipStreamSynchronize(s), "synchronize");
    }
};

spamm_status make_probe(const float* a, const float* b, int64_t n, int32_t leaf, const double* pa, const double* pb,
                        double ab_sumsq, float* e, void* ws, size_t ws_bytes, void* stream, Probe* p) {
    if (!make_geom(n, leaf, &p->g)) return fail(SPAMM_EINVAL, "bad size n=%lld leaf=%d", (long long)n, leaf);
    if (!pa || !pb) return fail(SPAMM_EINVAL, "null pyramid pointer");
    spamm_status st = check_mul_args(p->g, a, b, e);
    if (st != SPAMM_OK) return st;
    if (!(ab_sumsq > 0.0) || std::isinf(ab_sumsq))
        return fail(SPAMM_EINVAL, "||AB||_F^2 must be positive and finite (got %g)", ab_sumsq);
    if ((st = check_grid(p->g)) != SPAMM_OK) return st;
    if ((st = check_workspace(p->g, ws, ws_bytes)) != SPAMM_OK) return st;
    p->a = a;
    p->b = b;
    p->pa = pa;
    p->pb = pb;
    p->ab_sumsq = ab_sumsq;
    p->e = e;
    p->ws = ws;
    p->s = static_cast<hipStream_t>(stream);
    return SPAMM_OK;
}

}  // namespace

extern "C" {

int64_t spamm_mlp_param_count(void) { return spamm::MlpLayout{}.count; }

int64_t spamm_mlp_acts_floats(int32_t batch) { return batch < 1 ? 0 : spamm::MlpLayout::acts(batch).acts_total; }

spamm_status spamm_tau_features(const double* pyr_a, const double* pyr_b, int64_t n, int32_t leaf, double target,
                                float* features, void* stream) {
    g_last_error[0] = '\0';
    Geom g;
    if (!make_geom(n, leaf, &g)) return fail(SPAMM_EINVAL, "bad size n=%lld leaf=%d", (long long)n, leaf);
    if (!pyr_a || !pyr_b || !features) return fail(SPAMM_EINVAL, "null pointer");
    if (!(target > 0.0) || std::isinf(target)) return fail(SPAMM_EINVAL, "target must be positive and finite");
    return hip_check(spamm::launch_tau_features(pyr_a, pyr_b, g.bdim, g.lv, float(std::log10(target)), features,
                                                static_cast<hipStream_t>(stream)),
                     "features kernel");
}

spamm_status spamm_mlp_forward(const float* params, const float* x, int32_t batch, float* y, float* acts,
                               void* stream) {
    g_last_error[0] = '\0';
    if (!params || !x || !y || !acts) return fail(SPAMM_EINVAL, "null pointer");
    if (batch < 1) return fail(SPAMM_EINVAL, "batch must be >= 1");
    return hip_check(spamm::launch_mlp_forward(params, x, batch, acts, y, static_cast<hipStream_t>(stream)),
                     "network forward kernels");
}

spamm_status spamm_mlp_loss_grad(const float* params, const float* x, const float* t, int32_t batch, float* acts,
                                 float* grad, float* loss, void* stream) {
    g_last_error[0] = '\0';
    if (!params || !x || !t || !acts || !grad || !loss) return fail(SPAMM_EINVAL, "null pointer");
    if (batch < 1) return fail(SPAMM_EINVAL, "batch must be >= 1");
    return hip_check(
        spamm::launch_mlp_loss_grad(params, x, t, batch, acts, grad, loss, static_cast<hipStream_t>(stream)),
        "network gradient kernels");
}

spamm_status spamm_mlp_adam(float* params, const float* grad, float* m, float* v, int32_t step, float lr,
                            float beta1, float beta2, float eps, void* stream) {
    g_last_error[0] = '\0';
    if (!params || !grad || !m || !v) return fail(SPAMM_EINVAL, "null pointer");
    if (step < 1) return fail(SPAMM_EINVAL, "step counts from 1");
    const float c1 = float(1.0 - std::pow(double(beta1), double(step)));
    const float c2 = float(1.0 - std::pow(double(beta2), double(step)));
    return hip_check(spamm::launch_adam(params, grad, m, v, spamm::MlpLayout{}.count, lr, beta1, beta2, eps, c1, c2,
                                        static_cast<hipStream_t>(stream)),
                     "adam kernel");
}

size_t spamm_sumsq_scratch_bytes(void) { return sizeof(double) * spamm::kSumBlocks; }

spamm_status spamm_sumsq(const float* x, int64_t count, double* out, void* scratch, size_t scratch_bytes,
                         void* stream) {
    g_last_error[0] = '\0';
    if ((!x && count > 0) || !out || !scratch) return fail(SPAMM_EINVAL, "null pointer");
    if (count < 0) return fail(SPAMM_EINVAL, "count must be >= 0");
    if (scratch_bytes < spamm_sumsq_scratch_bytes())
        return fail(SPAMM_ENOSPACE, "scratch of %zu bytes, %zu needed", scratch_bytes, spamm_sumsq_scratch_bytes());
    return hip_check(
        spamm::launch_sumsq(x, count, static_cast<double*>(scratch), out, static_cast<hipStream_t>(stream)),
        "sumsq kernels");
}

spamm_status spamm_error_for_tau(const float* a, const float* b, int64_t n, int32_t leaf, double tau,
                                 const double* pyr_a, const double* pyr_b, double ab_sumsq, float* e_scratch,
                                 double* err_out, int64_t* dropped_out, void* workspace, size_t workspace_bytes,
                                 void* stream) {
    g_last_error[0] = '\0';
    Probe p;
    spamm_status st = make_probe(a, b, n, leaf, pyr_a, pyr_b, ab_sumsq, e_scratch, workspace, workspace_bytes,
                                 stream, &p);
    if (st != SPAMM_OK) return st;
    if (!err_out) return fail(SPAMM_EINVAL, "null err_out");
    if ((st = check_tau(tau)) != SPAMM_OK) return st;
    return p.error(tau, err_out, dropped_out);
}

spamm_status spamm_search_tau_for_error(const float* a, const float* b, int64_t n, int32_t leaf, double target,
                                        double tau_guess, int32_t max_evals, const double* pyr_a,
                                        const double* pyr_b, double ab_sumsq, float* e_scratch, double* tau_out,
                                        double* err_out, int64_t* pairs_out, int32_t* evals_out, void* workspace,
                                        size_t workspace_bytes, void* stream) {
    g_last_error[0] = '\0';
    Probe p;
    spamm_status st = make_probe(a, b, n, leaf, pyr_a, pyr_b, ab_sumsq, e_scratch, workspace, workspace_bytes,
                                 stream, &p);
    if (st != SPAMM_OK) return st;
    if (!tau_out) return fail(SPAMM_EINVAL, "null tau_out");
    if (!(target > 0.0)) return fail(SPAMM_EINVAL, "target must be > 0");
    if (max_evals < 1) return fail(SPAMM_EINVAL, "max_evals must be >= 1");
    if (std::isnan(tau_guess)) return fail(SPAMM_EINVAL, "tau_guess is NaN");

    int evals = 0;
    double pmin = 0.0, pmax = 0.0;
    if ((st = p.bounds(DBL_TRUE_MIN, &pmin, &pmax)) != SPAMM_OK) return st;
    double lo = 0.0, lo_err = 0.0;  // passing threshold (a product) and its error
    if (std::isinf(pmin)) {
        // every norm product is zero: SpAMM is exactly AB for every tau, and
        // the largest product is 0
        lo = 0.0;
    } else {
        // invariant: lo is a product with error <= target (the smallest positive
        // product keeps every nonzero pair: error 0); hi is a threshold whose
        // error exceeds the target, +inf standing for "above every product"
        lo = pmin;
        double hi = kInf;
        auto snap = [&](double x, double* out) { return p.bounds(x, out, nullptr); };
        auto eval = [&](double t, bool* pass, double* e) -> spamm_status {
            spamm_status r = p.error(t, e, nullptr);
            ++evals;
            *pass = *e <= target;
            return r;
        };
        bool pass = false;
        double e = 0.0, c = 0.0;
        if (tau_guess > 0.0 && evals < max_evals) {
            const double g0 = tau_guess < pmin ? pmin : (tau_guess > pmax ? pmax : tau_guess);
            if ((st = snap(g0, &c)) != SPAMM_OK) return st;
            if ((st = eval(c, &pass, &e)) != SPAMM_OK) return st;
            if (pass) {
                lo = c;
                lo_err = e;
                while (evals < max_evals) {  // grow upwards
                    const double up = lo * 4.0;
                    if (up > pmax) break;
                    if ((st = snap(up, &c)) != SPAMM_OK) return st;
                    if ((st = eval(c, &pass, &e)) != SPAMM_OK) return st;
                    if (!pass) {
                        hi = c;
                        break;
                    }
                    lo = c;
                    lo_err = e;
                }
            } else {
                hi = c;
                while (evals < max_evals) {  // grow downwards
                    const double down = hi / 4.0;
                    if (down <= pmin) break;
                    if ((st = snap(down, &c)) != SPAMM_OK) return st;
                    if (c >= hi) {  // no product in [down, hi): same mask as hi
                        hi = down;
                        continue;
                    }
                    if ((st = eval(c, &pass, &e)) != SPAMM_OK) return st;
                    if (pass) {
                        lo = c;
                        lo_err = e;
                        break;
                    }
                    hi = c;
                }
            }
        }
        for (int guard = 0; evals < max_evals && guard < 8192; ++guard) {
            double next = 0.0;  // the smallest product above lo
            if ((st = snap(std::nextafter(lo, kInf), &next)) != SPAMM_OK) return st;
            if (next >= hi) break;  // lo is the largest passing product
            double mid = std::isinf(hi) ? pmax : std::sqrt(lo) * std::sqrt(hi);
            if (!(mid > lo)) mid = next;
            if ((st = snap(mid, &c)) != SPAMM_OK) return st;
            if (c >= hi) {  // no product in [mid, hi): mid fails like hi
                hi = mid;
                continue;
            }
            if ((st = eval(c, &pass, &e)) != SPAMM_OK) return st;
            if (pass) {
                lo = c;
                lo_err = e;
            } else {
                hi = c;
            }
        }
    }
    int64_t kept = 0;
    if ((st = p.kept(lo, &kept)) != SPAMM_OK) return st;
    *tau_out = lo;
    if (err_out) *err_out = lo_err;
    if (pairs_out) *pairs_out = kept;
    if (evals_out) *evals_out = evals;
    return SPAMM_OK;
}

}  // extern "C"
