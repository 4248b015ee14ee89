// Coefficient training (Sec. III.C) and the matrix forward/backward used for fitting on
// matrices.
//
// fe_train_coeffs fits the L x 4 coefficients of the layer recursion to the Fermi function
// g(y) = 1/(1 + exp(beta0 (mu0 - y))) or to its entropy function on the model coordinate
// y in [0, 1], by Levenberg-Marquardt (Marquardt damping scaled by the running maximum of the
// Gram diagonal) with geodesic acceleration (Transtrum and Sethna): the second directional
// derivative of the residuals along the step is computed exactly (forward mode of second order in
// the residual kernel; a central difference for the Skip-SP2 / Max-SP2 models) and its
// correction is kept only when 2 |a| <= 0.75 |step|. Residuals and the Jacobian are
// evaluated on the GPU in FP64 (one lane per sample point), J^T J and J^T r on the GPU, the
// damped normal equations are solved on the host in FP64 (Cholesky). The damping follows Nielsen's
// update (gain ratio of actual to predicted cost reduction).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "fe_host.h"
#include "fe_variant.h"

using namespace fehost;

extern "C" int fe_matrix_forward(float* hist, int64_t n, const double* theta, int32_t L, float* P,
                                 void* stream);
extern "C" int fe_matrix_backward(const float* hist, int64_t n, const double* theta, int32_t L,
                                  const float* G, float* work, double* part, int32_t nblocks,
                                  double* grad, void* stream);

namespace {

constexpr double kLn2 = 0.69314718055994530942;

// Logistic g(y) = 1/(1 + exp(beta0 (mu0 - y))), evaluated without overflow.
double fermi_target(double y, double beta0, double mu0) {
    const double u = beta0 * (mu0 - y);
    if (u >= 0) {
        const double e = exp(-u);
        return e / (1.0 + e);
    }
    return 1.0 / (1.0 + exp(u));
}

// Entropy -g ln g - (1-g) ln(1-g) of the logistic, written in |u| to avoid ln 0.
double entropy_target(double y, double beta0, double mu0) {
    const double u = fabs(beta0 * (mu0 - y));
    const double t = exp(-u);
    return log1p(t) + u * t / (1.0 + t);
}

// n points as the (k + 1/2)/n quantiles of a density on [0, 1]: 1 (uniform), 1 + |g'| or
// sqrt(1 + g'^2), integrated by the trapezoid rule on a fine grid.
std::vector<double> sample_points(int n, double beta0, double mu0, int law) {
    const int grid = 1 << 20;
    std::vector<double> cdf(grid + 1);
    auto dens = [&](double y) {
        const double g = fermi_target(y, beta0, mu0);
        const double gp = beta0 * g * (1.0 - g);
        if (law == FE_SAMPLE_UNIFORM) return 1.0;
        if (law == FE_SAMPLE_ARCLEN) return sqrt(1.0 + gp * gp);
        return 1.0 + fabs(gp);
    };
    cdf[0] = 0.0;
    double prev = dens(0.0);
    for (int i = 1; i <= grid; ++i) {
        const double y = (double)i / grid;
        const double d = dens(y);
        cdf[i] = cdf[i - 1] + 0.5 * (prev + d) / grid;
        prev = d;
    }
    const double tot = cdf[grid];
    std::vector<double> out(n);
    int j = 0;
    for (int k = 0; k < n; ++k) {
        const double q = (k + 0.5) / n * tot;
        while (j < grid && cdf[j + 1] < q) ++j;
        const double c0 = cdf[j], c1 = cdf[j + 1];
        const double f = c1 > c0 ? (q - c0) / (c1 - c0) : 0.0;
        out[k] = ((double)j + f) / grid;
    }
    return out;
}

// In-place Cholesky of the symmetric positive definite P x P matrix a (lower part used);
// returns false if it is not positive definite.
bool cholesky(std::vector<double>& a, int P) {
    for (int j = 0; j < P; ++j) {
        double s = a[(size_t)j * P + j];
        for (int k = 0; k < j; ++k) s -= a[(size_t)j * P + k] * a[(size_t)j * P + k];
        if (!(s > 0.0)) return false;
        const double d = sqrt(s);
        a[(size_t)j * P + j] = d;
        for (int i = j + 1; i < P; ++i) {
            double t = a[(size_t)i * P + j];
            for (int k = 0; k < j; ++k) t -= a[(size_t)i * P + k] * a[(size_t)j * P + k];
            a[(size_t)i * P + j] = t / d;
        }
    }
    return true;
}

void chol_solve(const std::vector<double>& l, int P, std::vector<double>& x) {
    for (int i = 0; i < P; ++i) {
        double s = x[i];
        for (int k = 0; k < i; ++k) s -= l[(size_t)i * P + k] * x[k];
        x[i] = s / l[(size_t)i * P + i];
    }
    for (int i = P - 1; i >= 0; --i) {
        double s = x[i];
        for (int k = i + 1; k < P; ++k) s -= l[(size_t)k * P + i] * x[k];
        x[i] = s / l[(size_t)i * P + i];
    }
}

// Host FP64 evaluation of the scalar model (for the final error on a dense grid).
double model_value(const double* th, int L, int target, double mu0, double alpha, double y) {
    double x = target == FE_TARGET_ENTROPY ? alpha * (y - mu0) + mu0 : y;
    double A = 0.0;
    for (int i = 0; i < L; ++i) {
        A += th[4 * i + 3] * x;
        x = th[4 * i] * x * x + th[4 * i + 1] * x + th[4 * i + 2];
    }
    const double u = A + x;
    return target == FE_TARGET_ENTROPY ? 4.0 * kLn2 * u * (1.0 - u) : u;
}

struct DevBufs {
    double *y = nullptr, *tgt = nullptr, *r = nullptr, *JT = nullptr, *G = nullptr, *g = nullptr, *v = nullptr;
    double* coef = nullptr;
    void release() {
        for (double* p : {y, tgt, r, JT, G, g, v, coef})
            if (p) (void)hipFree(p);
    }
};

// Levenberg-Marquardt with geodesic acceleration over P coefficients and n residuals (see the
// file comment). launch(th, jac) enqueues the residuals at th into d.r and, if jac, the Jacobian
// transposed into d.JT, on stream s. If second is given (has_second), second(th, v) enqueues the
// exact second directional derivative of the residuals along v into d.v; otherwise it is
// estimated by a central difference. On return th holds the best coefficients, r their
// residuals (host), and it / lam the iterations and final damping.
template <class Launch, class Second>
hipError_t lm_run(int P, int n, std::vector<double>& th, std::vector<double>& r, DevBufs& d,
                  hipStream_t s, int max_iter, double tol, Launch launch, bool has_second,
                  Second second, int& it, double& lam) {
    std::vector<double> rp(n), rm(n), G((size_t)P * P), g(P), Gl((size_t)P * P), dmax(P, 0.0);
    auto eval = [&](const std::vector<double>& t, std::vector<double>& out, bool jac) -> hipError_t {
        hipError_t err = launch(t, jac);
        if (err == hipSuccess) err = hipMemcpyAsync(out.data(), d.r, sizeof(double) * n, hipMemcpyDeviceToHost, s);
        if (err == hipSuccess) err = hipStreamSynchronize(s);
        return err;
    };
    // J^T v for v on the host (copied to d.v), or already in d.v (v_on_device), or r (neither)
    auto gram = [&](bool full, const std::vector<double>* v, std::vector<double>& gout,
                    bool v_on_device = false) -> hipError_t {
        hipError_t err = hipSuccess;
        if (v) err = hipMemcpyAsync(d.v, v->data(), sizeof(double) * n, hipMemcpyHostToDevice, s);
        if (err == hipSuccess)
            err = fe::launch_gram(d.JT, (v || v_on_device) ? d.v : d.r, P, n, full ? d.G : nullptr,
                                  d.g, s);
        if (err == hipSuccess && full) err = hipMemcpyAsync(G.data(), d.G, sizeof(double) * P * P, hipMemcpyDeviceToHost, s);
        if (err == hipSuccess) err = hipMemcpyAsync(gout.data(), d.g, sizeof(double) * P, hipMemcpyDeviceToHost, s);
        if (err == hipSuccess) err = hipStreamSynchronize(s);
        return err;
    };
    auto cost = [](const std::vector<double>& v) {
        double c = 0.0;
        for (double x : v) c += x * x;
        return 0.5 * c;
    };
    auto maxabs = [](const std::vector<double>& v) {
        double m = 0.0;
        for (double x : v) m = std::max(m, fabs(x));
        return m;
    };

    lam = 1e-3;
    double nu = 2.0;
    it = 0;
    hipError_t e = eval(th, r, true);
    double C = cost(r);
    bool have_gram = false;
    std::vector<double> dl(P), acc(P), tn(P), tmp(P);
    for (; e == hipSuccess && it < max_iter; ++it) {
        if (maxabs(r) < tol) break;
        if (!have_gram) {
            e = gram(true, nullptr, g);
            if (e != hipSuccess) break;
            for (int p = 0; p < P; ++p)
                for (int q = 0; q < p; ++q) G[(size_t)p * P + q] = G[(size_t)q * P + p];
            double big = 0.0;
            for (int p = 0; p < P; ++p) {
                dmax[p] = std::max(dmax[p], G[(size_t)p * P + p]);
                big = std::max(big, dmax[p]);
            }
            for (int p = 0; p < P; ++p) dmax[p] = std::max(dmax[p], 1e-12 * big);
            have_gram = true;
        }
        Gl = G;
        for (int p = 0; p < P; ++p) Gl[(size_t)p * P + p] += lam * dmax[p];
        if (!cholesky(Gl, P)) {
            lam *= nu;
            nu *= 2.0;
            continue;
        }
        for (int p = 0; p < P; ++p) dl[p] = -g[p];
        chol_solve(Gl, P, dl);
        // geodesic acceleration (Transtrum and Sethna): the second directional derivative r''
        // of the residuals along dl, a = -(J^T J + lam D)^-1 J^T r'', step dl + a / 2, kept only
        // when 2 |a| / |dl| <= 0.75
        if (has_second) {
            e = second(th, dl);
            if (e != hipSuccess) break;
            e = gram(false, nullptr, tmp, true);
        } else {
            const double h = 0.1;
            for (int p = 0; p < P; ++p) tn[p] = th[p] + h * dl[p];
            e = eval(tn, rp, false);
            if (e != hipSuccess) break;
            for (int p = 0; p < P; ++p) tn[p] = th[p] - h * dl[p];
            e = eval(tn, rm, false);
            if (e != hipSuccess) break;
            for (int k = 0; k < n; ++k) rm[k] = (rp[k] - 2.0 * r[k] + rm[k]) / (h * h);
            e = gram(false, &rm, tmp);
        }
        if (e != hipSuccess) break;
        for (int p = 0; p < P; ++p) acc[p] = -tmp[p];
        chol_solve(Gl, P, acc);
        double na = 0.0, nd = 0.0;
        for (int p = 0; p < P; ++p) {
            na += acc[p] * acc[p];
            nd += dl[p] * dl[p];
        }
        if (2.0 * sqrt(na) > 0.75 * sqrt(nd)) {
            lam *= nu;
            nu *= 2.0;
            if (lam > 1e14) break;
            continue;
        }
        for (int p = 0; p < P; ++p) tn[p] = th[p] + dl[p] + 0.5 * acc[p];
        e = eval(tn, rp, true);
        if (e != hipSuccess) break;
        const double Cn = cost(rp);
        if (Cn < C) {
            // gain ratio against the reduction the linearised residuals predict for the velocity,
            // pred = -g.dl - dl.G.dl / 2; damping update of Nielsen (as used by Transtrum and
            // Sethna): lam *= max(1/3, 1 - (2 rho - 1)^3) on acceptance, doubling factors after
            // each rejection
            double pred = 0.0;
            for (int p = 0; p < P; ++p) {
                double gd = 0.0;
                for (int q = 0; q < P; ++q) gd += G[(size_t)p * P + q] * dl[q];
                pred -= g[p] * dl[p] + 0.5 * dl[p] * gd;
            }
            const double rho = pred > 0.0 ? (C - Cn) / pred : 1.0;
            const double t = 2.0 * rho - 1.0;
            lam = std::max(lam * std::max(1.0 / 3.0, 1.0 - t * t * t), 1e-15);
            nu = 2.0;
            th = tn;
            r = rp;
            C = Cn;
            have_gram = false;   // J at the new point is already on the device
        } else {
            lam *= nu;
            nu *= 2.0;
            if (lam > 1e14) break;
            e = eval(th, r, true);   // restore J at the current point
        }
    }
    return e;
}

// Refinement of the coefficients on a set of matrices (fe_train_spec's matrix set): damped
// Gauss-Newton steps on F = C_points + (w/2) sum_m ||P(X0_m) - Dref_m||_F^2 whose metric is the
// points' J^T J (scaled by the running Gram diagonal, as in the fit) and whose gradient holds both
// terms (the matrix term's from the FP32 backward pass); a step is kept when F decreases. th and
// r (the points' residuals) are updated in place.
template <class Launch>
int matrix_refine(const fe_train_spec* sp, int P, int n, std::vector<double>& th,
                  std::vector<double>& r, DevBufs& d, hipStream_t s, Launch launch, int& its,
                  int& accepted, double& loss0, double& loss1) {
    const int L = sp->L;
    const int64_t nm = sp->mat_n;
    const size_t nn = (size_t)nm * nm;
    const int nb = 256;
    float *hist = nullptr, *Pd = nullptr, *Gm = nullptr, *work = nullptr;
    double *part = nullptr, *gradd = nullptr, *ssq = nullptr;
    auto release = [&]() {
        for (void* q : {(void*)hist, (void*)Pd, (void*)Gm, (void*)work, (void*)part, (void*)gradd,
                        (void*)ssq})
            if (q) (void)hipFree(q);
    };
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&hist), sizeof(float) * (L + 1) * nn);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&Pd), sizeof(float) * nn);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&Gm), sizeof(float) * nn);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&work), sizeof(float) * 3 * nn);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&part), sizeof(double) * 4 * nb);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&gradd), sizeof(double) * P);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&ssq), sizeof(double));
    if (e != hipSuccess) {
        release();
        return hip_fail(e, "matrix refinement scratch");
    }
    // sum_m ||P(X0_m) - Dref_m||^2 at t and, if gm, its half-gradient sum_m J_m^T r_m
    auto mat_eval = [&](const std::vector<double>& t, double& loss, std::vector<double>* gm) -> int {
        loss = 0.0;
        if (gm) gm->assign(P, 0.0);
        std::vector<double> gh(P);
        for (int m = 0; m < sp->n_mats; ++m) {
            FE_HIP(hipMemcpyAsync(hist, sp->X0s[m], sizeof(float) * nn, hipMemcpyDeviceToDevice, s));
            int rc = fe_matrix_forward(hist, nm, t.data(), L, Pd, s);
            if (rc) return rc;
            FE_HIP(fe::launch_mat_residual(Pd, sp->Drefs[m], (int64_t)nn, gm ? Gm : nullptr, part, nb,
                                           ssq, s));
            double v = 0.0;
            FE_HIP(hipMemcpyAsync(&v, ssq, sizeof(double), hipMemcpyDeviceToHost, s));
            if (gm) {
                rc = fe_matrix_backward(hist, nm, t.data(), L, Gm, work, part, nb, gradd, s);
                if (rc) return rc;
                FE_HIP(hipMemcpyAsync(gh.data(), gradd, sizeof(double) * P, hipMemcpyDeviceToHost, s));
            }
            FE_HIP(hipStreamSynchronize(s));
            loss += v;
            if (gm)
                for (int p = 0; p < P; ++p) (*gm)[p] += gh[p];
        }
        return FE_OK;
    };
    auto points = [&](const std::vector<double>& t, std::vector<double>& out, bool jac) -> int {
        FE_HIP(launch(t, jac));
        FE_HIP(hipMemcpyAsync(out.data(), d.r, sizeof(double) * n, hipMemcpyDeviceToHost, s));
        FE_HIP(hipStreamSynchronize(s));
        return FE_OK;
    };
    const double w = sp->mat_weight;
    std::vector<double> G((size_t)P * P), g(P), gm(P), Gl((size_t)P * P), dl(P), tn(P), rn(n);
    std::vector<double> dmax(P, 0.0);
    double lm_ = 0.0;
    int rc = points(th, r, true);
    if (!rc) rc = mat_eval(th, lm_, &gm);
    loss0 = lm_;
    double lam = 1e-3;
    its = accepted = 0;
    bool fresh = true;   // J, G, g and gm belong to th
    for (; rc == FE_OK && its < sp->mat_iters; ++its) {
        if (fresh) {
            FE_HIP(fe::launch_gram(d.JT, d.r, P, n, d.G, d.g, s));
            FE_HIP(hipMemcpyAsync(G.data(), d.G, sizeof(double) * P * P, hipMemcpyDeviceToHost, s));
            FE_HIP(hipMemcpyAsync(g.data(), d.g, sizeof(double) * P, hipMemcpyDeviceToHost, s));
            FE_HIP(hipStreamSynchronize(s));
            for (int p = 0; p < P; ++p)
                for (int q = 0; q < p; ++q) G[(size_t)p * P + q] = G[(size_t)q * P + p];
            double big = 0.0;
            for (int p = 0; p < P; ++p) {
                dmax[p] = std::max(dmax[p], G[(size_t)p * P + p]);
                big = std::max(big, dmax[p]);
            }
            for (int p = 0; p < P; ++p) dmax[p] = std::max(dmax[p], 1e-12 * big);
            fresh = false;
        }
        double C = 0.0;
        for (double v : r) C += 0.5 * v * v;
        const double F = C + 0.5 * w * lm_;
        Gl = G;
        for (int p = 0; p < P; ++p) Gl[(size_t)p * P + p] += lam * dmax[p];
        if (!cholesky(Gl, P)) {
            lam *= 4.0;
            continue;
        }
        for (int p = 0; p < P; ++p) dl[p] = -(g[p] + w * gm[p]);
        chol_solve(Gl, P, dl);
        for (int p = 0; p < P; ++p) tn[p] = th[p] + dl[p];
        rc = points(tn, rn, false);
        double lmn = 0.0;
        if (!rc) rc = mat_eval(tn, lmn, nullptr);
        if (rc) break;
        double Cn = 0.0;
        for (double v : rn) Cn += 0.5 * v * v;
        if (Cn + 0.5 * w * lmn < F) {
            th = tn;
            ++accepted;
            lam = std::max(lam / 3.0, 1e-15);
            rc = points(th, r, true);
            if (!rc) rc = mat_eval(th, lm_, &gm);
            fresh = true;
        } else {
            lam *= 2.0;
            if (lam > 1e14) break;
        }
    }
    loss1 = lm_;
    if (!fresh && rc == FE_OK) rc = points(th, r, false);
    release();
    return rc;
}

// Device scratch of one fit: n points, P coefficients (with an optional coefficient buffer).
hipError_t alloc_fit(DevBufs& d, int n, int P, const std::vector<double>& y, const std::vector<double>& tg) {
    hipError_t e = hipSuccess;
    for (double** p : {&d.y, &d.tgt, &d.r, &d.v})
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(p), sizeof(double) * n);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&d.JT), sizeof(double) * (size_t)P * n);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&d.G), sizeof(double) * (size_t)P * P);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&d.g), sizeof(double) * P);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&d.coef), sizeof(double) * P);
    if (e == hipSuccess) e = hipMemcpy(d.y, y.data(), sizeof(double) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d.tgt, tg.data(), sizeof(double) * n, hipMemcpyHostToDevice);
    return e;
}

}  // namespace

extern "C" {

int fe_scalar_eval(const double* y, int32_t n, const double* theta, int32_t L, int32_t target,
                   double mu0, double alpha, const double* tgt, double* r, double* JT, void* stream) {
    if (!y || !r || !theta || n < 1) return fail(FE_ERR_ARG, "bad arguments");
    if (L < 1 || L > fe::scalar_max_layers()) return fail(FE_ERR_ARG, "L out of range for the scalar kernel");
    if (target != FE_TARGET_FERMI && target != FE_TARGET_ENTROPY) return fail(FE_ERR_ARG, "unknown target");
    fe::ScalarArgs a{};
    a.y = y; a.tgt = tgt; a.r = r; a.JT = JT; a.n = n; a.L = L; a.target = target;
    a.mu0 = mu0; a.alpha = alpha;
    memcpy(a.theta, theta, sizeof(double) * 4 * L);
    FE_HIP(fe::launch_scalar_eval(a, static_cast<hipStream_t>(stream)));
    return FE_OK;
}

int fe_scalar_second(const double* y, int32_t n, const double* theta, int32_t L, int32_t target,
                     double mu0, double alpha, const double* v, double* r2, void* stream) {
    if (!y || !r2 || !theta || !v || n < 1) return fail(FE_ERR_ARG, "bad arguments");
    if (L < 1 || L > fe::scalar_max_layers()) return fail(FE_ERR_ARG, "L out of range for the scalar kernel");
    if (target != FE_TARGET_FERMI && target != FE_TARGET_ENTROPY) return fail(FE_ERR_ARG, "unknown target");
    fe::ScalarArgs a{};
    a.y = y; a.tgt = nullptr; a.r = nullptr; a.JT = nullptr; a.vdir = v; a.r2 = r2;
    a.n = n; a.L = L; a.target = target; a.mu0 = mu0; a.alpha = alpha;
    memcpy(a.theta, theta, sizeof(double) * 4 * L);
    FE_HIP(fe::launch_scalar_eval(a, static_cast<hipStream_t>(stream)));
    return FE_OK;
}

int fe_train_coeffs(const fe_train_spec* spec, const double* theta_init, double* theta_out,
                    fe_train_report* rep, fe_workspace* ws, void* stream) {
    (void)ws;
    if (!spec || !theta_out) return fail(FE_ERR_ARG, "spec and theta_out are required");
    const int L = spec->L, n = spec->n_points, P = 4 * L;
    if (L < 1 || L > fe::scalar_max_layers()) return fail(FE_ERR_ARG, "L out of range");
    if (n < P) return fail(FE_ERR_ARG, "need at least 4L sample points");
    if (!(spec->beta0 > 0.0) || !(spec->mu0 > 0.0 && spec->mu0 < 1.0)) return fail(FE_ERR_ARG, "bad (beta0, mu0)");
    if (spec->target != FE_TARGET_FERMI && spec->target != FE_TARGET_ENTROPY) return fail(FE_ERR_ARG, "unknown target");
    if (spec->n_mats < 0) return fail(FE_ERR_ARG, "n_mats must be >= 0");
    if (spec->n_mats > 0) {
        if (spec->target != FE_TARGET_FERMI) return fail(FE_ERR_ARG, "the matrix set takes the Fermi target");
        if (!spec->X0s || !spec->Drefs) return fail(FE_ERR_ARG, "X0s and Drefs are required with n_mats > 0");
        if (spec->mat_n < 64 || spec->mat_n % 64 != 0) return fail(FE_ERR_ARG, "mat_n must be a positive multiple of 64");
        if (spec->mat_iters < 1) return fail(FE_ERR_ARG, "mat_iters must be >= 1");
        if (!(spec->mat_weight > 0.0) || !isfinite(spec->mat_weight)) return fail(FE_ERR_ARG, "mat_weight must be positive");
        for (int m = 0; m < spec->n_mats; ++m)
            if (!spec->X0s[m] || !spec->Drefs[m]) return fail(FE_ERR_ARG, "a matrix pointer is NULL");
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const double b0 = spec->beta0, m0 = spec->mu0;
    const double alpha = spec->target == FE_TARGET_ENTROPY ? spec->alpha : 1.0;

    std::vector<double> th(P);
    if (theta_init) {
        memcpy(th.data(), theta_init, sizeof(double) * P);
    } else {
        // SP2 embedding (Eq. sp2-mu, App. C) for as many layers as the slope needs
        // (Eq. layer count), identity layers after it
        const int nl = std::max(1, std::min(L, (int)lround(fe_layer_count(b0))));
        std::vector<double> sp(4 * nl);
        fe_sp2_coeffs(m0, nl, sp.data());
        for (int i = 0; i < L; ++i) {
            double* t = th.data() + 4 * i;
            if (i < nl) memcpy(t, sp.data() + 4 * i, sizeof(double) * 4);
            else { t[0] = 0.0; t[1] = 1.0; t[2] = 0.0; t[3] = 0.0; }
        }
    }
    std::vector<double> y = sample_points(n, b0, m0, spec->sampling);
    std::vector<double> tg(n);
    for (int k = 0; k < n; ++k)
        tg[k] = spec->target == FE_TARGET_ENTROPY ? entropy_target(y[k], b0, m0) : fermi_target(y[k], b0, m0);

    // Training scratch lives for this call only (the trainer is not on the expansion's path).
    DevBufs d;
    hipError_t e = alloc_fit(d, n, P, y, tg);
    if (e != hipSuccess) {
        d.release();
        return hip_fail(e, "trainer scratch");
    }
    fe::ScalarArgs sa{};
    sa.y = d.y; sa.tgt = d.tgt; sa.n = n; sa.L = L; sa.target = spec->target; sa.mu0 = m0; sa.alpha = alpha;
    auto launch = [&](const std::vector<double>& t, bool jac) -> hipError_t {
        memcpy(sa.theta, t.data(), sizeof(double) * P);
        sa.r = d.r;
        sa.JT = jac ? d.JT : nullptr;
        sa.r2 = nullptr;
        return fe::launch_scalar_eval(sa, s);
    };
    // exact r'' along v: forward mode of second order in the residual kernel, into d.v (d.r keeps
    // the residuals of the current point)
    auto second = [&](const std::vector<double>& t, const std::vector<double>& v) -> hipError_t {
        hipError_t err = hipMemcpyAsync(d.coef, v.data(), sizeof(double) * P, hipMemcpyHostToDevice, s);
        if (err != hipSuccess) return err;
        fe::ScalarArgs a2 = sa;
        memcpy(a2.theta, t.data(), sizeof(double) * P);
        a2.r = nullptr;
        a2.JT = nullptr;
        a2.vdir = d.coef;
        a2.r2 = d.v;
        return fe::launch_scalar_eval(a2, s);
    };
    std::vector<double> r(n);
    int it = 0, rc = FE_OK;
    double lam = 0.0;
    e = lm_run(P, n, th, r, d, s, spec->max_iter, spec->tol, launch, true, second, it, lam);
    if (e != hipSuccess) {
        d.release();
        return hip_fail(e, "trainer");
    }
    int mat_its = 0, mat_acc = 0;
    double ml0 = NAN, ml1 = NAN;
    if (spec->n_mats > 0) {
        rc = matrix_refine(spec, P, n, th, r, d, s, launch, mat_its, mat_acc, ml0, ml1);
        if (rc) {
            d.release();
            return rc;
        }
    }
    d.release();
    memcpy(theta_out, th.data(), sizeof(double) * P);
    double emax = 0.0, ss = 0.0;
    for (double v : r) {
        emax = std::max(emax, fabs(v));
        ss += v * v;
    }
    if (rep) {
        rep->iters = it;
        rep->rms = sqrt(ss / n);
        rep->max_err_points = emax;
        rep->lambda = lam;
        rep->mat_iters = mat_its;
        rep->mat_accepted = mat_acc;
        rep->mat_loss_start = ml0;
        rep->mat_loss_end = ml1;
        double gmax = 0.0;
        const int ng = 200001;
        for (int k = 0; k < ng; ++k) {
            const double yy = (double)k / (ng - 1);
            const double t = spec->target == FE_TARGET_ENTROPY ? entropy_target(yy, b0, m0) : fermi_target(yy, b0, m0);
            gmax = std::max(gmax, fabs(model_value(th.data(), L, spec->target, m0, alpha, yy) - t));
        }
        rep->max_err_grid = gmax;
    }
    if (emax >= spec->tol) rc = FE_ERR_NO_CONVERGENCE;
    if (rc) fail(rc, "the fit stopped above its tolerance (theta_out holds the best coefficients found)");
    return rc;
}

int fe_train_variant(const fe_train_spec* spec, const fe_qmodel* init, double* coef_out,
                     fe_train_report* rep, void* stream) {
    if (!spec || !coef_out) return fail(FE_ERR_ARG, "spec and coef_out are required");
    int rc = check_qmodel(init);
    if (rc) return rc;
    if (spec->target != FE_TARGET_FERMI) return fail(FE_ERR_ARG, "the variant trainer fits the Fermi target");
    if (spec->n_mats != 0) return fail(FE_ERR_ARG, "the variant trainer takes no matrix set");
    if (!(spec->beta0 > 0.0) || !(spec->mu0 > 0.0 && spec->mu0 < 1.0)) return fail(FE_ERR_ARG, "bad (beta0, mu0)");
    const int P = (int)qmodel_coef_count(init->arch, init->L, init->k, init->K), n = spec->n_points;
    if (n < P) return fail(FE_ERR_ARG, "need at least as many sample points as coefficients");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const double b0 = spec->beta0, m0 = spec->mu0;
    std::vector<double> th(init->coef, init->coef + P);
    std::vector<double> y = sample_points(n, b0, m0, spec->sampling);
    std::vector<double> tg(n);
    for (int k = 0; k < n; ++k) tg[k] = fermi_target(y[k], b0, m0);
    DevBufs d;
    hipError_t e = alloc_fit(d, n, P, y, tg);
    if (e != hipSuccess) {
        d.release();
        return hip_fail(e, "trainer scratch");
    }
    fe::VariantEvalArgs va{};
    va.y = d.y; va.tgt = d.tgt; va.r = d.r; va.coef = d.coef; va.n = n;
    va.arch = init->arch; va.L = init->L; va.k = init->k; va.K = init->K;
    auto launch = [&](const std::vector<double>& t, bool jac) -> hipError_t {
        hipError_t err = hipMemcpyAsync(d.coef, t.data(), sizeof(double) * P, hipMemcpyHostToDevice, s);
        va.JT = jac ? d.JT : nullptr;
        if (err == hipSuccess) err = fe::launch_variant_eval(va, s);
        return err;
    };
    std::vector<double> r(n);
    int it = 0;
    double lam = 0.0;
    auto no_second = [](const std::vector<double>&, const std::vector<double>&) {
        return hipErrorNotSupported;
    };
    e = lm_run(P, n, th, r, d, s, spec->max_iter, spec->tol, launch, false, no_second, it, lam);
    d.release();
    if (e != hipSuccess) return hip_fail(e, "trainer");
    memcpy(coef_out, th.data(), sizeof(double) * P);
    double emax = 0.0, ss = 0.0;
    for (double v : r) {
        emax = std::max(emax, fabs(v));
        ss += v * v;
    }
    if (rep) {
        rep->iters = it;
        rep->rms = sqrt(ss / n);
        rep->max_err_points = emax;
        rep->lambda = lam;
        rep->mat_iters = rep->mat_accepted = 0;
        rep->mat_loss_start = rep->mat_loss_end = NAN;
        double gmax = 0.0;
        const int ng = 200001;
        for (int k = 0; k < ng; ++k) {
            const double yy = (double)k / (ng - 1);
            const double f = qmodel_value(init->arch, init->L, init->k, init->K, th.data(), yy, nullptr);
            gmax = std::max(gmax, fabs(f - fermi_target(yy, b0, m0)));
        }
        rep->max_err_grid = gmax;
    }
    if (emax >= spec->tol) {
        fail(FE_ERR_NO_CONVERGENCE, "the fit stopped above its tolerance (coef_out holds the best coefficients found)");
        return FE_ERR_NO_CONVERGENCE;
    }
    return FE_OK;
}

int fe_matrix_forward(float* hist, int64_t n, const double* theta, int32_t L, float* P,
                      void* stream) {
    if (!hist || !P || !theta) return fail(FE_ERR_ARG, "bad arguments");
    if (n < 1 || n % fe::wide_tile() != 0) return fail(FE_ERR_ARG, "n must be a positive multiple of 64");
    if (L < 1 || L > fe::scalar_max_layers()) return fail(FE_ERR_ARG, "L out of range");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t nn = (size_t)n * n;
    for (int i = 0; i < L; ++i) {
        fe::WideArgs wa{};
        wa.np = n; wa.n = n;
        wa.X_in = hist + (size_t)i * nn;
        wa.X_out = hist + (size_t)(i + 1) * nn;
        wa.A = nullptr;
        wa.a = theta[4 * i]; wa.b = theta[4 * i + 1]; wa.c = theta[4 * i + 2];
        wa.d_next = 0.0;      // the accumulator is formed from the history below
        wa.last = 0;
        FE_HIP(fe::launch_layer_f32(wa, s));
    }
    fe::MatTheta mt{};
    memcpy(mt.v, theta, sizeof(double) * 4 * L);
    FE_HIP(fe::launch_fwd_out(hist, n, L, mt, P, s));
    return FE_OK;
}

int fe_matrix_backward(const float* hist, int64_t n, const double* theta, int32_t L,
                       const float* G, float* work, double* part, int32_t nblocks,
                       double* grad, void* stream) {
    if (!hist || !G || !work || !part || !grad || !theta) return fail(FE_ERR_ARG, "bad arguments");
    if (n < 1 || n % fe::wide_tile() != 0) return fail(FE_ERR_ARG, "n must be a positive multiple of 64");
    if (L < 1 || L > fe::scalar_max_layers()) return fail(FE_ERR_ARG, "L out of range");
    if (nblocks < 1) return fail(FE_ERR_ARG, "nblocks must be >= 1");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t nn = (size_t)n * n;
    float* Xb = work;            // adjoint of X_{i+1}
    float* Xb2 = work + nn;      // adjoint of X_i
    float* M = work + 2 * nn;    // Xb_{i+1} X_i
    FE_HIP(hipMemcpyAsync(Xb, G, sizeof(float) * nn, hipMemcpyDeviceToDevice, s));
    for (int i = L - 1; i >= 0; --i) {
        const float* Xi = hist + (size_t)i * nn;
        fe::WideArgs wa{};
        wa.np = n; wa.n = n; wa.plain = 1;
        wa.X_in = Xb; wa.B_in = Xi; wa.X_out = M;
        FE_HIP(fe::launch_layer_f32(wa, s));
        fe::BwdArgs ba{};
        ba.M = M; ba.Xb = Xb; ba.X = Xi; ba.G = G; ba.Xb_out = Xb2;
        ba.ca = (float)theta[4 * i]; ba.cb = (float)theta[4 * i + 1]; ba.cd = (float)theta[4 * i + 3];
        ba.n = n; ba.part = part;
        FE_HIP(fe::launch_bwd_elem(ba, nblocks, grad + 4 * i, s));
        std::swap(Xb, Xb2);
    }
    return FE_OK;
}

}  // extern "C"
