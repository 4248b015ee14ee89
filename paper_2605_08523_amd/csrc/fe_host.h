// Host-side state and helpers shared by the C ABI translation units.
#pragma once

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <string>
#include <vector>

#include "fe_internal.h"

struct fe_workspace {
    int device = 0;
    int64_t max_n = 0;
    int64_t np_cap = 0;           // largest padded size a single-matrix call may use
    size_t slot_bytes = 0;
    void* slot[2] = {nullptr, nullptr};           // 0: density, 1: entropy
    fe::Params* params = nullptr;                 // [2]
    fe::BoundsPartial* bparts = nullptr;          // [2][kMaxBoundsBlocks]
    fe::TracePartial* tparts = nullptr;           // [2][kMaxTiles]
    int n_cu = 0;                                 // compute units of the device
    float* sk_partial = nullptr;                  // stream-K partial tiles [2][n_cu][256*256]
    uint32_t* sk_flags = nullptr;                 // stream-K flags [n_cu]
    int* sk_err = nullptr;                        // stream-K wait failure flag
    uint32_t epoch = 0;                           // last stream-K launch epoch
    double* newton = nullptr;                     // [2] traces of the current chemical-potential iterate
    double* dots = nullptr;                       // [kMaxDotBlocks + 3] Frobenius-product partials, S, trD
    // batch capacity
    int32_t max_batch = 0;
    int64_t batch_elems = 0;                      // sum of padded sizes squared it can hold
    int64_t batch_tiles = 0;                      // tile-trace slots
    void* arena = nullptr;                        // 16 bytes per element (X, A, hi[2], lo[2])
    fe::BatchMat* bmats = nullptr;                // [max_batch]
    fe::Params* bparams = nullptr;                // [max_batch]
    fe::TracePartial* btparts = nullptr;          // [batch_tiles]
    uint64_t batch_gen = 0;                       // bumped by every batch plan created
};

namespace fehost {

// Message of the last error on this thread (one instance for the whole library).
inline std::string& last_error() {
    thread_local std::string msg = "no error";
    return msg;
}

inline int fail(int code, const std::string& msg) {
    last_error() = msg;
    return code;
}

inline int hip_fail(hipError_t e, const char* what) {
    return fail(FE_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define FE_HIP(call)                                         \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return hip_fail(e_, #call);    \
    } while (0)

inline constexpr int kMaxLayers = 4096;
inline constexpr double kDSkip = 1e-8;   // accumulator weights below this are skipped (Sec. V.A)

// Model-bank rule: the bank model with the fewest layers whose region of validity (Eq.
// conditions: beta' <= beta0 min(mu0/mu', (1 - mu0)/(1 - mu'))) holds an input with Gershgorin
// bounds [lo, hi], chemical potential mu and temperature kT (ties: the larger beta0); if none,
// the model with the widest region (the input is then clamped). Degenerate or unusable bounds
// (the expansion reports those) take the fewest layers.
inline int choose_bank_model(const fe_model* const* ms, int nbank, double lo, double hi, double mu,
                             double kT) {
    const double width = hi - lo;
    const bool usable = isfinite(lo) && isfinite(hi) && kT > 0.0;
    const bool degenerate = usable && !(width > 1e-300 * fmax(1.0, fabs(hi)));
    double mu_p = 0.5, beta_p = 0.0;
    if (usable && !degenerate) {
        mu_p = (hi - mu) / width;
        if (mu_p > 0.5) mu_p = 1.0 - mu_p;
        beta_p = width / kT;
    }
    int best = -1, widest = 0;
    double widest_b = -1.0;
    for (int k = 0; k < nbank; ++k) {
        const fe_model* m = ms[k];
        const double bmax = (mu_p > 0.0 && mu_p <= 0.5)
                                ? fmin(m->mu0 / mu_p, (1.0 - m->mu0) / (1.0 - mu_p)) * m->beta0
                                : 0.0;
        if (bmax > widest_b) {
            widest_b = bmax;
            widest = k;
        }
        const bool fits = !usable || degenerate || beta_p <= bmax;
        if (fits && (best < 0 || m->L < ms[best]->L ||
                     (m->L == ms[best]->L && m->beta0 > ms[best]->beta0)))
            best = k;
    }
    return best >= 0 ? best : widest;
}

// Argument checks shared by the single-matrix entry points.
inline int check_common(const double* H, int64_t n, int64_t ldh, double mu, double kT, fe_workspace* ws) {
    if (!ws) return fail(FE_ERR_ARG, "workspace is NULL");
    if (!H) return fail(FE_ERR_ARG, "H is NULL");
    if (n < 1) return fail(FE_ERR_ARG, "n must be >= 1");
    if (ldh < n) return fail(FE_ERR_ARG, "ldh < n");
    if (!(kT > 0.0) || !isfinite(kT)) return fail(FE_ERR_DOMAIN, "kT must be positive and finite");
    if (!isfinite(mu)) return fail(FE_ERR_DOMAIN, "mu must be finite");
    if (n > ws->max_n) return fail(FE_ERR_WORKSPACE, "n exceeds the workspace's max_n");
    return FE_OK;
}

// Waits for the stream, copies the rescale parameters of workspace slot `which` into *info and
// returns their status (a stream-K wait that gave up is reported by the trace reduction as
// FE_ERR_HIP).
inline int read_info(fe_workspace* ws, int which, hipStream_t s, fe_rescale_info* info) {
    FE_HIP(hipStreamSynchronize(s));
    fe::Params p;
    FE_HIP(hipMemcpy(&p, ws->params + which, sizeof(p), hipMemcpyDeviceToHost));
    info->emin = p.emin;
    info->emax = p.emax;
    info->mu_p = p.mu_p;
    info->beta_p = p.beta_p;
    info->beta_max = p.beta_max;
    info->scale = p.scale;
    info->shift = p.shift;
    info->flipped = p.flipped;
    info->clamped = p.clamped;
    info->degenerate = p.degenerate;
    info->status = p.status;
    if (p.status == FE_ERR_DOMAIN) return fail(FE_ERR_DOMAIN, "mu lies outside the Gershgorin bounds of H");
    if (p.status == FE_ERR_NONFINITE) return fail(FE_ERR_NONFINITE, "H holds a non-finite entry");
    if (p.status == FE_ERR_HIP)
        return fail(FE_ERR_HIP, "a stream-K workgroup gave up waiting for a partial tile (the "
                                "affected outputs are NaN)");
    return p.status;
}

// ---- Skip-SP2 / Max-SP2 models (coefficient layout of fe_qmodel) ----

inline int64_t qmodel_coef_count(int arch, int L, int k, int K) {
    if (arch == FE_ARCH_MAX) return (int64_t)L * (L + 3) / 2 + L + 2;
    return (int64_t)(1 + k + 2 * K) * L + K + 1;
}

inline int check_qmodel(const fe_qmodel* m) {
    if (!m || !m->coef) return fail(FE_ERR_ARG, "model or its coefficients are NULL");
    if (m->arch != FE_ARCH_MAX && m->arch != FE_ARCH_SKIP) return fail(FE_ERR_ARG, "unknown model family");
    if (m->L < 1 || m->L > 64) return fail(FE_ERR_ARG, "layer count out of range (1..64)");
    if (m->arch == FE_ARCH_SKIP && (m->k < 1 || m->k > 4 || m->K < 1 || m->K > 4))
        return fail(FE_ERR_ARG, "Skip-SP2 needs 1 <= k <= 4 and 1 <= K <= 4");
    if (!(m->beta0 > 0.0) || !(m->mu0 > 0.0 && m->mu0 < 1.0)) return fail(FE_ERR_ARG, "bad (beta0, mu0)");
    const int64_t P = qmodel_coef_count(m->arch, m->L, m->k, m->K);
    for (int64_t p = 0; p < P; ++p)
        if (!isfinite(m->coef[p])) return fail(FE_ERR_ARG, "non-finite coefficient");
    return FE_OK;
}

// Scalar model value at y in FP64; *zmax (if not null) receives the largest |operand| met.
inline double qmodel_value(int arch, int L, int k, int K, const double* c, double y, double* zmax) {
    std::vector<double> x(L + 1);
    x[0] = y;
    double zm = 0.0, f;
    if (arch == FE_ARCH_MAX) {
        int off = 0;
        for (int i = 0; i < L; ++i) {
            double z = c[off];
            for (int j = 0; j <= i; ++j) z += c[off + 1 + j] * x[j];
            zm = fmax(zm, fabs(z));
            x[i + 1] = z * z;
            off += i + 2;
        }
        f = c[off];
        for (int j = 0; j <= L; ++j) f += c[off + 1 + j] * x[j];
    } else {
        const int per = 1 + k + 2 * K;
        std::vector<double> A(c + (size_t)per * L, c + (size_t)per * L + K);
        for (int i = 0; i < L; ++i) {
            const double* ci = c + (size_t)per * i;
            double z = ci[0];
            for (int j = 0; j < k; ++j)
                if (i - j >= 0) z += ci[1 + j] * x[i - j];
            for (int l = 0; l < K; ++l) z += ci[1 + k + l] * A[l];
            for (int l = 0; l < K; ++l) A[l] += ci[1 + k + K + l] * x[i];
            zm = fmax(zm, fabs(z));
            x[i + 1] = z * z;
        }
        f = c[(size_t)per * L + K] * x[L];
        for (int l = 0; l < K; ++l) f += A[l];
    }
    if (zmax) *zmax = zm;
    return f;
}

// Squared-affine form of the layers for the 16-bit kernels (Eq. mlsp2 rewritten as in App. C).
// With s_i = b_i/(2a_i) and e_i = c_i - a_i s_i^2, layer i maps x to a_i (x + s_i)^2 + e_i, so
// its operand is Z_i = x_i + s_i and its epilogue forms the next operand from Y = Z_i^2 alone:
// Z_{i+1} = a_i Y + (e_i + s_{i+1}) I. The accumulator term d_{i+1} x_{i+1} = d_{i+1} Z_{i+1}
// - d_{i+1} s_{i+1} I is added as d_{i+1} Z_{i+1}, the constants being folded into the last
// layer: D = A + a_{L-1} Y + (e_{L-1} - sum_{i>=1} d_i s_i) I. No FP32 copy of the state is read
// or written, so the state is carried by the hi/lo split alone: 22 significant bits with FP16
// (used), 16 with BF16 (measured 2.3e-5 against the 1e-5 bar on a dense N = 128 matrix; BF16x2
// keeps the direct form). Not used (ok = false) when some |a_i| < 1e-6 or an operand would leave
// [-16, 16] on the unit interval; the epilogue weights (ca, cc, d_new per layer) and the
// rescale's operand shift s_0 are returned otherwise. dv(i) is the accumulator weight after the
// skip rule.
// The direct form is the default; FE_FORM=affine selects the squared-affine form (FP16x2). The
// affine state lives in the 22-bit split alone: 2x the direct form's error on the headline
// lattice and the batch, but 30x (5.4e-6 against 1.8e-7) on a dense random N = 8192 matrix, whose
// rescaled off-diagonal entries (~3e-5) sit below the FP16 normal range.
inline bool affine_allowed() {
    const char* f = getenv("FE_FORM");
    return f && strcmp(f, "affine") == 0;
}

struct AffineForm {
    bool ok = false;
    double op_shift = 0.0;
    std::vector<float> ca, cc, dnew;
};
template <class DV>
inline AffineForm affine_form(const fe_model* m, double alpha, DV dv) {
    AffineForm f;
    const int L = m->L;
    const double* th = m->theta;
    for (int i = 0; i < L; ++i)
        if (!(fabs(th[4 * i]) >= 1e-6)) return f;
    std::vector<double> s(L), e(L);
    for (int i = 0; i < L; ++i) {
        s[i] = th[4 * i + 1] / (2.0 * th[4 * i]);
        e[i] = th[4 * i + 2] - th[4 * i] * s[i] * s[i];
    }
    double zmax = 0.0;
    const int kPts = 1025;
    for (int k = 0; k < kPts; ++k) {
        double x = alpha * ((double)k / (kPts - 1) - m->mu0) + m->mu0;
        for (int i = 0; i < L; ++i) {
            const double z = x + s[i];
            zmax = fmax(zmax, fabs(z));
            x = th[4 * i] * z * z + e[i];
        }
    }
    if (!(zmax <= 16.0)) return f;
    double fold = 0.0;
    for (int i = 1; i < L; ++i) fold -= dv(i) * s[i];
    f.ca.resize(L);
    f.cc.resize(L);
    f.dnew.resize(L);
    for (int i = 0; i < L; ++i) {
        f.ca[i] = (float)th[4 * i];
        const bool last = i + 1 == L;
        f.cc[i] = (float)(last ? e[i] + fold : e[i] + s[i + 1]);
        f.dnew[i] = last ? 0.0f : (float)dv(i + 1);
    }
    f.op_shift = s[0];
    f.ok = true;
    return f;
}

// Accumulator schedule of the 16-bit layer kernels in the direct form (the default; the
// squared-affine form adds one term per layer). The recursion adds d_j X_j
// for j = 1 .. L-1 (d_0 X_0 is formed by the rescale; X_L is the output). Layer i's epilogue sees
// X_i (its input) and X_{i+1} (its output), so each term can be added by one of two layers; terms
// are paired, A += d_j X_j + d_{j+1} X_{j+1} at layer j, which halves the layers that read and
// write A.
// dv(j) is d_j after the skip rule; d_old[i], d_new[i] are layer i's weights of X_i, X_{i+1}.
template <class DV>
inline void pair_accumulator_terms(int L, DV dv, float* d_old, float* d_new) {
    for (int i = 0; i < L; ++i) d_old[i] = d_new[i] = 0.0f;
    for (int j = 1; j < L;) {
        if (dv(j) == 0.0) {
            ++j;
            continue;
        }
        d_old[j] = (float)dv(j);
        if (j + 1 < L) d_new[j] = (float)dv(j + 1);
        j += 2;
    }
}
template <class DV>
inline void pair_accumulator_terms(int L, DV dv, std::vector<float>& d_old, std::vector<float>& d_new) {
    d_old.assign(L, 0.0f);
    d_new.assign(L, 0.0f);
    pair_accumulator_terms(L, dv, d_old.data(), d_new.data());
}

inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

inline int check_model(const fe_model* m, const char* name) {
    if (!m) return fail(FE_ERR_ARG, std::string(name) + " is NULL");
    if (m->L < 1 || m->L > kMaxLayers) return fail(FE_ERR_ARG, std::string(name) + ": L out of range");
    if (!m->theta) return fail(FE_ERR_ARG, std::string(name) + ": theta is NULL");
    if (!(m->beta0 > 0.0) || !isfinite(m->beta0))
        return fail(FE_ERR_ARG, std::string(name) + ": beta0 must be positive");
    if (!(m->mu0 > 0.0 && m->mu0 < 1.0)) return fail(FE_ERR_ARG, std::string(name) + ": mu0 must lie in (0, 1)");
    for (int i = 0; i < 4 * m->L; ++i)
        if (!isfinite(m->theta[i])) return fail(FE_ERR_ARG, std::string(name) + ": non-finite coefficient");
    return FE_OK;
}

// Largest |x_i| over the layers for model inputs in [0, 1] (after the entropy rescale when
// alpha != 1): the 16-bit operands must stay well inside the FP16 range (hi is scaled by 2^11
// inside the product).
inline double layer_range(const fe_model* m, double alpha) {
    double mx = 0.0;
    const int kPts = 1025;
    for (int k = 0; k < kPts; ++k) {
        double y = (double)k / (kPts - 1);
        double x = alpha * (y - m->mu0) + m->mu0;
        mx = fmax(mx, fabs(x));
        for (int i = 0; i < m->L; ++i) {
            const double* t = m->theta + 4 * i;
            x = t[0] * x * x + t[1] * x + t[2];
            mx = fmax(mx, fabs(x));
        }
    }
    return mx;
}


}  // namespace fehost
