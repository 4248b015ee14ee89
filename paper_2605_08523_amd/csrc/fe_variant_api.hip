// C ABI of the Skip-SP2 and Max-SP2 expansions (Sec. III.A) and of the MLSP2 embeddings of
// App. C. The expansion shares the bounds, rescale and trace reduction with the MLSP2 path; per
// layer it runs one squaring (k_square) and one combine pass (k_combine), see k_variant.hip.
#include <math.h>
#include <string.h>

#include <vector>

#include "fe_host.h"
#include "fe_variant.h"

using namespace fehost;

namespace {

constexpr int64_t kVarTile = 128;   // the squaring's tile; the combine's 64 divides it

int variant_slots(const fe_qmodel* m) {
    return m->arch == FE_ARCH_MAX ? m->L + 1 : m->k + m->K;
}

// Workgroup slots of one data-parallel round of the squaring (two per CU) on the current device.
int square_slots() {
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return 2 * ncu;
}

// States, the hi/lo operand and the squaring's partial tiles (one round of slots at most).
int64_t variant_bytes(int64_t np, const fe_qmodel* m, int slots) {
    const int64_t e = np * np;
    return (int64_t)variant_slots(m) * e * (int64_t)sizeof(float) + 2 * e * (int64_t)sizeof(uint16_t) +
           (int64_t)slots * fe::kSquarePartTile * (int64_t)sizeof(float);
}

// Largest |operand| over the unit interval of the model coordinate (4097 points).
double variant_range(const fe_qmodel* m) {
    double zm = 0.0;
    for (int i = 0; i <= 4096; ++i) {
        double z = 0.0;
        (void)qmodel_value(m->arch, m->L, m->k, m->K, m->coef, i / 4096.0, &z);
        zm = fmax(zm, z);
    }
    return zm;
}

}  // namespace

extern "C" {

int fe_qmodel_coef_count(int32_t arch, int32_t L, int32_t k, int32_t K, int64_t* count) {
    if (!count) return fail(FE_ERR_ARG, "count is NULL");
    if (arch != FE_ARCH_MAX && arch != FE_ARCH_SKIP) return fail(FE_ERR_ARG, "unknown model family");
    if (L < 1 || (arch == FE_ARCH_SKIP && (k < 1 || K < 1))) return fail(FE_ERR_ARG, "bad shape");
    *count = qmodel_coef_count(arch, L, k, K);
    return FE_OK;
}

int fe_variant_scratch_bytes(int64_t n, const fe_qmodel* m, int64_t* bytes) {
    if (!bytes) return fail(FE_ERR_ARG, "bytes is NULL");
    if (n < 1) return fail(FE_ERR_ARG, "n must be >= 1");
    int rc = check_qmodel(m);
    if (rc) return rc;
    *bytes = variant_bytes(round_up(n, kVarTile), m, square_slots());
    return FE_OK;
}

int fe_expand_density_variant(const double* H, int64_t n, int64_t ldh, double mu, double kT,
                              const fe_qmodel* m, int32_t prec, void* scratch, int64_t scratch_bytes,
                              void* D, int32_t d_is_fp64, int64_t ldd, double* trD, double* trD2,
                              fe_rescale_info* info, fe_workspace* ws, void* stream) {
    int rc = check_common(H, n, ldh, mu, kT, ws);
    if (rc) return rc;
    rc = check_qmodel(m);
    if (rc) return rc;
    if (prec != FE_PREC_FP16X2 && prec != FE_PREC_BF16X2)
        return fail(FE_ERR_ARG, "the Skip-SP2 / Max-SP2 path runs the two-part 16-bit split modes only");
    if (D && ldd < n) return fail(FE_ERR_ARG, "ldd < n");
    const int64_t np = round_up(n, kVarTile);
    const int slots = square_slots();
    if (!scratch || scratch_bytes < variant_bytes(np, m, slots))
        return fail(FE_ERR_WORKSPACE, "scratch is smaller than fe_variant_scratch_bytes");
    if (fe::combine_tiles(np) > fe::kMaxTiles) return fail(FE_ERR_WORKSPACE, "too many tiles");
    if (variant_range(m) > 16.0) return fail(FE_ERR_RANGE, "operands exceed the 16-bit operand range");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int bf = prec == FE_PREC_BF16X2;
    const size_t e = (size_t)np * np;
    std::vector<float*> slot(variant_slots(m));
    for (size_t q = 0; q < slot.size(); ++q) slot[q] = static_cast<float*>(scratch) + q * e;
    uint16_t* hi = reinterpret_cast<uint16_t*>(static_cast<float*>(scratch) + slot.size() * e);
    uint16_t* lo = hi + e;
    float* parts = reinterpret_cast<float*>(lo + e);

    fe::Params* P = ws->params;
    FE_HIP(fe::launch_bounds_params(H, n, ldh, mu, kT, m->beta0, m->mu0, ws->bparts, P, s));
    // x_0 in FP32 (the rescale's accumulator output is pointed at the same slot with weight 1)
    float* x0 = slot[0];
    fe::RescaleArgs ra{};
    ra.H = H; ra.n = n; ra.ldh = ldh; ra.np = np; ra.P = P;
    ra.alpha = 1.0; ra.mu0 = m->mu0; ra.d0 = 1.0;
    ra.X32 = x0; ra.A32 = x0; ra.mode = 1; ra.bf16 = bf;
    FE_HIP(fe::launch_rescale(ra, s));

    const double* c = m->coef;
    const int L = m->L;
    auto base = [&]() {
        fe::CombineArgs a{};
        a.n = n; a.np = np; a.bf16 = bf; a.hi = hi; a.lo = lo; a.P = P;
        return a;
    };
    fe::CombineArgs fin = base();
    if (m->arch == FE_ARCH_MAX) {
        int off = 0;
        for (int i = 0; i < L; ++i) {
            fe::CombineArgs a = base();
            a.diag = (float)c[off];
            a.nterm = i + 1;
            for (int j = 0; j <= i; ++j) {
                a.term[j] = slot[j];
                a.w[j] = (float)c[off + 1 + j];
            }
            FE_HIP(fe::launch_combine(a, s));
            FE_HIP(fe::launch_square(hi, lo, np, slot[i + 1], bf, slots, parts, s));
            off += i + 2;
        }
        fin.diag = (float)c[off];
        fin.nterm = L + 1;
        for (int j = 0; j <= L; ++j) {
            fin.term[j] = slot[j];
            fin.w[j] = (float)c[off + 1 + j];
        }
    } else {
        const int k = m->k, K = m->K, per = 1 + k + 2 * K;
        const double* a0 = c + (size_t)per * L;
        float* const* ring = slot.data();            // x_i lives in ring[i % k]
        float* const* acc = slot.data() + k;         // A_{i,l} - a0_l I
        for (int i = 0; i < L; ++i) {
            const double* ci = c + (size_t)per * i;
            fe::CombineArgs a = base();
            double diag = ci[0];
            for (int l = 0; l < K; ++l) diag += ci[1 + k + l] * a0[l];
            a.diag = (float)diag;
            for (int j = 0; j < k && i - j >= 0; ++j) {
                a.term[a.nterm] = ring[(i - j) % k];
                a.w[a.nterm++] = (float)ci[1 + j];
            }
            if (i > 0)
                for (int l = 0; l < K; ++l) {
                    a.term[a.nterm] = acc[l];
                    a.w[a.nterm++] = (float)ci[1 + k + l];
                }
            a.nacc = K;
            for (int l = 0; l < K; ++l) {
                a.acc[l] = acc[l];
                a.g[l] = (float)ci[1 + k + K + l];
            }
            a.acc_src = ring[i % k];
            a.acc_first = i == 0;
            FE_HIP(fe::launch_combine(a, s));
            FE_HIP(fe::launch_square(hi, lo, np, ring[(i + 1) % k], bf, slots, parts, s));
        }
        double d = 0.0;
        for (int l = 0; l < K; ++l) d += a0[l];
        fin.diag = (float)d;
        fin.term[fin.nterm] = ring[L % k];
        fin.w[fin.nterm++] = (float)a0[K];
        for (int l = 0; l < K; ++l) {
            fin.term[fin.nterm] = acc[l];
            fin.w[fin.nterm++] = 1.0f;
        }
    }
    fin.out = 1;
    fin.D = D;
    fin.ldd = ldd;
    fin.out_mode = D ? (d_is_fp64 ? 1 : 0) : 2;
    fin.partials = ws->tparts;
    FE_HIP(fe::launch_combine(fin, s));
    FE_HIP(fe::launch_reduce_partials(ws->tparts, fe::combine_tiles(np), trD, trD2, nullptr, P,
                                      nullptr, s));
    if (info) return read_info(ws, 0, s, info);
    return FE_OK;
}

int fe_embed_mlsp2(const fe_model* src, int32_t arch, double* coef_out) {
    if (!coef_out) return fail(FE_ERR_ARG, "coef_out is NULL");
    int rc = check_model(src, "model");
    if (rc) return rc;
    if (arch != FE_ARCH_MAX && arch != FE_ARCH_SKIP) return fail(FE_ERR_ARG, "unknown model family");
    const int L = src->L;
    const double* th = src->theta;
    for (int i = 0; i < L; ++i)
        if (th[4 * i] == 0.0) return fail(FE_ERR_ARG, "a layer with a = 0 has no squared-affine form");
    // Per layer of the squared form: operand weight on x~_i, constant, accumulator weight on x~_i.
    // x~_{i+1} = (x_i + b_i/(2a_i))^2 and x_i = a_{i-1} x~_i + e_{i-1}, e_i = c_i - b_i^2/(4a_i);
    // the output A + x_L = const + sum_i d_i a_{i-1} x~_i (d_0 x~_0) + a_{L-1} x~_L.
    std::vector<double> w(L), k0(L), g(L);
    auto ev = [&](int i) { return th[4 * i + 2] - th[4 * i + 1] * th[4 * i + 1] / (4.0 * th[4 * i]); };
    double cst = ev(L - 1);
    for (int i = 0; i < L; ++i) {
        const double shift = th[4 * i + 1] / (2.0 * th[4 * i]);
        w[i] = i == 0 ? 1.0 : th[4 * (i - 1)];
        k0[i] = i == 0 ? shift : ev(i - 1) + shift;
        g[i] = i == 0 ? th[3] : th[4 * i + 3] * th[4 * (i - 1)];
        if (i > 0) cst += th[4 * i + 3] * ev(i - 1);
    }
    const double omega = th[4 * (L - 1)];
    if (arch == FE_ARCH_SKIP) {
        for (int i = 0; i < L; ++i) {
            double* o = coef_out + 4 * i;   // alpha_c, alpha_0, beta_1, gamma_1
            o[0] = k0[i];
            o[1] = w[i];
            o[2] = 0.0;
            o[3] = g[i];
        }
        coef_out[4 * L] = cst;
        coef_out[4 * L + 1] = omega;
        return FE_OK;
    }
    int off = 0;
    for (int i = 0; i < L; ++i) {
        coef_out[off] = k0[i];
        for (int j = 0; j <= i; ++j) coef_out[off + 1 + j] = j == i ? w[i] : 0.0;
        off += i + 2;
    }
    coef_out[off] = cst;
    for (int j = 0; j < L; ++j) coef_out[off + 1 + j] = g[j];
    coef_out[off + 1 + L] = omega;
    return FE_OK;
}

int fe_variant_eval(const double* y, int32_t n, const fe_qmodel* m, const double* coef,
                    const double* tgt, double* r, double* JT, void* stream) {
    if (!y || !r || !m || !coef || n < 1) return fail(FE_ERR_ARG, "bad arguments");
    if (m->arch != FE_ARCH_MAX && m->arch != FE_ARCH_SKIP) return fail(FE_ERR_ARG, "unknown model family");
    if (m->L < 1 || m->L > fe::kVariantMaxL) return fail(FE_ERR_ARG, "layer count out of range (1..64)");
    if (m->arch == FE_ARCH_SKIP && (m->k < 1 || m->k > fe::kVariantMaxK || m->K < 1 || m->K > fe::kVariantMaxK))
        return fail(FE_ERR_ARG, "Skip-SP2 needs 1 <= k <= 4 and 1 <= K <= 4");
    fe::VariantEvalArgs a{};
    a.y = y; a.tgt = tgt; a.r = r; a.JT = JT; a.coef = coef; a.n = n;
    a.arch = m->arch; a.L = m->L; a.k = m->k; a.K = m->K;
    FE_HIP(fe::launch_variant_eval(a, static_cast<hipStream_t>(stream)));
    return FE_OK;
}

}  // extern "C"
