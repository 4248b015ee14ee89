// Host side of the C ABI declared in include/fe.h: argument checks, the workspace, and the
// launch sequence of Alg. 2 (bounds -> rescale -> L layers -> traces) on the caller's stream.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "fe_internal.h"

namespace fe {
int small_f64_max_np();
}  // namespace fe

#include "fe_host.h"

using namespace fehost;

namespace {

constexpr int64_t kStreamKMinN = 1536;   // workspaces for n >= this carry stream-K buffers

// Schedule of the split-precision layer kernel (FE_SCHEDULE=dp|sk|sk2 overrides):
//  0 data-parallel, 128 x 128 tiles, one workgroup per upper tile;
//  1 stream-K over 256 x 256 tiles, one workgroup per CU;
//  2 stream-K over 128 x 128 tiles, two workgroups per CU (whole-tile rounds first when there
//    are two or more rounds).
// Order: a schedule forced by the tuner, FE_SCHEDULE, the tuned table (fe_autotune), then the
// default: 2 when every stream-K workgroup gets at least eight K-blocks (else the partial-tile
// traffic outweighs the balance: measured slower below N ~ 2000), otherwise 0. Only workspaces
// sized for n >= kStreamKMinN carry the stream-K buffers.
// Schedules chosen by fe_autotune: (device, precision, size) -> schedule, process-wide. A
// size uses the entry of the nearest tuned size within a factor sqrt(2).
struct TunedEntry {
    int device, prec;
    int64_t n;
    int schedule;
};
std::mutex g_tune_mu;
std::vector<TunedEntry> g_tuned;
// fe_debug_streamk_giveup: stream-K waits expect a flag value that is never written
std::atomic<int> g_sk_giveup{0};
// fe_debug_layer_events: HIP events around each layer launch of the split path (the last call's)
std::mutex g_ev_mu;
bool g_ev_on = false;
std::vector<hipEvent_t> g_ev;
int g_ev_used = 0;

// Event k of the layer timing pool (created on first use), or nullptr if timing is off.
hipEvent_t layer_event(int k) {
    std::lock_guard<std::mutex> lk(g_ev_mu);
    if (!g_ev_on) return nullptr;
    while ((int)g_ev.size() <= k) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        g_ev.push_back(e);
    }
    if (k + 1 > g_ev_used) g_ev_used = k + 1;
    return g_ev[k];
}
constexpr uint32_t kNeverEpoch = 0xFFFFFFFFu;   // no launch publishes this value
thread_local int t_forced_schedule = -1;   // set by the tuner around its timing runs

int tuned_schedule(int device, int prec, int64_t n) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    int best = -1;
    double dist = 0.5;   // |log2(n / n_tuned)|
    for (const TunedEntry& t : g_tuned) {
        if (t.device != device || t.prec != prec) continue;
        const double d = fabs(log2((double)n / (double)t.n));
        if (d <= dist) {
            dist = d;
            best = t.schedule;
        }
    }
    return best;
}

int use_streamk(int64_t n, const fe_workspace* ws, int prec) {
    if (!ws->sk_partial) return 0;
    if (t_forced_schedule >= 0) return t_forced_schedule;
    const char* env = getenv("FE_SCHEDULE");
    if (env && env[0] == 'd') return 0;
    if (env && env[0] == 's') return strcmp(env, "sk2") == 0 ? 2 : 1;
    const int tuned = tuned_schedule(ws->device, prec, n);
    if (tuned >= 0) return tuned;
    const int64_t np = round_up(n, 128), T = np / 128, ntiles = T * (T + 1) / 2, nk = np / 64;
    const int64_t grid = 2 * (int64_t)ws->n_cu;
    const int64_t rounds = ntiles / grid;
    const int64_t nsk = rounds >= 2 ? ntiles - (rounds - 1) * grid : ntiles;
    return nsk * nk >= 8 * grid ? 2 : 0;
}

// Slot carving for the precision modes (np x np elements each). three: the middle parts of the
// three-part BF16 split follow (20 B per element in all, within the slot's 24).
struct SplitBufs {
    float *X, *A;
    uint16_t *hi[2], *lo[2], *mid[2];
};
SplitBufs carve_split(void* base, int64_t np, bool three = false) {
    SplitBufs b;
    const size_t e = (size_t)np * np;
    b.X = static_cast<float*>(base);
    b.A = b.X + e;
    uint16_t* h = reinterpret_cast<uint16_t*>(b.A + e);
    b.hi[0] = h;
    b.hi[1] = h + e;
    b.lo[0] = h + 2 * e;
    b.lo[1] = h + 3 * e;
    b.mid[0] = three ? h + 4 * e : nullptr;
    b.mid[1] = three ? h + 5 * e : nullptr;
    return b;
}
struct WideBufs {
    void *X[2], *A;
};
WideBufs carve_wide(void* base, int64_t np, size_t elem) {
    WideBufs b;
    const size_t e = (size_t)np * np * elem;
    char* c = static_cast<char*>(base);
    b.X[0] = c;
    b.X[1] = c + e;
    b.A = c + 2 * e;
    return b;
}

// Runs Alg. 2 for one matrix on workspace slot `which`. alpha = 1 and entropy = 0 give the
// density; entropy = 1 gives S (no matrix output).
// noalloc: the caller cannot allocate (fe_expand_density_noalloc): the squared-affine form, whose
// tables live on the heap, is not used.
// final_correction (16-bit modes): the last layer is a correction layer, its product X^2 from the
// FP32 state by FP32 MFMA and its epilogue D = A + d X + (a X^2 + b X + c I) in FP64, written
// without rounding to FP32 when D is float64.
int run_expansion(const double* H, int64_t n, int64_t ldh, double mu, double kT, const fe_model* m,
                  int prec, double alpha, int entropy, void* D, int d_is_fp64, int64_t ldd,
                  double* trD, double* trD2, double* S, fe_rescale_info* info, fe_workspace* ws,
                  hipStream_t s, int which, bool noalloc = false,
                  bool final_correction = false) {
    int rc = check_common(H, n, ldh, mu, kT, ws);
    if (rc) return rc;
    rc = check_model(m, entropy ? "entropy model" : "model");
    if (rc) return rc;
    if (prec < FE_PREC_FP64 || prec > FE_PREC_BF16X3) return fail(FE_ERR_ARG, "unknown precision");
    if (noalloc && prec == FE_PREC_BF16X3)
        return fail(FE_ERR_ARG, "the entry point without allocation runs FP16x2, BF16x2, FP32 or FP64");
    if (!entropy && D && ldd < n) return fail(FE_ERR_ARG, "ldd < n");
    if (entropy && !(fabs(alpha) <= 1.0)) return fail(FE_ERR_ARG, "|alpha| must be <= 1");
    const bool split = prec == FE_PREC_FP16X2 || prec == FE_PREC_BF16X2 || prec == FE_PREC_BF16X3;
    const bool three = prec == FE_PREC_BF16X3;
    if (split && layer_range(m, alpha) > 16.0)
        return fail(FE_ERR_RANGE, "layer values exceed the 16-bit operand range");

    int out_mode = 2;
    if (!entropy && D) out_mode = d_is_fp64 ? 1 : 0;
    const double* th = m->theta;
    auto dval = [&](int i) {
        const double d = th[4 * i + 3];
        return (prec != FE_PREC_FP64 && fabs(d) < kDSkip) ? 0.0 : d;
    };

    fe::Params* P = ws->params + which;
    fe::BoundsPartial* bp = ws->bparts + (size_t)which * fe::kMaxBoundsBlocks;
    fe::TracePartial* tp = ws->tparts + (size_t)which * fe::kMaxTiles;
    FE_HIP(fe::launch_bounds_params(H, n, ldh, mu, kT, m->beta0, m->mu0, bp, P, s));

    int npart = 1;
    if (prec == FE_PREC_FP64 && round_up(n, 16) <= fe::small_f64_max_np()) {
        const int64_t np = round_up(n, 16);
        WideBufs b = carve_wide(ws->slot[which], np, sizeof(double));
        fe::RescaleArgs ra{};
        ra.H = H; ra.n = n; ra.ldh = ldh; ra.np = np; ra.P = P;
        ra.alpha = alpha; ra.mu0 = m->mu0; ra.d0 = 0.0;
        ra.X64 = static_cast<double*>(b.X[0]); ra.A64 = static_cast<double*>(b.A);
        ra.mode = 2;
        FE_HIP(fe::launch_rescale(ra, s));
        if (m->L > fe::kSmallMaxL) return fail(FE_ERR_ARG, "too many layers for the small FP64 path");
        fe::SmallArgs sa{};
        sa.n = n; sa.np = np; sa.X0 = static_cast<double*>(b.X[0]); sa.L = m->L;
        memcpy(sa.theta, th, sizeof(double) * 4 * m->L);
        sa.d0 = dval(0); sa.out_mode = out_mode; sa.entropy = entropy; sa.D = D; sa.ldd = ldd;
        sa.P = P; sa.partials = tp;
        FE_HIP(fe::launch_small_f64(sa, s));
    } else if (split) {
        fe::SplitPlan plan{};
        plan.streamk = three ? 0 : use_streamk(n, ws, prec);   // three parts: data-parallel
        plan.grid = plan.streamk == 2 ? 2 * ws->n_cu : ws->n_cu;
        plan.partial = ws->sk_partial;
        plan.own = ws->sk_partial ? ws->sk_partial + (size_t)ws->n_cu * 256 * 256 : nullptr;
        plan.flags = ws->sk_flags;
        plan.err = ws->sk_err;
        const int tile = fe::split_tile_for(plan.streamk);
        const int64_t np = round_up(n, tile);
        if (np > ws->np_cap) return fail(FE_ERR_WORKSPACE, "padded size exceeds the workspace");
        SplitBufs b = carve_split(ws->slot[which], np, three);
        const int bf = three ? 2 : prec == FE_PREC_BF16X2 ? 1 : 0;
        fe::RescaleArgs ra{};
        ra.H = H; ra.n = n; ra.ldh = ldh; ra.np = np; ra.P = P;
        ra.alpha = alpha; ra.mu0 = m->mu0; ra.d0 = dval(0);
        ra.X32 = b.X; ra.A32 = b.A; ra.hi = b.hi[0]; ra.lo = b.lo[0];
        ra.hi1 = b.hi[1]; ra.lo1 = b.lo[1];
        ra.mid = b.mid[0]; ra.mid1 = b.mid[1]; ra.three = three;
        ra.mode = 0; ra.bf16 = bf;
        // squared-affine layers on request (FE_FORM=affine, FP16x2, coefficients permitting);
        // BF16x2 always keeps the FP32 state (its 16-bit split would carry the state alone)
        const bool corr = final_correction;
        AffineForm af;
        if (!bf && !noalloc && !corr && affine_allowed()) af = affine_form(m, alpha, dval);
        ra.op_shift = af.ok ? af.op_shift : 0.0;
        FE_HIP(fe::launch_rescale(ra, s));
        const int T = (int)(np / tile);
        npart = T * (T + 1) / 2;
        if (npart > fe::kMaxTiles) return fail(FE_ERR_WORKSPACE, "too many tiles");
        float d_old[kMaxLayers], d_new[kMaxLayers];
        pair_accumulator_terms(m->L, dval, d_old, d_new);
        const int nsplit = corr ? m->L - 1 : m->L;   // layers on the 16-bit split
        if (hipEvent_t ev = layer_event(0)) {
            std::lock_guard<std::mutex> lk(g_ev_mu);
            g_ev_used = 1;
            FE_HIP(hipEventRecord(ev, s));
        }
        for (int i = 0; i < nsplit; ++i) {
            fe::LayerArgs la{};
            la.np = np; la.n = n;
            la.hi_in = b.hi[i & 1]; la.lo_in = b.lo[i & 1];
            la.hi_out = b.hi[(i + 1) & 1]; la.lo_out = b.lo[(i + 1) & 1];
            la.mid_in = b.mid[i & 1]; la.mid_out = b.mid[(i + 1) & 1];
            la.X = b.X; la.A = b.A;
            if (af.ok) {
                la.affine = 1;
                la.a = af.ca[i]; la.b = 0.0f; la.c = af.cc[i];
                la.d_old = 0.0f;
                la.d_new = af.dnew[i];
            } else {
                la.a = (float)th[4 * i]; la.b = (float)th[4 * i + 1]; la.c = (float)th[4 * i + 2];
                la.d_old = d_old[i];
                la.d_new = d_new[i];
            }
            la.last = (i + 1 == m->L);
            la.out_mode = out_mode; la.entropy = entropy; la.D = D; la.ldd = ldd;
            la.P = P; la.partials = tp;
            if (plan.streamk) {
                // flags start at 0, and kNeverEpoch is reserved: neither is ever published
                if (++ws->epoch == 0 || ws->epoch == kNeverEpoch) ws->epoch = 1;
                plan.epoch = ws->epoch;
                const bool giveup = g_sk_giveup.load() != 0;
                plan.wait_epoch = giveup ? kNeverEpoch : plan.epoch;
                plan.spin_limit = giveup ? 64 : (1 << 22);   // 1 << 22: ~0.2 s of sleeps
            }
            FE_HIP(fe::launch_layer_split(la, bf, plan, s));
            if (hipEvent_t ev = layer_event(i + 1)) FE_HIP(hipEventRecord(ev, s));
        }
        if (corr) {
            // the correction layer: the FP32 state X_{L-1} (upper triangle maintained by the
            // split layers) is mirrored to full, then one FP32 MFMA layer with the FP64 epilogue
            const int i = m->L - 1;
            FE_HIP(fe::launch_mirror_upper_f32(b.X, np, s));
            fe::WideArgs wa{};
            wa.np = np; wa.n = n;
            wa.X_in = b.X; wa.X_out = nullptr; wa.A = b.A;
            wa.a = th[4 * i]; wa.b = th[4 * i + 1]; wa.c = th[4 * i + 2]; wa.d_next = 0.0;
            wa.last = 1; wa.out_mode = out_mode; wa.entropy = entropy; wa.D = D; wa.ldd = ldd;
            wa.P = P; wa.partials = tp;
            wa.f64_epi = 1;
            wa.d_last = d_old[i];
            const int Tw = (int)(np / fe::wide_tile());
            npart = Tw * (Tw + 1) / 2;
            if (npart > fe::kMaxTiles) return fail(FE_ERR_WORKSPACE, "too many tiles");
            FE_HIP(fe::launch_layer_f32(wa, s));
        }
    } else {
        // FP64 beyond the one-workgroup size, or FP32: 64 x 64 tiled MFMA layers on X itself
        const bool f64 = prec == FE_PREC_FP64;
        const int tile = fe::wide_tile();
        const int64_t np = round_up(n, tile);
        if (np > ws->np_cap) return fail(FE_ERR_WORKSPACE, "padded size exceeds the workspace");
        WideBufs b = carve_wide(ws->slot[which], np, f64 ? sizeof(double) : sizeof(float));
        fe::RescaleArgs ra{};
        ra.H = H; ra.n = n; ra.ldh = ldh; ra.np = np; ra.P = P;
        ra.alpha = alpha; ra.mu0 = m->mu0; ra.d0 = dval(0);
        if (f64) {
            ra.X64 = static_cast<double*>(b.X[0]); ra.A64 = static_cast<double*>(b.A); ra.mode = 2;
        } else {
            ra.X32 = static_cast<float*>(b.X[0]); ra.A32 = static_cast<float*>(b.A); ra.mode = 1;
        }
        FE_HIP(fe::launch_rescale(ra, s));
        const int T = (int)(np / tile);
        npart = T * (T + 1) / 2;
        if (npart > fe::kMaxTiles) return fail(FE_ERR_WORKSPACE, "too many tiles");
        for (int i = 0; i < m->L; ++i) {
            fe::WideArgs wa{};
            wa.np = np; wa.n = n;
            wa.X_in = b.X[i & 1]; wa.X_out = b.X[(i + 1) & 1]; wa.A = b.A;
            wa.a = th[4 * i]; wa.b = th[4 * i + 1]; wa.c = th[4 * i + 2];
            wa.d_next = (i + 1 < m->L) ? dval(i + 1) : 0.0;
            wa.last = (i + 1 == m->L);
            wa.out_mode = out_mode; wa.entropy = entropy; wa.D = D; wa.ldd = ldd;
            wa.P = P; wa.partials = tp;
            FE_HIP(f64 ? fe::launch_layer_f64(wa, s) : fe::launch_layer_f32(wa, s));
        }
    }
    FE_HIP(fe::launch_reduce_partials(tp, npart, trD, trD2, S, P, ws->sk_err, s));
    if (info) return read_info(ws, which, s, info);
    return FE_OK;
}

}  // namespace

extern "C" {

const char* fe_last_error(void) { return last_error().c_str(); }

const char* fe_version(void) { return "fe-mi355x 0.1 (gfx950)"; }

int fe_workspace_create(int64_t max_n, int32_t max_batch, int64_t batch_elems, fe_workspace** out) {
    if (!out) return fail(FE_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (max_n < 1) return fail(FE_ERR_ARG, "max_n must be >= 1");
    if (max_batch < 0 || batch_elems < 0) return fail(FE_ERR_ARG, "negative batch capacity");
    fe_workspace* ws = new fe_workspace();
    FE_HIP(hipGetDevice(&ws->device));
    ws->max_n = max_n;
    ws->np_cap = round_up(max_n, 256);
    ws->slot_bytes = (size_t)ws->np_cap * ws->np_cap * 24;   // FP64 mode: 3 doubles per element
    hipError_t e = hipSuccess;
    for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipMalloc(&ws->slot[k], ws->slot_bytes);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&ws->params), 2 * sizeof(fe::Params));
    if (e == hipSuccess)
        e = hipMalloc(reinterpret_cast<void**>(&ws->bparts), 2 * fe::kMaxBoundsBlocks * sizeof(fe::BoundsPartial));
    if (e == hipSuccess)
        e = hipMalloc(reinterpret_cast<void**>(&ws->tparts), 2 * (size_t)fe::kMaxTiles * sizeof(fe::TracePartial));
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&ws->newton), 2 * sizeof(double));
    if (e == hipSuccess)
        e = hipMalloc(reinterpret_cast<void**>(&ws->dots), (fe::kMaxDotBlocks + 3) * sizeof(double));
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ws->n_cu, hipDeviceAttributeMultiprocessorCount, ws->device);
    if (e == hipSuccess && max_n >= kStreamKMinN) {
        e = hipMalloc(reinterpret_cast<void**>(&ws->sk_partial), 2 * (size_t)ws->n_cu * 256 * 256 * sizeof(float));
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&ws->sk_flags), 2 * (size_t)ws->n_cu * sizeof(uint32_t));
        if (e == hipSuccess) e = hipMemset(ws->sk_flags, 0, 2 * (size_t)ws->n_cu * sizeof(uint32_t));
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&ws->sk_err), sizeof(int));
        if (e == hipSuccess) e = hipMemset(ws->sk_err, 0, sizeof(int));
    }
    if (e == hipSuccess && max_batch > 0) {
        ws->max_batch = max_batch;
        ws->batch_elems = batch_elems;
        // tiles of either batch tile size (64: T(T+1)/2 with T = np / 64 <= np^2 / 4096 for
        // np >= 128, summed over the arena)
        ws->batch_tiles = batch_elems / 4096 + max_batch;
        e = hipMalloc(&ws->arena, (size_t)batch_elems * 16);
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&ws->bmats), (size_t)max_batch * sizeof(fe::BatchMat));
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&ws->bparams), (size_t)max_batch * sizeof(fe::Params));
        if (e == hipSuccess)
            e = hipMalloc(reinterpret_cast<void**>(&ws->btparts), (size_t)ws->batch_tiles * sizeof(fe::TracePartial));
    }
    if (e != hipSuccess) {
        fe_workspace_destroy(ws);
        return hip_fail(e, "hipMalloc (workspace)");
    }
    *out = ws;
    return FE_OK;
}

int fe_workspace_destroy(fe_workspace* ws) {
    if (!ws) return FE_OK;
    for (int k = 0; k < 2; ++k)
        if (ws->slot[k]) (void)hipFree(ws->slot[k]);
    if (ws->params) (void)hipFree(ws->params);
    if (ws->bparts) (void)hipFree(ws->bparts);
    if (ws->tparts) (void)hipFree(ws->tparts);
    if (ws->newton) (void)hipFree(ws->newton);
    if (ws->dots) (void)hipFree(ws->dots);
    if (ws->sk_partial) (void)hipFree(ws->sk_partial);
    if (ws->sk_flags) (void)hipFree(ws->sk_flags);
    if (ws->sk_err) (void)hipFree(ws->sk_err);
    if (ws->arena) (void)hipFree(ws->arena);
    if (ws->bmats) (void)hipFree(ws->bmats);
    if (ws->bparams) (void)hipFree(ws->bparams);
    if (ws->btparts) (void)hipFree(ws->btparts);
    delete ws;
    return FE_OK;
}

int fe_rescale(const double* H, int64_t n, int64_t ldh, double mu, double kT, const fe_model* m,
               float* X0, int64_t ldx, fe_rescale_info* info, fe_workspace* ws, void* stream) {
    int rc = check_common(H, n, ldh, mu, kT, ws);
    if (rc) return rc;
    rc = check_model(m, "model");
    if (rc) return rc;
    if (X0 && ldx < n) return fail(FE_ERR_ARG, "ldx < n");
    hipStream_t s = static_cast<hipStream_t>(stream);
    FE_HIP(fe::launch_bounds_params(H, n, ldh, mu, kT, m->beta0, m->mu0, ws->bparts, ws->params, s));
    if (X0) {
        const int64_t np = round_up(n, 16);
        WideBufs b = carve_wide(ws->slot[0], np, sizeof(float));
        fe::RescaleArgs ra{};
        ra.H = H; ra.n = n; ra.ldh = ldh; ra.np = np; ra.P = ws->params;
        ra.alpha = 1.0; ra.mu0 = m->mu0; ra.d0 = 0.0;
        ra.X32 = static_cast<float*>(b.X[0]); ra.A32 = static_cast<float*>(b.A);
        ra.mode = 1; ra.X0out = X0; ra.ldx = ldx;
        FE_HIP(fe::launch_rescale(ra, s));
    }
    if (info) return read_info(ws, 0, s, info);
    return FE_OK;
}

int fe_expand_density(const double* H, int64_t n, int64_t ldh, double mu, double kT,
                      const fe_model* m, int32_t prec, int32_t final_correction, void* D,
                      int32_t d_is_fp64, int64_t ldd, double* trD, double* trD2,
                      fe_rescale_info* info, fe_workspace* ws, void* stream) {
    if (final_correction != 0 && final_correction != 1)
        return fail(FE_ERR_ARG, "final_correction must be 0 or 1");
    const bool corr = final_correction &&
                      (prec == FE_PREC_FP16X2 || prec == FE_PREC_BF16X2 || prec == FE_PREC_BF16X3);
    return run_expansion(H, n, ldh, mu, kT, m, prec, 1.0, 0, D, d_is_fp64, ldd, trD, trD2, nullptr,
                         info, ws, static_cast<hipStream_t>(stream), 0, false, corr);
}

int fe_expand_density_filling(const double* H, int64_t n, int64_t ldh, double n_occ, double kT,
                              double mu_init, const fe_model* m, int32_t prec, double tol,
                              int32_t max_iter, void* D, int32_t d_is_fp64, int64_t ldd,
                              double* trD, double* trD2, double* mu_out, int32_t* iters_out,
                              fe_rescale_info* info, fe_workspace* ws, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!mu_out) return fail(FE_ERR_ARG, "mu_out is NULL");
    *mu_out = NAN;
    if (iters_out) *iters_out = 0;
    int rc = check_common(H, n, ldh, 0.0, kT, ws);
    if (rc) return rc;
    rc = check_model(m, "model");
    if (rc) return rc;
    if (!(n_occ > 0.0 && n_occ < (double)n)) return fail(FE_ERR_ARG, "n_occ must lie in (0, n)");
    if (!(tol > 0.0) || max_iter < 1) return fail(FE_ERR_ARG, "tol must be > 0 and max_iter >= 1");

    // Bracket: Tr D increases with mu, from ~0 below the Gershgorin interval to ~n above it.
    FE_HIP(fe::launch_bounds_params(H, n, ldh, 0.0, kT, m->beta0, m->mu0, ws->bparts, ws->params, s));
    FE_HIP(hipStreamSynchronize(s));
    fe::Params p;
    FE_HIP(hipMemcpy(&p, ws->params, sizeof(p), hipMemcpyDeviceToHost));
    if (p.status == FE_ERR_NONFINITE) return fail(FE_ERR_NONFINITE, "H holds a non-finite entry");
    double lo = p.emin, hi = p.emax;
    if (!(hi > lo)) {   // H = c I: any mu is admissible; bracket a window of temperatures
        lo = p.emin - 50.0 * kT;
        hi = p.emax + 50.0 * kT;
    }
    double mu = isfinite(mu_init) ? mu_init : 0.5 * (lo + hi);
    if (!(mu > lo && mu < hi)) return fail(FE_ERR_DOMAIN, "mu_init lies outside the Gershgorin bounds of H");

    // Newton on Tr D(mu) = n_occ with d Tr D / d mu = (Tr D - sum D_ij^2) / kT (Sec. IV.3), kept
    // inside the shrinking bracket: a step that leaves it, or a vanishing derivative (mu in a
    // gap at low temperature), is replaced by bisection.
    fe_rescale_info inf{};
    double t[2] = {0.0, 0.0};
    bool converged = false;
    for (int it = 1; it <= max_iter; ++it) {
        rc = run_expansion(H, n, ldh, mu, kT, m, prec, 1.0, 0, D, d_is_fp64, ldd, ws->newton,
                           ws->newton + 1, nullptr, &inf, ws, s, 0);
        if (rc < 0) return rc;
        FE_HIP(hipMemcpy(t, ws->newton, sizeof(t), hipMemcpyDeviceToHost));
        *mu_out = mu;
        if (iters_out) *iters_out = it;
        const double r = n_occ - t[0];
        if (fabs(r) <= tol) {
            converged = true;
            break;
        }
        if (r > 0.0) lo = mu;
        else hi = mu;
        const double deriv = (t[0] - t[1]) / kT;
        double next = deriv > 0.0 ? mu + r / deriv : NAN;
        if (!(next > lo && next < hi)) next = 0.5 * (lo + hi);
        mu = next;
    }
    if (trD) FE_HIP(hipMemcpyAsync(trD, ws->newton, sizeof(double), hipMemcpyDeviceToDevice, s));
    if (trD2) FE_HIP(hipMemcpyAsync(trD2, ws->newton + 1, sizeof(double), hipMemcpyDeviceToDevice, s));
    if (info) *info = inf;
    if (!converged) return fail(FE_ERR_NO_CONVERGENCE, "chemical potential not converged within max_iter");
    return rc;
}

int fe_model_select(const double* H, int64_t n, int64_t ldh, double mu, double kT,
                    const fe_model* bank, int32_t nbank, int32_t* index, fe_workspace* ws,
                    void* stream) {
    if (!index) return fail(FE_ERR_ARG, "index is NULL");
    if (!bank || nbank < 1) return fail(FE_ERR_ARG, "empty model bank");
    int rc = check_common(H, n, ldh, mu, kT, ws);
    if (rc) return rc;
    std::vector<const fe_model*> ms;
    for (int k = 0; k < nbank; ++k) {
        rc = check_model(&bank[k], "bank model");
        if (rc) return rc;
        ms.push_back(&bank[k]);
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    FE_HIP(fe::launch_bounds_params(H, n, ldh, mu, kT, bank[0].beta0, bank[0].mu0, ws->bparts,
                                    ws->params, s));
    FE_HIP(hipStreamSynchronize(s));
    fe::Params p;
    FE_HIP(hipMemcpy(&p, ws->params, sizeof(p), hipMemcpyDeviceToHost));
    if (p.status == FE_ERR_NONFINITE) return fail(FE_ERR_NONFINITE, "H holds a non-finite entry");
    *index = choose_bank_model(ms.data(), nbank, p.emin, p.emax, mu, kT);
    return FE_OK;
}

namespace {

// Times each schedule candidate on one expansion of H (1 warm-up + reps timed, HIP events on s),
// writes ms3[c] (NaN for candidates not run) and records the fastest for (device, prec, n).
int time_schedules(const double* H, int64_t n, int64_t ldh, double mu, double kT, const fe_model* m,
                   int32_t prec, int reps, double* ms3, int* best_out, fe_workspace* ws,
                   hipStream_t s) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    int rc = FE_OK;
    const int cands = ws->sk_partial ? 3 : 1;
    double best = 0.0;
    int best_s = -1;
    if (ms3)
        for (int c = 0; c < 3; ++c) ms3[c] = NAN;
    for (int c = 0; c < cands && e == hipSuccess && rc == FE_OK; ++c) {
        t_forced_schedule = c;
        float t = 0.0f;
        for (int rep = 0; rep <= reps && rc == FE_OK && e == hipSuccess; ++rep) {
            if (rep == 1) e = hipEventRecord(e0, s);   // the first run is a warm-up
            if (e == hipSuccess)
                rc = run_expansion(H, n, ldh, mu, kT, m, prec, 1.0, 0, nullptr, 0, n, nullptr,
                                   nullptr, nullptr, nullptr, ws, s, 0);
        }
        if (e == hipSuccess && rc == FE_OK) e = hipEventRecord(e1, s);
        if (e == hipSuccess && rc == FE_OK) e = hipEventSynchronize(e1);
        if (e == hipSuccess && rc == FE_OK) e = hipEventElapsedTime(&t, e0, e1);
        t_forced_schedule = -1;
        if (e != hipSuccess || rc != FE_OK) break;
        // a candidate whose stream-K waits gave up (status FE_ERR_HIP from the trace reduction)
        // produced no result: it is not timed and cannot be chosen
        fe::Params pc;
        e = hipMemcpy(&pc, ws->params, sizeof(pc), hipMemcpyDeviceToHost);
        if (e != hipSuccess) break;
        if (pc.status == FE_ERR_HIP) continue;
        const double per = t / reps;
        if (ms3) ms3[c] = per;
        if (best_s < 0 || per < best) {
            best = per;
            best_s = c;
        }
    }
    t_forced_schedule = -1;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(e, "autotune");
    if (rc != FE_OK) return rc;
    if (best_s < 0) return fail(FE_ERR_HIP, "autotune: no candidate schedule completed");
    if (best_out) *best_out = best_s;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (TunedEntry& t : g_tuned)
        if (t.device == ws->device && t.prec == prec && t.n == n) {
            t.schedule = best_s;
            return FE_OK;
        }
    g_tuned.push_back({ws->device, prec, n, best_s});
    return FE_OK;
}

}  // namespace

int fe_autotune_input(const double* H, int64_t n, int64_t ldh, double mu, double kT,
                      const fe_model* m, int32_t prec, int32_t* choice, double* ms,
                      fe_workspace* ws, void* stream) {
    if (prec != FE_PREC_FP16X2 && prec != FE_PREC_BF16X2)
        return fail(FE_ERR_ARG, "the tuner chooses among the 16-bit split schedules");
    int rc = check_common(H, n, ldh, mu, kT, ws);
    if (rc) return rc;
    rc = check_model(m, "model");
    if (rc) return rc;
    int best = 0;
    rc = time_schedules(H, n, ldh, mu, kT, m, prec, 2, ms, &best, ws,
                        static_cast<hipStream_t>(stream));
    if (rc == FE_OK && choice) *choice = best;
    return rc;
}

int fe_autotune(const int64_t* sizes, int32_t count, int32_t prec, int32_t* choice, double* ms,
                fe_workspace* ws, void* stream) {
    if (!sizes || count < 1) return fail(FE_ERR_ARG, "no sizes to tune");
    if (!ws) return fail(FE_ERR_ARG, "workspace is NULL");
    if (prec != FE_PREC_FP16X2 && prec != FE_PREC_BF16X2)
        return fail(FE_ERR_ARG, "the tuner chooses among the 16-bit split schedules");
    int64_t nmax = 0;
    for (int i = 0; i < count; ++i) {
        if (sizes[i] < 1) return fail(FE_ERR_ARG, "sizes must be >= 1");
        nmax = sizes[i] > nmax ? sizes[i] : nmax;
    }
    if (nmax > ws->max_n) return fail(FE_ERR_WORKSPACE, "a size exceeds the workspace's max_n");
    hipStream_t s = static_cast<hipStream_t>(stream);
    // the timing input: a random symmetric matrix and a short SP2 model with a small accumulator
    // weight on every layer, so that the accumulator is updated on every second layer as in the
    // trained models (those epilogues read and write A: they cost more than the others)
    double* H = nullptr;
    FE_HIP(hipMalloc(reinterpret_cast<void**>(&H), sizeof(double) * (size_t)nmax * nmax));
    std::vector<double> theta(4 * 6);
    fe_sp2_coeffs(0.5, 6, theta.data());
    for (int l = 0; l < 6; ++l) theta[4 * l + 3] = 1e-3;
    fe_model m{6, 100.0, 0.5, theta.data()};
    int rc = FE_OK;
    hipError_t e = hipSuccess;
    for (int i = 0; i < count && rc == FE_OK; ++i) {
        const int64_t n = sizes[i];
        e = fe::launch_fill_symmetric(H, n, 0x5eedULL + (uint64_t)n, s);
        if (e != hipSuccess) break;
        int best = 0;
        rc = time_schedules(H, n, n, 0.0, 0.1, &m, prec, 3, ms ? ms + 3 * i : nullptr, &best, ws, s);
        if (rc == FE_OK && choice) choice[i] = best;
    }
    (void)hipFree(H);
    if (e != hipSuccess) return hip_fail(e, "autotune");
    return rc;
}

int fe_autotune_lookup(int64_t n, int32_t prec, fe_workspace* ws, int32_t* schedule) {
    if (!ws || !schedule) return fail(FE_ERR_ARG, "workspace and schedule are required");
    if (n < 1) return fail(FE_ERR_ARG, "n must be >= 1");
    *schedule = use_streamk(n, ws, prec);
    return FE_OK;
}

int fe_autotune_clear(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned.clear();
    return FE_OK;
}

int fe_observable(const void* D, int32_t d_is_fp64, int64_t ldd, const double* A, int64_t lda,
                  int64_t n, double* out, fe_workspace* ws, void* stream) {
    if (!ws) return fail(FE_ERR_ARG, "workspace is NULL");
    if (!D || !A || !out) return fail(FE_ERR_ARG, "D, A and out must be non-NULL");
    if (n < 1 || ldd < n || lda < n) return fail(FE_ERR_ARG, "n < 1 or a leading dimension < n");
    FE_HIP(fe::launch_dot(D, d_is_fp64, ldd, A, lda, n, ws->dots, 0, 0.0, 0.0, nullptr, nullptr,
                          out, static_cast<hipStream_t>(stream)));
    return FE_OK;
}

int fe_free_energy(const double* H, int64_t n, int64_t ldh, double mu, double kT,
                   const fe_model* m, const fe_model* mS, double alpha, int32_t prec, void* D,
                   int32_t d_is_fp64, int64_t ldd, double* G, double* S, double* trD,
                   fe_rescale_info* info, fe_workspace* ws, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!G) return fail(FE_ERR_ARG, "G is NULL");
    int rc = check_common(H, n, ldh, mu, kT, ws);
    if (rc) return rc;
    double* dS = ws->dots + fe::kMaxDotBlocks;
    double* dtr = dS + 1;
    // entropy first on slot 1; afterwards that slot holds D when the caller passes none
    rc = run_expansion(H, n, ldh, mu, kT, mS ? mS : m, prec, alpha, 1, nullptr, 0, 0, nullptr,
                       nullptr, dS, nullptr, ws, s, 1);
    if (rc < 0) return rc;
    void* Dw = D;
    int64_t ldw = ldd;
    int w64 = d_is_fp64;
    if (!Dw) {
        Dw = ws->slot[1];
        ldw = n;
        w64 = 0;
    }
    rc = run_expansion(H, n, ldh, mu, kT, m, prec, 1.0, 0, Dw, w64, ldw, dtr, dtr + 1, nullptr,
                       info, ws, s, 0);
    if (rc < 0) return rc;
    FE_HIP(fe::launch_dot(Dw, w64, ldw, H, ldh, n, ws->dots, 1, mu, kT, dtr, dS, G, s));
    if (S) FE_HIP(hipMemcpyAsync(S, dS, sizeof(double), hipMemcpyDeviceToDevice, s));
    if (trD) FE_HIP(hipMemcpyAsync(trD, dtr, sizeof(double), hipMemcpyDeviceToDevice, s));
    return rc;
}

int fe_expand_entropy(const double* H, int64_t n, int64_t ldh, double mu, double kT,
                      const fe_model* mS, double alpha, int32_t prec, double* S,
                      fe_rescale_info* info, fe_workspace* ws, void* stream) {
    if (!S) return fail(FE_ERR_ARG, "S is NULL");
    return run_expansion(H, n, ldh, mu, kT, mS, prec, alpha, 1, nullptr, 0, 0, nullptr, nullptr, S,
                         info, ws, static_cast<hipStream_t>(stream), 1);
}

int fe_streamk_segments(int64_t np, int32_t schedule, int32_t grid, int32_t w, int32_t* geom,
                        int32_t* segs, int32_t cap, int32_t* count) {
    if (!geom || !count) return fail(FE_ERR_ARG, "geom and count are required");
    if (schedule != 1 && schedule != 2) return fail(FE_ERR_ARG, "schedule must be 1 or 2");
    const int tile = fe::split_tile_for(schedule);
    if (np < tile || np % tile != 0 || np > (int64_t)1 << 20)
        return fail(FE_ERR_ARG, "np must be a positive multiple of the schedule's tile");
    if (grid < 1) return fail(FE_ERR_ARG, "grid must be >= 1");
    if (segs && cap < 0) return fail(FE_ERR_ARG, "cap must be >= 0");
    const fe::SkGeometry G = fe::split_sk_geometry(np, schedule, grid);
    geom[0] = G.T; geom[1] = G.ntiles; geom[2] = G.nk; geom[3] = G.dp_tiles; geom[4] = G.groups;
    geom[5] = G.grid;
    *count = 0;
    if (w < 0 || w >= G.grid) return FE_OK;
    int k = 0;
    fe::sk_walk(G, w, [&](int pass, int t, int kb0, int kb1, int jlo) {
        if (segs && k < cap) {
            int32_t* q = segs + 5 * k;
            q[0] = pass; q[1] = t; q[2] = kb0; q[3] = kb1; q[4] = jlo;
        }
        ++k;
    });
    *count = k;
    return FE_OK;
}

int fe_debug_layer_events(int32_t enable) {
    std::lock_guard<std::mutex> lk(g_ev_mu);
    g_ev_on = enable != 0;
    g_ev_used = 0;
    return FE_OK;
}

int fe_debug_layer_events_read(double* ms, int32_t cap, int32_t* count) {
    if (!count) return fail(FE_ERR_ARG, "count is NULL");
    std::lock_guard<std::mutex> lk(g_ev_mu);
    *count = g_ev_used > 1 ? g_ev_used - 1 : 0;
    if (*count == 0 || !ms) return FE_OK;
    FE_HIP(hipEventSynchronize(g_ev[g_ev_used - 1]));
    for (int k = 0; k + 1 < g_ev_used && k < cap; ++k) {
        float t = 0.0f;
        FE_HIP(hipEventElapsedTime(&t, g_ev[k], g_ev[k + 1]));
        ms[k] = t;
    }
    return FE_OK;
}

int fe_debug_streamk_giveup(int32_t enable) {
    g_sk_giveup.store(enable ? 1 : 0);
    return FE_OK;
}

int fe_sp2_coeffs(double mu_p, int32_t L, double* theta_out) {
    if (!theta_out || L < 1) return fail(FE_ERR_ARG, "bad arguments");
    if (!(mu_p > 0.0 && mu_p < 1.0)) return fail(FE_ERR_DOMAIN, "mu' must lie in (0, 1)");
    double m = mu_p;
    for (int i = 0; i < L; ++i) {
        const double sq = m * m, up = 2.0 * m - m * m;
        double* t = theta_out + 4 * i;
        if (fabs(sq - mu_p) < fabs(up - mu_p)) {   // X^2 keeps the image of mu' closer
            t[0] = 1.0; t[1] = 0.0; t[2] = 0.0; t[3] = 0.0;
            m = sq;
        } else {                                   // 2X - X^2
            t[0] = -1.0; t[1] = 2.0; t[2] = 0.0; t[3] = 0.0;
            m = up;
        }
    }
    return FE_OK;
}

double fe_layer_count(double beta_p) {
    const double phi = 2.0 / (1.0 + sqrt(5.0));
    return log(beta_p / 4.0) / log(2.0 * phi);
}

}  // extern "C"

// ---- the entry point that allocates nothing --------------------------------------------------
//
// fe_expand_density_noalloc keeps what fe_expand_density keeps in a workspace (rescale parameters,
// Gershgorin and trace partials, and the padded matrices of one expansion) in `scratch`, a static
// device array of fixed size: the loader places one copy on every GPU the library runs on, held
// until the process ends. Host code never uses the array's name as an address: the device address
// of each GPU's copy comes from hipGetSymbolAddress on that GPU's first call and is kept per device.
// Every call on a GPU shares that copy; nothing in it must start at zero (every buffer is written
// before it is read within one call), and calls that overlap in time on one GPU race.

namespace {

constexpr size_t kNoAllocHeadBytes = (size_t)2 << 20;    // parameters and partials
constexpr size_t kNoAllocSlotBytes = (size_t)64 << 20;   // the padded matrices of one expansion
constexpr size_t kNoAllocParamsOff = 0;
constexpr size_t kNoAllocBoundsOff = 256;
constexpr size_t kNoAllocTracesOff =
    kNoAllocBoundsOff + ((fe::kMaxBoundsBlocks * sizeof(fe::BoundsPartial) + 255) / 256) * 256;
static_assert(2 * sizeof(fe::Params) <= kNoAllocBoundsOff, "parameter block");
static_assert(kNoAllocTracesOff + (size_t)fe::kMaxTiles * sizeof(fe::TracePartial) <= kNoAllocHeadBytes,
              "partials block");

}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocHeadBytes + kNoAllocSlotBytes];

namespace {

constexpr int kNoAllocMaxDevices = 64;
std::mutex g_noalloc_mu;
unsigned char* g_noalloc_ptr[kNoAllocMaxDevices] = {};

// Device address of this GPU's copy of `scratch` (the current device), looked up once per device.
int noalloc_scratch(int dev, unsigned char** out) {
    if (dev < 0 || dev >= kNoAllocMaxDevices) return fail(FE_ERR_ARG, "device index out of range");
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(FE_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_noalloc_ptr[dev] = static_cast<unsigned char*>(p);
    }
    *out = g_noalloc_ptr[dev];
    return FE_OK;
}

// Bytes of the padded matrices run_expansion carves from a slot for one density expansion of
// size n in precision prec on the data-parallel schedule.
size_t expansion_slot_bytes(int64_t n, int prec) {
    if (prec == FE_PREC_FP64 && round_up(n, 16) <= fe::small_f64_max_np()) {
        const size_t np = (size_t)round_up(n, 16);
        return 3 * np * np * sizeof(double);
    }
    if (prec == FE_PREC_FP16X2 || prec == FE_PREC_BF16X2) {
        const size_t np = (size_t)round_up(n, fe::split_tile_for(0));
        return 2 * np * np * sizeof(float) + 4 * np * np * sizeof(uint16_t);
    }
    const size_t np = (size_t)round_up(n, fe::wide_tile());
    return 3 * np * np * (prec == FE_PREC_FP64 ? sizeof(double) : sizeof(float));
}

}  // namespace

extern "C" int fe_expand_density_noalloc(const double* H, int64_t n, int64_t ldh, double mu,
                                         double kT, const fe_model* m, int32_t prec,
                                         int32_t final_correction, void* D, int32_t d_is_fp64,
                                         int64_t ldd, double* trD, double* trD2,
                                         fe_rescale_info* info, void* stream) {
    if (n < 1) return fail(FE_ERR_ARG, "n must be >= 1");
    if (final_correction != 0 && final_correction != 1)
        return fail(FE_ERR_ARG, "final_correction must be 0 or 1");
    if (prec < FE_PREC_FP64 || prec > FE_PREC_BF16X2) return fail(FE_ERR_ARG, "unknown precision");
    if (n > ((int64_t)1 << 16) || expansion_slot_bytes(n, prec) > kNoAllocSlotBytes)
        return fail(FE_ERR_WORKSPACE, "n exceeds the no-allocation scratch (64 MiB of matrices: "
                                      "n <= 2048 for FP16X2/BF16X2, 2304 for FP32, 1664 for FP64)");
    int dev = 0;
    FE_HIP(hipGetDevice(&dev));
    unsigned char* base = nullptr;
    int rc = noalloc_scratch(dev, &base);
    if (rc) return rc;
    // a workspace view of the static scratch: no stream-K buffers (data-parallel schedule), one slot
    fe_workspace w;
    w.device = dev;
    w.max_n = n;
    w.np_cap = (int64_t)1 << 40;   // the size check above replaces the slot-capacity check
    w.slot_bytes = kNoAllocSlotBytes;
    w.slot[0] = base + kNoAllocHeadBytes;
    w.params = reinterpret_cast<fe::Params*>(base + kNoAllocParamsOff);
    w.bparts = reinterpret_cast<fe::BoundsPartial*>(base + kNoAllocBoundsOff);
    w.tparts = reinterpret_cast<fe::TracePartial*>(base + kNoAllocTracesOff);
    const bool corr = final_correction && (prec == FE_PREC_FP16X2 || prec == FE_PREC_BF16X2);
    return run_expansion(H, n, ldh, mu, kT, m, prec, 1.0, 0, D, d_is_fp64, ldd, trD, trD2, nullptr,
                         info, &w, static_cast<hipStream_t>(stream), 0, true, corr);
}
