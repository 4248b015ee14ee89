// Host side of the batched expansion: a plan lays the batch out in the workspace arena
// (matrices sorted by decreasing padded size), uploads the per-matrix descriptors once and
// captures the whole launch sequence (bounds, rescale, L grouped layers, reductions, and the
// entropy pass when an entropy model is given) into one hipGraph that each launch replays.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "fe_host.h"

using namespace fehost;

struct fe_batch_plan {
    uint64_t gen = 0;       // workspace layout generation this plan was built for
    int count = 0;
    int total_tiles = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    fe_workspace* ws = nullptr;
};

namespace {

int check_item(const fe_batch_item& it, int i) {
    if (!it.H) return fail(FE_ERR_ARG, "batch item " + std::to_string(i) + ": H is NULL");
    if (it.n < 1) return fail(FE_ERR_ARG, "batch item " + std::to_string(i) + ": n < 1");
    if (it.ldh < it.n) return fail(FE_ERR_ARG, "batch item " + std::to_string(i) + ": ldh < n");
    if (it.D && it.ldd < it.n) return fail(FE_ERR_ARG, "batch item " + std::to_string(i) + ": ldd < n");
    return FE_OK;
}

// Enqueues one expansion pass (density or entropy) of the whole batch on `s`.
int enqueue_pass(fe_workspace* ws, int count, int total_tiles, int64_t max_np, const fe_model* m,
                 double alpha, int entropy, int bf, int prec, int32_t* status, hipStream_t s) {
    const double* th = m->theta;
    auto dval = [&](int i) {
        const double d = th[4 * i + 3];
        return (prec != FE_PREC_FP64 && fabs(d) < kDSkip) ? 0.0 : d;
    };
    if (!entropy) FE_HIP(fe::launch_batch_bounds(ws->bmats, count, m->beta0, m->mu0, ws->bparams, s));
    FE_HIP(fe::launch_batch_rescale(ws->bmats, count, max_np, ws->bparams, alpha, m->mu0, dval(0), bf, s));
    std::vector<float> d_old, d_new;
    pair_accumulator_terms(m->L, dval, d_old, d_new);
    for (int i = 0; i < m->L; ++i) {
        fe::BatchLayerArgs q{};
        q.mats = ws->bmats;
        q.count = count;
        q.parity = i & 1;
        q.a = (float)th[4 * i];
        q.b = (float)th[4 * i + 1];
        q.c = (float)th[4 * i + 2];
        q.d_old = d_old[i];
        q.d_new = d_new[i];
        q.last = (i + 1 == m->L);
        q.entropy = entropy;
        q.P = ws->bparams;
        q.partials = ws->btparts;
        FE_HIP(fe::launch_batch_layer(q, total_tiles, bf, s));
    }
    FE_HIP(fe::launch_batch_reduce(ws->bmats, count, ws->btparts, ws->bparams, entropy, status, s));
    return FE_OK;
}

}  // namespace

extern "C" {

int fe_batch_plan_create(const fe_batch_item* items, int32_t count, const fe_model* m,
                         const fe_model* mS, double alpha, int32_t prec, int32_t* status,
                         fe_workspace* ws, fe_batch_plan** out) {
    if (!out) return fail(FE_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!ws) return fail(FE_ERR_ARG, "workspace is NULL");
    if (!items || count < 1) return fail(FE_ERR_ARG, "empty batch");
    if (count > ws->max_batch) return fail(FE_ERR_WORKSPACE, "batch larger than the workspace's max_batch");
    int rc = check_model(m, "model");
    if (rc) return rc;
    if (prec != FE_PREC_FP16X2 && prec != FE_PREC_BF16X2)
        return fail(FE_ERR_ARG, "batched expansion supports the FP16x2 and BF16x2 modes");
    if (layer_range(m, 1.0) > 16.0) return fail(FE_ERR_RANGE, "layer values exceed the 16-bit operand range");
    if (mS) {
        rc = check_model(mS, "entropy model");
        if (rc) return rc;
        if (mS->beta0 != m->beta0 || mS->mu0 != m->mu0)
            return fail(FE_ERR_ARG, "the entropy model must share (beta0, mu0) with the density model");
        if (!(fabs(alpha) <= 1.0)) return fail(FE_ERR_ARG, "|alpha| must be <= 1");
        if (layer_range(mS, alpha) > 16.0)
            return fail(FE_ERR_RANGE, "entropy layer values exceed the 16-bit operand range");
    }
    for (int i = 0; i < count; ++i) {
        rc = check_item(items[i], i);
        if (rc) return rc;
    }
    const int64_t bt = fe::batch_tile();
    std::vector<int> order(count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return items[a].n > items[b].n; });
    std::vector<fe::BatchMat> mats(count);
    int64_t elems = 0, tiles = 0, max_np = 0;
    for (int k = 0; k < count; ++k) {
        const fe_batch_item& it = items[order[k]];
        const int64_t np = round_up(it.n, bt);
        const int64_t T = np / bt;
        elems += np * np;
        tiles += T * (T + 1) / 2;
        max_np = std::max(max_np, np);
    }
    if (elems > ws->batch_elems) return fail(FE_ERR_WORKSPACE, "batch exceeds the workspace arena");
    if (tiles > ws->batch_tiles || tiles > (int64_t)0x7fffffff)
        return fail(FE_ERR_WORKSPACE, "batch has too many tiles for the workspace");
    char* arena = static_cast<char*>(ws->arena);
    int64_t off = 0, t0 = 0;
    for (int k = 0; k < count; ++k) {
        const fe_batch_item& it = items[order[k]];
        fe::BatchMat& bm = mats[k];
        memset(&bm, 0, sizeof(bm));
        const int64_t np = round_up(it.n, bt);
        const size_t e = (size_t)np * np;
        bm.H = it.H;
        bm.n = it.n;
        bm.ldh = it.ldh;
        bm.np = np;
        bm.mu = it.mu;
        bm.kT = it.kT;
        bm.X = reinterpret_cast<float*>(arena + off * 16);
        bm.A = bm.X + e;
        uint16_t* h = reinterpret_cast<uint16_t*>(bm.A + e);
        bm.hi[0] = h;
        bm.hi[1] = h + e;
        bm.lo[0] = h + 2 * e;
        bm.lo[1] = h + 3 * e;
        bm.D = it.D;
        bm.ldd = it.ldd;
        bm.d_is_fp64 = it.d_is_fp64;
        bm.item = order[k];
        bm.trD = it.trD;
        bm.trD2 = it.trD2;
        bm.S = it.S;
        bm.tile0 = (int32_t)t0;
        off += (int64_t)e;
        t0 += (np / bt) * (np / bt + 1) / 2;
    }
    FE_HIP(hipMemcpy(ws->bmats, mats.data(), sizeof(fe::BatchMat) * count, hipMemcpyHostToDevice));

    fe_batch_plan* plan = new fe_batch_plan();
    plan->gen = ++ws->batch_gen;   // earlier plans on this workspace become stale
    plan->count = count;
    plan->total_tiles = (int)tiles;
    plan->ws = ws;
    hipStream_t cs;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete plan;
        return hip_fail(e, "hipStreamCreate");
    }
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    const int bf = prec == FE_PREC_BF16X2;
    if (e == hipSuccess) {
        rc = enqueue_pass(ws, count, (int)tiles, max_np, m, 1.0, 0, bf, prec, status, cs);
        if (rc == FE_OK && mS) rc = enqueue_pass(ws, count, (int)tiles, max_np, mS, alpha, 1, bf, prec, status, cs);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(cs, &g);
        plan->graph = g;
        if (rc == FE_OK && e2 != hipSuccess) rc = hip_fail(e2, "hipStreamEndCapture");
        if (rc == FE_OK) {
            e2 = hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0);
            if (e2 != hipSuccess) rc = hip_fail(e2, "hipGraphInstantiate");
        }
    } else {
        rc = hip_fail(e, "hipStreamBeginCapture");
    }
    (void)hipStreamDestroy(cs);
    if (rc != FE_OK) {
        fe_batch_plan_destroy(plan);
        return rc;
    }
    *out = plan;
    return FE_OK;
}

int fe_batch_plan_launch(fe_batch_plan* plan, void* stream) {
    if (!plan || !plan->exec) return fail(FE_ERR_ARG, "invalid plan");
    if (plan->gen != plan->ws->batch_gen)
        return fail(FE_ERR_WORKSPACE, "a newer batch plan has replaced this one in the workspace");
    FE_HIP(hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream)));
    return FE_OK;
}

int fe_batch_plan_destroy(fe_batch_plan* plan) {
    if (!plan) return FE_OK;
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    delete plan;
    return FE_OK;
}

int fe_batched_expand(const fe_batch_item* items, int32_t count, const fe_model* m,
                      const fe_model* mS, double alpha, int32_t prec, int32_t* status,
                      fe_workspace* ws, void* stream) {
    fe_batch_plan* plan = nullptr;
    int rc = fe_batch_plan_create(items, count, m, mS, alpha, prec, status, ws, &plan);
    if (rc) return rc;
    rc = fe_batch_plan_launch(plan, stream);
    if (rc == FE_OK) {
        hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
        if (e != hipSuccess) rc = hip_fail(e, "hipStreamSynchronize");
    }
    fe_batch_plan_destroy(plan);
    return rc;
}

}  // extern "C"
