// Host side of the batched expansion: a plan lays the batch out in the workspace arena
// (matrices sorted by decreasing layer count, then decreasing padded size), uploads the
// per-matrix descriptors and the coefficient tables once and captures the whole launch sequence
// (bounds, rescale, the layers, reductions, and the entropy pass when requested) into one
// hipGraph that each launch replays. The layers of a pass run as one grouped launch per layer, or
// as one queue launch over all layers (batch_queue.h). With a model bank every matrix runs the model with the
// fewest layers whose region of validity (Eq. conditions) contains its (beta', mu').
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <numeric>
#include <vector>

#include "batch_queue.h"
#include "fe_host.h"

using namespace fehost;

struct fe_batch_plan {
    uint64_t gen = 0;       // workspace layout generation this plan was built for
    int count = 0;
    int tile = 128;         // tile size of the layer kernel (128 or 64)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    fe_workspace* ws = nullptr;
    void* tables = nullptr; // device coefficient tables of both passes
    void* maps = nullptr;   // device XCD-affine tile maps of the layer launches
    int launch = FE_BATCH_LAUNCH_QUEUE;    // one queue launch, or one grouped launch per layer
    int default_launch = FE_BATCH_LAUNCH_QUEUE;   // the form chosen at creation (by batch size)
    void* queues = nullptr; // device work queues and counters of the queue launch (both passes)
    // what a rebuild with another tile size needs (host copies)
    std::vector<fe_batch_item> items;
    std::vector<int> model;
    std::vector<std::vector<double>> theta;   // density models, then entropy models
    std::vector<fe_model> dens, ent;
    double alpha = 1.0;
    int32_t prec = 0;
    int32_t* status = nullptr;
};

namespace {

// fe_debug_batch_queue_giveup: every wait of the queue launch expects a count never reached
std::atomic<int> g_queue_giveup{0};

int check_item(const fe_batch_item& it, int i) {
    if (!it.H) return fail(FE_ERR_ARG, "batch item " + std::to_string(i) + ": H is NULL");
    if (it.n < 1) return fail(FE_ERR_ARG, "batch item " + std::to_string(i) + ": n < 1");
    if (it.ldh < it.n) return fail(FE_ERR_ARG, "batch item " + std::to_string(i) + ": ldh < n");
    if (it.D && it.ldd < it.n) return fail(FE_ERR_ARG, "batch item " + std::to_string(i) + ": ldd < n");
    return FE_OK;
}

// Host image of one pass's coefficient tables (layout of fe::BatchCoef).
struct PassTables {
    std::vector<float> coef;
    std::vector<int32_t> L;
    std::vector<float> d0;
    std::vector<double> shift0;
    int max_L = 0;
};

// Per model the layer weights of the single-matrix path, in the same form (squared-affine when
// the coefficients allow it, decided with the same alpha) so both give bitwise equal results.
PassTables make_tables(const std::vector<const fe_model*>& ms, int prec, double alpha) {
    PassTables t;
    for (const fe_model* m : ms) t.max_L = std::max(t.max_L, (int)m->L);
    t.coef.assign(ms.size() * t.max_L * 8, 0.0f);
    for (size_t k = 0; k < ms.size(); ++k) {
        const fe_model* m = ms[k];
        const double* th = m->theta;
        auto dval = [&](int i) {
            const double d = th[4 * i + 3];
            return (prec != FE_PREC_FP64 && fabs(d) < kDSkip) ? 0.0 : d;
        };
        AffineForm af;
        if (prec == FE_PREC_FP16X2 && affine_allowed()) af = affine_form(m, alpha, dval);
        std::vector<float> d_old, d_new;
        pair_accumulator_terms(m->L, dval, d_old, d_new);
        for (int l = 0; l < m->L; ++l) {
            float* c = &t.coef[(k * t.max_L + l) * 8];
            if (af.ok) {
                c[0] = af.ca[l];
                c[2] = af.cc[l];
                c[4] = af.dnew[l];
                c[5] = 1.0f;
            } else {
                c[0] = (float)th[4 * l];
                c[1] = (float)th[4 * l + 1];
                c[2] = (float)th[4 * l + 2];
                c[3] = d_old[l];
                c[4] = d_new[l];
            }
        }
        t.L.push_back(m->L);
        t.d0.push_back((float)dval(0));
        t.shift0.push_back(af.ok ? af.op_shift : 0.0);
    }
    return t;
}

// XCD-affine tile map of the layer launches over the matrices [0, k) of the sorted batch (those
// still active): each matrix's tiles go to one XCD, the matrices dealt in batch order to the XCD
// with the least work so far (work ~ tiles x K length); workgroup 8 i + x takes the i-th tile of
// XCD x (the hardware deals consecutive workgroups to consecutive XCDs on this 8-XCD chip, so
// workgroups 8 i + x, i = 0, 1, ..., share one XCD: XCD x itself when the dispatch starts at XCD 0,
// another one otherwise), empty slots are (-1, -1).
constexpr int kXcds = 8;
std::vector<int32_t> xcd_map(const std::vector<fe::BatchMat>& mats, int k, int tile) {
    std::vector<std::vector<int32_t>> lists(kXcds);
    std::vector<double> load(kXcds, 0.0);
    for (int m = 0; m < k; ++m) {
        const int64_t T = mats[m].np / tile, nt = T * (T + 1) / 2;
        int x = 0;
        for (int y = 1; y < kXcds; ++y)
            if (load[y] < load[x]) x = y;
        load[x] += (double)nt * (double)mats[m].np;
        for (int64_t t = 0; t < nt; ++t) {
            lists[x].push_back(m);
            lists[x].push_back((int32_t)t);
        }
    }
    size_t maxlen = 0;
    for (const auto& l : lists) maxlen = std::max(maxlen, l.size() / 2);
    std::vector<int32_t> map(2 * kXcds * maxlen, -1);
    for (int x = 0; x < kXcds; ++x)
        for (size_t i = 0; i < lists[x].size() / 2; ++i) {
            map[2 * (kXcds * i + x)] = lists[x][2 * i];
            map[2 * (kXcds * i + x) + 1] = lists[x][2 * i + 1];
        }
    return map;
}

// The queue (XCD) of each matrix of the sorted batch for the queue launch: dealt in batch order
// to the queue with the least work so far, as in xcd_map.
std::vector<int> deal_queues(const std::vector<fe::BatchMat>& mats, int tile, int nq) {
    std::vector<double> load(nq, 0.0);
    std::vector<int> q(mats.size());
    for (size_t m = 0; m < mats.size(); ++m) {
        const int64_t T = mats[m].np / tile, nt = T * (T + 1) / 2;
        int x = 0;
        for (int y = 1; y < nq; ++y)
            if (load[y] < load[x]) x = y;
        load[x] += (double)nt * (double)mats[m].np;
        q[m] = x;
    }
    return q;
}

// Host image of one pass's queues: items {matrix, tile, layer, need} per queue, layer-major, and
// the queue offsets. L[k]: layer count of model k in this pass.
struct PassQueues {
    std::vector<int32_t> items;   // 4 per item
    std::vector<int32_t> qoff;    // nq + 1
    int64_t longest = 0;
};
PassQueues make_queues(const std::vector<fe::BatchMat>& mats, const std::vector<int>& queue_of,
                       const std::vector<int32_t>& L, int max_L, int tile, int nq) {
    PassQueues pq;
    pq.qoff.assign(nq + 1, 0);
    for (int x = 0; x < nq; ++x) {
        pq.qoff[x] = (int32_t)(pq.items.size() / 4);
        for (int l = 0; l < max_L; ++l)
            for (size_t m = 0; m < mats.size(); ++m) {
                if (queue_of[m] != x || L[mats[m].model] <= l) continue;
                const int64_t T = mats[m].np / tile, nt = T * (T + 1) / 2;
                for (int64_t t = 0; t < nt; ++t) {
                    pq.items.push_back((int32_t)m);
                    pq.items.push_back((int32_t)t);
                    pq.items.push_back(l);
                    pq.items.push_back((int32_t)(l * nt));
                }
            }
        const int64_t len = (int64_t)(pq.items.size() / 4) - pq.qoff[x];
        pq.longest = std::max(pq.longest, len);
    }
    pq.qoff[nq] = (int32_t)(pq.items.size() / 4);
    return pq;
}

// Queues of the queue launch on the current device (its XCD count), and whether the launch's
// assumptions hold there (fe::batch_queue_probe, run once per device).
int queue_support(int* nq_out, bool* ok) {
    static std::mutex mu;
    static std::vector<int> state;   // per device: 0 unknown, 1 available, 2 unavailable
    static std::vector<int> nqs;
    int dev = 0, nq = 0;
    FE_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    if ((int)state.size() <= dev) {
        state.resize(dev + 1, 0);
        nqs.resize(dev + 1, 1);
    }
    if (state[dev] == 0) {
        if (hipDeviceGetAttribute(&nq, hipDeviceAttributeNumberOfXccs, dev) != hipSuccess || nq < 1)
            nq = 1;
        bool good = false;
        FE_HIP(fe::batch_queue_probe(nq, &good));
        state[dev] = good ? 1 : 2;
        nqs[dev] = nq;
    }
    *nq_out = nqs[dev];
    *ok = state[dev] == 1;
    return FE_OK;
}

// Device view of one pass's queues for a launch.
struct QueueLaunch {
    fe::BatchQueue q{};
    int64_t grid = 0;   // queues x longest queue
};

// One layer launch: its tile map on the device and the number of workgroups.
struct LayerLaunch {
    const int32_t* map;
    int grid;
};

// Enqueues one expansion pass (density or entropy) of the whole batch on `s`: with `queue`, all
// layers in one queue launch; else launches[l] is layer l's grouped launch (grid 0: no matrix has
// that many layers).
int enqueue_pass(fe_workspace* ws, int count, int64_t max_np, const fe::BatchCoef& cf,
                 const std::vector<LayerLaunch>& launches, const QueueLaunch* queue, double alpha,
                 int entropy, int bf, int tile, int32_t* status, hipStream_t s) {
    if (!entropy) FE_HIP(fe::launch_batch_bounds(ws->bmats, count, ws->bparams, s));
    FE_HIP(fe::launch_batch_rescale(ws->bmats, count, max_np, ws->bparams, alpha, cf, bf, s));
    if (queue) {
        fe::BatchLayerArgs q{};
        q.mats = ws->bmats;
        q.count = count;
        q.entropy = entropy;
        q.cf = cf;
        q.P = ws->bparams;
        q.partials = ws->btparts;
        FE_HIP(fe::launch_batch_queue_reset(queue->q, count, s));
        FE_HIP(fe::launch_batch_queue(q, queue->q, queue->grid, bf, tile, s));
        FE_HIP(fe::launch_batch_queue_check(ws->bmats, count, queue->q, cf, ws->bparams, tile, s));
        FE_HIP(fe::launch_batch_reduce(ws->bmats, count, ws->btparts, ws->bparams, entropy, status,
                                       tile, s));
        return FE_OK;
    }
    for (int l = 0; l < cf.max_L; ++l) {
        if (launches[l].grid == 0) break;
        fe::BatchLayerArgs q{};
        q.mats = ws->bmats;
        q.map = launches[l].map;
        q.count = count;
        q.parity = l & 1;
        q.layer = l;
        q.entropy = entropy;
        q.cf = cf;
        q.P = ws->bparams;
        q.partials = ws->btparts;
        FE_HIP(fe::launch_batch_layer(q, launches[l].grid, bf, tile, s));
    }
    FE_HIP(fe::launch_batch_reduce(ws->bmats, count, ws->btparts, ws->bparams, entropy, status,
                                   tile, s));
    return FE_OK;
}

// Bytes of the arena per padded element: X, A, hi[2], lo[2] (and mid[2] for three parts).
int64_t arena_bytes_per_elem(int32_t prec) { return prec == FE_PREC_BF16X3 ? 20 : 16; }

// Descriptors of the batch in the arena, in `order`; model[i] is item i's model index.
std::vector<fe::BatchMat> layout(const fe_batch_item* items, const std::vector<int>& order,
                                 const std::vector<int>& model,
                                 const std::vector<const fe_model*>& ms, fe_workspace* ws,
                                 int64_t bt, int32_t prec, int64_t* tiles_out,
                                 int64_t* max_np_out) {
    const bool three = prec == FE_PREC_BF16X3;
    const int64_t bpe = arena_bytes_per_elem(prec);
    const int64_t pad = fe::kBatchPad;
    std::vector<fe::BatchMat> mats(order.size());
    char* arena = static_cast<char*>(ws->arena);
    int64_t off = 0, t0 = 0, max_np = 0;
    for (size_t k = 0; k < order.size(); ++k) {
        const fe_batch_item& it = items[order[k]];
        fe::BatchMat& bm = mats[k];
        memset(&bm, 0, sizeof(bm));
        const int64_t np = round_up(it.n, pad);
        const size_t e = (size_t)np * np;
        bm.H = it.H;
        bm.n = it.n;
        bm.ldh = it.ldh;
        bm.np = np;
        bm.mu = it.mu;
        bm.kT = it.kT;
        bm.model = model[order[k]];
        bm.beta0 = ms[bm.model]->beta0;
        bm.mu0 = ms[bm.model]->mu0;
        bm.X = reinterpret_cast<float*>(arena + off * bpe);
        bm.A = bm.X + e;
        uint16_t* h = reinterpret_cast<uint16_t*>(bm.A + e);
        bm.hi[0] = h;
        bm.hi[1] = h + e;
        bm.lo[0] = h + 2 * e;
        bm.lo[1] = h + 3 * e;
        bm.mid[0] = three ? h + 4 * e : nullptr;
        bm.mid[1] = three ? h + 5 * e : nullptr;
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
        max_np = std::max(max_np, np);
    }
    *tiles_out = t0;
    *max_np_out = max_np;
    return mats;
}

int check_batch(const fe_batch_item* items, int count, int32_t prec, fe_workspace* ws) {
    if (!ws) return fail(FE_ERR_ARG, "workspace is NULL");
    if (!items || count < 1) return fail(FE_ERR_ARG, "empty batch");
    if (count > ws->max_batch) return fail(FE_ERR_WORKSPACE, "batch larger than the workspace's max_batch");
    const int64_t bt = 64;   // the larger tile count of the two tile sizes
    int64_t elems = 0, tiles = 0;
    for (int i = 0; i < count; ++i) {
        int rc = check_item(items[i], i);
        if (rc) return rc;
        const int64_t np = round_up(items[i].n, (int64_t)fe::kBatchPad), T = np / bt;
        elems += np * np;
        tiles += T * (T + 1) / 2;
    }
    if (elems * arena_bytes_per_elem(prec) > ws->batch_elems * 16)
        return fail(FE_ERR_WORKSPACE, "batch exceeds the workspace arena");
    if (tiles > ws->batch_tiles || tiles > (int64_t)0x7fffffff)
        return fail(FE_ERR_WORKSPACE, "batch has too many tiles for the workspace");
    return FE_OK;
}

// Releases a plan's graph and tables (before a rebuild or on destruction).
void release_plan(fe_batch_plan* plan) {
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    if (plan->tables) (void)hipFree(plan->tables);
    if (plan->maps) (void)hipFree(plan->maps);
    if (plan->queues) (void)hipFree(plan->queues);
    plan->exec = nullptr;
    plan->graph = nullptr;
    plan->tables = nullptr;
    plan->maps = nullptr;
    plan->queues = nullptr;
}

// Builds and captures `plan` for its stored inputs with layer tiles of `tile` (128 or 64): item i
// runs model dens[model[i]] (and ent[model[i]] for the entropy pass when ent is non-empty).
int build_plan(fe_batch_plan* plan, int tile) {
    release_plan(plan);
    const fe_batch_item* items = plan->items.data();
    const int count = plan->count;
    const std::vector<int>& model = plan->model;
    std::vector<const fe_model*> dens, ent;
    for (const fe_model& m : plan->dens) dens.push_back(&m);
    for (const fe_model& m : plan->ent) ent.push_back(&m);
    const double alpha = plan->alpha;
    const int32_t prec = plan->prec;
    int32_t* status = plan->status;
    fe_workspace* ws = plan->ws;
    std::vector<int> order(count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const int la = dens[model[a]]->L, lb = dens[model[b]]->L;
        if (la != lb) return la > lb;
        return items[a].n > items[b].n;
    });
    int64_t tiles = 0, max_np = 0;
    std::vector<fe::BatchMat> mats = layout(items, order, model, dens, ws, tile, prec, &tiles, &max_np);
    if (tiles > ws->batch_tiles) return fail(FE_ERR_WORKSPACE, "batch has too many tiles for the workspace");
    const PassTables td = make_tables(dens, prec, 1.0);
    PassTables te;
    if (!ent.empty()) te = make_tables(ent, prec, alpha);
    // active tiles per layer (the sorted order makes them a prefix in both passes)
    auto active_tiles = [&](const PassTables& t) {
        std::vector<int> act(t.max_L, 0);
        for (int l = 0; l < t.max_L; ++l) {
            int64_t a = 0;
            bool prefix = true;
            for (int k = 0; k < count; ++k) {
                const bool on = t.L[mats[k].model] > l;
                if (!on) prefix = false;
                else if (!prefix) return std::vector<int>();   // not a prefix
                else a = (k + 1 < count) ? mats[k + 1].tile0 : tiles;
            }
            act[l] = (int)a;
        }
        return act;
    };
    const std::vector<int> act_d = active_tiles(td);
    const std::vector<int> act_e = ent.empty() ? std::vector<int>() : active_tiles(te);
    if (act_d.empty() || (!ent.empty() && act_e.empty()))
        return fail(FE_ERR_ARG, "entropy and density models must order the batch the same way");
    // active matrices per layer (a prefix), and one XCD-affine map per distinct prefix
    auto active_mats = [&](const PassTables& t) {
        std::vector<int> k(t.max_L, 0);
        for (int l = 0; l < t.max_L; ++l)
            while (k[l] < count && t.L[mats[k[l]].model] > l) ++k[l];
        return k;
    };
    const std::vector<int> km_d = active_mats(td);
    const std::vector<int> km_e = ent.empty() ? std::vector<int>() : active_mats(te);
    std::vector<int> prefixes(km_d.begin(), km_d.end());
    prefixes.insert(prefixes.end(), km_e.begin(), km_e.end());
    std::sort(prefixes.begin(), prefixes.end());
    prefixes.erase(std::unique(prefixes.begin(), prefixes.end()), prefixes.end());
    std::vector<int32_t> all_maps;
    std::vector<size_t> map_off(count + 1, 0), map_len(count + 1, 0);
    for (int k : prefixes) {
        if (k == 0) continue;
        const std::vector<int32_t> mp = xcd_map(mats, k, tile);
        map_off[k] = all_maps.size();
        map_len[k] = mp.size() / 2;
        all_maps.insert(all_maps.end(), mp.begin(), mp.end());
    }
    // earlier plans on this workspace become stale before its shared descriptors are replaced,
    // and no launch of them may still be reading those descriptors
    plan->gen = ++ws->batch_gen;
    FE_HIP(hipDeviceSynchronize());
    FE_HIP(hipMemcpy(ws->bmats, mats.data(), sizeof(fe::BatchMat) * count, hipMemcpyHostToDevice));
    {
        hipError_t em = hipMalloc(&plan->maps, std::max<size_t>(4, all_maps.size() * 4));
        if (em == hipSuccess && !all_maps.empty())
            em = hipMemcpy(plan->maps, all_maps.data(), all_maps.size() * 4, hipMemcpyHostToDevice);
        if (em != hipSuccess) return hip_fail(em, "batch tile maps");
    }
    auto launches_of = [&](const std::vector<int>& km) {
        std::vector<LayerLaunch> v(km.size());
        for (size_t l = 0; l < km.size(); ++l) {
            const int k = km[l];
            v[l].map = k ? static_cast<const int32_t*>(plan->maps) + map_off[k] : nullptr;
            v[l].grid = k ? (int)map_len[k] : 0;
        }
        return v;
    };
    const std::vector<LayerLaunch> ll_d = launches_of(km_d);
    const std::vector<LayerLaunch> ll_e = launches_of(km_e);

    plan->tile = tile;
    // device tables: [density coef | L | d0 | shift0 | entropy ...], 256-byte aligned parts
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t cd = al(td.coef.size() * 4), ld = al(td.L.size() * 4), dd = al(td.d0.size() * 4);
    const size_t sd = al(td.shift0.size() * 8);
    const size_t ce = al(te.coef.size() * 4), le = al(te.L.size() * 4), de = al(te.d0.size() * 4);
    const size_t se = al(te.shift0.size() * 8);
    hipError_t e = hipMalloc(&plan->tables, cd + ld + dd + sd + ce + le + de + se + 256);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc (batch tables)");
    char* base = static_cast<char*>(plan->tables);
    auto up = [&](size_t off, const void* src, size_t bytes) {
        return bytes ? hipMemcpy(base + off, src, bytes, hipMemcpyHostToDevice) : hipSuccess;
    };
    fe::BatchCoef cfd{reinterpret_cast<const float*>(base), reinterpret_cast<const int32_t*>(base + cd),
                      reinterpret_cast<const float*>(base + cd + ld),
                      reinterpret_cast<const double*>(base + cd + ld + dd), td.max_L};
    const size_t eo = cd + ld + dd + sd;
    fe::BatchCoef cfe{reinterpret_cast<const float*>(base + eo),
                      reinterpret_cast<const int32_t*>(base + eo + ce),
                      reinterpret_cast<const float*>(base + eo + ce + le),
                      reinterpret_cast<const double*>(base + eo + ce + le + de), te.max_L};
    e = up(0, td.coef.data(), td.coef.size() * 4);
    if (e == hipSuccess) e = up(cd, td.L.data(), td.L.size() * 4);
    if (e == hipSuccess) e = up(cd + ld, td.d0.data(), td.d0.size() * 4);
    if (e == hipSuccess) e = up(cd + ld + dd, td.shift0.data(), td.shift0.size() * 8);
    if (e == hipSuccess) e = up(eo, te.coef.data(), te.coef.size() * 4);
    if (e == hipSuccess) e = up(eo + ce, te.L.data(), te.L.size() * 4);
    if (e == hipSuccess) e = up(eo + ce + le, te.d0.data(), te.d0.size() * 4);
    if (e == hipSuccess) e = up(eo + ce + le + de, te.shift0.data(), te.shift0.size() * 8);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy (batch tables)");
    // queue launch: per pass the items of every queue, then both passes' counters
    QueueLaunch qd, qe;
    int nq = 1;
    bool queue_ok = false;
    if (plan->launch == FE_BATCH_LAUNCH_QUEUE) {
        int rcq = queue_support(&nq, &queue_ok);
        if (rcq != FE_OK) return rcq;
        if (!queue_ok) plan->launch = FE_BATCH_LAUNCH_LAYERS;   // the default falls back
    }
    const bool queued = plan->launch == FE_BATCH_LAUNCH_QUEUE;
    if (queued) {
        const std::vector<int> queue_of = deal_queues(mats, tile, nq);
        const PassQueues pd = make_queues(mats, queue_of, td.L, td.max_L, tile, nq);
        PassQueues pe;
        if (!ent.empty()) pe = make_queues(mats, queue_of, te.L, te.max_L, tile, nq);
        if (pd.longest * nq > 0x7fffffff || pe.longest * nq > 0x7fffffff)
            return fail(FE_ERR_WORKSPACE, "batch has too many work items for one queue launch");
        const size_t id = al(pd.items.size() * 4), ie = al(pe.items.size() * 4);
        const size_t od = al(pd.qoff.size() * 4), oe = al(pe.qoff.size() * 4);
        const size_t cn = al((size_t)fe::batch_queue_counters(nq, count) * 4);
        e = hipMalloc(&plan->queues, id + ie + od + oe + cn + 256);
        if (e != hipSuccess) return hip_fail(e, "hipMalloc (batch queues)");
        char* qb = static_cast<char*>(plan->queues);
        auto upq = [&](size_t off, const std::vector<int32_t>& v) {
            return v.empty() ? hipSuccess
                             : hipMemcpy(qb + off, v.data(), v.size() * 4, hipMemcpyHostToDevice);
        };
        e = upq(0, pd.items);
        if (e == hipSuccess) e = upq(id, pe.items);
        if (e == hipSuccess) e = upq(id + ie, pd.qoff);
        if (e == hipSuccess) e = upq(id + ie + od, pe.qoff);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy (batch queues)");
        int32_t* counters = reinterpret_cast<int32_t*>(qb + id + ie + od + oe);
        auto view = [&](QueueLaunch& v, size_t items_off, size_t qoff_off, int64_t longest) {
            v.q.items = reinterpret_cast<const int4*>(qb + items_off);
            v.q.qoff = reinterpret_cast<const int32_t*>(qb + qoff_off);
            v.q.nq = nq;
            v.q.ticket = counters;
            v.q.done = counters + nq;
            v.q.err = counters + nq + count;
            const bool giveup = g_queue_giveup.load() != 0;
            // 1 << 20 polls, each after up to 16 x 512 clocks of sleep: ~5 s
            v.q.spin_limit = giveup ? 64 : (1 << 20);
            v.q.need_offset = giveup ? (1 << 30) : 0;
            v.grid = longest * nq;
        };
        view(qd, 0, id + ie, pd.longest);
        if (!ent.empty()) view(qe, id, id + ie + od, pe.longest);
    }
    hipStream_t cs;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
    int rc = FE_OK;
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    const int bf = prec == FE_PREC_BF16X3 ? 2 : prec == FE_PREC_BF16X2 ? 1 : 0;
    if (e == hipSuccess) {
        rc = enqueue_pass(ws, count, max_np, cfd, ll_d, queued ? &qd : nullptr, 1.0, 0, bf,
                          tile, status, cs);
        if (rc == FE_OK && !ent.empty())
            rc = enqueue_pass(ws, count, max_np, cfe, ll_e, queued ? &qe : nullptr, alpha, 1, bf,
                              tile, status, cs);
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
    return rc;
}

// A new plan holding copies of its inputs, built with 128 x 128 layer tiles.
int create_plan(const fe_batch_item* items, int count, const std::vector<int>& model,
                const std::vector<const fe_model*>& dens, const std::vector<const fe_model*>& ent,
                double alpha, int32_t prec, int32_t* status, fe_workspace* ws,
                fe_batch_plan** out) {
    fe_batch_plan* plan = new fe_batch_plan();
    plan->count = count;
    plan->ws = ws;
    plan->items.assign(items, items + count);
    plan->model = model;
    plan->theta.reserve(dens.size() + ent.size());
    for (const fe_model* m : dens) {
        plan->theta.emplace_back(m->theta, m->theta + 4 * m->L);
        plan->dens.push_back({m->L, m->beta0, m->mu0, plan->theta.back().data()});
    }
    for (const fe_model* m : ent) {
        plan->theta.emplace_back(m->theta, m->theta + 4 * m->L);
        plan->ent.push_back({m->L, m->beta0, m->mu0, plan->theta.back().data()});
    }
    plan->alpha = alpha;
    plan->prec = prec;
    plan->status = status;
    // Default launch form: the queue launch when the first layer alone holds at least one 128 x 128
    // tile per resident workgroup slot (two per CU); a smaller batch is bound by its chain of
    // layers, where the per-layer launches hand each layer over faster (measured: 64 matrices of
    // N <= 300, 0.63 against 1.0 ms; 256 of N <= 384, 2.09 against 1.84 ms the other way round).
    {
        int64_t tiles = 0;
        for (int i = 0; i < count; ++i) {
            const int64_t T = (items[i].n + 127) / 128;
            tiles += T * (T + 1) / 2;
        }
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 256;
        plan->launch = tiles >= 2 * (int64_t)cus ? FE_BATCH_LAUNCH_QUEUE : FE_BATCH_LAUNCH_LAYERS;
        plan->default_launch = plan->launch;
    }
    const int rc = build_plan(plan, 128);
    if (rc != FE_OK) {
        fe_batch_plan_destroy(plan);
        return rc;
    }
    *out = plan;
    return FE_OK;
}

int check_16bit_model(const fe_model* m, double alpha, const char* what) {
    int rc = check_model(m, what);
    if (rc) return rc;
    if (layer_range(m, alpha) > 16.0)
        return fail(FE_ERR_RANGE, std::string(what) + ": layer values exceed the 16-bit operand range");
    return FE_OK;
}

}  // namespace

extern "C" {

int fe_batch_plan_create(const fe_batch_item* items, int32_t count, const fe_model* m,
                         const fe_model* mS, double alpha, int32_t prec, int32_t* status,
                         fe_workspace* ws, fe_batch_plan** out) {
    if (!out) return fail(FE_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (prec != FE_PREC_FP16X2 && prec != FE_PREC_BF16X2 && prec != FE_PREC_BF16X3)
        return fail(FE_ERR_ARG, "batched expansion supports the FP16x2, BF16x2 and BF16x3 modes");
    int rc = check_batch(items, count, prec, ws);
    if (rc) return rc;
    rc = check_16bit_model(m, 1.0, "model");
    if (rc) return rc;
    if (mS) {
        if (!(fabs(alpha) <= 1.0)) return fail(FE_ERR_ARG, "|alpha| must be <= 1");
        rc = check_16bit_model(mS, alpha, "entropy model");
        if (rc) return rc;
        if (mS->beta0 != m->beta0 || mS->mu0 != m->mu0)
            return fail(FE_ERR_ARG, "the entropy model must share (beta0, mu0) with the density model");
    }
    std::vector<int> model(count, 0);
    std::vector<const fe_model*> dens{m}, ent;
    if (mS) ent.push_back(mS);
    return create_plan(items, count, model, dens, ent, alpha, prec, status, ws, out);
}

int fe_batch_plan_create_bank(const fe_batch_item* items, int32_t count, const fe_model* bank,
                              int32_t nbank, int32_t with_entropy, double alpha, int32_t prec,
                              int32_t* status, int32_t* chosen, fe_workspace* ws,
                              fe_batch_plan** out) {
    if (!out) return fail(FE_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (prec != FE_PREC_FP16X2 && prec != FE_PREC_BF16X2 && prec != FE_PREC_BF16X3)
        return fail(FE_ERR_ARG, "batched expansion supports the FP16x2, BF16x2 and BF16x3 modes");
    int rc = check_batch(items, count, prec, ws);
    if (rc) return rc;
    if (!bank || nbank < 1) return fail(FE_ERR_ARG, "empty model bank");
    if (with_entropy && !(fabs(alpha) <= 1.0)) return fail(FE_ERR_ARG, "|alpha| must be <= 1");
    std::vector<const fe_model*> ms;
    for (int k = 0; k < nbank; ++k) {
        rc = check_16bit_model(&bank[k], 1.0, "bank model");
        if (rc) return rc;
        if (with_entropy) {
            rc = check_16bit_model(&bank[k], alpha, "bank model (entropy)");
            if (rc) return rc;
        }
        ms.push_back(&bank[k]);
    }
    // (beta', mu') of every item from its Gershgorin bounds: one bounds pass, synchronized.
    std::vector<int> provisional(count, 0), order(count);
    std::iota(order.begin(), order.end(), 0);
    int64_t tiles = 0, max_np = 0;
    std::vector<fe::BatchMat> mats = layout(items, order, provisional, ms, ws, 128, prec, &tiles, &max_np);
    // the descriptors are shared by every plan on the workspace: older plans become stale first,
    // and none of their launches may still be reading them
    ++ws->batch_gen;
    FE_HIP(hipDeviceSynchronize());
    FE_HIP(hipMemcpy(ws->bmats, mats.data(), sizeof(fe::BatchMat) * count, hipMemcpyHostToDevice));
    FE_HIP(fe::launch_batch_bounds(ws->bmats, count, ws->bparams, nullptr));
    std::vector<fe::Params> P(count);
    FE_HIP(hipMemcpy(P.data(), ws->bparams, sizeof(fe::Params) * count, hipMemcpyDeviceToHost));
    std::vector<int> model(count, 0);
    for (int i = 0; i < count; ++i) {
        model[i] = choose_bank_model(ms.data(), nbank, P[i].emin, P[i].emax, items[i].mu, items[i].kT);
        if (chosen) chosen[i] = model[i];
    }
    std::vector<const fe_model*> ent;
    if (with_entropy) ent = ms;
    return create_plan(items, count, model, ms, ent, alpha, prec, status, ws, out);
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
    release_plan(plan);
    delete plan;
    return FE_OK;
}

int fe_batch_plan_retile(fe_batch_plan* plan, int32_t tile) {
    if (!plan) return fail(FE_ERR_ARG, "invalid plan");
    if (tile != 64 && tile != 128) return fail(FE_ERR_ARG, "tile must be 64 or 128");
    if (tile == 64 && plan->prec == FE_PREC_BF16X3)
        return fail(FE_ERR_ARG, "the three-part BF16 split runs 128 x 128 tiles only");
    FE_HIP(hipDeviceSynchronize());   // a launch of the old graph may still be reading its tables
    return build_plan(plan, tile);
}

int fe_batch_plan_set_launch(fe_batch_plan* plan, int32_t launch) {
    if (!plan) return fail(FE_ERR_ARG, "invalid plan");
    if (launch != FE_BATCH_LAUNCH_LAYERS && launch != FE_BATCH_LAUNCH_QUEUE)
        return fail(FE_ERR_ARG, "launch must be FE_BATCH_LAUNCH_LAYERS or FE_BATCH_LAUNCH_QUEUE");
    if (launch == FE_BATCH_LAUNCH_QUEUE) {
        int nq = 1;
        bool ok = false;
        const int rc = queue_support(&nq, &ok);
        if (rc != FE_OK) return rc;
        if (!ok)
            return fail(FE_ERR_ARG, "the queue launch is unavailable on this device (workgroups are "
                                    "not dealt to its XCDs round-robin)");
    }
    FE_HIP(hipDeviceSynchronize());   // as in fe_batch_plan_retile
    plan->launch = launch;
    return build_plan(plan, plan->tile);
}

int fe_batch_plan_autotune(fe_batch_plan* plan, void* stream, int32_t* tile, double* ms) {
    if (!plan) return fail(FE_ERR_ARG, "invalid plan");
    hipStream_t s = static_cast<hipStream_t>(stream);
    FE_HIP(hipDeviceSynchronize());   // as in fe_batch_plan_retile
    int nq = 1;
    bool queue_ok = false;
    {
        const int rc = queue_support(&nq, &queue_ok);
        if (rc != FE_OK) return rc;
    }
    // candidates: tile x launch form (the three-part split has the 128 x 128 tile only)
    struct Cand {
        int tile, launch;
        double ms;
    };
    std::vector<Cand> cands;
    for (int t : {128, 64}) {
        if (t == 64 && plan->prec == FE_PREC_BF16X3) continue;
        if (queue_ok) cands.push_back({t, FE_BATCH_LAUNCH_QUEUE, NAN});
        cands.push_back({t, FE_BATCH_LAUNCH_LAYERS, NAN});
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    FE_HIP(hipEventCreate(&e0));
    hipError_t e = hipEventCreate(&e1);
    int rc = FE_OK;
    for (size_t c = 0; c < cands.size() && rc == FE_OK && e == hipSuccess; ++c) {
        plan->launch = cands[c].launch;
        rc = build_plan(plan, cands[c].tile);
        if (rc != FE_OK) break;
        for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {   // one warm-up, three timed
            if (rep == 1) e = hipEventRecord(e0, s);
            if (e == hipSuccess) e = hipGraphLaunch(plan->exec, s);
        }
        float t = 0.0f;
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        cands[c].ms = t / 3.0;
    }
    (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess || rc != FE_OK) {
        // leave the plan usable: the default form at 128 x 128
        plan->launch = queue_ok ? plan->default_launch : FE_BATCH_LAUNCH_LAYERS;
        (void)build_plan(plan, 128);
        return e != hipSuccess ? hip_fail(e, "batch autotune") : rc;
    }
    size_t best = 0;
    for (size_t c = 1; c < cands.size(); ++c)
        if (cands[c].ms < cands[best].ms) best = c;
    if (ms) {
        ms[0] = ms[1] = NAN;
        for (const Cand& c : cands) {
            double& m = ms[c.tile == 128 ? 0 : 1];
            if (!(m <= c.ms)) m = c.ms;   // the faster launch form of each tile size
        }
    }
    if (tile) *tile = cands[best].tile;
    if (plan->tile == cands[best].tile && plan->launch == cands[best].launch) return FE_OK;
    plan->launch = cands[best].launch;
    return build_plan(plan, cands[best].tile);
}

int fe_batch_plan_get(const fe_batch_plan* plan, int32_t* tile, int32_t* launch) {
    if (!plan) return fail(FE_ERR_ARG, "invalid plan");
    if (tile) *tile = plan->tile;
    if (launch) *launch = plan->launch;
    return FE_OK;
}

int fe_batch_queue_layout(int32_t count, const int64_t* np, const int32_t* L, int32_t tile,
                          int32_t nq, int32_t* items, int64_t cap, int32_t* qoff, int64_t* nitems) {
    if (count < 1 || !np || !L || !qoff || !nitems) return fail(FE_ERR_ARG, "bad arguments");
    if (tile != 64 && tile != 128) return fail(FE_ERR_ARG, "tile must be 64 or 128");
    if (nq < 1 || nq > 16) return fail(FE_ERR_ARG, "nq must be 1 .. 16");
    std::vector<fe::BatchMat> mats(count);
    std::vector<int32_t> Lm(count);
    int max_L = 0;
    for (int i = 0; i < count; ++i) {
        if (np[i] < tile || np[i] % tile != 0 || L[i] < 1)
            return fail(FE_ERR_ARG, "np must be a positive multiple of the tile, L >= 1");
        memset(&mats[i], 0, sizeof(mats[i]));
        mats[i].np = np[i];
        mats[i].model = i;   // one "model" per matrix: its layer count
        Lm[i] = L[i];
        max_L = std::max(max_L, (int)L[i]);
    }
    const PassQueues pq = make_queues(mats, deal_queues(mats, tile, nq), Lm, max_L, tile, nq);
    *nitems = (int64_t)pq.items.size() / 4;
    for (int x = 0; x <= nq; ++x) qoff[x] = pq.qoff[x];
    if (items) {
        if (cap < *nitems) return fail(FE_ERR_ARG, "items too small");
        memcpy(items, pq.items.data(), pq.items.size() * sizeof(int32_t));
    }
    return FE_OK;
}

int fe_debug_batch_queue_giveup(int32_t enable) {
    g_queue_giveup.store(enable ? 1 : 0);
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
