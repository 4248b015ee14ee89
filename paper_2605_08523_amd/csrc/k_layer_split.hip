// One layer of the recursion X <- a X^2 + b X + c I, A <- A + d X (Eq. mlsp2) for a symmetric X
// held as X = hi + lo / s with 16-bit hi/lo (Sec. V.A, Eq. emulated matmul), on CDNA4 MFMA.
//
// Design (gfx950):
//  * Only tiles (I, J) with I <= J are computed (X^2 is symmetric); the epilogue writes the tile
//    and its mirror, so every stored matrix stays exactly symmetric.
//  * X^2 is accumulated in FP32 from three products per K step in one accumulator,
//        s X^2 ~ (s hi_I) hi_J + hi_I lo_J + lo_I hi_J,
//    the lo*lo term being below 2^-22 relative for FP16. By symmetry the B operand of tile
//    (I, J) is the row panel J, so both operands are row panels with K contiguous.
//  * The epilogue is fused (see split_common.h): Y goes through LDS, one row-major pass applies
//    a Y + b X + c delta_ij, updates A and writes the next hi/lo (and, in the direct form, the FP32
//    master X); a transposed pass writes the mirror tile. The last layer writes D and FP64
//    traces. In the squared-affine form (FP16x2 default) the operand is the shifted state
//    x + b/(2a), so b = 0 and X is neither read nor written.
//  * Three schedules:
//      data-parallel: one workgroup per upper tile (128 x 128, four 64 x 64 wave tiles);
//      stream-K over 128 x 128 tiles, two persistent workgroups per CU: the (tile, K-block)
//        iterations left after the whole-tile rounds are split evenly. A workgroup that stops
//        inside a tile publishes its FP32 partial; the workgroup that finishes the tile adds the
//        earlier workgroups' partials in a fixed order in its epilogue (accumulators stay in
//        registers);
//      stream-K over 256 x 256 tiles (eight 128 x 64 wave tiles, two LDS stages filled by
//        direct global-to-LDS loads, fragment reads interleaved with the MFMAs), one
//        workgroup per CU: the same; its K loop holds no prefetch registers, so the 128
//        accumulators per lane also stay in registers through the wait and the epilogue.
//    A workgroup only ever waits for workgroups with smaller ids, which were dispatched earlier,
//    and every wait is bounded.
#include "split_common.h"
#include "streamk_plan.h"

namespace fe {
namespace {

using namespace split;

using CfgDP = Cfg<128, 2, 2, 64, 128, 1>;
using CfgSK = Cfg<256, 2, 4, 32, 128, 2, 1>;   // direct-to-LDS operand staging
using CfgSK2 = Cfg<128, 2, 2, 64, 128, 1>;   // stream-K over 128 x 128 tiles, two workgroups per CU
// Three-part BF16 split: six panels of 32-deep K-blocks in one LDS stage (61 KiB), so two
// workgroups still fit per CU; data-parallel only.
using CfgDP3 = Cfg<128, 2, 2, 32, 128, 1, 0, 3>;


template <class C>
__device__ inline void zero(Acc<C>& acc) {
#pragma unroll
    for (int mb = 0; mb < C::MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < C::NB; ++nb)
#pragma unroll
            for (int j = 0; j < 16; ++j) acc.v[mb][nb][j] = 0.0f;
}

template <bool BF, class C>
__global__ void __launch_bounds__(C::NT) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_layer_dp(LayerArgs p) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int T = (int)(p.np / C::BM);
    const int t = xcd_tile(blockIdx.x, gridDim.x);   // tiles [0, gridDim.x)
    int I, J;
    tile_coords(t, T, I, J);
    Acc<C> acc;
    zero(acc);
    if constexpr (C::NS == 3)
        kloop3<C>(p.hi_in, p.mid_in, p.lo_in, p.np, (int64_t)I * C::BM, (int64_t)J * C::BM, 0,
                  (int)(p.np / C::BK), acc, reinterpret_cast<uint16_t*>(smem));
    else
        kloop<BF, C>(p.hi_in, p.lo_in, p.np, (int64_t)I * C::BM, (int64_t)J * C::BM, 0,
                     (int)(p.np / C::BK), acc, reinterpret_cast<uint16_t*>(smem));
    epilogue<BF, C>(p, acc, reinterpret_cast<float*>(smem), I, J, t);
}

// Thread 0 waits until the workgroups of group g with indices jlo .. j-1 have published their
// partials of the current tile (each publishes exactly once: a group never has more workgroups
// than iterations, so every range is non-empty). Their ids g + NG jlo, ..., w - NG are all smaller
// than w. Bounded: a wait that gives up sets *err and returns true for the whole workgroup (the
// caller's epilogue then writes NaN for the whole tile, so that no plausible value is built from
// partials that may belong to an earlier layer). Ends with a barrier.
__device__ inline bool wait_published(const SplitPlan& sk, int g, int NG, int jlo, int w) {
    __shared__ int gave_up_all;
    if (threadIdx.x == 0) {
        bool gave_up = false;
        for (int wp = g + NG * jlo; wp < w && !gave_up; wp += NG) {
            int spins = 0;
            while (__hip_atomic_load(sk.flags + wp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) !=
                   sk.wait_epoch) {
                if (++spins > sk.spin_limit) {
                    atomicOr(sk.err, 1);
                    gave_up = true;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        gave_up_all = gave_up ? 1 : 0;
    }
    // The partials are read after this barrier, i.e. after the flags were seen, with
    // device-coherent loads.
    __syncthreads();
    return gave_up_all != 0;
}

template <bool BF, class C>
__global__ void __launch_bounds__(C::NT) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_layer_sk(LayerArgs p, SplitPlan sk) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    // Accumulators stay in registers through the wait when the K loop leaves room for them
    // (small tiles, or the direct-to-LDS loop, which holds no prefetch registers); otherwise
    // (128 per lane next to a register-prefetch loop) they are staged to memory after the K loop.
    constexpr bool kRegEpi = C::MB * C::NB <= 4 || C::DMA;
    const int tid = threadIdx.x;
    const int w = blockIdx.x;
    const int T = (int)(p.np / C::BM);
    const int ntiles = T * (T + 1) / 2;
    const int nk = (int)(p.np / C::BK);
    constexpr size_t TILE = (size_t)C::BM * C::BM;
    float* own = sk.own + (size_t)w * TILE;
    float* pub = sk.partial + (size_t)w * TILE;
    float* sY = reinterpret_cast<float*>(smem);

    // Tiles [0, dp_tiles) were computed whole by a data-parallel launch before this one; the
    // walk over the rest is in streamk_plan.h (shared with the host-side plan checks).
    SkGeometry G;
    G.T = T;
    G.ntiles = ntiles;
    G.nk = nk;
    G.dp_tiles = sk.dp_tiles;
    G.groups = sk.groups;
    G.grid = sk.grid;
    const int NG = sk.groups, g = w % NG, j = w / NG;
    sk_walk(G, w, [&](int pass, int t, int kb0, int kb1, int jlo) {
        int I, J;
        tile_coords(t, T, I, J);
        // Earlier workgroups of the group with indices jlo .. j-1 hold the first kb0 blocks of
        // this tile; their partial slots are NG tiles apart. The epilogue adds them in a fixed
        // order, so the result does not depend on timing.
        const float* parts = sk.partial + (size_t)(g + NG * jlo) * TILE;
        Acc<C> acc;
        zero(acc);
        kloop<BF, C>(p.hi_in, p.lo_in, p.np, (int64_t)I * C::BM, (int64_t)J * C::BM, kb0, kb1, acc,
                     reinterpret_cast<uint16_t*>(smem));
        if (pass == 0) {
            // Publication: every wave waits until its device-coherent stores of the partial
            // have completed, then one flag store (device-coherent too) announces the tile.
            // No release fence: on this chip it writes back the whole L2, and the readers'
            // acquire would invalidate it; the partial needs neither (see store_coherent).
            store_tile<BF, C, true>(acc, pub);
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            if (tid == 0)
                __hip_atomic_store(sk.flags + w, sk.epoch, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        } else if constexpr (kRegEpi) {
            const bool gave_up = wait_published(sk, g, NG, jlo, w);
            epilogue<BF, C, 1>(p, acc, sY, I, J, t, parts, (size_t)NG * TILE, j - jlo, gave_up);
        } else {
            store_tile<BF, C, false>(acc, own);
            const bool gave_up = wait_published(sk, g, NG, jlo, w);
            epilogue_mem<BF, C, 1>(p, own, parts, (size_t)NG * TILE, j - jlo, sY, I, J, t,
                                   gave_up);
        }
    });
}

template <class K>
hipError_t set_lds(K kern, size_t bytes, bool& done) {
    if (done) return hipSuccess;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess) done = true;
    return e;
}

template <bool BF, class C = CfgDP>
hipError_t launch_dp(const LayerArgs& a, hipStream_t s) {
    auto kern = k_layer_dp<BF, C>;
    static bool done = false;
    hipError_t e = set_lds(kern, C::LDS_BYTES, done);
    if (e != hipSuccess) return e;
    const int T = (int)(a.np / C::BM);
    hipLaunchKernelGGL(kern, dim3(T * (T + 1) / 2), dim3(C::NT), C::LDS_BYTES, s, a);
    return hipGetLastError();
}

template <bool BF, class C>
hipError_t launch_sk(const LayerArgs& a, const SplitPlan& sk, hipStream_t s) {
    auto kern = k_layer_sk<BF, C>;
    static bool done = false;
    hipError_t e = set_lds(kern, C::LDS_BYTES, done);
    if (e != hipSuccess) return e;
    // One workgroup per CU, but never more workgroups per group than the group's (tile,
    // K-block) iterations: then every range is non-empty and each tile's earlier contributors
    // all publish (sk_plan). Configurations that stage their accumulators through memory run
    // stream-K alone; the others run all but the last full round of tiles as whole tiles in a
    // data-parallel launch first (their K walks stay in step, which the L2 rewards).
    constexpr bool reg_epi = C::MB * C::NB <= 4;
    const SkGeometry G = sk_plan(a.np, C::BM, C::BK, sk.grid, reg_epi);
    SplitPlan plan = sk;
    plan.grid = G.grid;
    plan.groups = G.groups;
    plan.dp_tiles = G.dp_tiles;
    if (plan.grid < 1) return hipErrorInvalidValue;
    if constexpr (reg_epi) {
        if (plan.dp_tiles > 0) {
            auto dkern = k_layer_dp<BF, C>;
            static bool ddone = false;
            e = set_lds(dkern, C::LDS_BYTES, ddone);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(dkern, dim3(plan.dp_tiles), dim3(C::NT), C::LDS_BYTES, s, a);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    hipLaunchKernelGGL(kern, dim3(plan.grid), dim3(C::NT), C::LDS_BYTES, s, a, plan);
    return hipGetLastError();
}

}  // namespace

int split_tile_for(int streamk) {
    static_assert(CfgDP3::BM == CfgDP::BM, "the three-part split runs the data-parallel tile");
    return streamk == 1 ? CfgSK::BM : streamk == 2 ? CfgSK2::BM : CfgDP::BM;
}

SkGeometry split_sk_geometry(int64_t np, int streamk, int grid) {
    if (streamk == 1) return sk_plan(np, CfgSK::BM, CfgSK::BK, grid, CfgSK::MB * CfgSK::NB <= 4);
    return sk_plan(np, CfgSK2::BM, CfgSK2::BK, grid, CfgSK2::MB * CfgSK2::NB <= 4);
}

hipError_t launch_layer_split(const LayerArgs& a, int bf16, const SplitPlan& plan, hipStream_t s) {
    if (bf16 == 2) {   // three-part BF16 split: data-parallel schedule only
        if (plan.streamk != 0) return hipErrorInvalidValue;
        return launch_dp<true, CfgDP3>(a, s);
    }
    if (plan.streamk == 1)
        return bf16 ? launch_sk<true, CfgSK>(a, plan, s) : launch_sk<false, CfgSK>(a, plan, s);
    if (plan.streamk == 2)
        return bf16 ? launch_sk<true, CfgSK2>(a, plan, s) : launch_sk<false, CfgSK2>(a, plan, s);
    return bf16 ? launch_dp<true>(a, s) : launch_dp<false>(a, s);
}

}  // namespace fe
