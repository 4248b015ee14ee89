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
//    a Y + b X + c delta_ij, updates A with the next layer's d and writes the master and the next
//    hi/lo; a transposed pass writes the mirror tile. The last layer writes D and FP64 traces.
//  * Two schedules:
//      data-parallel: one workgroup per upper tile (128 x 128, four 64 x 64 wave tiles), used when
//        the matrix is small;
//      stream-K: one persistent workgroup per CU (256 x 256 tiles, four 128 x 128 wave tiles,
//        double-buffered LDS); the (tile, K-block) iterations are split evenly. Every segment
//        stores its FP32 partial tile to memory (so the 256 accumulator registers die right after
//        the K loop): a workgroup that stops inside a tile publishes it, the workgroup that
//        finishes the tile runs the epilogue from memory, adding the earlier workgroups' partials
//        in a fixed order. A workgroup only ever waits for workgroups with smaller ids, which were
//        dispatched earlier, and every wait is bounded.
#include "split_common.h"

namespace fe {
namespace {

using namespace split;

using CfgDP = Cfg<128, 2, 2, 32, 64, 1>;
using CfgSK = Cfg<256, 2, 2, 32, 128, 2>;

constexpr int kSpinLimit = 1 << 22;   // ~0.2 s of s_sleep before a wait gives up

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
    int I, J;
    tile_coords(blockIdx.x, T, I, J);
    Acc<C> acc;
    zero(acc);
    kloop<BF, C>(p.hi_in, p.lo_in, p.np, (int64_t)I * C::BM, (int64_t)J * C::BM, 0,
                 (int)(p.np / C::BK), acc, reinterpret_cast<uint16_t*>(smem));
    epilogue<BF, C>(p, acc, reinterpret_cast<float*>(smem), I, J, blockIdx.x);
}

template <bool BF, class C>
__global__ void __launch_bounds__(C::NT) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_layer_sk(LayerArgs p, SplitPlan sk) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int tid = threadIdx.x;
    const int w = blockIdx.x, G = sk.grid;
    const int T = (int)(p.np / C::BM);
    const int ntiles = T * (T + 1) / 2;
    const int nk = (int)(p.np / C::BK);
    const int64_t total = (int64_t)ntiles * nk;
    const int64_t a_w = total * w / G, b_w = total * (w + 1) / G;
    constexpr size_t TILE = (size_t)C::BM * C::BM;
    float* own = sk.own + (size_t)w * TILE;
    float* pub = sk.partial + (size_t)w * TILE;

    // Segments of [a_w, b_w): if the range stops inside its last tile, that tail segment is
    // computed and published first, so that the workgroup finishing that tile never waits behind
    // this workgroup's own waits (no chains of waits across the grid). Then the remaining
    // segments, each of which finishes a tile, in order.
    const int t_last = (int)((b_w - 1) / nk);
    const int64_t tail_start = (int64_t)t_last * nk > a_w ? (int64_t)t_last * nk : a_w;
    const bool publishes = b_w < (int64_t)(t_last + 1) * nk;
    const int64_t own_end = publishes ? tail_start : b_w;
    for (int pass = publishes ? 0 : 1; pass < 2; ++pass) {
        int64_t it = pass == 0 ? tail_start : a_w;
        const int64_t stop = pass == 0 ? b_w : own_end;
        while (it < stop) {
            const int t = (int)(it / nk);
            const int kb0 = (int)(it - (int64_t)t * nk);
            const int64_t rest = stop - it;
            const int kb1 = (int)((int64_t)kb0 + rest < nk ? kb0 + rest : nk);
            int I, J;
            tile_coords(t, T, I, J);
            {
                Acc<C> acc;
                zero(acc);
                kloop<BF, C>(p.hi_in, p.lo_in, p.np, (int64_t)I * C::BM, (int64_t)J * C::BM, kb0,
                             kb1, acc, reinterpret_cast<uint16_t*>(smem));
                // The accumulators leave registers here: the published partial of the tile this
                // workgroup stops inside, or its own share of a tile it finishes.
                store_tile<BF, C>(acc, pass == 0 ? pub : own);
            }
            if (pass == 0) {
                __threadfence();
                __syncthreads();
                if (tid == 0)
                    __hip_atomic_store(sk.flags + w, sk.epoch, __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_AGENT);
            } else {
                // Earlier workgroups wlo..w-1 hold the first kb0 blocks of this tile; their
                // partial slots are contiguous. Wait for all of them; the epilogue adds them in a
                // fixed order, so the result does not depend on timing.
                int wlo = w;
                if (kb0 > 0) {
                    while (wlo > 0 && total * wlo / G > (int64_t)t * nk) --wlo;
                    if (tid == 0) {
                        // every workgroup wlo..w-1 has a non-empty range inside this tile (the
                        // grid never exceeds the iteration count), so each publishes exactly once
                        bool gave_up = false;
                        for (int wp = wlo; wp < w && !gave_up; ++wp) {
                            int spins = 0;
                            while (__hip_atomic_load(sk.flags + wp, __ATOMIC_ACQUIRE,
                                                     __HIP_MEMORY_SCOPE_AGENT) != sk.epoch) {
                                if (++spins > kSpinLimit) {
                                    atomicOr(sk.err, 1);
                                    gave_up = true;
                                    break;
                                }
                                __builtin_amdgcn_s_sleep(2);
                            }
                        }
                    }
                }
                __syncthreads();
                if (kb0 > 0) __threadfence();
                epilogue_mem<BF, C>(p, own, sk.partial + (size_t)wlo * TILE, w - wlo,
                                    reinterpret_cast<float*>(smem), I, J, t);
            }
            it += kb1 - kb0;
        }
    }
}

template <class K>
hipError_t set_lds(K kern, size_t bytes, bool& done) {
    if (done) return hipSuccess;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess) done = true;
    return e;
}

template <bool BF>
hipError_t launch_dp(const LayerArgs& a, hipStream_t s) {
    using C = CfgDP;
    auto kern = k_layer_dp<BF, C>;
    static bool done = false;
    hipError_t e = set_lds(kern, C::LDS_BYTES, done);
    if (e != hipSuccess) return e;
    const int T = (int)(a.np / C::BM);
    hipLaunchKernelGGL(kern, dim3(T * (T + 1) / 2), dim3(C::NT), C::LDS_BYTES, s, a);
    return hipGetLastError();
}

template <bool BF>
hipError_t launch_sk(const LayerArgs& a, const SplitPlan& sk, hipStream_t s) {
    using C = CfgSK;
    auto kern = k_layer_sk<BF, C>;
    static bool done = false;
    hipError_t e = set_lds(kern, C::LDS_BYTES, done);
    if (e != hipSuccess) return e;
    // One workgroup per CU, but never more workgroups than (tile, K-block) iterations: then
    // every workgroup's range is non-empty and each tile's earlier contributors all publish.
    const int64_t T = a.np / C::BM;
    const int64_t total = T * (T + 1) / 2 * (a.np / C::BK);
    SplitPlan plan = sk;
    if (plan.grid > total) plan.grid = (int)total;
    if (plan.grid < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(kern, dim3(plan.grid), dim3(C::NT), C::LDS_BYTES, s, a, plan);
    return hipGetLastError();
}

}  // namespace

int split_tile_for(int streamk) { return streamk ? CfgSK::BM : CfgDP::BM; }

hipError_t launch_layer_split(const LayerArgs& a, int bf16, const SplitPlan& plan, hipStream_t s) {
    if (plan.streamk) return bf16 ? launch_sk<true>(a, plan, s) : launch_sk<false>(a, plan, s);
    return bf16 ? launch_dp<true>(a, s) : launch_dp<false>(a, s);
}

}  // namespace fe
