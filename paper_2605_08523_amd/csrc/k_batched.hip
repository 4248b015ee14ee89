// Batched expansion of many Hamiltonians of uneven size (Alg. 2 applied to each matrix of a
// batch): batched Gershgorin bounds and rescale parameters, batched rescale/split, one grouped
// launch per layer covering every upper tile of every matrix, and per-matrix trace reductions.
// Matrices are padded to multiples of the tile; the padding is zero off the diagonal, is never
// rewritten (so X stays block diagonal) and is masked out of D and the traces.
#include <math.h>

#include <algorithm>
#include <vector>

#include "batch_queue.h"
#include "split_common.h"

namespace fe {
namespace {

using namespace split;
// 128 x 128 tiles over eight waves of 32 x 64 (four waves per SIMD with two workgroups per CU):
// each workgroup's K loop here is short (2 to 12 blocks) and waits on its loads more than on the
// MFMA pipes, so more waves per CU hide more of that latency (1.08x over four waves of 64 x 64
// on the batch of 1024); the epilogue keeps two groups of loads in flight per thread (register
// budget of four waves per SIMD).
using CfgB = Cfg<128, 4, 2, 64, 128, 1>;
constexpr int kBatchEpiGroups = 2;
// 64 x 64 tiles (32 x 32 per wave): less padding for small N. Three waves per SIMD (the 128 x 128
// tile: four): at four its code spills ~10 registers, and three run small-matrix batches 4-6%
// faster.
using CfgB64 = Cfg<64, 2, 2, 32, 64, 1>;
// Three-part BF16 split: the same 128 x 128 tile and eight waves, six panels of 32-deep K-blocks
// in one LDS stage.
using CfgB3 = Cfg<128, 4, 2, 32, 128, 1, 0, 3>;

__device__ inline double wsum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline double wmin(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline double wmax(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// One workgroup of 16 waves per matrix: Gershgorin bounds (one wave per row, each row summed in
// the same order as the single-matrix prologue, so both give the same bounds) and the rescale
// parameters of Sec. IV.1.
constexpr int kBoundsWaves = 16;
__global__ void __launch_bounds__(kBoundsWaves * 64)
k_batch_bounds(const BatchMat* mats, int count, Params* P) {
    const int b = blockIdx.x;
    if (b >= count) return;
    const BatchMat m = mats[b];
    const double beta0 = m.beta0, mu0 = m.mu0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double lo = INFINITY, hi = -INFINITY;
    int bad = 0;
    for (int64_t i = wave; i < m.n; i += kBoundsWaves) {
        const double* row = m.H + i * m.ldh;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int64_t j = lane;
        for (; j + 192 < m.n; j += 256) {
            s0 += fabs(row[j]);
            s1 += fabs(row[j + 64]);
            s2 += fabs(row[j + 128]);
            s3 += fabs(row[j + 192]);
        }
        for (; j < m.n; j += 64) s0 += fabs(row[j]);
        const double s = wsum((s0 + s1) + (s2 + s3));
        const double d = row[i];
        const double r = s - fabs(d);
        if (!isfinite(s)) bad = 1;
        lo = fmin(lo, d - r);
        hi = fmax(hi, d + r);
    }
    __shared__ double slo[kBoundsWaves], shi[kBoundsWaves];
    __shared__ int sbad[kBoundsWaves];
    if (lane == 0) {
        slo[wave] = lo;
        shi[wave] = hi;
        sbad[wave] = bad;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int w = 1; w < kBoundsWaves; ++w) {
        lo = fmin(lo, slo[w]);
        hi = fmax(hi, shi[w]);
        bad |= sbad[w];
    }
    const double mu = m.mu, kT = m.kT;
    Params p;
    p.emin = lo;
    p.emax = hi;
    p.flipped = p.clamped = p.degenerate = 0;
    p.status = FE_OK;
    const double width = hi - lo;
    if (bad || !isfinite(lo) || !isfinite(hi)) {
        p.status = FE_ERR_NONFINITE;
        p.mu_p = p.beta_p = p.beta_max = p.scale = p.shift = NAN;
    } else if (!(kT > 0.0)) {
        p.status = FE_ERR_DOMAIN;
        p.mu_p = p.beta_p = p.beta_max = p.scale = p.shift = NAN;
    } else if (width <= 1e-300 * fmax(1.0, fabs(hi))) {
        double y = mu0 + (mu - lo) / (kT * beta0);
        p.degenerate = 1;
        if (!(y >= 0.0 && y <= 1.0)) {
            p.clamped = 1;
            y = fmin(1.0, fmax(0.0, y));
        }
        p.mu_p = NAN;
        p.beta_p = INFINITY;
        p.beta_max = NAN;
        p.scale = 0.0;
        p.shift = y;
    } else if (!(lo < mu && mu < hi)) {
        p.status = FE_ERR_DOMAIN;
        p.mu_p = p.beta_p = p.beta_max = p.scale = p.shift = NAN;
    } else {
        double mu_p = (hi - mu) / width;
        double beta_p = width / kT;
        const int flip = mu_p > 0.5;
        if (flip) mu_p = 1.0 - mu_p;
        const double bmax = fmin(mu0 / mu_p, (1.0 - mu0) / (1.0 - mu_p)) * beta0;
        if (beta_p > bmax) {
            beta_p = bmax;
            p.clamped = 1;
            p.status = FE_WARN_BETA_CLAMPED;
        }
        const double r = beta_p / beta0;
        p.scale = flip ? r / width : -r / width;
        p.shift = flip ? r * (-lo / width - mu_p) + mu0 : r * (hi / width - mu_p) + mu0;
        p.mu_p = mu_p;
        p.beta_p = beta_p;
        p.beta_max = bmax;
        p.flipped = flip;
    }
    P[b] = p;
}

// Rescale and split of every matrix: blockIdx.y selects the matrix, blockIdx.x a chunk; four
// consecutive columns per thread (16-byte stores; np is a multiple of the tile), the same
// per-element arithmetic as the single-matrix rescale.
template <bool BF>
__global__ void __launch_bounds__(256)
k_batch_rescale(const BatchMat* mats, int count, const Params* P, double alpha, BatchCoef cf,
                int three) {
    const int b = blockIdx.y;
    if (b >= count) return;
    const BatchMat m = mats[b];
    const double mu0 = m.mu0;
    const float d0 = cf.d0[m.model];
    const double s0 = cf.shift0[m.model];
    const double scale = P[b].scale, shift = P[b].shift;
    const uint32_t qrow = (uint32_t)(m.np / 4), quads = (uint32_t)(m.np * m.np / 4);
    for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < quads; q += gridDim.x * blockDim.x) {
        const uint32_t i = q / qrow, j0 = 4 * (q - i * qrow);
        const int64_t e0 = (int64_t)i * m.np + j0;
        double x[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t j = j0 + k;
            x[k] = 0.0;
            if (i < m.n && j < m.n) {
                double v = scale * m.H[i * m.ldh + j] + (i == j ? shift : 0.0);
                x[k] = alpha * v + (i == j ? (1.0 - alpha) * mu0 : 0.0);
            }
        }
        floatx4 xf, af;
        uint16_t h[4], l[4], md[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            xf[k] = (float)x[k];
            af[k] = d0 * xf[k];
            const float xs = i == j0 + k ? (float)(x[k] + s0) : xf[k];
            if (three) split3(xs, h[k], md[k], l[k]);
            else split16<BF>(xs, h[k], l[k]);
        }
        *reinterpret_cast<floatx4*>(m.X + e0) = xf;
        *reinterpret_cast<floatx4*>(m.A + e0) = af;
        auto pack = [](const uint16_t* v) {
            return u32x2{(uint32_t)v[0] | ((uint32_t)v[1] << 16), (uint32_t)v[2] | ((uint32_t)v[3] << 16)};
        };
        *reinterpret_cast<u32x2*>(m.hi[0] + e0) = pack(h);
        *reinterpret_cast<u32x2*>(m.lo[0] + e0) = pack(l);
        if (three) *reinterpret_cast<u32x2*>(m.mid[0] + e0) = pack(md);
        // the other buffer's padding too (no epilogue writes it)
        if (i >= m.n || j0 + 3 >= m.n) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (i < m.n && j0 + k < m.n) continue;
                m.hi[1][e0 + k] = h[k];
                m.lo[1][e0 + k] = l[k];
                if (three) m.mid[1][e0 + k] = md[k];
            }
        }
    }
}

// Layer `layer` of upper tile t of matrix `lo`: the same K loop and fused epilogue as the
// single-matrix kernel. poisoned: the tile's inputs could not be waited for (queue launch);
// its outputs are NaN.
// mats, Ls, coef: q.mats, q.cf.L and q.cf.coef, which the queue kernel passes as separate
// no-alias arguments: its atomics precede these loads, and only with the arguments' no-alias
// guarantee does the compiler know them unwritten and load them into scalar registers (else the
// descriptors take vector registers throughout the tile's code, which then spills).
template <bool BF, class C>
__device__ __attribute__((always_inline)) inline void batch_tile(
    const BatchLayerArgs& q, const BatchMat* __restrict__ mats, const int32_t* __restrict__ Ls,
    const float* __restrict__ coef, int lo, int t, int layer, bool poisoned, unsigned char* smem) {
    const BatchMat& m = mats[lo];
    const int L = Ls[m.model];
    const float* cf = coef + ((size_t)m.model * q.cf.max_L + layer) * 8;
    const int T = (int)(m.np / C::BM);
    const int parity = layer & 1;
    int I, J;
    tile_coords(t, T, I, J);
    LayerArgs p;
    p.np = m.np;
    p.n = m.n;
    p.hi_in = m.hi[parity];
    p.lo_in = m.lo[parity];
    p.hi_out = m.hi[parity ^ 1];
    p.lo_out = m.lo[parity ^ 1];
    p.mid_in = m.mid[parity];
    p.mid_out = m.mid[parity ^ 1];
    p.X = m.X;
    p.A = m.A;
    p.a = cf[0];
    p.b = cf[1];
    p.c = cf[2];
    p.d_old = cf[3];
    p.d_new = cf[4];
    p.affine = cf[5] != 0.0f;
    p.last = layer == L - 1;
    p.entropy = q.entropy;
    p.D = m.D;
    p.ldd = m.ldd;
    p.out_mode = q.entropy ? 2 : (m.D ? (m.d_is_fp64 ? 1 : 0) : 2);
    p.P = q.P + lo;
    p.partials = q.partials + m.tile0;
    Acc<C> acc;
#pragma unroll
    for (int mb = 0; mb < C::MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < C::NB; ++nb)
#pragma unroll
            for (int j = 0; j < 16; ++j) acc.v[mb][nb][j] = 0.0f;
    // K-blocks wholly in the padding add only zero products to the real block (X is block
    // diagonal there), and the padded part of the tile is not stored: they are skipped.
    const int kend = (int)((p.n + C::BK - 1) / C::BK);
    if constexpr (C::NS == 3)
        kloop3<C>(p.hi_in, p.mid_in, p.lo_in, p.np, (int64_t)I * C::BM, (int64_t)J * C::BM, 0, kend,
                  acc, reinterpret_cast<uint16_t*>(smem));
    else
        kloop<BF, C>(p.hi_in, p.lo_in, p.np, (int64_t)I * C::BM, (int64_t)J * C::BM, 0, kend, acc,
                     reinterpret_cast<uint16_t*>(smem));
    epilogue<BF, C, C::BM == 128 ? kBatchEpiGroups : 8>(p, acc, reinterpret_cast<float*>(smem), I, J,
                                                        t, nullptr, 0, 0, poisoned);
}

// One layer for every upper tile of every matrix. Workgroup g takes the (matrix, tile) of its slot
// in the plan's map, which keeps all tiles of a matrix on one XCD (the hardware deals consecutive
// workgroups to consecutive XCDs, so workgroups g and g + 8 share one), so the matrix's operand
// panels are fetched into one L2 instead of eight; without
// a map it finds its matrix by binary search over the tile prefix sums.
template <bool BF, class C>
__global__ void __launch_bounds__(C::NT)
__attribute__((amdgpu_waves_per_eu(C::BM == 128 ? 4 : 3, C::BM == 128 ? 4 : 3)))
k_batch_layer(BatchLayerArgs q) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int g = blockIdx.x;
    int lo, t;
    if (q.map) {
        lo = q.map[2 * g];
        t = q.map[2 * g + 1];
        if (lo < 0) return;   // an empty slot; whole workgroup leaves
    } else {
        lo = 0;
        int hi = q.count - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (q.mats[mid].tile0 <= g) lo = mid;
            else hi = mid - 1;
        }
        t = g - q.mats[lo].tile0;
    }
    if (q.layer >= q.cf.L[q.mats[lo].model]) return;   // not launched for such matrices
    batch_tile<BF, C>(q, q.mats, q.cf.L, q.cf.coef, lo, t, q.layer, false, smem);
}

// Every layer of every matrix of a pass in one launch (the queue protocol is described with
// BatchQueue): each workgroup takes the next ticket of its XCD's queue, waits until the item's
// matrix has completed its previous layer, computes the item, and once every wave's stores of it
// have completed counts it done. The wait is bounded: one that gives up marks the matrix and
// raises the abort flag, after which no wait blocks; such an item is computed with NaN outputs.
// Workgroups beyond their queue's length leave at once.
template <bool BF, class C>
__global__ void __launch_bounds__(C::NT)
__attribute__((amdgpu_waves_per_eu(C::BM == 128 ? 4 : 3, C::BM == 128 ? 4 : 3)))
k_batch_queue(BatchLayerArgs q, BatchQueue Q, const BatchMat* __restrict__ mats,
              const int32_t* __restrict__ Ls, const float* __restrict__ coef) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    __shared__ int4 s_item;
    __shared__ int s_gave_up;
    if (threadIdx.x == 0) {
        int x;
        asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID, 0, 4)" : "=s"(x));
        int4 it = make_int4(-1, 0, 0, 0);   // none: no queue for this XCD (the completion check
                                            // reports the matrices), or the queue is exhausted
        if (x < Q.nq) {
            const int q0 = Q.qoff[x], total = Q.qoff[x + 1] - q0;
            const int k = __hip_atomic_fetch_add(Q.ticket + x, 1, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
            if (k < total) it = Q.items[q0 + k];
        }
        int gave_up = 0;
        if (it.x >= 0) {
            int32_t* const abort_flag = Q.err + q.count;
            int spins = 0, backoff = 1;
            const int need = it.w + Q.need_offset;
            while (__hip_atomic_load(Q.done + it.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                   need) {
                if (++spins > Q.spin_limit ||
                    __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    __hip_atomic_store(Q.err + it.x, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    gave_up = 1;
                    break;
                }
                // Back off (up to ~16 x 512 clocks between polls): where most workgroups wait
                // (small batches), tight polling of a few counters slows the producers' updates.
                for (int k = 0; k < backoff; ++k) __builtin_amdgcn_s_sleep(8);
                if (backoff < 16) backoff *= 2;
            }
        }
        s_item = it;
        s_gave_up = gave_up;
    }
    // Lines of the matrix that this CU's L1 holds from before its producers' stores are stale:
    // wave 0 invalidates the L1 and waits for that before the barrier, after which every wave
    // loads. The invalidate takes agent scope: the workgroup-scope one leaves the L1 alone when a
    // workgroup's waves share one CU (measured: it does not stop stale reads here).
    if (threadIdx.x < 64) asm volatile("buffer_inv sc1\n\ts_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    const int mat = __builtin_amdgcn_readfirstlane(s_item.x);
    if (mat < 0) return;   // nothing to do; whole workgroup leaves
    const int t = __builtin_amdgcn_readfirstlane(s_item.y);
    const int layer = __builtin_amdgcn_readfirstlane(s_item.z);
    const bool gave_up = __builtin_amdgcn_readfirstlane(s_gave_up) != 0;
    batch_tile<BF, C>(q, mats, Ls, coef, mat, t, layer, gave_up, smem);
    // This wave's stores of the item have completed (in the XCD's L2). The memory clobber keeps
    // the compiler from sinking any of them below the wait.
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x == 0)
        __hip_atomic_fetch_add(Q.done + mat, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// XCD of workgroup b (one wave each), for the check that the queue launch's assumptions hold.
__global__ void __launch_bounds__(64) k_xcc_probe(int32_t* out, int n) {
    if (threadIdx.x != 0 || (int)blockIdx.x >= n) return;
    int x;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID, 0, 4)" : "=s"(x));
    out[blockIdx.x] = x;
}

__global__ void __launch_bounds__(256) k_batch_queue_reset(int32_t* p, int64_t n) {
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = 0;
}

__global__ void __launch_bounds__(256)
k_batch_queue_check(const BatchMat* mats, int count, BatchQueue Q, BatchCoef cf, Params* P,
                    int tile) {
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= count) return;
    const BatchMat& m = mats[b];
    const int64_t T = m.np / tile;
    const int64_t want = (int64_t)cf.L[m.model] * (T * (T + 1) / 2);
    if ((Q.done[b] != want || Q.err[b] != 0) && P[b].status >= 0) P[b].status = FE_ERR_HIP;
}

// Per-matrix fixed-order reduction of the tile traces into Tr, sum of squares, and S (entropy).
__global__ void __launch_bounds__(64)
k_batch_reduce(const BatchMat* mats, int count, const TracePartial* partials, const Params* P,
               int entropy, int32_t* status, int tile) {
    const int b = blockIdx.x;
    if (b >= count) return;
    const BatchMat m = mats[b];
    const int T = (int)(m.np / tile);
    const int nt = T * (T + 1) / 2;
    double tr = 0.0, sq = 0.0;
    for (int k = threadIdx.x; k < nt; k += 64) {
        tr += partials[m.tile0 + k].tr;
        sq += partials[m.tile0 + k].sq;
    }
    tr = wsum(tr);
    sq = wsum(sq);
    if (threadIdx.x == 0) {
        const double bad = P[b].status < 0 ? NAN : 0.0;
        if (entropy) {
            if (m.S) *m.S = 4.0 * 0.69314718055994530942 * (tr - sq) + bad;
        } else {
            if (m.trD) *m.trD = tr + bad;
            if (m.trD2) *m.trD2 = sq + bad;
        }
        if (status && (!entropy || P[b].status < 0)) status[m.item] = P[b].status;
    }
}

}  // namespace

hipError_t launch_batch_bounds(const BatchMat* mats, int count, Params* P, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_bounds, dim3(count), dim3(kBoundsWaves * 64), 0, s, mats, count, P);
    return hipGetLastError();
}

hipError_t launch_batch_rescale(const BatchMat* mats, int count, int64_t max_np, const Params* P,
                                double alpha, BatchCoef cf, int bf16, hipStream_t s) {
    int chunks = (int)((max_np * max_np / 4 + 1023) / 1024);
    if (chunks < 1) chunks = 1;
    if (chunks > 64) chunks = 64;
    dim3 grid(chunks, count);
    if (bf16)
        hipLaunchKernelGGL(k_batch_rescale<true>, grid, dim3(256), 0, s, mats, count, P, alpha, cf,
                           bf16 == 2 ? 1 : 0);
    else
        hipLaunchKernelGGL(k_batch_rescale<false>, grid, dim3(256), 0, s, mats, count, P, alpha, cf, 0);
    return hipGetLastError();
}

template <bool BF, class C>
hipError_t launch_layer_t(const BatchLayerArgs& q, int grid, hipStream_t s) {
    auto kern = k_batch_layer<BF, C>;
    static bool done = false;
    if (!done) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)C::LDS_BYTES);
        if (e != hipSuccess) return e;
        done = true;
    }
    hipLaunchKernelGGL(kern, dim3(grid), dim3(C::NT), C::LDS_BYTES, s, q);
    return hipGetLastError();
}

hipError_t launch_batch_layer(const BatchLayerArgs& q, int grid, int bf16, int tile,
                              hipStream_t s) {
    if (grid < 1) return hipErrorInvalidValue;
    if (bf16 == 2)   // three-part BF16 split: 128 x 128 tiles only
        return tile == 128 ? launch_layer_t<true, CfgB3>(q, grid, s) : hipErrorInvalidValue;
    if (tile == 64)
        return bf16 ? launch_layer_t<true, CfgB64>(q, grid, s)
                    : launch_layer_t<false, CfgB64>(q, grid, s);
    if (tile != 128) return hipErrorInvalidValue;
    return bf16 ? launch_layer_t<true, CfgB>(q, grid, s)
                : launch_layer_t<false, CfgB>(q, grid, s);
}

template <bool BF, class C>
hipError_t queue_t(const BatchLayerArgs& q, const BatchQueue& Q, int64_t grid, hipStream_t s) {
    auto kern = k_batch_queue<BF, C>;
    static bool done = false;
    if (!done) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)C::LDS_BYTES);
        if (e != hipSuccess) return e;
        done = true;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(C::NT), C::LDS_BYTES, s, q, Q, q.mats,
                       q.cf.L, q.cf.coef);
    return hipGetLastError();
}

hipError_t launch_batch_queue_reset(const BatchQueue& Q, int count, hipStream_t s) {
    const int64_t n = batch_queue_counters(Q.nq, count);
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 256);
    hipLaunchKernelGGL(k_batch_queue_reset, dim3(blocks), dim3(256), 0, s, Q.ticket, n);
    return hipGetLastError();
}

hipError_t launch_batch_queue(const BatchLayerArgs& q, const BatchQueue& Q, int64_t grid, int bf16,
                              int tile, hipStream_t s) {
    if (grid < 1 || grid > 0x7fffffff) return hipErrorInvalidValue;
    if (bf16 == 2) return tile == 128 ? queue_t<true, CfgB3>(q, Q, grid, s) : hipErrorInvalidValue;
    if (tile == 64)
        return bf16 ? queue_t<true, CfgB64>(q, Q, grid, s) : queue_t<false, CfgB64>(q, Q, grid, s);
    if (tile != 128) return hipErrorInvalidValue;
    return bf16 ? queue_t<true, CfgB>(q, Q, grid, s) : queue_t<false, CfgB>(q, Q, grid, s);
}

hipError_t batch_queue_probe(int nq, bool* ok) {
    *ok = false;
    if (nq < 1 || nq > 16) return hipSuccess;
    const int n = 64 * nq;
    int32_t* d = nullptr;
    hipError_t e = hipMalloc(&d, n * sizeof(int32_t));
    if (e != hipSuccess) return e;
    std::vector<int32_t> h(n, -1);
    hipLaunchKernelGGL(k_xcc_probe, dim3(n), dim3(64), 0, nullptr, d, n);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpy(h.data(), d, n * sizeof(int32_t), hipMemcpyDeviceToHost);
    (void)hipFree(d);
    if (e != hipSuccess) return e;
    // round-robin from whichever XCD the dispatcher's pointer is at (it carries over from the
    // previous dispatch: measured starts at XCD 0 and at XCD 7)
    bool good = h[0] >= 0 && h[0] < nq;
    for (int b = 0; b < n; ++b) good = good && h[b] == (h[0] + b) % nq;
    *ok = good;
    return hipSuccess;
}

hipError_t launch_batch_queue_check(const BatchMat* mats, int count, const BatchQueue& Q,
                                    BatchCoef cf, Params* P, int tile, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_queue_check, dim3((count + 255) / 256), dim3(256), 0, s, mats, count,
                       Q, cf, P, tile);
    return hipGetLastError();
}

hipError_t launch_batch_reduce(const BatchMat* mats, int count, const TracePartial* partials,
                               const Params* P, int entropy, int32_t* status, int tile,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_batch_reduce, dim3(count), dim3(64), 0, s, mats, count, partials, P,
                       entropy, status, tile);
    return hipGetLastError();
}

}  // namespace fe
