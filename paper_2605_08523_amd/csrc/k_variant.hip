// Kernels of the Skip-SP2 and Max-SP2 expansions (Sec. III.A: Eq. maxsp2, Alg. maxsp2-1d and the
// Skip-SP2 layer with k skips and K accumulators).
//
// Every layer of both families squares an affine combination of stored matrices. On the GPU a
// layer is two passes:
//  * k_square: Z^2 of the split operand Z = hi + lo / s by the same MFMA K loop as the MLSP2
//    layer (three 16-bit products, FP32 accumulation, upper 128 x 128 tiles), stored in FP32;
//  * k_combine: one HBM-bound pass over the upper 64 x 64 tiles that forms the next operand
//    z = diag delta_ij + sum_t w_t S_t from the stored states (x_j, accumulators), updates the
//    accumulators, and writes z as hi/lo together with its mirror tile (through LDS); in its last
//    use it forms the result f and writes D with FP64 trace partials.
// The scalar kernel evaluates the same models at sample points with a reverse-mode Jacobian
// (FP64, one lane per point) for the coefficient trainer.
#include <algorithm>

#include "fe_variant.h"
#include "split_common.h"

namespace fe {
namespace {

using namespace split;
using CfgQ = Cfg<128, 2, 2, 64, 128, 1>;

template <bool BF, class C>
__global__ void __launch_bounds__(C::NT) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_square(const uint16_t* __restrict__ hi, const uint16_t* __restrict__ lo, int64_t np,
         float* __restrict__ out) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int T = (int)(np / C::BM);
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    int I, J;
    tile_coords(t, T, I, J);
    Acc<C> acc;
#pragma unroll
    for (int mb = 0; mb < C::MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < C::NB; ++nb)
#pragma unroll
            for (int j = 0; j < 16; ++j) acc.v[mb][nb][j] = 0.0f;
    const int64_t I0 = (int64_t)I * C::BM, J0 = (int64_t)J * C::BM;
    kloop<BF, C>(hi, lo, np, I0, J0, 0, (int)(np / C::BK), acc, reinterpret_cast<uint16_t*>(smem));
    // 32x32 MFMA result layout: acc[j] of lane l is row 8(j/4) + 4(l/32) + j%4, column l%32, so
    // for each j the 64 lanes store two 128-byte row segments.
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / C::WN, wn = wave % C::WN;
    const float inv_s = BF ? 1.0f : (1.0f / 2048.0f);
    const bool diag = I == J;
#pragma unroll
    for (int mb = 0; mb < C::MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < C::NB; ++nb) {
            const int c = wn * C::WAVE_N + nb * 32 + (lane & 31);
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int r = wm * C::WAVE_M + mb * 32 + 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3);
                if (!diag || c >= r) out[(I0 + r) * np + J0 + c] = acc.v[mb][nb][j] * inv_s;
            }
        }
}

// The tiles left after the whole rounds of the data-parallel launch (a partial round would
// leave most CUs idle): tile tile0 + w / nsplit, K-blocks of segment w % nsplit, its FP32 partial
// (row-major 128 x 128) to parts[w]; k_square_reduce adds the nsplit partials of each tile in
// segment order and stores the elements on or above the diagonal.
template <bool BF, class C>
__global__ void __launch_bounds__(C::NT) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_square_part(const uint16_t* __restrict__ hi, const uint16_t* __restrict__ lo, int64_t np,
              int tile0, int nsplit, float* __restrict__ parts) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int T = (int)(np / C::BM);
    const int w = blockIdx.x;
    int I, J;
    tile_coords(tile0 + w / nsplit, T, I, J);
    const int nk = (int)(np / C::BK), sg = w % nsplit;
    const int kb0 = (int)((int64_t)sg * nk / nsplit), kb1 = (int)((int64_t)(sg + 1) * nk / nsplit);
    Acc<C> acc;
#pragma unroll
    for (int mb = 0; mb < C::MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < C::NB; ++nb)
#pragma unroll
            for (int j = 0; j < 16; ++j) acc.v[mb][nb][j] = 0.0f;
    kloop<BF, C>(hi, lo, np, (int64_t)I * C::BM, (int64_t)J * C::BM, kb0, kb1, acc,
                 reinterpret_cast<uint16_t*>(smem));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / C::WN, wn = wave % C::WN;
    const float inv_s = BF ? 1.0f : (1.0f / 2048.0f);
    float* out = parts + (size_t)w * C::BM * C::BM;
#pragma unroll
    for (int mb = 0; mb < C::MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < C::NB; ++nb) {
            const int c = wn * C::WAVE_N + nb * 32 + (lane & 31);
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int r = wm * C::WAVE_M + mb * 32 + 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3);
                out[r * C::BM + c] = acc.v[mb][nb][j] * inv_s;
            }
        }
}

// One block per 1024 elements (256 threads x 4) of a split tile: kReduceBlocks blocks per tile.
constexpr int kReduceBlocks = 128 * 128 / 1024;

template <class C>
__global__ void __launch_bounds__(256)
k_square_reduce(int64_t np, int tile0, int nsplit, const float* __restrict__ parts,
                float* __restrict__ out) {
    const int T = (int)(np / C::BM);
    const int tl = blockIdx.x / kReduceBlocks;
    int I, J;
    tile_coords(tile0 + tl, T, I, J);
    const bool diag = I == J;
    const float* p = parts + (size_t)tl * nsplit * C::BM * C::BM;
    {
        const int e = (blockIdx.x % kReduceBlocks) * 1024 + threadIdx.x * 4;
        float v[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        for (int q = 0; q < nsplit; ++q)
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] += p[(size_t)q * C::BM * C::BM + e + k];
        const int r = e / C::BM, c = e % C::BM;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (!diag || c + k >= r)
                out[((int64_t)I * C::BM + r) * np + (int64_t)J * C::BM + c + k] = v[k];
    }
}

constexpr int kCT = 64;   // combine tile
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ inline void tile_of(int t, int T, int& I, int& J) {
    I = 0;
    while (t >= T - I) {
        t -= T - I;
        ++I;
    }
    J = I + t;
}

template <bool BF>
__global__ void __launch_bounds__(256) k_combine(CombineArgs a) {
    __shared__ float sZ[kCT][kCT + 1];
    __shared__ double red[8];
    const int tid = threadIdx.x;
    const int T = (int)(a.np / kCT);
    int I, J;
    tile_of(blockIdx.x, T, I, J);
    const bool diag = I == J;
    const int64_t I0 = (int64_t)I * kCT, J0 = (int64_t)J * kCT, np = a.np, n = a.n;
    const int cg = (tid & 15) * 4;
    const bool result = a.out != 0;
    const int flip = result ? a.P->flipped : 0;
    double tr = 0.0, sq = 0.0;
#pragma unroll 1
    for (int q = 0; q < 4; ++q) {
        const int r = (tid >> 4) + 16 * q;
        const int64_t gr = I0 + r, gi = gr * np + J0 + cg;
        floatx4 z;
#pragma unroll
        for (int k = 0; k < 4; ++k) z[k] = (gr == J0 + cg + k) ? a.diag : 0.0f;
        // terms in groups of four, the group's loads issued before its FMAs (Max-SP2 reads up
        // to L + 1 states per element)
        int t = 0;
        for (; t + 4 <= a.nterm; t += 4) {
            floatx4 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = *reinterpret_cast<const floatx4*>(a.term[t + u] + gi);
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int k = 0; k < 4; ++k) z[k] = fmaf(a.w[t + u], v[u][k], z[k]);
        }
        for (; t < a.nterm; ++t) {
            const floatx4 v = *reinterpret_cast<const floatx4*>(a.term[t] + gi);
#pragma unroll
            for (int k = 0; k < 4; ++k) z[k] = fmaf(a.w[t], v[k], z[k]);
        }
        if (a.nacc > 0) {
            const floatx4 src = *reinterpret_cast<const floatx4*>(a.acc_src + gi);
            for (int l = 0; l < a.nacc; ++l) {
                floatx4 v = a.acc_first ? floatx4{0.0f, 0.0f, 0.0f, 0.0f}
                                        : *reinterpret_cast<const floatx4*>(a.acc[l] + gi);
#pragma unroll
                for (int k = 0; k < 4; ++k) v[k] = fmaf(a.g[l], src[k], v[k]);
                *reinterpret_cast<floatx4*>(a.acc[l] + gi) = v;
            }
        }
        const bool full = !diag || cg >= r;
        if (!result) {
            if (full) {
                u32x2 h, l;
                split4<BF>(z, h, l);
                *reinterpret_cast<u32x2*>(a.hi + gi) = h;
                *reinterpret_cast<u32x2*>(a.lo + gi) = l;
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if (cg + k < r) continue;
                    uint16_t h, l;
                    split16<BF>(z[k], h, l);
                    a.hi[gi + k] = h;
                    a.lo[gi + k] = l;
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int64_t gc = J0 + cg + k;
                double v = (double)z[k];
                if (flip) v = (gr == gc ? 1.0 : 0.0) - v;
                z[k] = (float)v;
                if ((!diag || cg + k >= r) && gr < n && gc < n) {
                    const double vo = (double)z[k];
                    if (gr == gc) tr += vo;
                    sq += (gr == gc ? 1.0 : 2.0) * vo * vo;
                    if (a.out_mode == 0) reinterpret_cast<float*>(a.D)[gr * a.ldd + gc] = z[k];
                    else if (a.out_mode == 1) reinterpret_cast<double*>(a.D)[gr * a.ldd + gc] = vo;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) sZ[r][cg + k] = z[k];
    }
    __syncthreads();
    // Mirror: output row J0 + c, columns I0 + rr .. rr + 3 hold z(rr .. rr + 3, c).
    if (!result || a.out_mode != 2) {
#pragma unroll 1
        for (int q = 0; q < 4; ++q) {
            const int c = (tid >> 4) + 16 * q;
            const int rr = cg;
            if (diag && rr >= c) continue;   // the mirror of a diagonal tile is its strict lower part
            floatx4 v;
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] = sZ[rr + k][c];
            const int64_t orow = J0 + c, oi = orow * np + I0 + rr;
            if (!result) {
                if (!diag || rr + 3 < c) {
                    u32x2 h, l;
                    split4<BF>(v, h, l);
                    *reinterpret_cast<u32x2*>(a.hi + oi) = h;
                    *reinterpret_cast<u32x2*>(a.lo + oi) = l;
                } else {
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        if (rr + k >= c) continue;
                        uint16_t h, l;
                        split16<BF>(v[k], h, l);
                        a.hi[oi + k] = h;
                        a.lo[oi + k] = l;
                    }
                }
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int64_t ocol = I0 + rr + k;
                    if ((diag && rr + k >= c) || orow >= n || ocol >= n) continue;
                    if (a.out_mode == 0) reinterpret_cast<float*>(a.D)[orow * a.ldd + ocol] = v[k];
                    else reinterpret_cast<double*>(a.D)[orow * a.ldd + ocol] = (double)v[k];
                }
            }
        }
    }
    if (result) {
        tr = wave_sum(tr);
        sq = wave_sum(sq);
        const int lane = tid & 63, wave = tid >> 6;
        if (lane == 0) {
            red[2 * wave] = tr;
            red[2 * wave + 1] = sq;
        }
        __syncthreads();
        if (tid == 0) {
            double t0 = 0.0, s0 = 0.0;
            for (int w = 0; w < 4; ++w) {
                t0 += red[2 * w];
                s0 += red[2 * w + 1];
            }
            a.partials[blockIdx.x].tr = t0;
            a.partials[blockIdx.x].sq = s0;
        }
    }
}

// Scalar models at one point per lane with reverse-mode derivatives (coefficient layout of
// fe_qmodel).
//  Max-SP2: s_i = delta_i + sum_{j<=i} theta_{i,j} x_j, x_{i+1} = s_i^2, f = c + sum_j gamma_j x_j.
//    xb_j = gamma_j + sum_{i>=j} sb_i theta_{i,j}, sb_i = 2 s_i xb_{i+1};
//    df/d delta_i = sb_i, df/d theta_{i,j} = sb_i x_j, df/dc = 1, df/d gamma_j = x_j.
//  Skip-SP2: s_i = alpha_c_i + sum_{j<k} alpha_{i,j} x_{i-j} + sum_l beta_{i,l} A_{i,l},
//    x_{i+1} = s_i^2, A_{i+1,l} = A_{i,l} + gamma_{i,l} x_i, A_{0,l} = a0_l,
//    f = omega x_L + sum_l A_{L,l}. Backward per layer, last first: sb_i = 2 s_i xb_{i+1};
//    the accumulator step gives df/d gamma_{i,l} = Ab_l x_i, xb_i += gamma_{i,l} Ab_l; the operand
//    gives df/d alpha_c_i = sb_i, df/d alpha_{i,j} = sb_i x_{i-j}, xb_{i-j} += sb_i alpha_{i,j},
//    df/d beta_{i,l} = sb_i A_{i,l}, Ab_l += sb_i beta_{i,l}; finally df/d a0_l = Ab_l.
__global__ void __launch_bounds__(128) k_variant_eval(VariantEvalArgs a) {
    const int kpt = blockIdx.x * blockDim.x + threadIdx.x;
    if (kpt >= a.n) return;
    const int L = a.L;
    const double* c = a.coef;
    double x[kVariantMaxL + 1], s[kVariantMaxL], xb[kVariantMaxL + 1];
    x[0] = a.y[kpt];
    double f;
    if (a.arch == 1) {
        int off = 0;
        for (int i = 0; i < L; ++i) {
            double z = c[off];
            for (int j = 0; j <= i; ++j) z += c[off + 1 + j] * x[j];
            s[i] = z;
            x[i + 1] = z * z;
            off += i + 2;
        }
        f = c[off];
        for (int j = 0; j <= L; ++j) f += c[off + 1 + j] * x[j];
        a.r[kpt] = f - (a.tgt ? a.tgt[kpt] : 0.0);
        if (!a.JT) return;
        double* JT = a.JT;
        const size_t n = a.n;
        JT[(size_t)off * n + kpt] = 1.0;
        for (int j = 0; j <= L; ++j) {
            xb[j] = c[off + 1 + j];
            JT[(size_t)(off + 1 + j) * n + kpt] = x[j];
        }
        for (int i = L - 1; i >= 0; --i) {
            off -= i + 2;
            const double sb = 2.0 * s[i] * xb[i + 1];
            JT[(size_t)off * n + kpt] = sb;
            for (int j = 0; j <= i; ++j) {
                JT[(size_t)(off + 1 + j) * n + kpt] = sb * x[j];
                xb[j] += sb * c[off + 1 + j];
            }
        }
        return;
    }
    const int k = a.k, K = a.K, per = 1 + k + 2 * K;
    double A[kVariantMaxK], Ah[kVariantMaxL][kVariantMaxK];
    for (int l = 0; l < K; ++l) A[l] = c[per * L + l];
    for (int i = 0; i < L; ++i) {
        const double* ci = c + per * i;
        double z = ci[0];
        for (int j = 0; j < k; ++j)
            if (i - j >= 0) z += ci[1 + j] * x[i - j];
        for (int l = 0; l < K; ++l) {
            z += ci[1 + k + l] * A[l];
            Ah[i][l] = A[l];
        }
        for (int l = 0; l < K; ++l) A[l] += ci[1 + k + K + l] * x[i];
        s[i] = z;
        x[i + 1] = z * z;
    }
    const double omega = c[per * L + K];
    f = omega * x[L];
    for (int l = 0; l < K; ++l) f += A[l];
    a.r[kpt] = f - (a.tgt ? a.tgt[kpt] : 0.0);
    if (!a.JT) return;
    double* JT = a.JT;
    const size_t n = a.n;
    double Ab[kVariantMaxK];
    for (int l = 0; l < K; ++l) Ab[l] = 1.0;
    for (int j = 0; j < L; ++j) xb[j] = 0.0;
    xb[L] = omega;
    JT[(size_t)(per * L + K) * n + kpt] = x[L];
    for (int i = L - 1; i >= 0; --i) {
        const double* ci = c + per * i;
        const int p0 = per * i;
        const double sb = 2.0 * s[i] * xb[i + 1];
        for (int l = 0; l < K; ++l) {
            JT[(size_t)(p0 + 1 + k + K + l) * n + kpt] = Ab[l] * x[i];
            xb[i] += ci[1 + k + K + l] * Ab[l];
        }
        JT[(size_t)p0 * n + kpt] = sb;
        for (int j = 0; j < k; ++j) {
            const bool in = i - j >= 0;
            JT[(size_t)(p0 + 1 + j) * n + kpt] = in ? sb * x[i - j] : 0.0;
            if (in) xb[i - j] += sb * ci[1 + j];
        }
        for (int l = 0; l < K; ++l) {
            JT[(size_t)(p0 + 1 + k + l) * n + kpt] = sb * Ah[i][l];
            Ab[l] += sb * ci[1 + k + l];
        }
    }
    for (int l = 0; l < K; ++l) JT[(size_t)(per * L + l) * n + kpt] = Ab[l];
}

template <class Kern>
hipError_t set_lds_once(Kern kern, size_t bytes, bool& done) {
    if (done) return hipSuccess;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess) done = true;
    return e;
}

template <bool BF>
hipError_t launch_square_t(const uint16_t* hi, const uint16_t* lo, int64_t np, float* out,
                           int slots, float* parts, hipStream_t s) {
    using C = CfgQ;
    auto kern = k_square<BF, C>;
    auto kpart = k_square_part<BF, C>;
    static bool done = false, done_p = false;
    hipError_t e = set_lds_once(kern, C::LDS_BYTES, done);
    if (e == hipSuccess) e = set_lds_once(kpart, C::LDS_BYTES, done_p);
    if (e != hipSuccess) return e;
    const int T = (int)(np / C::BM), ntiles = T * (T + 1) / 2, nk = (int)(np / C::BK);
    SquareSplit sp = square_split(ntiles, nk, slots);
    if (sp.dp > 0)
        hipLaunchKernelGGL(kern, dim3(sp.dp), dim3(C::NT), C::LDS_BYTES, s, hi, lo, np, out);
    if (sp.tail > 0) {
        hipLaunchKernelGGL(kpart, dim3(sp.tail * sp.nsplit), dim3(C::NT), C::LDS_BYTES, s, hi, lo,
                           np, sp.dp, sp.nsplit, parts);
        hipLaunchKernelGGL(k_square_reduce<C>, dim3(sp.tail * kReduceBlocks), dim3(256), 0, s, np,
                           sp.dp, sp.nsplit, (const float*)parts, out);
    }
    return hipGetLastError();
}

}  // namespace

int combine_tiles(int64_t np) {
    const int T = (int)(np / kCT);
    return T * (T + 1) / 2;
}

hipError_t launch_combine(const CombineArgs& a, hipStream_t s) {
    if (a.np % kCT != 0 || a.nterm < 0 || a.nterm > kCombineMaxTerms || a.nacc < 0 ||
        a.nacc > kCombineMaxAcc)
        return hipErrorInvalidValue;
    const int tiles = combine_tiles(a.np);
    if (a.bf16)
        hipLaunchKernelGGL(k_combine<true>, dim3(tiles), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_combine<false>, dim3(tiles), dim3(256), 0, s, a);
    return hipGetLastError();
}

SquareSplit square_split(int ntiles, int nk, int slots) {
    SquareSplit sp;
    const int rounds = slots > 0 ? ntiles / slots : 0;
    const int tail = ntiles - rounds * slots;
    if (rounds >= 1 && tail > 0 && 4 * tail <= slots) {
        sp.dp = rounds * slots;
        sp.tail = tail;
        sp.nsplit = std::min(slots / tail, nk);
    } else {
        sp.dp = ntiles;
    }
    return sp;
}

hipError_t launch_square(const uint16_t* hi, const uint16_t* lo, int64_t np, float* out, int bf16,
                         int slots, float* parts, hipStream_t s) {
    if (np % CfgQ::BM != 0) return hipErrorInvalidValue;
    return bf16 ? launch_square_t<true>(hi, lo, np, out, slots, parts, s)
                : launch_square_t<false>(hi, lo, np, out, slots, parts, s);
}

hipError_t launch_variant_eval(const VariantEvalArgs& a, hipStream_t s) {
    if (a.L < 1 || a.L > kVariantMaxL || (a.arch == 2 && (a.K < 1 || a.K > kVariantMaxK || a.k < 1 ||
                                                          a.k > kVariantMaxK)))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_variant_eval, dim3((a.n + 127) / 128), dim3(128), 0, s, a);
    return hipGetLastError();
}

}  // namespace fe
