// The whole recursion of Eq. (mlsp2) in FP64 for a matrix of padded size np <= 128, inside one
// workgroup: X lives in LDS (np x (np+1) doubles <= 129 KiB), each wave owns a set of 16 x 16
// upper-triangle blocks of X^2 (FP64 MFMA 16x16x4), and keeps the accumulator A of its blocks in
// registers across all layers. One launch runs every layer and the final output step
// (D = A + X, I - D when flipped; FP64 traces), so a small matrix costs one launch.
#include "fe_internal.h"

namespace fe {
namespace {

typedef double double4v __attribute__((ext_vector_type(4)));

constexpr int kSmallThreads = 512;   // 8 waves, two per SIMD
constexpr int kSmallWaves = kSmallThreads / 64;
constexpr int kSmallMaxNp = 128;
constexpr int kBlocksPerWave = (kSmallMaxNp / 16) * (kSmallMaxNp / 16 + 1) / 2 / kSmallWaves + 1;  // 5

__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__global__ void __launch_bounds__(kSmallThreads) k_small_f64(SmallArgs p) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    double* sX = reinterpret_cast<double*>(smem);
    const int np = (int)p.np;
    const int ld = np + 1;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nb = np / 16;                      // 16 x 16 blocks per side
    const int nblk = nb * (nb + 1) / 2;

    for (int e = tid; e < np * np; e += kSmallThreads) {
        const int i = e / np, j = e % np;
        sX[i * ld + j] = p.X0[e];
    }

    // blocks owned by this wave: wave, wave + 8, ...; (bi, bj) with bi <= bj
    int bi[kBlocksPerWave], bj[kBlocksPerWave];
#pragma unroll
    for (int s = 0; s < kBlocksPerWave; ++s) {
        int b = wave + s * kSmallWaves, i = 0;
        if (b < nblk) {
            while (b >= nb - i) {
                b -= nb - i;
                ++i;
            }
            bi[s] = i;
            bj[s] = i + b;
        } else {
            bi[s] = bj[s] = -1;
        }
    }
    __syncthreads();

    // accumulator of the owned elements: A = d0 X0
    double4v Areg[kBlocksPerWave];
    // FP64 MFMA 16x16x4 result layout: acc[i] of lane l holds D[4 i + l / 16][l % 16]
    const int lr = lane >> 4, lc = lane & 15;
#pragma unroll
    for (int s = 0; s < kBlocksPerWave; ++s) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            Areg[s][i] = 0.0;
            if (bi[s] >= 0) Areg[s][i] = p.d0 * sX[(bi[s] * 16 + 4 * i + lr) * ld + bj[s] * 16 + lc];
        }
    }

    const int ar = lane & 15, ak = lane >> 4;     // MFMA operand: row (of the 16-block), k
    for (int layer = 0; layer < p.L; ++layer) {
        const double ca = p.theta[4 * layer + 0], cb = p.theta[4 * layer + 1];
        const double cc = p.theta[4 * layer + 2];
        const double dn = (layer + 1 < p.L) ? p.theta[4 * (layer + 1) + 3] : 0.0;
        double4v acc[kBlocksPerWave];
#pragma unroll
        for (int s = 0; s < kBlocksPerWave; ++s) acc[s] = (double4v){0.0, 0.0, 0.0, 0.0};
        for (int k0 = 0; k0 < np; k0 += 4) {
#pragma unroll
            for (int s = 0; s < kBlocksPerWave; ++s) {
                if (bi[s] >= 0) {
                    const double a = sX[(bi[s] * 16 + ar) * ld + k0 + ak];
                    const double b = sX[(bj[s] * 16 + ar) * ld + k0 + ak];
                    acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[s], 0, 0, 0);
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < kBlocksPerWave; ++s) {
            if (bi[s] < 0) continue;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = bi[s] * 16 + 4 * i + lr, c = bj[s] * 16 + lc;
                if (r > c) continue;
                const double x = sX[r * ld + c];
                const double xn = ca * acc[s][i] + cb * x + (r == c ? cc : 0.0);
                Areg[s][i] += dn * xn;
                sX[r * ld + c] = xn;
                sX[c * ld + r] = xn;
            }
        }
        __syncthreads();
    }

    // output: D = A + X (I - D if flipped), traces in FP64
    const int flip = (!p.entropy) ? p.P->flipped : 0;
    double tr = 0.0, sq = 0.0;
#pragma unroll
    for (int s = 0; s < kBlocksPerWave; ++s) {
        if (bi[s] < 0) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = bi[s] * 16 + 4 * i + lr, c = bj[s] * 16 + lc;
            if (r > c || r >= p.n || c >= p.n) continue;
            double v = Areg[s][i] + sX[r * ld + c];
            if (flip) v = (r == c ? 1.0 : 0.0) - v;
            if (!p.entropy && p.out_mode == 0) v = (double)(float)v;
            if (r == c) tr += v;
            sq += (r == c ? 1.0 : 2.0) * v * v;
            if (!p.entropy) {
                if (p.out_mode == 0) {
                    float* D = reinterpret_cast<float*>(p.D);
                    D[(int64_t)r * p.ldd + c] = (float)v;
                    D[(int64_t)c * p.ldd + r] = (float)v;
                } else if (p.out_mode == 1) {
                    double* D = reinterpret_cast<double*>(p.D);
                    D[(int64_t)r * p.ldd + c] = v;
                    D[(int64_t)c * p.ldd + r] = v;
                }
            }
        }
    }
    tr = wave_sum(tr);
    sq = wave_sum(sq);
    __syncthreads();
    double* red = sX;
    if (lane == 0) {
        red[2 * wave] = tr;
        red[2 * wave + 1] = sq;
    }
    __syncthreads();
    if (tid == 0) {
        double t = 0.0, q = 0.0;
        for (int w = 0; w < kSmallWaves; ++w) {
            t += red[2 * w];
            q += red[2 * w + 1];
        }
        p.partials[0].tr = t;
        p.partials[0].sq = q;
    }
}

}  // namespace

int small_f64_max_np() { return kSmallMaxNp; }

hipError_t launch_small_f64(const SmallArgs& a, hipStream_t s) {
    if (a.np > kSmallMaxNp || a.np % 16 != 0) return hipErrorInvalidValue;
    const size_t lds = (size_t)a.np * (a.np + 1) * sizeof(double);
    static bool attr_done = false;
    if (!attr_done) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_small_f64),
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)((size_t)kSmallMaxNp * (kSmallMaxNp + 1) * sizeof(double)));
        if (e != hipSuccess) return e;
        attr_done = true;
    }
    hipLaunchKernelGGL(k_small_f64, dim3(1), dim3(kSmallThreads), lds, s, a);
    return hipGetLastError();
}

}  // namespace fe
