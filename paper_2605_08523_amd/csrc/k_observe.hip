// Frobenius products for observables and the free energy: <A> = 2 Tr(D A) = 2 sum_ij D_ij A_ij
// for symmetric D and A (Sec. II.A, Eq. observables), and G = 2 (Tr[D H] - mu Tr D) - 2 kT S
// (Sec. III.B). One pass over D and A (bound by HBM bandwidth), FP64 accumulation, per-block
// partials reduced in a fixed order (deterministic).
#include "fe_internal.h"

namespace fe {
namespace {

constexpr int kDotThreads = 256;

__device__ inline double block_sum(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kDotThreads / 64; ++w) t += red[w];
    return t;
}

// Partial sums of D_ij A_ij over rows [b R, b R + R) for block b.
template <typename TD>
__global__ void __launch_bounds__(kDotThreads)
k_dot_rows(const TD* __restrict__ D, int64_t ldd, const double* __restrict__ A, int64_t lda,
           int64_t n, int rows, double* __restrict__ partials) {
    __shared__ double red[kDotThreads / 64];
    const int64_t r0 = (int64_t)blockIdx.x * rows;
    const int64_t r1 = r0 + rows < n ? r0 + rows : n;
    double acc = 0.0;
    for (int64_t r = r0; r < r1; ++r) {
        const TD* d = D + r * ldd;
        const double* a = A + r * lda;
        for (int64_t c = threadIdx.x; c < n; c += kDotThreads) acc += (double)d[c] * a[c];
    }
    const double t = block_sum(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// One block: sum of the partials in order. mode 0: out = 2 sum (an observable). mode 1: the
// free energy out = 2 (sum - mu trD) - 2 kT S from device scalars trD and S.
__global__ void __launch_bounds__(kDotThreads)
k_dot_final(const double* __restrict__ partials, int count, int mode, double mu, double kT,
            const double* trD, const double* S, double* out) {
    __shared__ double red[kDotThreads / 64];
    double acc = 0.0;
    // fixed assignment of partials to threads and a fixed tree: deterministic
    for (int i = threadIdx.x; i < count; i += kDotThreads) acc += partials[i];
    const double t = block_sum(acc, red);
    if (threadIdx.x == 0) *out = mode == 0 ? 2.0 * t : 2.0 * (t - mu * *trD) - 2.0 * kT * *S;
}

}  // namespace

hipError_t launch_dot(const void* D, int d_is_fp64, int64_t ldd, const double* A, int64_t lda,
                      int64_t n, double* partials, int mode, double mu, double kT,
                      const double* trD, const double* S, double* out, hipStream_t s) {
    const int rows = (int)((n + kMaxDotBlocks - 1) / kMaxDotBlocks);
    const int blocks = (int)((n + rows - 1) / rows);
    if (d_is_fp64)
        hipLaunchKernelGGL(k_dot_rows<double>, dim3(blocks), dim3(kDotThreads), 0, s,
                           static_cast<const double*>(D), ldd, A, lda, n, rows, partials);
    else
        hipLaunchKernelGGL(k_dot_rows<float>, dim3(blocks), dim3(kDotThreads), 0, s,
                           static_cast<const float*>(D), ldd, A, lda, n, rows, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(kDotThreads), 0, s, partials, blocks, mode, mu,
                       kT, trD, S, out);
    return hipGetLastError();
}

}  // namespace fe
