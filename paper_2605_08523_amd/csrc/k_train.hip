// Device kernels of the coefficient trainer (Sec. III.C):
//  * the scalar model at sample points (Eq. mlsp2; for the entropy target Eq. entropy expansion
//    and its output layer), the residuals against the target values and the Jacobian with
//    respect to the 4L coefficients by reverse-mode differentiation, FP64, one lane per point;
//  * Gram products J^T J and J^T v for the Levenberg-Marquardt normal equations;
//  * the elementwise part of the backward pass of the FP32 matrix recursion.
#include <math.h>

#include "fe_internal.h"

namespace fe {
namespace {

// Reverse mode through the layers for one point: forward x_0..x_L (kept per lane), output
// u = A_L + x_L with A_L = sum_i d_i x_i; adjoint xb_L = 1, xb_i = d_i + xb_{i+1}(2 a_i x_i + b_i);
// du/da_i = xb_{i+1} x_i^2, du/db_i = xb_{i+1} x_i, du/dc_i = xb_{i+1}, du/dd_i = x_i.
// Entropy target: s = 4 ln2 u (1 - u), ds = 4 ln2 (1 - 2u) du.
__global__ void __launch_bounds__(256)
k_scalar_eval(ScalarArgs a) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    const int L = a.L;
    const double y = a.y[k];
    double x = a.target == 1 ? a.alpha * (y - a.mu0) + a.mu0 : y;
    double xs[kScalarMaxL + 1];
    double A = 0.0;
    for (int i = 0; i < L; ++i) {
        xs[i] = x;
        A += a.theta[4 * i + 3] * x;
        x = a.theta[4 * i] * x * x + a.theta[4 * i + 1] * x + a.theta[4 * i + 2];
    }
    xs[L] = x;
    const double u = A + x;
    double out = u, fac = 1.0;
    if (a.target == 1) {
        const double k4 = 4.0 * 0.69314718055994530942;
        out = k4 * u * (1.0 - u);
        fac = k4 * (1.0 - 2.0 * u);
    }
    if (a.r) a.r[k] = out - (a.tgt ? a.tgt[k] : 0.0);
    if (a.r2) {
        // second derivative of the output along theta + t v at t = 0 (forward mode, second
        // order): with x' and x'' the first and second t-derivatives of a state,
        //   x_{i+1}'  = va x^2 + 2 a x x' + vb x + b x' + vc,
        //   x_{i+1}'' = 4 va x x' + 2 a (x'^2 + x x'') + 2 vb x' + b x'',
        //   A'  += vd x + d x',   A'' += 2 vd x' + d x''
        // (the input does not depend on theta, so x_0' = x_0'' = 0)
        const double* v = a.vdir;
        double xd = 0.0, xdd = 0.0, Ad = 0.0, Add = 0.0;
        for (int i = 0; i < L; ++i) {
            const double xi = xs[i];
            const double ca = a.theta[4 * i], cb = a.theta[4 * i + 1], cd = a.theta[4 * i + 3];
            const double va = v[4 * i], vb = v[4 * i + 1], vc = v[4 * i + 2], vd = v[4 * i + 3];
            Ad += vd * xi + cd * xd;
            Add += 2.0 * vd * xd + cd * xdd;
            const double nd = va * xi * xi + 2.0 * ca * xi * xd + vb * xi + cb * xd + vc;
            const double ndd = 4.0 * va * xi * xd + 2.0 * ca * (xd * xd + xi * xdd) + 2.0 * vb * xd +
                               cb * xdd;
            xd = nd;
            xdd = ndd;
        }
        const double ud = Ad + xd, udd = Add + xdd;
        double o2 = udd;
        if (a.target == 1) {
            const double k4 = 4.0 * 0.69314718055994530942;
            o2 = k4 * (-2.0 * ud * ud + (1.0 - 2.0 * u) * udd);
        }
        a.r2[k] = o2;
    }
    if (!a.JT) return;
    double xb = 1.0;   // adjoint of x_{i+1}
    for (int i = L - 1; i >= 0; --i) {
        const double xi = xs[i];
        double* col = a.JT + (size_t)4 * i * a.n + k;   // J^T[4i + c][k]
        col[0] = fac * xb * xi * xi;
        col[(size_t)a.n] = fac * xb * xi;
        col[(size_t)2 * a.n] = fac * xb;
        col[(size_t)3 * a.n] = fac * xi;
        xb = a.theta[4 * i + 3] + xb * (2.0 * a.theta[4 * i] * xi + a.theta[4 * i + 1]);
    }
}

// G[p][q] = sum_k JT[p][k] JT[q][k] for q >= p (one block per pair) and g[p] = sum_k JT[p][k] v[k]
// (blocks with q == P). Fixed-order tree reduction.
__global__ void __launch_bounds__(256)
k_gram(const double* JT, const double* v, int P, int n, double* G, double* g) {
    int pair = blockIdx.x, p = 0;
    // blocks 0 .. P(P+1)/2 - 1: pairs (p, q >= p); then P blocks for J^T v
    const int npairs = P * (P + 1) / 2;
    const double* a;
    const double* b;
    double* dst;
    if (pair < npairs) {
        while (pair >= P - p) {
            pair -= P - p;
            ++p;
        }
        const int q = p + pair;
        if (!G) return;
        a = JT + (size_t)p * n;
        b = JT + (size_t)q * n;
        dst = G + (size_t)p * P + q;
    } else {
        p = pair - npairs;
        if (!g || p >= P) return;
        a = JT + (size_t)p * n;
        b = v;
        dst = g + p;
    }
    double s = 0.0;
    for (int k = threadIdx.x; k < n; k += 256) s += a[k] * b[k];
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *dst = red[0];
}

// Backward of one layer of the FP32 matrix recursion, given M = Xb_{i+1} X_i:
//   grad a_i = <M, X_i>, grad b_i = <Xb_{i+1}, X_i>, grad c_i = tr Xb_{i+1}, grad d_i = <G, X_i>,
//   Xb_i = a_i (M + M^T) + b_i Xb_{i+1} + d_i G.
// Partial sums per block (FP64) are reduced in a fixed order by k_bwd_reduce.
__global__ void __launch_bounds__(256)
k_bwd_elem(BwdArgs a) {
    const int64_t n = a.n;
    const int64_t total = n * n;
    double sa = 0.0, sb = 0.0, sc = 0.0, sd = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t i = e / n, j = e - i * n;
        const float m = a.M[e], mt = a.M[j * n + i];
        const float xb = a.Xb[e], x = a.X[e], gg = a.G[e];
        sa += (double)m * x;
        sb += (double)xb * x;
        if (i == j) sc += xb;
        sd += (double)gg * x;
        a.Xb_out[e] = a.ca * (m + mt) + a.cb * xb + a.cd * gg;
    }
    __shared__ double red[4][256];
    red[0][threadIdx.x] = sa;
    red[1][threadIdx.x] = sb;
    red[2][threadIdx.x] = sc;
    red[3][threadIdx.x] = sd;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int c = 0; c < 4; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 4) a.part[(size_t)blockIdx.x * 4 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void __launch_bounds__(64)
k_bwd_reduce(const double* part, int nblocks, double* grad4) {
    if (threadIdx.x >= 4) return;
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += part[(size_t)b * 4 + threadIdx.x];
    grad4[threadIdx.x] = s;
}

// P = A + X_L from the forward history (A = sum_i d_i X_i), and G-weighted output pieces.
__global__ void __launch_bounds__(256)
k_fwd_out(const float* hist, int64_t n, int L, MatTheta th, float* P) {
    const int64_t total = n * n;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        double A = 0.0;
        for (int i = 0; i < L; ++i) A += th.v[4 * i + 3] * (double)hist[(size_t)i * total + e];
        P[e] = (float)(A + (double)hist[(size_t)L * total + e]);
    }
}

// Residual of a matrix fit: G = P - Dref (FP32, the backward pass's input) and per-block FP64
// partial sums of (P - Dref)^2, reduced in a fixed order by k_sumsq_reduce.
__global__ void __launch_bounds__(256)
k_mat_residual(const float* P, const double* Dref, int64_t total, float* G, double* part) {
    double s = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const double r = (double)P[e] - Dref[e];
        if (G) G[e] = (float)r;
        s += r * r;
    }
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(64) k_sumsq_reduce(const double* part, int nblocks, double* out) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += part[b];
    *out = s;
}

}  // namespace

int scalar_max_layers() { return kScalarMaxL; }

hipError_t launch_mat_residual(const float* P, const double* Dref, int64_t total, float* G,
                               double* part, int nblocks, double* sumsq, hipStream_t s) {
    hipLaunchKernelGGL(k_mat_residual, dim3(nblocks), dim3(256), 0, s, P, Dref, total, G, part);
    hipLaunchKernelGGL(k_sumsq_reduce, dim3(1), dim3(64), 0, s, part, nblocks, sumsq);
    return hipGetLastError();
}

hipError_t launch_scalar_eval(const ScalarArgs& a, hipStream_t s) {
    if (a.L < 1 || a.L > kScalarMaxL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_scalar_eval, dim3((a.n + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_gram(const double* JT, const double* v, int P, int n, double* G, double* g,
                       hipStream_t s) {
    const int blocks = P * (P + 1) / 2 + P;
    hipLaunchKernelGGL(k_gram, dim3(blocks), dim3(256), 0, s, JT, v, P, n, G, g);
    return hipGetLastError();
}

hipError_t launch_bwd_elem(const BwdArgs& a, int nblocks, double* grad4, hipStream_t s) {
    hipLaunchKernelGGL(k_bwd_elem, dim3(nblocks), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_bwd_reduce, dim3(1), dim3(64), 0, s, a.part, nblocks, grad4);
    return hipGetLastError();
}

hipError_t launch_fwd_out(const float* hist, int64_t n, int L, const MatTheta& th, float* P, hipStream_t s) {
    int64_t blocks = (n * n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fwd_out, dim3((unsigned)blocks), dim3(256), 0, s, hist, n, L, th, P);
    return hipGetLastError();
}

}  // namespace fe
