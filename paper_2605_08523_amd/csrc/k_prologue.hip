// Prologue of the expansion: Gershgorin bounds, rescale parameters and the rescaled start matrix
// (Sec. IV.1, Eqs. H', mu', beta', flip, conditions, H0; Alg. 2 first steps), plus the
// deterministic reduction of per-tile traces (Sec. IV.3, Eq. tr(D^2); Eq. entropy expansion-s).
#include <math.h>

#include "fe_internal.h"
#include "split_common.h"

namespace fe {
namespace {

constexpr int kBoundsThreads = 256;

__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline double wave_min(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline int wave_or(int v) {
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, 64);
    return v;
}

// One wave per row: r_i = sum_{j != i} |h_ij|, row bounds h_ii -/+ r_i; min/max over the
// block's rows into one partial. A non-finite entry makes the row sum non-finite.
__global__ void __launch_bounds__(kBoundsThreads)
k_gershgorin(const double* __restrict__ H, int64_t n, int64_t ldh, BoundsPartial* partials) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int kWaves = kBoundsThreads / 64;
    double lo = INFINITY, hi = -INFINITY;
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * kWaves + wave; i < n; i += (int64_t)gridDim.x * kWaves) {
        const double* row = H + i * ldh;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int64_t j = lane;
        for (; j + 192 < n; j += 256) {
            s0 += fabs(row[j]);
            s1 += fabs(row[j + 64]);
            s2 += fabs(row[j + 128]);
            s3 += fabs(row[j + 192]);
        }
        for (; j < n; j += 64) s0 += fabs(row[j]);
        double s = wave_sum((s0 + s1) + (s2 + s3));
        const double d = row[i];
        const double r = s - fabs(d);
        if (!isfinite(s)) bad = 1;
        lo = fmin(lo, d - r);
        hi = fmax(hi, d + r);
    }
    __shared__ double slo[kWaves], shi[kWaves];
    __shared__ int sbad[kWaves];
    if (lane == 0) {
        slo[wave] = lo;
        shi[wave] = hi;
        sbad[wave] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kWaves; ++w) {
            lo = fmin(lo, slo[w]);
            hi = fmax(hi, shi[w]);
            bad |= sbad[w];
        }
        partials[blockIdx.x].lo = lo;
        partials[blockIdx.x].hi = hi;
        partials[blockIdx.x].nonfinite = bad;
    }
}

// Reduce the partial bounds and compute the rescale of Sec. IV.1 in FP64 on the device.
__global__ void __launch_bounds__(256)
k_params(const BoundsPartial* partials, int count, double mu, double kT, double beta0, double mu0,
         Params* P) {
    double lo = INFINITY, hi = -INFINITY;
    int bad = 0;
    for (int k = threadIdx.x; k < count; k += blockDim.x) {
        lo = fmin(lo, partials[k].lo);
        hi = fmax(hi, partials[k].hi);
        bad |= partials[k].nonfinite;
    }
    lo = wave_min(lo);
    hi = wave_max(hi);
    bad = wave_or(bad);
    __shared__ double slo[4], shi[4];
    __shared__ int sbad[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        slo[wave] = lo;
        shi[wave] = hi;
        sbad[wave] = bad;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int w = 1; w < (int)(blockDim.x / 64); ++w) {
        lo = fmin(lo, slo[w]);
        hi = fmax(hi, shi[w]);
        bad |= sbad[w];
    }
    Params p;
    p.emin = lo;
    p.emax = hi;
    p.flipped = 0;
    p.clamped = 0;
    p.degenerate = 0;
    p.status = FE_OK;
    const double width = hi - lo;
    if (bad || !isfinite(lo) || !isfinite(hi)) {
        p.status = FE_ERR_NONFINITE;
        p.mu_p = p.beta_p = p.beta_max = NAN;
        p.scale = p.shift = NAN;
    } else if (width <= 1e-300 * fmax(1.0, fabs(hi))) {
        // H = c I: the model coordinate of every eigenvalue is y = mu0 + (mu - c)/(kT beta0).
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
        p.mu_p = p.beta_p = p.beta_max = NAN;
        p.scale = p.shift = NAN;
    } else {
        double mu_p = (hi - mu) / width;           // Eq. mu'
        double beta_p = width / kT;                // Eq. beta'
        const int flip = mu_p > 0.5;               // Eq. flip (strict)
        if (flip) mu_p = 1.0 - mu_p;
        const double bmax = fmin(mu0 / mu_p, (1.0 - mu0) / (1.0 - mu_p)) * beta0;  // Eq. conditions
        if (beta_p > bmax) {
            beta_p = bmax;
            p.clamped = 1;
            p.status = FE_WARN_BETA_CLAMPED;
        }
        const double r = beta_p / beta0;
        // X0 = r (H' - mu' I) + mu0 I with H' = (emax I - H)/width, or its flip (H - emin I)/width.
        p.scale = flip ? r / width : -r / width;
        p.shift = flip ? r * (-lo / width - mu_p) + mu0 : r * (hi / width - mu_p) + mu0;
        p.mu_p = mu_p;
        p.beta_p = beta_p;
        p.beta_max = bmax;
        p.flipped = flip;
    }
    *P = p;
}

template <bool BF>
__device__ inline void split16(float x, uint16_t& h, uint16_t& l) {
    if constexpr (!BF) {
        const _Float16 hh = (_Float16)x;
        const float r = x - (float)hh;             // exact in FP32
        const _Float16 ll = (_Float16)(r * 2048.0f);
        h = __builtin_bit_cast(uint16_t, hh);
        l = __builtin_bit_cast(uint16_t, ll);
    } else {
        const __bf16 hh = (__bf16)x;
        const float r = x - (float)hh;
        const __bf16 ll = (__bf16)r;
        h = __builtin_bit_cast(uint16_t, hh);
        l = __builtin_bit_cast(uint16_t, ll);
    }
}

template <bool BF>
__device__ inline void rescale_quad(const RescaleArgs& a, double scale, double shift, int64_t i,
                                    int64_t j0) {
    const int64_t e0 = i * a.np + j0;
    double x[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t j = j0 + k;
        x[k] = 0.0;
        if (i < a.n && j < a.n) {
            double v = scale * a.H[i * a.ldh + j] + (i == j ? shift : 0.0);
            v = a.alpha * v + (i == j ? (1.0 - a.alpha) * a.mu0 : 0.0);
            if (a.X0out) a.X0out[i * a.ldx + j] = (float)v;
            x[k] = v;
        }
    }
    if (a.mode == 2) {
        *reinterpret_cast<double2*>(a.X64 + e0) = double2{x[0], x[1]};
        *reinterpret_cast<double2*>(a.X64 + e0 + 2) = double2{x[2], x[3]};
        *reinterpret_cast<double2*>(a.A64 + e0) = double2{a.d0 * x[0], a.d0 * x[1]};
        *reinterpret_cast<double2*>(a.A64 + e0 + 2) = double2{a.d0 * x[2], a.d0 * x[3]};
        return;
    }
    const float d0f = (float)a.d0;
    split::floatx4 xf, af;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        xf[k] = (float)x[k];
        af[k] = d0f * xf[k];
    }
    *reinterpret_cast<split::floatx4*>(a.X32 + e0) = xf;
    *reinterpret_cast<split::floatx4*>(a.A32 + e0) = af;
    if (a.mode != 0) return;
    uint16_t h[4], l[4], md[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float xs = i == j0 + k ? (float)(x[k] + a.op_shift) : xf[k];
        if (a.three) split::split3(xs, h[k], md[k], l[k]);
        else split16<BF>(xs, h[k], l[k]);
    }
    auto pack = [](const uint16_t* v) {
        return split::u32x2{(uint32_t)v[0] | ((uint32_t)v[1] << 16), (uint32_t)v[2] | ((uint32_t)v[3] << 16)};
    };
    *reinterpret_cast<split::u32x2*>(a.hi + e0) = pack(h);
    *reinterpret_cast<split::u32x2*>(a.lo + e0) = pack(l);
    if (a.three) *reinterpret_cast<split::u32x2*>(a.mid + e0) = pack(md);
    // the other buffer's padding (rows or columns >= n), which no layer epilogue writes
    if (i >= a.n || j0 + 3 >= a.n) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (i < a.n && j0 + k < a.n) continue;
            if (a.hi1) {
                a.hi1[e0 + k] = h[k];
                a.lo1[e0 + k] = l[k];
            }
            if (a.three && a.mid1) a.mid1[e0 + k] = md[k];
        }
    }
}

// The rescaled start matrix X0 (FP32 or FP64 master), the accumulator A = d0 X0 and, for the
// 16-bit modes, the split operands, over the padded np x np matrix (zero padding). Four
// consecutive columns per thread (16-byte stores; np is a multiple of 4), quads in a grid-stride
// loop.
template <bool BF>
__global__ void __launch_bounds__(256) k_rescale(RescaleArgs a) {
    const Params* P = a.P;
    const double scale = P->scale, shift = P->shift;
    const int64_t qrow = a.np / 4, quads = a.np * qrow;
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    if (quads <= 0xffffffffLL) {
        for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < quads; q += step) {
            const uint32_t i = (uint32_t)q / (uint32_t)qrow, jq = (uint32_t)q - i * (uint32_t)qrow;
            rescale_quad<BF>(a, scale, shift, i, 4 * (int64_t)jq);
        }
    } else {
        for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < quads; q += step) {
            const int64_t i = q / qrow;
            rescale_quad<BF>(a, scale, shift, i, 4 * (q - i * qrow));
        }
    }
}

__global__ void __launch_bounds__(256)
k_reduce(const TracePartial* partials, int count, double* out_tr, double* out_sq, double* out_S,
         Params* P, int* err) {
    // Fixed-order reduction: thread t sums partials t, t+256, ...; then a tree over threads.
    __shared__ double st[256], ss[256];
    double tr = 0.0, sq = 0.0;
    for (int k = threadIdx.x; k < count; k += 256) {
        tr += partials[k].tr;
        sq += partials[k].sq;
    }
    st[threadIdx.x] = tr;
    ss[threadIdx.x] = sq;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            st[threadIdx.x] += st[threadIdx.x + w];
            ss[threadIdx.x] += ss[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (err && *err) {
            // a stream-K wait gave up: the tiles it finished hold NaN; report it here too
            *err = 0;
            if (P->status >= 0) P->status = FE_ERR_HIP;
        }
        const double bad = (P->status < 0) ? NAN : 0.0;
        if (out_tr) *out_tr = st[0] + bad;
        if (out_sq) *out_sq = ss[0] + bad;
        if (out_S) *out_S = 4.0 * 0.69314718055994530942 * (st[0] - ss[0]) + bad;
    }
}

__global__ void __launch_bounds__(256) k_fill_symmetric(double* H, int64_t n, uint64_t seed) {
    const double off = 1.0 / sqrt((double)n);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * n;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / n, j = e - i * n;
        const uint64_t a = (uint64_t)(i < j ? i : j), b = (uint64_t)(i < j ? j : i);
        // splitmix64 of the unordered pair and the seed
        uint64_t z = seed + 0x9e3779b97f4a7c15ULL * (a * 0x100000001b3ULL + b + 1);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
        z ^= z >> 31;
        const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
        H[e] = i == j ? u : u * off;
    }
}

}  // namespace

hipError_t launch_bounds_params(const double* H, int64_t n, int64_t ldh, double mu, double kT,
                                double beta0, double mu0, BoundsPartial* partials, Params* P,
                                hipStream_t s) {
    int64_t blocks = (n + 3) / 4;
    if (blocks > kMaxBoundsBlocks) blocks = kMaxBoundsBlocks;
    hipLaunchKernelGGL(k_gershgorin, dim3((unsigned)blocks), dim3(kBoundsThreads), 0, s, H, n, ldh,
                       partials);
    hipLaunchKernelGGL(k_params, dim3(1), dim3(256), 0, s, partials, (int)blocks, mu, kT, beta0,
                       mu0, P);
    return hipGetLastError();
}

hipError_t launch_rescale(const RescaleArgs& a, hipStream_t s) {
    if (a.np % 4 != 0) return hipErrorInvalidValue;
    int64_t total = a.np * a.np / 4;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (a.bf16)
        hipLaunchKernelGGL(k_rescale<true>, dim3((unsigned)blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_rescale<false>, dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fill_symmetric(double* H, int64_t n, uint64_t seed, hipStream_t s) {
    int64_t blocks = (n * n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_fill_symmetric, dim3((unsigned)blocks), dim3(256), 0, s, H, n, seed);
    return hipGetLastError();
}

hipError_t launch_reduce_partials(const TracePartial* partials, int count, double* out_tr,
                                  double* out_sq, double* out_S, Params* P, int* err,
                                  hipStream_t s) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, s, partials, count, out_tr, out_sq, out_S,
                       P, err);
    return hipGetLastError();
}

}  // namespace fe
