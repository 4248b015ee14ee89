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
__global__ void __launch_bounds__(256) k_rescale(RescaleArgs a) {
    const Params* P = a.P;
    const double scale = P->scale, shift = P->shift;
    const int64_t total = a.np * a.np;
    const float d0f = (float)a.d0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / a.np, j = e - i * a.np;
        double x = 0.0;
        if (i < a.n && j < a.n) {
            x = scale * a.H[i * a.ldh + j] + (i == j ? shift : 0.0);
            x = a.alpha * x + (i == j ? (1.0 - a.alpha) * a.mu0 : 0.0);
            if (a.X0out) a.X0out[i * a.ldx + j] = (float)x;
        }
        if (a.mode == 2) {
            a.X64[e] = x;
            a.A64[e] = a.d0 * x;
        } else {
            const float xf = (float)x;
            a.X32[e] = xf;
            a.A32[e] = d0f * xf;
            if (a.mode == 0) {
                const float xs = i == j ? (float)(x + a.op_shift) : xf;
                const bool pad = i >= a.n || j >= a.n;
                uint16_t h, l;
                if (a.three) {
                    uint16_t m;
                    split::split3(xs, h, m, l);
                    a.mid[e] = m;
                    if (pad && a.mid1) a.mid1[e] = m;
                } else {
                    split16<BF>(xs, h, l);
                }
                a.hi[e] = h;
                a.lo[e] = l;
                if (a.hi1 && pad) {
                    a.hi1[e] = h;
                    a.lo1[e] = l;
                }
            }
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
    int64_t total = a.np * a.np;
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
