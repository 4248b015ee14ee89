// FP32 and FP64 layer kernels of the recursion X <- a X^2 + b X + c I, A <- A + d X
// (Eq. mlsp2), and the plain product C = L R^T used by the coefficient trainer.
//
// 64 x 64 output tiles, four waves of 32 x 32; FP32 uses v_mfma_f32_32x32x2f32 (one 32 x 32
// block per wave), FP64 uses v_mfma_f64_16x16x4f64 (2 x 2 blocks per wave). The operands of
// tile (I, J) are the row panels I and J (X is symmetric, so column panel J = row panel J^T).
// Register prefetch of the next K block overlaps the MFMAs on the current one. The layer form
// computes only upper tiles and writes each tile and its mirror through an LDS-staged epilogue.
#include "fe_internal.h"

namespace fe {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double double4v __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;

// v_mfma_f32_32x32x2f32: lane l supplies A[l % 32][l / 32] and B[l / 32][l % 32];
// acc[j] of lane l holds D[8 (j/4) + 4 (l/32) + j%4][l % 32].
template <>
struct Mfma<float> {
    static constexpr int BLK = 32, KSTEP = 2, NACC = 16;
    using acc_t = floatx16;
    __device__ static acc_t zero() {
        acc_t z;
#pragma unroll
        for (int j = 0; j < 16; ++j) z[j] = 0.0f;
        return z;
    }
    __device__ static acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
    }
    __device__ static int arow(int lane) { return lane & 31; }
    __device__ static int akk(int lane) { return lane >> 5; }
    __device__ static int crow(int lane, int j) { return 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3); }
    __device__ static int ccol(int lane) { return lane & 31; }
};

// v_mfma_f64_16x16x4f64: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16];
// acc[i] of lane l holds D[4 i + l / 16][l % 16].
template <>
struct Mfma<double> {
    static constexpr int BLK = 16, KSTEP = 4, NACC = 4;
    using acc_t = double4v;
    __device__ static acc_t zero() { return (acc_t){0.0, 0.0, 0.0, 0.0}; }
    __device__ static acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static int arow(int lane) { return lane & 15; }
    __device__ static int akk(int lane) { return lane >> 4; }
    __device__ static int crow(int lane, int j) { return 4 * j + (lane >> 4); }
    __device__ static int ccol(int lane) { return lane & 15; }
};

constexpr int BM = 64;        // tile
constexpr int NT = 256;       // 4 waves, 2 x 2 of 32 x 32

__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <typename T>
__global__ void __launch_bounds__(NT) k_wide(WideArgs p) {
    using M = Mfma<T>;
    constexpr int BK = 16;                       // K per LDS stage
    constexpr int LDK = BK + 1;                  // odd row stride: conflict-free column reads
    constexpr int NBW = 32 / M::BLK;             // MFMA blocks per wave side
    constexpr int LDY = BM + 1;
    __shared__ T sA[BM * LDK], sB[BM * LDK];
    __shared__ T sY[BM * LDY];
    __shared__ double red[8];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t np = p.np;
    const int T_ = (int)(np / BM);
    int I, J;
    if (p.plain) {
        I = blockIdx.x / T_;
        J = blockIdx.x % T_;
    } else {
        int rem = blockIdx.x, i = 0;
        while (rem >= T_ - i) {
            rem -= T_ - i;
            ++i;
        }
        I = i;
        J = i + rem;
    }
    const bool diag = !p.plain && I == J;
    const int64_t I0 = (int64_t)I * BM, J0 = (int64_t)J * BM;
    const T* __restrict__ Lm = static_cast<const T*>(p.X_in);
    const T* __restrict__ Rm = p.plain ? static_cast<const T*>(p.B_in) : Lm;

    // global -> LDS: 64 rows x 16 K of each panel = 1024 elements, 4 per thread
    constexpr int PER = BM * BK / NT;
    T ra[PER], rb[PER];
    auto gload = [&](int kb) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + q * NT, row = e / BK, k = e % BK;
            ra[q] = Lm[(I0 + row) * np + (int64_t)kb * BK + k];
            rb[q] = Rm[(J0 + row) * np + (int64_t)kb * BK + k];
        }
    };
    auto sstore = [&]() {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + q * NT, row = e / BK, k = e % BK;
            sA[row * LDK + k] = ra[q];
            sB[row * LDK + k] = rb[q];
        }
    };

    typename M::acc_t acc[NBW][NBW];
#pragma unroll
    for (int x = 0; x < NBW; ++x)
#pragma unroll
        for (int y = 0; y < NBW; ++y) acc[x][y] = M::zero();

    const int nk = (int)(np / BK);
    gload(0);
    sstore();
    __syncthreads();
    for (int kb = 0; kb < nk; ++kb) {
        if (kb + 1 < nk) gload(kb + 1);
#pragma unroll
        for (int k0 = 0; k0 < BK; k0 += M::KSTEP) {
            T av[NBW], bv[NBW];
#pragma unroll
            for (int x = 0; x < NBW; ++x) {
                av[x] = sA[(wm * 32 + x * M::BLK + M::arow(lane)) * LDK + k0 + M::akk(lane)];
                bv[x] = sB[(wn * 32 + x * M::BLK + M::arow(lane)) * LDK + k0 + M::akk(lane)];
            }
#pragma unroll
            for (int x = 0; x < NBW; ++x)
#pragma unroll
                for (int y = 0; y < NBW; ++y) acc[x][y] = M::mma(av[x], bv[y], acc[x][y]);
        }
        __syncthreads();
        if (kb + 1 < nk) {
            sstore();
            __syncthreads();
        }
    }

    // stage the 64 x 64 product tile in LDS
#pragma unroll
    for (int x = 0; x < NBW; ++x)
#pragma unroll
        for (int y = 0; y < NBW; ++y)
#pragma unroll
            for (int j = 0; j < M::NACC; ++j) {
                const int r = wm * 32 + x * M::BLK + M::crow(lane, j);
                const int c = wn * 32 + y * M::BLK + M::ccol(lane);
                sY[r * LDY + c] = acc[x][y][j];
            }
    __syncthreads();

    if (p.plain) {
        T* C = static_cast<T*>(p.X_out);
        for (int e = tid; e < BM * BM; e += NT) {
            const int r = e / BM, c = e % BM;
            C[(I0 + r) * np + J0 + c] = sY[r * LDY + c];
        }
        return;
    }

    const T ca = (T)p.a, cb = (T)p.b, cc = (T)p.c, dn = (T)p.d_next;
    const bool last = p.last != 0, ent = p.entropy != 0;
    const int flip = (last && !ent) ? p.P->flipped : 0;
    const bool f64e = last && p.f64_epi;   // FP64 epilogue of a correction layer (T = float)
    const int64_t n = p.n;
    T* __restrict__ Xo = static_cast<T*>(p.X_out);
    T* __restrict__ A = static_cast<T*>(p.A);
    // Last-layer value at upper position gi (row gr, column gc) from the product y:
    // D = A + d_last X + (a y + b X + c delta), in FP64 for the correction layer (then not
    // rounded: the layer's D is formed in FP64 from FP32 products and FP32 state), else in T.
    auto last_value = [&](T y, int64_t gi, int64_t gr, int64_t gc) -> double {
        double v;
        if (f64e) {
            const double x = (double)Lm[gi];
            v = (double)A[gi] + p.d_last * x + (p.a * (double)y + p.b * x + (gr == gc ? p.c : 0.0));
        } else {
            const T xn = ca * y + cb * Lm[gi] + (gr == gc ? cc : (T)0);
            v = (double)A[gi] + (double)xn;
        }
        if (flip) v = (gr == gc ? 1.0 : 0.0) - v;
        // FP32 mode carries FP32 values (so the tile and its mirror hold the same number)
        return (ent || sizeof(T) == 8 || f64e) ? v : (double)(float)v;
    };
    double tr = 0.0, sq = 0.0;
    for (int e = tid; e < BM * BM; e += NT) {
        const int r = e / BM, c = e % BM;
        if (diag && r > c) continue;
        const int64_t gr = I0 + r, gc = J0 + c, gi = gr * np + gc;
        const T y = sY[r * LDY + c];
        if (!last) {
            const T xn = ca * y + cb * Lm[gi] + (gr == gc ? cc : (T)0);
            if (dn != (T)0) A[gi] += dn * xn;
            Xo[gi] = xn;
            sY[r * LDY + c] = xn;
        } else {
            const double vo = last_value(y, gi, gr, gc);
            if (gr < n && gc < n) {
                if (gr == gc) tr += vo;
                sq += (gr == gc ? 1.0 : 2.0) * vo * vo;
                if (!ent) {
                    if (p.out_mode == 0)
                        reinterpret_cast<float*>(p.D)[gr * p.ldd + gc] = (float)vo;
                    else if (p.out_mode == 1)
                        reinterpret_cast<double*>(p.D)[gr * p.ldd + gc] = vo;
                }
            }
            if (!f64e) sY[r * LDY + c] = (T)vo;   // the correction layer keeps y and recomputes
        }
    }
    __syncthreads();
    if (!(last && (ent || p.out_mode == 2))) {
        for (int e = tid; e < BM * BM; e += NT) {
            const int r = e % BM, c = e / BM;
            if (diag && !(r < c)) continue;
            const T v = sY[r * LDY + c];
            const int64_t orow = J0 + c, ocol = I0 + r;
            if (!last) {
                Xo[orow * np + ocol] = v;
            } else if (orow < n && ocol < n) {
                // the mirror of an FP64 correction value is recomputed from the same operands,
                // so D stays exactly symmetric
                const double vo = f64e ? last_value(v, (I0 + r) * np + J0 + c, I0 + r, J0 + c)
                                       : (double)v;
                if (p.out_mode == 0)
                    reinterpret_cast<float*>(p.D)[orow * p.ldd + ocol] = (float)vo;
                else
                    reinterpret_cast<double*>(p.D)[orow * p.ldd + ocol] = vo;
            }
        }
    }
    if (last) {
        tr = wave_sum(tr);
        sq = wave_sum(sq);
        if (lane == 0) {
            red[2 * wave] = tr;
            red[2 * wave + 1] = sq;
        }
        __syncthreads();
        if (tid == 0) {
            double t = 0.0, s = 0.0;
            for (int w = 0; w < 4; ++w) {
                t += red[2 * w];
                s += red[2 * w + 1];
            }
            p.partials[blockIdx.x].tr = t;
            p.partials[blockIdx.x].sq = s;
        }
    }
}

// Lower triangle of an np x np FP32 matrix from its upper triangle (X[i][j] = X[j][i] for
// i > j), through 64 x 64 LDS tiles: workgroup (I, J), I >= J, reads the upper tile (J, I) row by
// row and writes its transpose into the lower tile (I, J); diagonal tiles copy within the tile.
__global__ void __launch_bounds__(256) k_mirror_upper(float* X, int64_t np) {
    __shared__ float t[BM][BM + 1];
    int rem = blockIdx.x, i = 0;
    const int T_ = (int)(np / BM);
    while (rem >= T_ - i) {   // upper-tile enumeration: tile (i, i + rem) is the source
        rem -= T_ - i;
        ++i;
    }
    const int64_t R0 = (int64_t)i * BM, C0 = (int64_t)(i + rem) * BM;   // source tile, R0 <= C0
    for (int e = threadIdx.x; e < BM * BM; e += 256) {
        const int r = e / BM, c = e % BM;
        t[r][c] = X[(R0 + r) * np + C0 + c];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < BM * BM; e += 256) {
        const int r = e / BM, c = e % BM;   // destination (C0 + r, R0 + c) = source (R0 + c, C0 + r)
        if (R0 == C0 && !(r > c)) continue;
        X[(C0 + r) * np + R0 + c] = t[c][r];
    }
}

template <typename T>
hipError_t launch(const WideArgs& a, hipStream_t s) {
    if (a.np % BM != 0) return hipErrorInvalidValue;
    const int T_ = (int)(a.np / BM);
    const int grid = a.plain ? T_ * T_ : T_ * (T_ + 1) / 2;
    hipLaunchKernelGGL(k_wide<T>, dim3(grid), dim3(NT), 0, s, a);
    return hipGetLastError();
}

}  // namespace

int wide_tile() { return BM; }
hipError_t launch_layer_f32(const WideArgs& a, hipStream_t s) { return launch<float>(a, s); }
hipError_t launch_layer_f64(const WideArgs& a, hipStream_t s) { return launch<double>(a, s); }
hipError_t launch_mirror_upper_f32(float* X, int64_t np, hipStream_t s) {
    if (np % BM != 0) return hipErrorInvalidValue;
    const int T_ = (int)(np / BM);
    hipLaunchKernelGGL(k_mirror_upper, dim3(T_ * (T_ + 1) / 2), dim3(256), 0, s, X, np);
    return hipGetLastError();
}

}  // namespace fe
