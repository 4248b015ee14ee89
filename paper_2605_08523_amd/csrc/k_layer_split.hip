// One layer of the recursion X <- a X^2 + b X + c I, A <- A + d X (Eq. mlsp2) for a symmetric X
// held as X = hi + s^-1 lo with 16-bit hi/lo (Sec. V.A, Eq. emulated matmul), on CDNA4 MFMA.
//
// Design (gfx950):
//  * Only tiles (I, J) with I <= J are computed (X^2 is symmetric); the epilogue writes the
//    tile and its mirror, so every stored matrix stays exactly symmetric.
//  * X^2 is accumulated in FP32 from three products per K step in one accumulator,
//        s Y = (s hi_I) hi_J + hi_I lo_J + lo_I hi_J,
//    where lo is stored pre-scaled by s = 2^11 for FP16 (keeps it out of the FP16 subnormals)
//    and s = 1 for BF16. The lo*lo term is dropped (below 2^-22 relative for FP16).
//    By symmetry the B operand of tile (I, J) is the row panel J, so both operands are read as
//    row panels with K contiguous.
//  * The epilogue is fused: Y goes through LDS, then one row-major pass computes
//    X' = a Y + b X + c delta_ij, updates A with the next layer's d, writes the FP32 master and
//    the next layer's hi/lo, and a second (transposed) pass writes the mirror tile. On the last
//    layer it writes D = A + X' (I - D when the spectrum was flipped) and per-tile FP64 traces.
//  * Workgroup ids are remapped so that each XCD (8 per chip, one L2 each) receives a
//    contiguous range of tiles.
#include "fe_internal.h"

namespace fe {
namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));   // 16 bytes of 16-bit operands

template <bool BF>
__device__ inline void split16(float x, uint16_t& h, uint16_t& l) {
    if constexpr (!BF) {
        const _Float16 hh = (_Float16)x;
        const float r = x - (float)hh;
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

// hi scaled by s = 2^11 (FP16; exact power-of-two scaling) or unchanged (BF16, s = 1).
template <bool BF>
__device__ inline u32x4 scale_hi(u32x4 ah) {
    if constexpr (!BF) {
        const half8 h = __builtin_bit_cast(half8, ah) * (_Float16)2048.0f;
        return __builtin_bit_cast(u32x4, h);
    } else {
        return ah;
    }
}

// acc += (s hi_a) hi_b + hi_a lo_b + lo_a hi_b  (three 32x32x16 MFMAs, FP32 accumulate)
template <bool BF>
__device__ inline floatx16 mfma3(u32x4 ahs, u32x4 ah, u32x4 al, u32x4 bh, u32x4 bl, floatx16 acc) {
    if constexpr (!BF) {
        acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(half8, ahs),
                                                     __builtin_bit_cast(half8, bh), acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(half8, ah),
                                                     __builtin_bit_cast(half8, bl), acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(half8, al),
                                                     __builtin_bit_cast(half8, bh), acc, 0, 0, 0);
    } else {
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, ahs),
                                                      __builtin_bit_cast(bf16x8, bh), acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, ah),
                                                      __builtin_bit_cast(bf16x8, bl), acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, al),
                                                      __builtin_bit_cast(bf16x8, bh), acc, 0, 0, 0);
    }
    return acc;
}

__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Map a workgroup id to a tile (I, J), I <= J, of the T x T tile grid. Ids are first remapped so
// that the hardware's round-robin over the 8 XCDs hands each XCD a contiguous logical range,
// then the logical id walks the upper triangle row by row.
__device__ inline void tile_of(int w, int T, int ntiles, int& I, int& J, int& logical) {
    const int q = ntiles >> 3, r = ntiles & 7, x = w & 7;
    logical = x * q + (x < r ? x : r) + (w >> 3);
    int rem = logical, i = 0;
    while (rem >= T - i) {
        rem -= T - i;
        ++i;
    }
    I = i;
    J = i + rem;
}

template <bool BF, int BM, int WM, int WN, int BK, int EC, int OCC>
__global__ void __launch_bounds__(WM * WN * 64) __attribute__((amdgpu_waves_per_eu(OCC, OCC)))
k_layer_split(LayerArgs p) {
    constexpr int NT = WM * WN * 64;
    constexpr int LDK = BK + 8;                 // padded LDS row (halves): 16-B aligned, no conflicts
    constexpr int WAVE_M = BM / WM, WAVE_N = BM / WN;
    constexpr int MB = WAVE_M / 32, NB = WAVE_N / 32;
    constexpr int CPR = BK / 8;                 // 16-byte chunks per panel row
    constexpr int CH = BM * CPR / NT;           // chunks per thread per array
    constexpr int LDY = BM + 1;                 // epilogue staging row (floats)
    static_assert(BM * CPR % NT == 0, "load split");
    static_assert(WAVE_M % 32 == 0 && WAVE_N % 32 == 0, "wave tile");
    static_assert(BM % EC == 0 && EC % 32 == 0 && (EC * BM) % NT == 0, "epilogue chunk");

    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    uint16_t* sAh = reinterpret_cast<uint16_t*>(smem);
    uint16_t* sAl = sAh + BM * LDK;
    uint16_t* sBh = sAl + BM * LDK;
    uint16_t* sBl = sBh + BM * LDK;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int64_t np = p.np;
    const int T = (int)(np / BM);
    const int ntiles = T * (T + 1) / 2;
    int I, J, logical;
    tile_of(blockIdx.x, T, ntiles, I, J, logical);
    const bool diag = (I == J);
    const int64_t I0 = (int64_t)I * BM, J0 = (int64_t)J * BM;

    // ---- K loop: global -> registers (next stage) while MFMAs consume LDS (this stage) -------
    const uint16_t* __restrict__ hin = p.hi_in;
    const uint16_t* __restrict__ lin = p.lo_in;
    // Thread -> (row, 16-byte chunk) of the BM x BK panel slab, CH chunks per thread per array.
    int64_t goffI[CH], goffJ[CH];
    int soff[CH];
#pragma unroll
    for (int q = 0; q < CH; ++q) {
        const int cidx = tid + q * NT;
        const int row = cidx / CPR, kc = cidx % CPR;
        goffI[q] = (I0 + row) * np + kc * 8;
        goffJ[q] = (J0 + row) * np + kc * 8;
        soff[q] = row * LDK + kc * 8;
    }
    u32x4 pAh[CH], pAl[CH], pBh[CH], pBl[CH];

    floatx16 acc[MB][NB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int j = 0; j < 16; ++j) acc[mb][nb][j] = 0.0f;

    const int nk = (int)(np / BK);
#pragma unroll
    for (int q = 0; q < CH; ++q) {
        pAh[q] = *reinterpret_cast<const u32x4*>(hin + goffI[q]);
        pAl[q] = *reinterpret_cast<const u32x4*>(lin + goffI[q]);
        pBh[q] = *reinterpret_cast<const u32x4*>(hin + goffJ[q]);
        pBl[q] = *reinterpret_cast<const u32x4*>(lin + goffJ[q]);
    }
#pragma unroll
    for (int q = 0; q < CH; ++q) {
        *reinterpret_cast<u32x4*>(sAh + soff[q]) = pAh[q];
        *reinterpret_cast<u32x4*>(sAl + soff[q]) = pAl[q];
        *reinterpret_cast<u32x4*>(sBh + soff[q]) = pBh[q];
        *reinterpret_cast<u32x4*>(sBl + soff[q]) = pBl[q];
    }
    __syncthreads();
    const int frag_row = lane & 31, frag_k = (lane >> 5) * 8;
    for (int kb = 0; kb < nk; ++kb) {
        const bool more = kb + 1 < nk;
        if (more) {
            const int64_t k0 = (int64_t)(kb + 1) * BK;
#pragma unroll
            for (int q = 0; q < CH; ++q) {
                pAh[q] = *reinterpret_cast<const u32x4*>(hin + goffI[q] + k0);
                pAl[q] = *reinterpret_cast<const u32x4*>(lin + goffI[q] + k0);
                pBh[q] = *reinterpret_cast<const u32x4*>(hin + goffJ[q] + k0);
                pBl[q] = *reinterpret_cast<const u32x4*>(lin + goffJ[q] + k0);
            }
        }
#pragma unroll
        for (int ks = 0; ks < BK / 16; ++ks) {
            u32x4 ah[MB], al[MB], bh[NB], bl[NB];
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                const int o = (wm * WAVE_M + mb * 32 + frag_row) * LDK + ks * 16 + frag_k;
                ah[mb] = *reinterpret_cast<const u32x4*>(sAh + o);
                al[mb] = *reinterpret_cast<const u32x4*>(sAl + o);
            }
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const int o = (wn * WAVE_N + nb * 32 + frag_row) * LDK + ks * 16 + frag_k;
                bh[nb] = *reinterpret_cast<const u32x4*>(sBh + o);
                bl[nb] = *reinterpret_cast<const u32x4*>(sBl + o);
            }
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                const u32x4 ahs = scale_hi<BF>(ah[mb]);
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    acc[mb][nb] = mfma3<BF>(ahs, ah[mb], al[mb], bh[nb], bl[nb], acc[mb][nb]);
            }
        }
        __syncthreads();
        if (more) {
#pragma unroll
            for (int q = 0; q < CH; ++q) {
                *reinterpret_cast<u32x4*>(sAh + soff[q]) = pAh[q];
                *reinterpret_cast<u32x4*>(sAl + soff[q]) = pAl[q];
                *reinterpret_cast<u32x4*>(sBh + soff[q]) = pBh[q];
                *reinterpret_cast<u32x4*>(sBl + soff[q]) = pBl[q];
            }
            __syncthreads();
        }
    }

    // ---- fused epilogue ------------------------------------------------------------------
    const float inv_s = BF ? 1.0f : (1.0f / 2048.0f);
    const float ca = p.a, cb = p.b, cc = p.c, dn = p.d_next;
    const bool last = p.last != 0;
    const bool ent = p.entropy != 0;
    const int flip = last ? p.P->flipped : 0;
    const int64_t n = p.n;
    float* __restrict__ X = p.X;
    float* __restrict__ A = p.A;
    float* sY = reinterpret_cast<float*>(smem);
    double tr = 0.0, sq = 0.0;

#pragma unroll 1
    for (int ch = 0; ch < BM / EC; ++ch) {
        const int R0 = ch * EC;
        // phase 1: accumulators -> LDS (only the blocks whose rows fall in this chunk)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            const int rb = wm * WAVE_M + mb * 32;
            if (rb >= R0 && rb < R0 + EC) {
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    const int cl = wn * WAVE_N + nb * 32 + (lane & 31);
#pragma unroll
                    for (int j = 0; j < 16; ++j) {
                        const int r = rb + 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3);
                        sY[(r - R0) * LDY + cl] = acc[mb][nb][j] * inv_s;
                    }
                }
            }
        }
        __syncthreads();
        // phase 2: row-major pass over the chunk (coalesced along columns)
#pragma unroll 4
        for (int e = tid; e < EC * BM; e += NT) {
            const int rl = e / BM, c = e % BM, r = R0 + rl;
            if (diag && r > c) continue;
            const int64_t gr = I0 + r, gc = J0 + c;
            const int64_t gi = gr * np + gc;
            const float y = sY[rl * LDY + c];
            const float x = X[gi];
            const float xn = fmaf(ca, y, fmaf(cb, x, gr == gc ? cc : 0.0f));
            if (!last) {
                X[gi] = xn;
                if (dn != 0.0f) A[gi] = fmaf(dn, xn, A[gi]);
                uint16_t h, l;
                split16<BF>(xn, h, l);
                p.hi_out[gi] = h;
                p.lo_out[gi] = l;
                sY[rl * LDY + c] = xn;
            } else {
                double v = (double)A[gi] + (double)xn;
                if (flip && !ent) v = (gr == gc ? 1.0 : 0.0) - v;
                const float vf = ent ? 0.0f : (float)v;
                const double vo = ent ? v : (double)vf;
                if (gr < n && gc < n) {
                    if (gr == gc) tr += vo;
                    sq += (gr == gc ? 1.0 : 2.0) * vo * vo;
                    if (!ent) {
                        if (p.out_mode == 0)
                            reinterpret_cast<float*>(p.D)[gr * p.ldd + gc] = vf;
                        else if (p.out_mode == 1)
                            reinterpret_cast<double*>(p.D)[gr * p.ldd + gc] = (double)vf;
                    }
                }
                sY[rl * LDY + c] = vf;
            }
        }
        __syncthreads();
        // phase 3: mirror pass, writes tile (J, I) = (I, J)^T (coalesced along the output row)
        if (!(last && (ent || p.out_mode == 2))) {
#pragma unroll 4
            for (int e = tid; e < EC * BM; e += NT) {
                const int rl = e % EC, c = e / EC, r = R0 + rl;
                if (diag && !(r < c)) continue;
                const float v = sY[rl * LDY + c];
                const int64_t orow = J0 + c, ocol = I0 + r;
                if (!last) {
                    uint16_t h, l;
                    split16<BF>(v, h, l);
                    p.hi_out[orow * np + ocol] = h;
                    p.lo_out[orow * np + ocol] = l;
                } else if (orow < n && ocol < n) {
                    if (p.out_mode == 0)
                        reinterpret_cast<float*>(p.D)[orow * p.ldd + ocol] = v;
                    else
                        reinterpret_cast<double*>(p.D)[orow * p.ldd + ocol] = (double)v;
                }
            }
        }
        __syncthreads();
    }

    if (last) {
        tr = wave_sum(tr);
        sq = wave_sum(sq);
        double* red = reinterpret_cast<double*>(smem);
        if (lane == 0) {
            red[2 * wave] = tr;
            red[2 * wave + 1] = sq;
        }
        __syncthreads();
        if (tid == 0) {
            double t = 0.0, s = 0.0;
            for (int w = 0; w < NT / 64; ++w) {
                t += red[2 * w];
                s += red[2 * w + 1];
            }
            p.partials[logical].tr = t;
            p.partials[logical].sq = s;
        }
    }
}

template <bool BF, int BM, int WM, int WN, int BK, int EC, int OCC>
hipError_t launch_cfg(const LayerArgs& a, hipStream_t s) {
    constexpr int NT = WM * WN * 64;
    constexpr size_t kloop = (size_t)4 * BM * (BK + 8) * sizeof(uint16_t);
    constexpr size_t epi = (size_t)EC * (BM + 1) * sizeof(float);
    constexpr size_t lds = kloop > epi ? kloop : epi;
    auto kern = k_layer_split<BF, BM, WM, WN, BK, EC, OCC>;
    static bool attr_done = false;
    if (!attr_done) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr_done = true;
    }
    const int T = (int)(a.np / BM);
    const int ntiles = T * (T + 1) / 2;
    hipLaunchKernelGGL(kern, dim3(ntiles), dim3(NT), lds, s, a);
    return hipGetLastError();
}

}  // namespace

int split_tile_ok(int tile) { return tile == 128 || tile == 256; }

hipError_t launch_layer_split(const LayerArgs& a, int bf16, int tile, hipStream_t s) {
    if (tile == 256) {
        return bf16 ? launch_cfg<true, 256, 2, 2, 32, 64, 1>(a, s) : launch_cfg<false, 256, 2, 2, 32, 64, 1>(a, s);
    }
    return bf16 ? launch_cfg<true, 128, 2, 2, 32, 64, 2>(a, s) : launch_cfg<false, 128, 2, 2, 32, 64, 2>(a, s);
}

}  // namespace fe
