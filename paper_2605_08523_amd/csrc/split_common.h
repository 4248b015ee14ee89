// Device building blocks shared by the split-precision layer kernels (data-parallel and
// stream-K): operand split, the three-product MFMA step, the LDS-staged K loop and the fused
// epilogue of one upper-triangle tile.
#pragma once

#include "fe_internal.h"

namespace fe {
namespace split {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));   // 8 16-bit operands

// x = hi + lo / s with s = 2^11 for FP16 (keeps lo out of the FP16 subnormals) and s = 1 for BF16;
// x - hi is exact in FP32, lo is its rounding.
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

// hi scaled by s (exact power-of-two scaling for FP16; identity for BF16).
template <bool BF>
__device__ inline u32x4 scale_hi(u32x4 ah) {
    if constexpr (!BF) {
        const half8 h = __builtin_bit_cast(half8, ah) * (_Float16)2048.0f;
        return __builtin_bit_cast(u32x4, h);
    } else {
        return ah;
    }
}

// acc += (s hi_a) hi_b + hi_a lo_b + lo_a hi_b  (three 32x32x16 MFMAs, FP32 accumulate) = s (X^2)
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

// Tile t of the row-major walk over the upper triangle of a T x T tile grid.
__device__ inline void tile_coords(int t, int T, int& I, int& J) {
    int rem = t, i = 0;
    while (rem >= T - i) {
        rem -= T - i;
        ++i;
    }
    I = i;
    J = i + rem;
}

// Compile-time shape of one kernel configuration.
template <int BM_, int WM_, int WN_, int BK_, int EC_, int STAGES_>
struct Cfg {
    static constexpr int BM = BM_, WM = WM_, WN = WN_, BK = BK_, EC = EC_, STAGES = STAGES_;
    static constexpr int NT = WM * WN * 64;
    static constexpr int LDK = BK + 8;                // padded LDS row (16-bit elements)
    static constexpr int WAVE_M = BM / WM, WAVE_N = BM / WN;
    static constexpr int MB = WAVE_M / 32, NB = WAVE_N / 32;
    static constexpr int CPR = BK / 8;                // 16-byte chunks per panel row
    static constexpr int CH = BM * CPR / NT;          // chunks per thread per array
    static constexpr int LDY = BM + 1;                // epilogue staging row (floats)
    static constexpr size_t STAGE_ELEMS = (size_t)4 * BM * LDK;
    static constexpr size_t KLOOP_BYTES = STAGES * STAGE_ELEMS * sizeof(uint16_t);
    static constexpr size_t EPI_BYTES = (size_t)EC * LDY * sizeof(float);
    static constexpr size_t LDS_BYTES = KLOOP_BYTES > EPI_BYTES ? KLOOP_BYTES : EPI_BYTES;
    static_assert(BM * CPR % NT == 0, "load split");
    static_assert(WAVE_M % 32 == 0 && WAVE_N % 32 == 0, "wave tile");
    static_assert(BM % EC == 0 && EC % 32 == 0 && (EC * BM) % NT == 0, "epilogue chunk");
};

template <class C>
struct Acc {
    floatx16 v[C::MB][C::NB];
};

// acc += s * (rows I0..I0+BM) (rows J0..J0+BM)^T over K blocks [kb0, kb1) of the current layer's
// hi/lo operands. STAGES = 1: single LDS buffer with register prefetch (two barriers per block);
// STAGES = 2: double-buffered LDS (one barrier per block).
template <bool BF, class C>
__device__ inline void kloop(const uint16_t* __restrict__ hin, const uint16_t* __restrict__ lin,
                             int64_t np, int64_t I0, int64_t J0, int kb0, int kb1, Acc<C>& acc,
                             uint16_t* smem) {
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));   // keep address arithmetic inside a caller's persistent loop
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave / C::WN, wn = wave % C::WN;
    int64_t goffI[C::CH], goffJ[C::CH];
    int soff[C::CH];
#pragma unroll
    for (int q = 0; q < C::CH; ++q) {
        const int cidx = tid + q * C::NT;
        const int row = cidx / C::CPR, kc = cidx % C::CPR;
        goffI[q] = (I0 + row) * np + kc * 8;
        goffJ[q] = (J0 + row) * np + kc * 8;
        soff[q] = row * C::LDK + kc * 8;
    }
    u32x4 pAh[C::CH], pAl[C::CH], pBh[C::CH], pBl[C::CH];
    auto gl = [&](int kb) {
        const int64_t k0 = (int64_t)kb * C::BK;
#pragma unroll
        for (int q = 0; q < C::CH; ++q) {
            pAh[q] = *reinterpret_cast<const u32x4*>(hin + goffI[q] + k0);
            pAl[q] = *reinterpret_cast<const u32x4*>(lin + goffI[q] + k0);
            pBh[q] = *reinterpret_cast<const u32x4*>(hin + goffJ[q] + k0);
            pBl[q] = *reinterpret_cast<const u32x4*>(lin + goffJ[q] + k0);
        }
    };
    auto st = [&](uint16_t* buf) {
        uint16_t* sAh = buf;
        uint16_t* sAl = sAh + C::BM * C::LDK;
        uint16_t* sBh = sAl + C::BM * C::LDK;
        uint16_t* sBl = sBh + C::BM * C::LDK;
#pragma unroll
        for (int q = 0; q < C::CH; ++q) {
            *reinterpret_cast<u32x4*>(sAh + soff[q]) = pAh[q];
            *reinterpret_cast<u32x4*>(sAl + soff[q]) = pAl[q];
            *reinterpret_cast<u32x4*>(sBh + soff[q]) = pBh[q];
            *reinterpret_cast<u32x4*>(sBl + soff[q]) = pBl[q];
        }
    };
    const int frag_row = lane & 31, frag_k = (lane >> 5) * 8;
    auto compute = [&](const uint16_t* buf) {
        const uint16_t* sAh = buf;
        const uint16_t* sAl = sAh + C::BM * C::LDK;
        const uint16_t* sBh = sAl + C::BM * C::LDK;
        const uint16_t* sBl = sBh + C::BM * C::LDK;
#pragma unroll
        for (int ks = 0; ks < C::BK / 16; ++ks) {
            u32x4 ah[C::MB], al[C::MB], bh[C::NB], bl[C::NB];
#pragma unroll
            for (int mb = 0; mb < C::MB; ++mb) {
                const int o = (wm * C::WAVE_M + mb * 32 + frag_row) * C::LDK + ks * 16 + frag_k;
                ah[mb] = *reinterpret_cast<const u32x4*>(sAh + o);
                al[mb] = *reinterpret_cast<const u32x4*>(sAl + o);
            }
#pragma unroll
            for (int nb = 0; nb < C::NB; ++nb) {
                const int o = (wn * C::WAVE_N + nb * 32 + frag_row) * C::LDK + ks * 16 + frag_k;
                bh[nb] = *reinterpret_cast<const u32x4*>(sBh + o);
                bl[nb] = *reinterpret_cast<const u32x4*>(sBl + o);
            }
#pragma unroll
            for (int mb = 0; mb < C::MB; ++mb) {
                const u32x4 ahs = scale_hi<BF>(ah[mb]);
#pragma unroll
                for (int nb = 0; nb < C::NB; ++nb)
                    acc.v[mb][nb] = mfma3<BF>(ahs, ah[mb], al[mb], bh[nb], bl[nb], acc.v[mb][nb]);
            }
            // keep one K step's operands live at a time (the scheduler would otherwise hoist the
            // next step's LDS reads and spill the accumulators)
            __builtin_amdgcn_sched_barrier(0);
        }
    };

    if constexpr (C::STAGES == 1) {
        gl(kb0);
        st(smem);
        __syncthreads();
        for (int kb = kb0; kb < kb1; ++kb) {
            const bool more = kb + 1 < kb1;
            if (more) gl(kb + 1);
            compute(smem);
            __syncthreads();
            if (more) {
                st(smem);
                __syncthreads();
            }
        }
    } else {
        uint16_t* buf0 = smem;
        uint16_t* buf1 = smem + C::STAGE_ELEMS;
        gl(kb0);
        st(buf0);
        if (kb0 + 1 < kb1) gl(kb0 + 1);
        __syncthreads();
        for (int kb = kb0; kb < kb1; ++kb) {
            uint16_t* cur = ((kb - kb0) & 1) ? buf1 : buf0;
            uint16_t* nxt = ((kb - kb0) & 1) ? buf0 : buf1;
            if (kb + 1 < kb1) st(nxt);          // nxt was last read before the previous barrier
            if (kb + 2 < kb1) gl(kb + 2);
            compute(cur);
            __syncthreads();
        }
    }
}

// Fused epilogue of tile (I, J), I <= J, from the accumulators (which hold s X^2):
//   X' = a X^2 + b X + c delta_ij;  A += d_next X';  write the FP32 master, the next layer's
//   hi/lo (tile and mirror).  On the last layer: D = A + X' (delta_ij - D if flipped), written to
//   the tile and its mirror, or (entropy) U = A + X' traced only; FP64 partial traces per tile.
template <bool BF, class C>
__device__ inline void epilogue(const LayerArgs& p, const Acc<C>& acc, float* sY, int I, int J,
                                int tile_index) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / C::WN, wn = wave % C::WN;
    const int64_t np = p.np;
    const int64_t I0 = (int64_t)I * C::BM, J0 = (int64_t)J * C::BM;
    const bool diag = (I == J);
    const float inv_s = BF ? 1.0f : (1.0f / 2048.0f);
    const float ca = p.a, cb = p.b, cc = p.c, dn = p.d_next;
    const bool last = p.last != 0;
    const bool ent = p.entropy != 0;
    const int flip = (last && !ent) ? p.P->flipped : 0;
    const int64_t n = p.n;
    float* __restrict__ X = p.X;
    float* __restrict__ A = p.A;
    double tr = 0.0, sq = 0.0;

#pragma unroll 1
    for (int ch = 0; ch < C::BM / C::EC; ++ch) {
        const int R0 = ch * C::EC;
#pragma unroll
        for (int mb = 0; mb < C::MB; ++mb) {
            const int rb = wm * C::WAVE_M + mb * 32;
            if (rb >= R0 && rb < R0 + C::EC) {
#pragma unroll
                for (int nb = 0; nb < C::NB; ++nb) {
                    const int cl = wn * C::WAVE_N + nb * 32 + (lane & 31);
#pragma unroll
                    for (int j = 0; j < 16; ++j) {
                        // 32x32 MFMA result layout: acc[j] of lane l is row 8(j/4) + 4(l/32) + j%4, column l%32
                        const int r = rb + 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3);
                        sY[(r - R0) * C::LDY + cl] = acc.v[mb][nb][j] * inv_s;
                    }
                }
            }
        }
        __syncthreads();
#pragma unroll 4
        for (int e = tid; e < C::EC * C::BM; e += C::NT) {
            const int rl = e / C::BM, c = e % C::BM, r = R0 + rl;
            if (diag && r > c) continue;
            const int64_t gr = I0 + r, gc = J0 + c;
            const int64_t gi = gr * np + gc;
            const float y = sY[rl * C::LDY + c];
            const float x = X[gi];
            const float xn = fmaf(ca, y, fmaf(cb, x, gr == gc ? cc : 0.0f));
            if (!last) {
                X[gi] = xn;
                if (dn != 0.0f) A[gi] = fmaf(dn, xn, A[gi]);
                uint16_t h, l;
                split16<BF>(xn, h, l);
                p.hi_out[gi] = h;
                p.lo_out[gi] = l;
                sY[rl * C::LDY + c] = xn;
            } else {
                double v = (double)A[gi] + (double)xn;
                if (flip) v = (gr == gc ? 1.0 : 0.0) - v;
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
                sY[rl * C::LDY + c] = vf;
            }
        }
        __syncthreads();
        if (!(last && (ent || p.out_mode == 2))) {
#pragma unroll 4
            for (int e = tid; e < C::EC * C::BM; e += C::NT) {
                const int rl = e % C::EC, c = e / C::EC, r = R0 + rl;
                if (diag && !(r < c)) continue;
                const float v = sY[rl * C::LDY + c];
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
        double* red = reinterpret_cast<double*>(sY);
        if (lane == 0) {
            red[2 * wave] = tr;
            red[2 * wave + 1] = sq;
        }
        __syncthreads();
        if (tid == 0) {
            double t = 0.0, s = 0.0;
            for (int w = 0; w < C::NT / 64; ++w) {
                t += red[2 * w];
                s += red[2 * w + 1];
            }
            p.partials[tile_index].tr = t;
            p.partials[tile_index].sq = s;
        }
        __syncthreads();
    }
}

// Store the accumulators of a BM x BM tile (scaled by 1/s, i.e. as X^2) row-major into dst.
// Each store instruction writes two 128-byte row segments.
template <bool BF, class C>
__device__ inline void store_tile(const Acc<C>& acc, float* __restrict__ dst) {
    int tid = threadIdx.x;
    // Opaque to the optimiser: inside a persistent loop the 256 element offsets below would
    // otherwise be hoisted out of the loop and kept in (spilled) registers.
    asm volatile("" : "+v"(tid));
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave / C::WN, wn = wave % C::WN;
    const float inv_s = BF ? 1.0f : (1.0f / 2048.0f);
#pragma unroll
    for (int mb = 0; mb < C::MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < C::NB; ++nb) {
            const int rb = wm * C::WAVE_M + mb * 32 + 4 * (lane >> 5);
            const int cl = wn * C::WAVE_N + nb * 32 + (lane & 31);
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int r = rb + 8 * (j >> 2) + (j & 3);
                dst[r * C::BM + cl] = acc.v[mb][nb][j] * inv_s;
            }
        }
}

// Fused epilogue of tile (I, J), I <= J, reading X^2 from memory: Y = Y0 + parts[0] + ... +
// parts[nparts-1] (row-major BM x BM FP32 tiles, added in this order). Same outputs as
// `epilogue`; X' is staged through LDS (EC rows at a time) for the transposed mirror pass.
template <bool BF, class C>
__device__ inline void epilogue_mem(const LayerArgs& p, const float* __restrict__ Y0,
                                    const float* __restrict__ parts, int nparts, float* sY, int I,
                                    int J, int tile_index) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t np = p.np;
    const int64_t I0 = (int64_t)I * C::BM, J0 = (int64_t)J * C::BM;
    const bool diag = (I == J);
    const float ca = p.a, cb = p.b, cc = p.c, dn = p.d_next;
    const bool last = p.last != 0;
    const bool ent = p.entropy != 0;
    const int flip = (last && !ent) ? p.P->flipped : 0;
    const int64_t n = p.n;
    float* __restrict__ X = p.X;
    float* __restrict__ A = p.A;
    double tr = 0.0, sq = 0.0;

#pragma unroll 1
    for (int ch = 0; ch < C::BM / C::EC; ++ch) {
        const int R0 = ch * C::EC;
#pragma unroll 4
        for (int e = tid; e < C::EC * C::BM; e += C::NT) {
            const int rl = e / C::BM, c = e % C::BM, r = R0 + rl;
            if (diag && r > c) continue;
            const int loc = r * C::BM + c;
            float y = Y0[loc];
            for (int q = 0; q < nparts; ++q) y += parts[(size_t)q * C::BM * C::BM + loc];
            const int64_t gr = I0 + r, gc = J0 + c;
            const int64_t gi = gr * np + gc;
            const float x = X[gi];
            const float xn = fmaf(ca, y, fmaf(cb, x, gr == gc ? cc : 0.0f));
            if (!last) {
                X[gi] = xn;
                if (dn != 0.0f) A[gi] = fmaf(dn, xn, A[gi]);
                uint16_t h, l;
                split16<BF>(xn, h, l);
                p.hi_out[gi] = h;
                p.lo_out[gi] = l;
                sY[rl * C::LDY + c] = xn;
            } else {
                double v = (double)A[gi] + (double)xn;
                if (flip) v = (gr == gc ? 1.0 : 0.0) - v;
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
                sY[rl * C::LDY + c] = vf;
            }
        }
        __syncthreads();
        if (!(last && (ent || p.out_mode == 2))) {
#pragma unroll 4
            for (int e = tid; e < C::EC * C::BM; e += C::NT) {
                const int rl = e % C::EC, c = e / C::EC, r = R0 + rl;
                if (diag && !(r < c)) continue;
                const float v = sY[rl * C::LDY + c];
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
        double* red = reinterpret_cast<double*>(sY);
        if (lane == 0) {
            red[2 * wave] = tr;
            red[2 * wave + 1] = sq;
        }
        __syncthreads();
        if (tid == 0) {
            double t = 0.0, s = 0.0;
            for (int w = 0; w < C::NT / 64; ++w) {
                t += red[2 * w];
                s += red[2 * w + 1];
            }
            p.partials[tile_index].tr = t;
            p.partials[tile_index].sq = s;
        }
        __syncthreads();
    }
}

}  // namespace split
}  // namespace fe
