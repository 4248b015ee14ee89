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
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));   // 4 16-bit values

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

// Three-part BF16 split (FE_PREC_BF16X3): x = h + m + l with h = bf16(x), m = bf16(x - h),
// l = bf16(x - h - m); both differences are exact in FP32, so h + m + l carries 24 significant
// bits of x (its FP32 value up to the last bit or two).
__device__ inline void split3(float x, uint16_t& h, uint16_t& m, uint16_t& l) {
    const __bf16 hh = (__bf16)x;
    const float r1 = x - (float)hh;
    const __bf16 mm = (__bf16)r1;
    const float r2 = r1 - (float)mm;
    const __bf16 ll = (__bf16)r2;
    h = __builtin_bit_cast(uint16_t, hh);
    m = __builtin_bit_cast(uint16_t, mm);
    l = __builtin_bit_cast(uint16_t, ll);
}

// acc += hh + hm + mh + hl + lh + mm over one 32x32x16 step (six BF16 MFMAs, FP32 accumulate):
// every product of parts down to 2^-16 of the leading one; the dropped ml, lm, ll are below
// 2^-24 relative.
__device__ inline floatx16 mfma6(const u32x4* a, const u32x4* b, floatx16 acc) {
#define FE_MFMA_BF(x, y) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, x), __builtin_bit_cast(bf16x8, y), acc, 0, 0, 0)
    FE_MFMA_BF(a[0], b[0]);
    FE_MFMA_BF(a[0], b[1]);
    FE_MFMA_BF(a[1], b[0]);
    FE_MFMA_BF(a[0], b[2]);
    FE_MFMA_BF(a[2], b[0]);
    FE_MFMA_BF(a[1], b[1]);
#undef FE_MFMA_BF
    return acc;
}

__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Tile t of a blocked walk over the upper triangle of a T x T tile grid: blocks of B x B tiles
// (bi, bj >= bi) in row-major block order, row-major inside a block (its upper part on the
// diagonal). A run of consecutive tiles (what one XCD's workgroups hold at a time) then touches
// fewer distinct row panels than a run of the plain row-major walk.
constexpr int kTileBlock = 8;
__device__ inline void tile_coords(int t, int T, int& I, int& J) {
    constexpr int B = kTileBlock;
    const int NB = (T + B - 1) / B;
    int rem = t;
    I = J = 0;
    for (int bi = 0; bi < NB; ++bi) {
        const int r0 = bi * B, h = T - r0 < B ? T - r0 : B;
        for (int bj = bi; bj < NB; ++bj) {
            const int c0 = bj * B, w = T - c0 < B ? T - c0 : B;
            const int cnt = bj == bi ? h * (h + 1) / 2 : h * w;
            if (rem < cnt) {
                if (bj != bi) {
                    I = r0 + rem / w;
                    J = c0 + rem % w;
                } else {
                    int i = 0;
                    while (rem >= h - i) {
                        rem -= h - i;
                        ++i;
                    }
                    I = r0 + i;
                    J = r0 + i + rem;
                }
                return;
            }
            rem -= cnt;
        }
    }
}

// Tile of data-parallel workgroup b among ntiles: the hardware deals workgroups to the 8 XCDs
// round-robin, so the workgroups b with one value of b % 8 share an XCD (which one depends on where
// the dispatch starts); each XCD is given a contiguous run of tiles.
__device__ inline int xcd_tile(int b, int ntiles) {
    const int per = ntiles / 8;
    return b < 8 * per ? (b % 8) * per + b / 8 : b;
}

// Compile-time shape of one kernel configuration. DMA = 1: operands go from global memory straight
// to LDS (no register staging), in unpadded rows whose 16-byte chunks are XOR-swizzled.
// NS = 3: three-part BF16 split (three operand arrays per panel), register-staged loop only.
template <int BM_, int WM_, int WN_, int BK_, int EC_, int STAGES_, int DMA_ = 0, int NS_ = 2>
struct Cfg {
    static constexpr int BM = BM_, WM = WM_, WN = WN_, BK = BK_, EC = EC_, STAGES = STAGES_;
    static constexpr int DMA = DMA_;
    static constexpr int NS = NS_;                    // operand parts (2: hi/lo, 3: hi/mid/lo)
    static constexpr int NT = WM * WN * 64;
    static constexpr int LDK = DMA ? BK : BK + 8;     // LDS row (16-bit elements)
    static constexpr int WAVE_M = BM / WM, WAVE_N = BM / WN;
    static constexpr int MB = WAVE_M / 32, NB = WAVE_N / 32;
    static constexpr int CPR = BK / 8;                // 16-byte chunks per panel row
    static constexpr int CH = BM * CPR / NT;          // chunks per thread per array
    static constexpr int LDY = BM + 4;                // epilogue staging row (floats, 16-B aligned)
    static constexpr size_t STAGE_ELEMS = (size_t)2 * NS * BM * LDK;
    static constexpr size_t KLOOP_BYTES = STAGES * STAGE_ELEMS * sizeof(uint16_t);
    static constexpr size_t EPI_BYTES = (size_t)EC * LDY * sizeof(float);
    static constexpr size_t LDS_BYTES = KLOOP_BYTES > EPI_BYTES ? KLOOP_BYTES : EPI_BYTES;
    static_assert(BM * CPR % NT == 0, "load split");
    static_assert(WAVE_M % 32 == 0 && WAVE_N % 32 == 0, "wave tile");
    static_assert(BM % EC == 0 && EC % 32 == 0 && (EC * BM) % NT == 0, "epilogue chunk");
    static_assert(EC % 16 == 0 && LDY % 4 == 0, "vectorised epilogue");
    static_assert(!DMA || (STAGES == 2 && BK >= 16 && BK <= 64 && (4 * BM * BK / 512) % (NT / 64) == 0),
                  "direct-to-LDS staging");
    static_assert(NS == 2 || (NS == 3 && STAGES == 1 && !DMA), "three-part split: one register-staged stage");
};

// N groups of (M MFMAs, one LDS read) for the scheduler.
template <int N, int M>
__device__ inline void sgb_interleave() {
    if constexpr (N > 0) {
        __builtin_amdgcn_sched_group_barrier(0x008, M, 0);
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
        sgb_interleave<N - 1, M>();
    }
}

template <class C>
struct Acc {
    floatx16 v[C::MB][C::NB];
};

// Direct-to-LDS form of the K loop (C::DMA): each lane's global_load_lds_dwordx4 moves one
// 16-byte chunk, and the 64 chunks of one instruction land in 1 KiB of LDS in lane order. A stage
// holds the four BM x BK operand panels (A hi, A lo, B hi, B lo) in unpadded rows; chunk c of row
// r sits at position c ^ ((r / RP) % CPR) of its row (RP rows per 128 bytes), so the eight rows
// that a quarter-wave's fragment read touches fall on distinct banks. Two stages: block kb + 1
// is in flight while block kb is multiplied. The barrier is a bare s_barrier after an explicit
// wait for this wave's own loads (a full __syncthreads would also drain everything else in
// flight); the fragment reads of the next K step are interleaved with the current step's MFMAs.
template <bool BF, class C>
__device__ inline void kloop_dma(const uint16_t* __restrict__ hin, const uint16_t* __restrict__ lin,
                                 int64_t np, int64_t I0, int64_t J0, int kb0, int kb1, Acc<C>& acc,
                                 uint16_t* smem) {
    typedef __attribute__((address_space(3))) void lds_void;
    typedef const __attribute__((address_space(1))) void global_void;
    constexpr int CPR = C::BK / 8, RP = 8 / CPR > 0 ? 8 / CPR : 1, RPI = 64 / CPR;
    constexpr int IPA = C::BM / RPI;                      // 1-KiB instructions per panel and stage
    constexpr int NW = C::NT / 64, IPW = 4 * IPA / NW;    // per wave and stage
    constexpr int PANEL = C::BM * C::BK, STAGE = 4 * PANEL;
    static_assert((RPI / RP) % CPR == 0, "a lane's chunk position is the same in every instruction");
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave / C::WN, wn = wave % C::WN;
    auto swz = [](int r, int c) { return c ^ ((r / RP) % CPR); };
    // Instruction q of this wave covers panel a, rows blk * RPI .. + RPI - 1: a wave-uniform base
    // (scalar registers) plus the lane's offset, the same for every q.
    const int wave_u = __builtin_amdgcn_readfirstlane(wave);
    const uint32_t lane_off = (uint32_t)((lane / CPR) * np + swz(lane / CPR, lane % CPR) * 8);
    const uint16_t* src[IPW];
    int dst[IPW];
#pragma unroll
    for (int q = 0; q < IPW; ++q) {
        const int gi = wave_u + q * NW, a = gi / IPA, blk = gi % IPA;
        src[q] = ((a & 1) ? lin : hin) + ((a < 2 ? I0 : J0) + blk * RPI) * np;
        dst[q] = a * PANEL + blk * RPI * C::BK;
    }
    auto issue = [&](int kb, uint16_t* stage) {
        const int64_t k0 = (int64_t)kb * C::BK;
#pragma unroll
        for (int q = 0; q < IPW; ++q)
            __builtin_amdgcn_global_load_lds((global_void*)(src[q] + k0 + lane_off),
                                             (lds_void*)(stage + dst[q]), 16, 0, 0);
    };
    const int frag_row = lane & 31, frag_c = lane >> 5;
    struct Frag {
        u32x4 ah[C::MB], al[C::MB], bh[C::NB], bl[C::NB];
    };
    auto ld = [&](const uint16_t* stage, int ks, Frag& f) {
#pragma unroll
        for (int mb = 0; mb < C::MB; ++mb) {
            const int r = wm * C::WAVE_M + mb * 32 + frag_row;
            const int o = r * C::BK + swz(r, ks * 2 + frag_c) * 8;
            f.ah[mb] = *reinterpret_cast<const u32x4*>(stage + o);
            f.al[mb] = *reinterpret_cast<const u32x4*>(stage + PANEL + o);
        }
#pragma unroll
        for (int nb = 0; nb < C::NB; ++nb) {
            const int r = wn * C::WAVE_N + nb * 32 + frag_row;
            const int o = r * C::BK + swz(r, ks * 2 + frag_c) * 8;
            f.bh[nb] = *reinterpret_cast<const u32x4*>(stage + 2 * PANEL + o);
            f.bl[nb] = *reinterpret_cast<const u32x4*>(stage + 3 * PANEL + o);
        }
    };
    auto mm = [&](const Frag& f) {
#pragma unroll
        for (int mb = 0; mb < C::MB; ++mb) {
            const u32x4 ahs = scale_hi<BF>(f.ah[mb]);
#pragma unroll
            for (int nb = 0; nb < C::NB; ++nb)
                acc.v[mb][nb] = mfma3<BF>(ahs, f.ah[mb], f.al[mb], f.bh[nb], f.bl[nb], acc.v[mb][nb]);
        }
    };
    // Scheduling of one step: the hi scaling first, then each fragment read of the next step
    // between MFMAs of this one.
    constexpr int NDS = 2 * (C::MB + C::NB), NMF = 3 * C::MB * C::NB;
    constexpr int PER = NMF >= 2 * NDS ? 2 : 1;   // MFMAs between two fragment reads
    static_assert(NMF >= PER * NDS, "interleave pattern");
    auto pattern = [&](bool reads) {
        __builtin_amdgcn_sched_group_barrier(0x002, 4 * C::MB, 0);
        if (reads) {
            sgb_interleave<NDS, PER>();
            __builtin_amdgcn_sched_group_barrier(0x008, NMF - PER * NDS, 0);
        } else {
            __builtin_amdgcn_sched_group_barrier(0x008, NMF, 0);
        }
        __builtin_amdgcn_sched_barrier(0);
    };
    constexpr int KS = C::BK / 16;
    static_assert(KS % 2 == 0, "two fragment sets");
    auto compute = [&](const uint16_t* stage) {
        Frag f0, f1;
        ld(stage, 0, f0);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int ks = 0; ks < KS; ks += 2) {
            ld(stage, ks + 1, f1);
            mm(f0);
            pattern(true);
            if (ks + 2 < KS) {
                ld(stage, ks + 2, f0);
                mm(f1);
                pattern(true);
            } else {
                mm(f1);
                pattern(false);
            }
        }
    };
    if (kb0 < kb1) issue(kb0, smem);
    for (int kb = kb0; kb < kb1; ++kb) {
        uint16_t* cur = smem + ((kb - kb0) & 1) * STAGE;
        uint16_t* nxt = smem + (((kb - kb0) & 1) ^ 1) * STAGE;
        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this wave's chunks of block kb landed
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();          // ... and every wave's; nxt is no longer read
        asm volatile("" ::: "memory");
        if (kb + 1 < kb1) issue(kb + 1, nxt);
        compute(cur);
    }
    asm volatile("" ::: "memory");
    __syncthreads();
}

// acc += s * (rows I0..I0+BM) (rows J0..J0+BM)^T over K blocks [kb0, kb1) of the current layer's
// hi/lo operands. STAGES = 1: single LDS buffer with register prefetch (two barriers per block);
// STAGES = 2: double-buffered LDS (one barrier per block); DMA: see kloop_dma. Ends with a
// barrier.
template <bool BF, class C>
__device__ inline void kloop(const uint16_t* __restrict__ hin, const uint16_t* __restrict__ lin,
                             int64_t np, int64_t I0, int64_t J0, int kb0, int kb1, Acc<C>& acc,
                             uint16_t* smem) {
    if constexpr (C::DMA) {
        kloop_dma<BF, C>(hin, lin, np, I0, J0, kb0, kb1, acc, smem);
        return;
    }
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
    struct Frag {
        u32x4 ah[C::MB], al[C::MB], bh[C::NB], bl[C::NB];
    };
    auto ld = [&](const uint16_t* buf, int ks, Frag& f) {
        const uint16_t* sAh = buf;
        const uint16_t* sAl = sAh + C::BM * C::LDK;
        const uint16_t* sBh = sAl + C::BM * C::LDK;
        const uint16_t* sBl = sBh + C::BM * C::LDK;
#pragma unroll
        for (int mb = 0; mb < C::MB; ++mb) {
            const int o = (wm * C::WAVE_M + mb * 32 + frag_row) * C::LDK + ks * 16 + frag_k;
            f.ah[mb] = *reinterpret_cast<const u32x4*>(sAh + o);
            f.al[mb] = *reinterpret_cast<const u32x4*>(sAl + o);
        }
#pragma unroll
        for (int nb = 0; nb < C::NB; ++nb) {
            const int o = (wn * C::WAVE_N + nb * 32 + frag_row) * C::LDK + ks * 16 + frag_k;
            f.bh[nb] = *reinterpret_cast<const u32x4*>(sBh + o);
            f.bl[nb] = *reinterpret_cast<const u32x4*>(sBl + o);
        }
    };
    auto mm = [&](const Frag& f) {
#pragma unroll
        for (int mb = 0; mb < C::MB; ++mb) {
            const u32x4 ahs = scale_hi<BF>(f.ah[mb]);
#pragma unroll
            for (int nb = 0; nb < C::NB; ++nb)
                acc.v[mb][nb] = mfma3<BF>(ahs, f.ah[mb], f.al[mb], f.bh[nb], f.bl[nb], acc.v[mb][nb]);
        }
    };
    // Small wave tiles read the next K step's fragments from LDS while the current step's
    // MFMAs run (two fragment sets live); large ones keep one set (register budget). The
    // scheduling barriers stop the compiler from hoisting further LDS reads, which would spill
    // the accumulators.
    constexpr int KS = C::BK / 16;
    constexpr bool kPipe = C::MB * C::NB <= 4 && KS % 2 == 0;
    auto compute = [&](const uint16_t* buf) {
        if constexpr (kPipe) {
            Frag f0, f1;
            ld(buf, 0, f0);
#pragma unroll
            for (int ks = 0; ks < KS; ks += 2) {
                ld(buf, ks + 1, f1);
                mm(f0);
                __builtin_amdgcn_sched_barrier(0);
                if (ks + 2 < KS) ld(buf, ks + 2, f0);
                mm(f1);
                __builtin_amdgcn_sched_barrier(0);
            }
        } else {
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                Frag f;
                ld(buf, ks, f);
                mm(f);
                __builtin_amdgcn_sched_barrier(0);
            }
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

// K loop of the three-part BF16 split (C::NS = 3): acc += the six products of rows I0..I0+BM and
// rows J0..J0+BM over K blocks [kb0, kb1) of the hi/mid/lo operands (same block order as kloop,
// so an element's sum does not depend on the tile's wave layout). One LDS stage holding the six
// BM x BK panels, register prefetch of the next block, one fragment set (register budget).
// Ends with a barrier.
template <class C>
__device__ inline void kloop3(const uint16_t* __restrict__ hin, const uint16_t* __restrict__ min,
                              const uint16_t* __restrict__ lin, int64_t np, int64_t I0, int64_t J0,
                              int kb0, int kb1, Acc<C>& acc, uint16_t* smem) {
    static_assert(C::NS == 3, "three-part split");
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave / C::WN, wn = wave % C::WN;
    constexpr int P = C::BM * C::LDK;   // one panel in LDS
    const uint16_t* src[3] = {hin, min, lin};
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
    u32x4 pA[3][C::CH], pB[3][C::CH];
    auto gl = [&](int kb) {
        const int64_t k0 = (int64_t)kb * C::BK;
#pragma unroll
        for (int q = 0; q < C::CH; ++q)
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                pA[t][q] = *reinterpret_cast<const u32x4*>(src[t] + goffI[q] + k0);
                pB[t][q] = *reinterpret_cast<const u32x4*>(src[t] + goffJ[q] + k0);
            }
    };
    auto st = [&](uint16_t* buf) {   // panels: A hi, mid, lo, then B hi, mid, lo
#pragma unroll
        for (int q = 0; q < C::CH; ++q)
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                *reinterpret_cast<u32x4*>(buf + t * P + soff[q]) = pA[t][q];
                *reinterpret_cast<u32x4*>(buf + (3 + t) * P + soff[q]) = pB[t][q];
            }
    };
    const int frag_row = lane & 31, frag_k = (lane >> 5) * 8;
    auto compute = [&](const uint16_t* buf) {
#pragma unroll
        for (int ks = 0; ks < C::BK / 16; ++ks) {
            u32x4 fa[C::MB][3], fb[C::NB][3];
#pragma unroll
            for (int mb = 0; mb < C::MB; ++mb) {
                const int o = (wm * C::WAVE_M + mb * 32 + frag_row) * C::LDK + ks * 16 + frag_k;
#pragma unroll
                for (int t = 0; t < 3; ++t) fa[mb][t] = *reinterpret_cast<const u32x4*>(buf + t * P + o);
            }
#pragma unroll
            for (int nb = 0; nb < C::NB; ++nb) {
                const int o = (wn * C::WAVE_N + nb * 32 + frag_row) * C::LDK + ks * 16 + frag_k;
#pragma unroll
                for (int t = 0; t < 3; ++t)
                    fb[nb][t] = *reinterpret_cast<const u32x4*>(buf + (3 + t) * P + o);
            }
#pragma unroll
            for (int mb = 0; mb < C::MB; ++mb)
#pragma unroll
                for (int nb = 0; nb < C::NB; ++nb) acc.v[mb][nb] = mfma6(fa[mb], fb[nb], acc.v[mb][nb]);
            __builtin_amdgcn_sched_barrier(0);
        }
    };
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
}

// Four consecutive values split into hi/lo, each packed for one 8-byte store.
template <bool BF>
__device__ inline void split4(floatx4 v, u32x2& h, u32x2& l) {
    uint16_t h0, l0, h1, l1, h2, l2, h3, l3;
    split16<BF>(v[0], h0, l0);
    split16<BF>(v[1], h1, l1);
    split16<BF>(v[2], h2, l2);
    split16<BF>(v[3], h3, l3);
    h = u32x2{(unsigned)h0 | ((unsigned)h1 << 16), (unsigned)h2 | ((unsigned)h3 << 16)};
    l = u32x2{(unsigned)l0 | ((unsigned)l1 << 16), (unsigned)l2 | ((unsigned)l3 << 16)};
}

// Four consecutive values in three BF16 parts, each packed for one 8-byte store.
__device__ inline void split4x3(floatx4 v, u32x2& h, u32x2& m, u32x2& l) {
    uint16_t hh[4], mm[4], ll[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) split3(v[k], hh[k], mm[k], ll[k]);
    h = u32x2{(unsigned)hh[0] | ((unsigned)hh[1] << 16), (unsigned)hh[2] | ((unsigned)hh[3] << 16)};
    m = u32x2{(unsigned)mm[0] | ((unsigned)mm[1] << 16), (unsigned)mm[2] | ((unsigned)mm[3] << 16)};
    l = u32x2{(unsigned)ll[0] | ((unsigned)ll[1] << 16), (unsigned)ll[2] | ((unsigned)ll[3] << 16)};
}

// Next-layer operands of four consecutive elements at `o`: hi/lo, or hi/mid/lo (C::NS = 3).
template <bool BF, class C>
__device__ inline void store_split4(const LayerArgs& p, int64_t o, floatx4 v) {
    if constexpr (C::NS == 3) {
        u32x2 h, m, l;
        split4x3(v, h, m, l);
        *reinterpret_cast<u32x2*>(p.hi_out + o) = h;
        *reinterpret_cast<u32x2*>(p.mid_out + o) = m;
        *reinterpret_cast<u32x2*>(p.lo_out + o) = l;
    } else {
        u32x2 h, l;
        split4<BF>(v, h, l);
        *reinterpret_cast<u32x2*>(p.hi_out + o) = h;
        *reinterpret_cast<u32x2*>(p.lo_out + o) = l;
    }
}
// ... of one element.
template <bool BF, class C>
__device__ inline void store_split1(const LayerArgs& p, int64_t o, float v) {
    if constexpr (C::NS == 3) {
        uint16_t h, m, l;
        split3(v, h, m, l);
        p.hi_out[o] = h;
        p.mid_out[o] = m;
        p.lo_out[o] = l;
    } else {
        uint16_t h, l;
        split16<BF>(v, h, l);
        p.hi_out[o] = h;
        p.lo_out[o] = l;
    }
}

// Device-coherent (agent scope) 32-bit accesses. Each one is coherent across the XCDs' L2
// caches by itself (global_store/load with sc1), so data handed between workgroups this way needs
// no cache-wide write-back or invalidate: those would also throw away the operand panels that
// every other workgroup of the XCD is streaming through the same L2.
__device__ inline void store_coherent(float* p, float v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline float load_coherent(const float* p) {
    return __hip_atomic_load(const_cast<float*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Buffer resource over [base, base + bytes) for raw buffer accesses (lanes outside the range
// read zero and drop their stores).
__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                             0x00020000);
}
constexpr int kCoherentAux = 16;   // cache policy sc1: device-coherent access

// Four consecutive floats at byte offset off of a buffer, read device-coherently (16 bytes).
__device__ inline floatx4 load4_coherent(__amdgpu_buffer_rsrc_t rs, int off) {
    return __builtin_bit_cast(floatx4, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, kCoherentAux));
}

// One chunk (tile rows R0 .. R0+EC-1) of the fused epilogue of tile (I, J), I <= J:
//   Y = X^2 (from sY, or from the row-major BM x BM tile Y0 in memory if Y0 is set) plus the
//   partial tiles parts[0..nparts-1] (part_stride floats apart, written by other workgroups and
//   read device-coherently, added in this order);
//   X' = a Y + b X + c delta_ij;  A += d_old X + d_new X';  write the FP32 master and the next layer's
//   hi/lo for the tile (row-major pass, four columns per thread) and its mirror (transposed pass
//   through sY, four rows per thread). With p.affine (squared-affine form) X' is the next operand
//   itself: X is neither read nor written (b = d_old = 0). On the last layer: D = A + X' (delta_ij - D if flipped)
//   written to the tile and its mirror, or (entropy) U = A + X' traced only; FP64 trace sums
//   accumulate in tr, sq. Diagonal tiles keep only the upper triangle of X and A, and their lower
//   half of hi/lo (or D) comes from the mirror pass, so every stored matrix is exactly symmetric.
//   poisoned: every output of the tile is NaN (a stream-K wait gave up).
//   Padding (rows or columns >= n): four-column groups that lie wholly in it are neither read nor
//   written, so the padded part of every stored matrix keeps the values the rescale gave it
//   (zero off the diagonal): X stays block diagonal, and the real block never sees a padded
//   value. (Groups that straddle n are computed whole: their padded entries come out zero.)
// Ends with a barrier (sY is free again).
template <bool BF, class C, int UMAX>
__device__ inline void epi_chunk(const LayerArgs& p, float* sY, int R0, int I, int J,
                                 const float* __restrict__ Y0, const float* __restrict__ parts,
                                 size_t part_stride, int nparts, double& tr, double& sq,
                                 bool poisoned) {
    const int tid = threadIdx.x;
    const int64_t np = p.np;
    const int64_t I0 = (int64_t)I * C::BM, J0 = (int64_t)J * C::BM;
    const bool diag = (I == J);
    // poisoned: the tile's partials could not be trusted (a stream-K wait gave up); a NaN weight
    // makes every output of the tile NaN
    const float ca = poisoned ? __builtin_nanf("") : p.a;
    const float cb = p.b, cc = p.c, dold = p.d_old, dnew = p.d_new;
    const bool upd = dold != 0.0f || dnew != 0.0f;
    const bool last = p.last != 0;
    const bool ent = p.entropy != 0;
    const int flip = (last && !ent) ? p.P->flipped : 0;
    const int64_t n = p.n;
    float* __restrict__ X = p.X;
    float* __restrict__ A = p.A;
    constexpr int G = C::BM / 4;                  // four-column groups per tile row
    constexpr int PER = C::EC * G / C::NT;        // groups per thread in this chunk
    constexpr int U = (PER % 4 == 0 && UMAX >= 4) ? 4 : (PER % 2 == 0 && UMAX >= 2) ? 2 : 1;
    const uint32_t part_bytes = (uint32_t)(C::BM * C::BM * sizeof(float));
    const bool load_a = last || upd;
    const bool use_x = p.affine == 0;   // squared-affine form: no FP32 state besides A

    // Row-major pass: groups of four consecutive columns, 16-byte accesses, in batches of U
    // groups per thread. The loads of batch i + 1 are issued before the stores of batch i: the
    // vector-memory counter is in order and counts stores too, so a wait for loads issued after
    // a batch's stores would also wait for those stores to complete.
    constexpr int NBATCH = PER / U;
    struct Batch {
        floatx4 y[U], x[U], a[U], p[U];
    };
    auto load_batch = [&](int b0, Batch& bt) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = tid + (b0 + u) * C::NT;
            const int rl = e / G, c = (e % G) * 4, r = R0 + rl;
            const int loc = r * C::BM + c;
            const int64_t gi = (I0 + r) * np + J0 + c;
            const bool live = I0 + r < n && J0 + c < n;
            bt.y[u] = Y0 ? *reinterpret_cast<const floatx4*>(Y0 + loc)
                         : *reinterpret_cast<const floatx4*>(sY + rl * C::LDY + c);
            if (nparts > 0)
                bt.p[u] = load4_coherent(make_rsrc(parts, part_bytes), loc * (int)sizeof(float));
            const floatx4 z{0.0f, 0.0f, 0.0f, 0.0f};
            bt.x[u] = (use_x && live) ? *reinterpret_cast<const floatx4*>(X + gi) : z;
            bt.a[u] = (load_a && live) ? *reinterpret_cast<const floatx4*>(A + gi) : z;
        }
    };
    auto finish_batch = [&](int b0, Batch& bt) {
        floatx4* y = bt.y;
        floatx4* x = bt.x;
        floatx4* a = bt.a;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (nparts > 0) {
                // parts in order: the first was loaded with the batch, the rest now
                const int e = tid + (b0 + u) * C::NT;
                const int loc = (R0 + e / G) * C::BM + (e % G) * 4;
#pragma unroll
                for (int k = 0; k < 4; ++k) y[u][k] += bt.p[u][k];
                for (int q = 1; q < nparts; ++q) {
                    const floatx4 v = load4_coherent(
                        make_rsrc(parts + (size_t)q * part_stride, part_bytes), loc * (int)sizeof(float));
#pragma unroll
                    for (int k = 0; k < 4; ++k) y[u][k] += v[k];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = tid + (b0 + u) * C::NT;
            const int rl = e / G, c = (e % G) * 4, r = R0 + rl;
            if (diag && c + 3 < r) continue;   // entirely below the diagonal
            float* srow = sY + rl * C::LDY + c;
            const int64_t gr = I0 + r, gc = J0 + c;
            const int64_t gi = gr * np + gc;
            if (!last && (gr >= n || gc >= n)) {   // wholly in the padding: left as it is
                *reinterpret_cast<floatx4*>(srow) = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
                continue;
            }
            floatx4 xn;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                xn[k] = fmaf(ca, y[u][k], fmaf(cb, x[u][k], gr == gc + k ? cc : 0.0f));
            const bool full = !diag || c >= r;
            if (!last) {
                if (full) {
                    if (use_x) *reinterpret_cast<floatx4*>(X + gi) = xn;
                    if (upd) {
                        floatx4 a4;
#pragma unroll
                        for (int k = 0; k < 4; ++k)
                            a4[k] = fmaf(dnew, xn[k], fmaf(dold, x[u][k], a[u][k]));
                        *reinterpret_cast<floatx4*>(A + gi) = a4;
                    }
                    store_split4<BF, C>(p, gi, xn);
                } else {
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        if (c + k < r) continue;
                        if (use_x) X[gi + k] = xn[k];
                        if (upd) A[gi + k] = fmaf(dnew, xn[k], fmaf(dold, x[u][k], a[u][k]));
                        store_split1<BF, C>(p, gi + k, xn[k]);
                    }
                }
                *reinterpret_cast<floatx4*>(srow) = xn;
            } else {
                floatx4 out;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int64_t gck = gc + k;
                    double v = (double)a[u][k] + (double)dold * (double)x[u][k] + (double)xn[k];
                    if (flip) v = (gr == gck ? 1.0 : 0.0) - v;
                    const float vf = ent ? 0.0f : (float)v;
                    const double vo = ent ? v : (double)vf;
                    if ((!diag || c + k >= r) && gr < n && gck < n) {
                        if (gr == gck) tr += vo;
                        sq += (gr == gck ? 1.0 : 2.0) * vo * vo;
                        if (!ent) {
                            if (p.out_mode == 0)
                                reinterpret_cast<float*>(p.D)[gr * p.ldd + gck] = vf;
                            else if (p.out_mode == 1)
                                reinterpret_cast<double*>(p.D)[gr * p.ldd + gck] = (double)vf;
                        }
                    }
                    out[k] = vf;
                }
                *reinterpret_cast<floatx4*>(srow) = out;
            }
        }
    };
    Batch bA, bB;
    load_batch(0, bA);
#pragma unroll
    for (int bi = 0; bi < NBATCH; ++bi) {
        if (bi & 1) {
            if (bi + 1 < NBATCH) load_batch((bi + 1) * U, bA);
            finish_batch(bi * U, bB);
        } else {
            if (bi + 1 < NBATCH) load_batch((bi + 1) * U, bB);
            finish_batch(bi * U, bA);
        }
    }
    __syncthreads();
    if (!last) {
        // Mirror: output row J0 + c, four consecutive output columns I0 + r .. r+3 per thread;
        // four neighbouring threads cover 16 contiguous columns of one output row.
        constexpr int RG = C::EC / 4;
#pragma unroll 2
        for (int e = tid; e < C::BM * RG; e += C::NT) {
            const int c = (e >> 2) % C::BM;
            const int rl = ((((e >> 2) / C::BM) << 2) + (e & 3)) * 4, r = R0 + rl;
            if (diag && r >= c) continue;   // nothing strictly below the diagonal
            floatx4 v;
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] = sY[(rl + k) * C::LDY + c];
            if (J0 + c >= n || I0 + r >= n) continue;   // wholly in the padding
            const int64_t oi = (J0 + c) * np + I0 + r;
            if (!diag || r + 3 < c) {
                store_split4<BF, C>(p, oi, v);
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if (r + k >= c) continue;
                    store_split1<BF, C>(p, oi + k, v[k]);
                }
            }
        }
    } else if (!(ent || p.out_mode == 2)) {
#pragma unroll 4
        for (int e = tid; e < C::EC * C::BM; e += C::NT) {
            const int rl = e % C::EC, c = e / C::EC, r = R0 + rl;
            if (diag && !(r < c)) continue;
            const float v = sY[rl * C::LDY + c];
            const int64_t orow = J0 + c, ocol = I0 + r;
            if (orow < n && ocol < n) {
                if (p.out_mode == 0)
                    reinterpret_cast<float*>(p.D)[orow * p.ldd + ocol] = v;
                else
                    reinterpret_cast<double*>(p.D)[orow * p.ldd + ocol] = (double)v;
            }
        }
    }
    __syncthreads();
}

// Per-tile FP64 trace partials of the last layer, reduced over the workgroup in a fixed order.
template <class C>
__device__ inline void write_traces(const LayerArgs& p, double tr, double sq, float* sY,
                                    int tile_index) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
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

// Fused epilogue of tile (I, J), I <= J, from the accumulators (which hold s X^2), plus optional
// partial tiles of other workgroups (see epi_chunk). The accumulators go through sY EC rows at a
// time. UMAX bounds the groups whose loads a thread keeps in flight (register budget).
template <bool BF, class C, int UMAX = 8>
__device__ inline void epilogue(const LayerArgs& p, const Acc<C>& acc, float* sY, int I, int J,
                                int tile_index, const float* __restrict__ parts = nullptr,
                                size_t part_stride = 0, int nparts = 0, bool poisoned = false) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / C::WN, wn = wave % C::WN;
    const float inv_s = BF ? 1.0f : (1.0f / 2048.0f);
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
        epi_chunk<BF, C, UMAX>(p, sY, R0, I, J, nullptr, parts, part_stride, nparts, tr, sq,
                               poisoned);
    }
    if (p.last) write_traces<C>(p, tr, sq, sY, tile_index);
}

// Store the accumulators of a BM x BM tile (scaled by 1/s, i.e. as X^2) row-major into dst,
// with device-coherent stores if COHERENT (a tile another workgroup reads), else plain ones.
// Each store instruction writes two 128-byte row segments.
template <bool BF, class C, bool COHERENT>
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
                if constexpr (COHERENT)
                    store_coherent(dst + r * C::BM + cl, acc.v[mb][nb][j] * inv_s);
                else
                    dst[r * C::BM + cl] = acc.v[mb][nb][j] * inv_s;
            }
        }
}

// Fused epilogue of tile (I, J), I <= J, reading X^2 from memory: Y = Y0 + parts[0] + ... +
// parts[nparts-1] (Y0 row-major BM x BM, written by this workgroup; see epi_chunk).
template <bool BF, class C, int UMAX = 8>
__device__ inline void epilogue_mem(const LayerArgs& p, const float* __restrict__ Y0,
                                    const float* __restrict__ parts, size_t part_stride,
                                    int nparts, float* sY, int I, int J, int tile_index,
                                    bool poisoned = false) {
    double tr = 0.0, sq = 0.0;
#pragma unroll 1
    for (int ch = 0; ch < C::BM / C::EC; ++ch)
        epi_chunk<BF, C, UMAX>(p, sY, ch * C::EC, I, J, Y0, parts, part_stride, nparts, tr, sq,
                               poisoned);
    if (p.last) write_traces<C>(p, tr, sq, sY, tile_index);
}

}  // namespace split
}  // namespace fe
