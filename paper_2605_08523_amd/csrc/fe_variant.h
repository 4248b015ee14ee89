// Internal interface of the Skip-SP2 / Max-SP2 expansions (Sec. III.A): launch arguments of the
// square and combine kernels and of the scalar model with its reverse-mode Jacobian.
#pragma once

#include "fe_internal.h"

namespace fe {

constexpr int kCombineMaxTerms = 66;   // Max-SP2 output over x_0 .. x_64
constexpr int kCombineMaxAcc = 4;
constexpr int kVariantMaxL = 64;
constexpr int kVariantMaxK = 4;        // Skip-SP2 skips and accumulators

// One pass over the upper 64 x 64 tiles of the FP32 state matrices:
//   z = diag * delta_ij + sum_t w[t] term[t]          (terms read before any update)
//   acc[l] = (acc_first ? 0 : acc[l]) + g[l] * acc_src
// out = 0: z is the next operand, split into hi/lo and written with its mirror;
// out = 1: z is the result f, written to D (I - f if the spectrum was flipped) with FP64 trace
// partials per tile. Only elements on or above the diagonal of the states are read.
struct CombineArgs {
    int64_t n, np;
    int nterm;
    const float* term[kCombineMaxTerms];
    float w[kCombineMaxTerms];
    float diag;
    int nacc;
    float* acc[kCombineMaxAcc];
    float g[kCombineMaxAcc];
    const float* acc_src;
    int acc_first;
    int out;
    int bf16;
    uint16_t* hi;
    uint16_t* lo;
    void* D;
    int64_t ldd;
    int out_mode;   // 0: float32 D, 1: float64 D, 2: traces only
    const Params* P;
    TracePartial* partials;
};
hipError_t launch_combine(const CombineArgs& a, hipStream_t s);
int combine_tiles(int64_t np);   // upper 64 x 64 tiles (= trace partials written by out = 1)

// out = Z^2 for Z = hi + lo / s (split operand), FP32, upper 128 x 128 tiles, elements on or
// above the diagonal; np a multiple of 128. Whole rounds of `slots` tiles run data-parallel; a
// small last round (at most slots / 4 tiles) is split along K over the slots, its partials
// (parts: at most slots tiles of 128 x 128 floats) added in a fixed order.
struct SquareSplit {
    int dp = 0;       // tiles of the data-parallel launch
    int tail = 0;     // tiles split along K
    int nsplit = 0;   // segments per split tile
};
SquareSplit square_split(int ntiles, int nk, int slots);
constexpr int64_t kSquarePartTile = 128 * 128;   // floats per partial tile
hipError_t launch_square(const uint16_t* hi, const uint16_t* lo, int64_t np, float* out, int bf16,
                         int slots, float* parts, hipStream_t s);

// Scalar Skip-SP2 / Max-SP2 model at n device points and, if JT is not null, its Jacobian
// transposed (JT[p][k], coefficient p in the layout of fe_qmodel). coef is a device array.
struct VariantEvalArgs {
    const double* y;
    const double* tgt;
    double* r;
    double* JT;
    const double* coef;
    int n, arch, L, k, K;
};
hipError_t launch_variant_eval(const VariantEvalArgs& a, hipStream_t s);

}  // namespace fe
