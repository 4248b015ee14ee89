// Internal declarations shared by the HIP translation units of libfe.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fe.h"
#include "streamk_plan.h"

namespace fe {

// Device-resident rescale parameters, produced by the prologue kernels and read by the rescale
// and final-layer kernels so that no host round trip is needed between them.
struct Params {
    double emin, emax;
    double mu_p, beta_p, beta_max;
    double scale, shift;   // X0 = scale * H + shift * I
    int32_t flipped, clamped, degenerate, status;
};

// Per-block partial results of the Gershgorin pass.
struct BoundsPartial {
    double lo, hi;
    int32_t nonfinite, pad;
};

// Per-tile partial traces of the last layer, reduced in a fixed order.
struct TracePartial {
    double tr, sq;   // sum of diagonal entries, sum of squared entries
};

// A slot of device scratch for one matrix (layout depends on the precision mode).
struct Slot {
    void* base;
    size_t bytes;
};

constexpr int kMaxBoundsBlocks = 4096;
constexpr int kMaxTiles = 1 << 16;

// ---- launchers (one per translation unit; all asynchronous on `s`) ------------------------

// Gershgorin bounds and the rescale parameters of Sec. IV.1 into *P.
hipError_t launch_bounds_params(const double* H, int64_t n, int64_t ldh, double mu, double kT,
                                double beta0, double mu0, BoundsPartial* partials, Params* P,
                                hipStream_t s);

// X0 = scale H + shift I into the working copies of a padded np x np matrix. Entries outside
// n x n are zero. `alpha` rescales towards mu0 for the entropy input:
// Y0 = alpha X0 + (1 - alpha) mu0 I (alpha = 1 for the density).
// mode 0: 16-bit split (X32, A32, hi, lo; T16 selected by bf16 flag)
// mode 1: FP32 (X32, A32)
// mode 2: FP64 (X64, A64)
struct RescaleArgs {
    const double* H;
    int64_t n, ldh, np;
    const Params* P;
    double alpha, mu0, d0;
    float* X32;
    float* A32;
    double* X64;
    double* A64;
    uint16_t* hi;
    uint16_t* lo;
    uint16_t* hi1;      // mode 0, optional: the other operand buffer; its padding (rows or
    uint16_t* lo1;      // columns >= n), which no layer epilogue writes, is written here too
    uint16_t* mid;      // mode 0 with three parts (BF16x3): the middle part, and the other
    uint16_t* mid1;     // buffer's (padding only)
    int three;          // mode 0: three-part BF16 split (hi/mid/lo) instead of hi/lo
    int mode;
    int bf16;
    double op_shift;    // mode 0: the hi/lo operand is X0 + op_shift I (squared-affine form)
    float* X0out;       // optional float32 n x n copy of X0 (fe_rescale)
    int64_t ldx;
};
hipError_t launch_rescale(const RescaleArgs& a, hipStream_t s);
// A random symmetric n x n matrix (row-major, FP64) for timing runs: diagonal U[-1, 1],
// off-diagonal U[-1, 1] / sqrt(n), from a hash of (min(i, j), max(i, j), seed).
hipError_t launch_fill_symmetric(double* H, int64_t n, uint64_t seed, hipStream_t s);

// One layer of the split-precision (FP16x2 / BF16x2 / BF16x3) recursion with the fused epilogue.
struct LayerArgs {
    int64_t np;             // padded size, multiple of the tile size
    int64_t n;              // real size (for output masking and traces)
    const uint16_t* hi_in;  // current operands (np x np, full symmetric)
    const uint16_t* lo_in;
    const uint16_t* mid_in; // three-part BF16 split only: the middle part
    uint16_t* hi_out;       // next-layer operands (unused on the last layer)
    uint16_t* lo_out;
    uint16_t* mid_out;
    float* X;               // FP32 master (upper triangle maintained), in place
    float* A;               // accumulator (upper triangle maintained), in place
    float a, b, c;          // this layer's coefficients
    float d_old, d_new;     // A += d_old X + d_new X' (X the layer's input, X' its output; 0 0 = skip)
    int affine;             // 1: squared-affine form, the operand is the state (X not read or written)
    int last;               // 1 on the last layer
    int out_mode;           // last layer: 0 = D float32, 1 = D float64, 2 = traces only
    int entropy;            // last layer: partials hold U traces for S (no D written)
    void* D;
    int64_t ldd;
    const Params* P;        // flip flag for the last layer
    TracePartial* partials; // one per tile on the last layer
};
// Schedule of the split-precision layer kernel.
struct SplitPlan {
    int streamk;          // 0: one workgroup per 128 x 128 upper tile; 1: persistent stream-K
    int grid;             // stream-K workgroups (one per CU)
    int groups;           // stream-K groups (8: one per XCD), set by the launcher
    int dp_tiles;         // leading tiles computed whole (data-parallel rounds), set by the launcher
    float* partial;       // stream-K published partial tiles, grid x 256 x 256 floats
    float* own;           // stream-K per-workgroup staging of finished tiles, grid x 256 x 256 floats
    uint32_t* flags;      // stream-K publication flags, one per workgroup (zero-initialised)
    uint32_t epoch;       // value written to a flag by this launch (distinct per launch)
    uint32_t wait_epoch;  // value a waiting workgroup expects (= epoch; another value only to
                          // exercise the give-up path from the host)
    int spin_limit;       // sleeps before a wait gives up
    int* err;             // set to 1 if a bounded wait gave up
};
int split_tile_for(int streamk);
// The stream-K plan the launcher uses for a padded size np, schedule 1 or 2, at most grid
// workgroups (host; see streamk_plan.h).
SkGeometry split_sk_geometry(int64_t np, int streamk, int grid);
// bf16: 0 FP16x2, 1 BF16x2, 2 three-part BF16 (data-parallel plan only; LayerArgs mid_* set).
hipError_t launch_layer_split(const LayerArgs& a, int bf16, const SplitPlan& plan, hipStream_t s);

// Whole recursion for np <= 128 in FP64 inside one workgroup's LDS. The coefficients travel
// by value with the launch.
constexpr int kSmallMaxL = 96;
struct SmallArgs {
    int64_t n, np;
    const double* X0;       // np x np FP64 start matrix (full)
    double theta[4 * kSmallMaxL];
    int L;
    double d0;
    int out_mode;           // 0 = D float32, 1 = D float64, 2 = traces only
    int entropy;
    void* D;
    int64_t ldd;
    const Params* P;
    TracePartial* partials; // one entry
};
hipError_t launch_small_f64(const SmallArgs& a, hipStream_t s);

// FP32 / FP64 tiled MFMA kernels (64 x 64 tiles) in two forms:
//  layer form (plain = 0): one layer of the recursion on X itself (operands = the full symmetric
//    X_in, ping-pong with X_out), upper tiles only, fused epilogue as in the split kernel;
//  product form (plain = 1): C = X_in B_in^T for row-major np x np operands over all tiles, written
//    row-major to X_out (used by the trainer's backward pass, where B_in = X is symmetric).
struct WideArgs {
    int64_t np, n;
    const void* X_in;       // layer: full symmetric X; product: left operand
    const void* B_in;       // product: right operand (rows)
    void* X_out;            // layer: next X (full); product: C
    void* A;                // accumulator, upper triangle (layer form)
    double a, b, c, d_next;
    int last, out_mode, entropy;
    void* D;
    int64_t ldd;
    const Params* P;
    TracePartial* partials;
    int plain;
    int f64_epi;            // last layer of the FP32 kernel as a correction layer: FP64 epilogue,
    double d_last;          //   D = A + d_last X + (a Y + b X + c I) in FP64, not rounded to FP32
};
int wide_tile();
// X[i][j] = X[j][i] for i > j (np x np FP32, np a multiple of wide_tile()).
hipError_t launch_mirror_upper_f32(float* X, int64_t np, hipStream_t s);
hipError_t launch_layer_f32(const WideArgs& a, hipStream_t s);
hipError_t launch_layer_f64(const WideArgs& a, hipStream_t s);

// ---- batches of matrices of uneven size --------------------------------------------------
// One matrix of a batch on the device (padded to a multiple of the 128-row tile).
struct BatchMat {
    const double* H;
    int64_t n, ldh, np;
    double mu, kT;
    double beta0, mu0;      // training point of the model this matrix runs with
    float* X;
    float* A;
    uint16_t* hi[2];
    uint16_t* lo[2];
    uint16_t* mid[2];       // three-part BF16 split only
    void* D;
    int64_t ldd;
    int32_t d_is_fp64;
    int32_t item;           // index of the caller's item (status slot)
    double* trD;
    double* trD2;
    double* S;
    int32_t tile0;          // first tile of this matrix in the grouped grid
    int32_t model;          // index of its model in the pass's coefficient tables
};
// Coefficients of one pass (density or entropy) for every model of a batch: layer l of model k
// at coef[(k * max_L + l) * 8 + {0, 1, 2, 3, 4}] = a, b, c, d_old, d_new (accumulator terms
// paired as in the single-matrix kernels); model k has L[k] layers and initial weight d0[k].
struct BatchCoef {
    const float* coef;      // [model][layer][8]: a, b, c, d_old, d_new, affine flag (LayerArgs)
    const int32_t* L;
    const float* d0;
    const double* shift0;   // operand shift of the rescale (squared-affine form), per model
    int max_L;
};
struct BatchLayerArgs {
    const BatchMat* mats;
    const int32_t* map;     // per workgroup (matrix, tile) pairs, (-1, -1) for an empty slot; or
                            // NULL: workgroup g takes tile g of the grouped grid
    int count;
    int parity;             // hi/lo buffer read by this layer
    int layer;
    int entropy;
    BatchCoef cf;
    const Params* P;
    TracePartial* partials;
};
constexpr int kBatchPad = 128;   // batch matrices are padded to a multiple of this
// Bounds and rescale parameters of every matrix with its own (beta0, mu0).
hipError_t launch_batch_bounds(const BatchMat* mats, int count, Params* P, hipStream_t s);
// bf16 (here and below): 0 FP16x2, 1 BF16x2, 2 three-part BF16 (BatchMat mid[] set; 128 tiles).
hipError_t launch_batch_rescale(const BatchMat* mats, int count, int64_t max_np, const Params* P,
                                double alpha, BatchCoef cf, int bf16, hipStream_t s);
// One layer over `grid` workgroups: with q.map, the slots of the map (the tiles of the matrices
// whose model has more than q.layer layers, each matrix on one XCD); without, the first `grid`
// tiles of the grouped grid.
hipError_t launch_batch_layer(const BatchLayerArgs& q, int grid, int bf16, int tile,
                              hipStream_t s);   // tile 128 or 64
hipError_t launch_batch_reduce(const BatchMat* mats, int count, const TracePartial* partials,
                               const Params* P, int entropy, int32_t* status, int tile,
                               hipStream_t s);

// ---- coefficient training --------------------------------------------------------------
constexpr int kScalarMaxL = 96;
struct ScalarArgs {
    const double* y;        // sample points (model coordinate), n
    const double* tgt;      // target values or NULL (residual = model)
    double* r;              // out: model - target, n
    double* JT;             // out (or NULL): Jacobian transposed, 4L x n
    const double* vdir;     // device 4L direction v (read when r2 is set)
    double* r2;             // out (or NULL): second directional derivative of the model along v
    int n, L, target;       // target 0: Fermi, 1: entropy
    double mu0, alpha;
    double theta[4 * kScalarMaxL];
};
int scalar_max_layers();
hipError_t launch_scalar_eval(const ScalarArgs& a, hipStream_t s);
hipError_t launch_gram(const double* JT, const double* v, int P, int n, double* G, double* g,
                       hipStream_t s);
struct MatTheta {
    double v[4 * kScalarMaxL];
};
struct BwdArgs {
    const float* M;         // Xb_{i+1} X_i
    const float* Xb;        // Xb_{i+1}
    const float* X;         // X_i
    const float* G;         // dLoss/dP
    float* Xb_out;          // Xb_i
    float ca, cb, cd;       // a_i, b_i, d_i
    int64_t n;
    double* part;           // per-block partial sums, nblocks x 4
};
hipError_t launch_bwd_elem(const BwdArgs& a, int nblocks, double* grad4, hipStream_t s);
// G = P - Dref (FP32; G may be NULL) and *sumsq = sum (P - Dref)^2 in FP64 over `total` entries
// (nblocks partial sums in part, reduced in a fixed order).
hipError_t launch_mat_residual(const float* P, const double* Dref, int64_t total, float* G,
                               double* part, int nblocks, double* sumsq, hipStream_t s);
hipError_t launch_fwd_out(const float* hist, int64_t n, int L, const MatTheta& th, float* P,
                          hipStream_t s);

// Frobenius product sum_ij D_ij A_ij over n x n (D float32 or float64, A float64) into at most
// kMaxDotBlocks partials, then one fixed-order reduction: mode 0 writes out = 2 sum (Eq.
// observables); mode 1 writes the free energy out = 2 (sum - mu *trD) - 2 kT *S.
constexpr int kMaxDotBlocks = 2048;
hipError_t launch_dot(const void* D, int d_is_fp64, int64_t ldd, const double* A, int64_t lda,
                      int64_t n, double* partials, int mode, double mu, double kT,
                      const double* trD, const double* S, double* out, hipStream_t s);

// Deterministic reduction of tile partials: out_tr = sum tr, out_sq = sum sq; if entropy,
// out_S = 4 ln2 (sum tr - sum sq). If err is set and *err != 0 (a stream-K wait gave up in this
// expansion), the outputs are NaN, P->status becomes FE_ERR_HIP and *err is cleared.
hipError_t launch_reduce_partials(const TracePartial* partials, int count, double* out_tr,
                                  double* out_sq, double* out_S, Params* P, int* err,
                                  hipStream_t s);

}  // namespace fe
