/*
 * fe.h -- C ABI of the MI355X (gfx950) finite-temperature Fermi-operator expansion library.
 *
 * The library evaluates the learned recursive expansion of the Fermi-Dirac density matrix
 * D = [exp(beta (H - mu I)) + I]^-1 (Sec. II.A) and of the electronic entropy
 * S = -Tr[D ln D + (I - D) ln(I - D)] (Sec. III.B, Eq. entropy-matrix, per spin, k_B = 1)
 * for a dense symmetric Hamiltonian H, following Alg. 2 of the paper:
 *   1. Gershgorin spectral bounds of H,
 *   2. affine rescale to the model coordinate with the spectrum flip and the region-of-validity
 *      clamp (Sec. IV.1, Eqs. H', mu', beta', H0, conditions, flip),
 *   3. L layers  A <- A + d_i X,  X <- a_i X^2 + b_i X + c_i I   (Eq. mlsp2, Alg. 1),
 *   4. D = A + X (I - (A + X) if the spectrum was flipped), Tr D and sum_ij D_ij^2
 *      (Sec. IV.3, Eq. tr(D^2)),
 *   5. the entropy expansion with its own coefficients on Y0 = alpha X0 + (1 - alpha) mu0 I
 *      and S = 4 ln2 (Tr U - sum_ij U_ij^2), U = A_S + Y (Eq. entropy expansion and its
 *      output layer).
 *
 * Conventions for every entry point:
 *   - Matrices are dense, row-major, float64 unless stated, with a leading dimension (ld) in
 *     elements >= n. H must be exactly symmetric; only its values are read.
 *   - "device" pointers are HIP device memory owned by the caller. The library never frees
 *     them. "host" pointers are ordinary host memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream). Every call is
 *     asynchronous on that stream unless its comment says it synchronizes.
 *   - The expansions allocate no device memory: it is allocated by fe_workspace_create, by
 *     batch plans (their tables and captured graph, when created or rebuilt), and by the
 *     trainers and fe_autotune (scratch for the call, freed before they return);
 *     fe_expand_density_noalloc uses no workspace at all. A workspace must not be used by two
 *     calls that overlap in time (e.g. on two streams).
 *   - Return value: FE_OK (0), a positive warning (the result is still produced), or a
 *     negative error (nothing was enqueued, unless stated). fe_last_error() gives a message.
 *   - Conditions found on the device (non-finite H, mu outside the spectral bounds) cannot be
 *     returned by an asynchronous call: the device turns the result into NaN so that it cannot
 *     be mistaken for a value, and the status is reported in fe_rescale_info.status when the
 *     caller asks for the info (which synchronizes).
 */
#ifndef FE_H
#define FE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------------------- */
#define FE_OK                  0
#define FE_WARN_BETA_CLAMPED   1   /* beta' above the model's region of validity was clamped to
                                      beta_max (Eq. conditions); D is then the density matrix at
                                      the clamped temperature, as the paper's reference code does */
#define FE_ERR_ARG            -1   /* bad argument (null pointer, n < 1, ld < n, L < 1, ...) */
#define FE_ERR_DOMAIN         -2   /* kT <= 0, or mu outside (eps_min, eps_max) */
#define FE_ERR_HIP            -3   /* a HIP runtime call failed */
#define FE_ERR_NONFINITE      -4   /* H holds a NaN or an infinity */
#define FE_ERR_NO_CONVERGENCE -5   /* a fit or an iteration did not reach its tolerance */
#define FE_ERR_WORKSPACE      -6   /* the workspace is too small for the request */
#define FE_ERR_RANGE          -7   /* the model's layer values leave the 16-bit operand range */

/* ---- precision of the layer products ---------------------------------------------- */
#define FE_PREC_FP64    0   /* FP64 MFMA products, FP64 storage */
#define FE_PREC_FP32    1   /* FP32 MFMA products, FP32 storage */
#define FE_PREC_FP16X2  2   /* X = hi + 2^-11 lo with FP16 hi/lo; X^2 from three FP16 MFMA products
                               (hi*hi, hi*lo, lo*hi) with FP32 accumulation; the lo*lo term is
                               dropped (Sec. V.A, Eq. emulated matmul). FP32 master copy of X. */
#define FE_PREC_BF16X2  3   /* same with BF16 hi/lo (no lo scaling) */
#define FE_PREC_BF16X3  4   /* X = hi + mid + lo with BF16 parts (24 significant bits); X^2 from six
                               BF16 MFMA products (hi*hi, hi*mid, mid*hi, hi*lo, lo*hi, mid*mid)
                               with FP32 accumulation, the dropped terms below 2^-24 relative
                               (the split products of Sec. V.A carried to a third part). FP32
                               master copy of X; data-parallel schedule; not for the variants,
                               the tuners or fe_expand_density_noalloc. */

/* ---- model: one coefficient table ---------------------------------------------------- */
typedef struct {
    int32_t L;            /* number of layers, >= 1 */
    double beta0;         /* training inverse temperature in the model coordinate (> 0) */
    double mu0;           /* training chemical potential in the model coordinate, in (0, 1) */
    const double* theta;  /* host, L x 4 row-major: theta[4i + 0..3] = (a_i, b_i, c_i, d_i) of
                             Eq. (mlsp2): x <- a x^2 + b x + c, A <- A + d x */
} fe_model;

/* ---- result of the rescale (Sec. IV.1) ------------------------------------------------ */
typedef struct {
    double emin, emax;    /* Gershgorin bounds of H */
    double mu_p;          /* mu' after the flip, in [0, 1/2] */
    double beta_p;        /* beta' after the clamp */
    double beta_max;      /* min(mu0/mu', (1 - mu0)/(1 - mu')) beta0 (Eq. conditions) */
    double scale, shift;  /* X0 = scale * H + shift * I */
    int32_t flipped;      /* 1 if mu' > 1/2 and the spectrum was flipped (Eq. flip) */
    int32_t clamped;      /* 1 if beta' was clamped */
    int32_t degenerate;   /* 1 if eps_max == eps_min (H = c I): X0 = y I with the exact y */
    int32_t status;       /* FE_OK, FE_WARN_BETA_CLAMPED, FE_ERR_DOMAIN or FE_ERR_NONFINITE */
} fe_rescale_info;

/* ---- workspace ------------------------------------------------------------------------ */
typedef struct fe_workspace fe_workspace;

/* Allocate device scratch for matrices up to max_n (single-matrix calls) and for batches of up
 * to max_batch matrices whose padded sizes sum to at most batch_elems elements (0 and 0 for no
 * batch capacity). Allocates on the current HIP device. */
int fe_workspace_create(int64_t max_n, int32_t max_batch, int64_t batch_elems, fe_workspace** ws);
int fe_workspace_destroy(fe_workspace* ws);

/* ---- single matrix ---------------------------------------------------------------------- */

/* Steps 1-2 of Alg. 2 (Gershgorin bounds, Eqs. H', mu', beta', flip, conditions, H0).
 * H: device, n x n (ld ldh). X0: device float32 n x n (ld ldx) or NULL: receives
 * X0 = (beta'/beta0)(H' - mu' I) + mu0 I. info: host or NULL; if non-NULL the call
 * synchronizes the stream and fills it. Returns FE_WARN_BETA_CLAMPED if clamped (only when
 * info is given), or the info's error status. */
int fe_rescale(const double* H, int64_t n, int64_t ldh, double mu, double kT, const fe_model* m,
               float* X0, int64_t ldx, fe_rescale_info* info, fe_workspace* ws, void* stream);

/* Density matrix by Alg. 2 (steps 1-4) with model m in precision prec (FE_PREC_*).
 * final_correction: 0 or 1. With 1 and a 16-bit split precision, the last layer is a correction
 *    layer: its product X^2 comes from the FP32 copy of the state by FP32 MFMA (FP32 inputs and
 *    accumulation) instead of the 16-bit split, and its output D = A + d X + (a X^2 + b X + c I)
 *    (I - D if flipped) is formed in FP64; a float64 D then receives these FP64 values. The
 *    correction layer costs one FP32 matrix product (2 N^3 at the FP32 MFMA rate). Ignored for
 *    FE_PREC_FP32 and FE_PREC_FP64 (their layers are already FP32 / FP64 throughout).
 * D: device, n x n (ld ldd), float32 if d_is_fp64 == 0 else float64; exactly symmetric.
 *    Without the correction layer, the 16-bit and FP32 modes give FP32 values (also when D is
 *    float64).
 * trD, trD2: device float64 scalars or NULL: Tr D and sum_ij D_ij^2 accumulated in FP64.
 * info: as for fe_rescale (synchronizes when non-NULL). */
int fe_expand_density(const double* H, int64_t n, int64_t ldh, double mu, double kT,
                      const fe_model* m, int32_t prec, int32_t final_correction, void* D,
                      int32_t d_is_fp64, int64_t ldd, double* trD, double* trD2,
                      fe_rescale_info* info, fe_workspace* ws, void* stream);

/* fe_expand_density without a workspace, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid allocation). It allocates
 * nothing: its scratch (rescale parameters, partial sums and the padded matrices of one
 * expansion) is a static device array of 66 MiB that the library holds on every GPU it runs on
 * until the process ends. Limit: the padded matrices must fit 64 MiB, i.e. n <= 2048 for
 * FE_PREC_FP16X2 / FE_PREC_BF16X2, n <= 2304 for FE_PREC_FP32, n <= 1664 for FE_PREC_FP64;
 * larger n returns FE_ERR_WORKSPACE; FE_PREC_BF16X3 returns FE_ERR_ARG. Always the data-parallel schedule and the direct layer form.
 * All calls on one GPU share that GPU's array: calls that overlap in time on one GPU (other
 * streams or threads) race and must be serialised by the caller. Arguments, outputs and
 * synchronisation as for fe_expand_density (H, D, trD, trD2 device; info host or NULL),
 * final_correction included. */
int fe_expand_density_noalloc(const double* H, int64_t n, int64_t ldh, double mu, double kT,
                              const fe_model* m, int32_t prec, int32_t final_correction, void* D,
                              int32_t d_is_fp64, int64_t ldd, double* trD, double* trD2,
                              fe_rescale_info* info, void* stream);

/* Model-bank selection for one matrix: the bank model with the fewest layers whose region of
 * validity (Eq. conditions) holds the (beta', mu') of H at (mu, kT) (ties: the larger beta0); if
 * none does, the one with the widest region (an expansion with it clamps beta' and warns).
 * bank: host array of nbank models. index: host, receives the chosen position. Runs the
 * Gershgorin pass on the device and synchronizes the stream. */
int fe_model_select(const double* H, int64_t n, int64_t ldh, double mu, double kT,
                    const fe_model* bank, int32_t nbank, int32_t* index, fe_workspace* ws,
                    void* stream);

/* Density matrix at a prescribed occupation (Sec. IV.3): the chemical potential solving
 * Tr D(mu) = n_occ is found by Newton iterations with d Tr D / d mu = beta (Tr D - sum D_ij^2)
 * (Eq. drho traced), each iterate one full expansion as in fe_expand_density; steps that leave
 * the current bracket, or a vanishing derivative, fall back to bisection of the bracket (which
 * starts as the Gershgorin interval of H).
 * n_occ: target Tr D, in (0, n). mu_init: starting guess strictly inside the Gershgorin bounds,
 *   or NaN for their midpoint. tol: stop when |Tr D - n_occ| <= tol. max_iter: >= 1.
 * D, d_is_fp64, ldd, trD, trD2: as for fe_expand_density, for the final iterate.
 * mu_out: host, the final mu. iters_out: host or NULL, expansions run. info: host or NULL, the
 *   final iterate's rescale info. Synchronizes the stream once per iterate.
 * Returns FE_ERR_NO_CONVERGENCE after max_iter iterates (D, mu_out hold the last one),
 * FE_ERR_DOMAIN if mu_init lies outside the bounds, else as fe_expand_density. */
int fe_expand_density_filling(const double* H, int64_t n, int64_t ldh, double n_occ, double kT,
                              double mu_init, const fe_model* m, int32_t prec, double tol,
                              int32_t max_iter, void* D, int32_t d_is_fp64, int64_t ldd,
                              double* trD, double* trD2, double* mu_out, int32_t* iters_out,
                              fe_rescale_info* info, fe_workspace* ws, void* stream);

/* Entropy by Alg. 2 (steps 1-2 and 5) with entropy coefficients mS (trained at the same
 * (beta0, mu0) as the density model, or the density model itself) and rescale alpha
 * (Sec. III.B; |alpha| <= 1). S: device float64 scalar (per spin, k_B = 1). */
int fe_expand_entropy(const double* H, int64_t n, int64_t ldh, double mu, double kT,
                      const fe_model* mS, double alpha, int32_t prec, double* S,
                      fe_rescale_info* info, fe_workspace* ws, void* stream);

/* Expectation value <A> = 2 Tr(D A) = 2 sum_ij D_ij A_ij of a symmetric observable (Sec. II.A,
 * Eq. observables; the 2 counts spin). D: device n x n (ld ldd), float32 (d_is_fp64 = 0) or
 * float64; A: device float64 n x n (ld lda). out: device float64 scalar. FP64 accumulation in a
 * fixed order (deterministic). Asynchronous on stream. */
int fe_observable(const void* D, int32_t d_is_fp64, int64_t ldd, const double* A, int64_t lda,
                  int64_t n, double* out, fe_workspace* ws, void* stream);

/* Electronic free energy G = 2 Tr[D (H - mu I)] - 2 kT S (Sec. III.B; S per spin channel,
 * k_B = 1): the entropy expansion with mS (or m when mS is NULL) and rescale alpha, the density
 * expansion with m, then the Frobenius product Tr[D H] of D as stored. D: device output as for
 * fe_expand_density, or NULL (then the workspace holds it, in float32). G: device float64 scalar; S, trD:
 * device float64 scalars or NULL. info: as for fe_expand_density (the density expansion's).
 * Asynchronous on stream unless info is given. */
int fe_free_energy(const double* H, int64_t n, int64_t ldh, double mu, double kT,
                   const fe_model* m, const fe_model* mS, double alpha, int32_t prec, void* D,
                   int32_t d_is_fp64, int64_t ldd, double* G, double* S, double* trD,
                   fe_rescale_info* info, fe_workspace* ws, void* stream);

/* ---- batches of matrices of uneven size ------------------------------------------------ */

/* One Hamiltonian of a batch. All pointers are device memory owned by the caller. */
typedef struct {
    const double* H;      /* n x n, leading dimension ldh >= n */
    int64_t n, ldh;
    double mu, kT;        /* chemical potential and temperature of this matrix */
    void* D;              /* n x n density matrix (ld ldd) or NULL for traces only */
    int64_t ldd;
    int32_t d_is_fp64;    /* D is float64 (else float32) */
    double* trD;          /* Tr D or NULL */
    double* trD2;         /* sum_ij D_ij^2 or NULL */
    double* S;            /* entropy or NULL (needs an entropy model) */
} fe_batch_item;

typedef struct fe_batch_plan fe_batch_plan;

/* Alg. 2 for every item of a batch (a batch of independent problems; the method is the same as
 * for one matrix). The plan lays the batch out in the workspace (which must have been created
 * with max_batch >= count and batch_elems >= sum of padded sizes squared (x 20/16 for
 * FE_PREC_BF16X3, whose arrays take 20 B per element instead of 16), padding to multiples
 * of 128), uploads the descriptors (synchronously) and captures the launch sequence into a HIP
 * graph: batched bounds and rescale, the layers (all in one queue launch, or one grouped launch
 * per layer: fe_batch_plan_set_launch), per-matrix traces, then the entropy pass if mS is not NULL (mS must share beta0 and
 * mu0 with m). Precision: FE_PREC_FP16X2, FE_PREC_BF16X2 or FE_PREC_BF16X3 (128 x 128 tiles only;
 * 20 instead of 16 B of the arena per padded element). status: device int32[count] or NULL,
 * receives each item's rescale status (FE_OK, FE_WARN_BETA_CLAMPED, FE_ERR_DOMAIN,
 * FE_ERR_NONFINITE); items with an error get NaN outputs. A workspace holds one batch layout: a
 * new plan makes earlier plans on it stale (their launch returns FE_ERR_WORKSPACE). The items'
 * pointers are captured; launching replays the graph on `stream` (asynchronous). */
int fe_batch_plan_create(const fe_batch_item* items, int32_t count, const fe_model* m,
                         const fe_model* mS, double alpha, int32_t prec, int32_t* status,
                         fe_workspace* ws, fe_batch_plan** plan);
/* A plan over a bank of models (the model-bank selection of Sec. IV.1's region of validity,
 * Eq. conditions): item i runs the bank model with the fewest layers whose region contains its
 * (beta', mu'), i.e. beta' <= beta0 min(mu0/mu', (1 - mu0)/(1 - mu')) with beta' and mu' from
 * the item's Gershgorin bounds (ties: the larger beta0); an item no model covers runs the model
 * with the widest region and reports FE_WARN_BETA_CLAMPED. bank: host array of nbank models.
 * with_entropy: also compute S[i] with each item's model (Sec. III.B reuse of the Fermi
 * coefficients) and rescale alpha. chosen: host int32[count] or NULL, receives the model index
 * per item. Synchronizes once (the bounds are read back to choose); otherwise as
 * fe_batch_plan_create. */
int fe_batch_plan_create_bank(const fe_batch_item* items, int32_t count, const fe_model* bank,
                              int32_t nbank, int32_t with_entropy, double alpha, int32_t prec,
                              int32_t* status, int32_t* chosen, fe_workspace* ws,
                              fe_batch_plan** plan);
int fe_batch_plan_launch(fe_batch_plan* plan, void* stream);

/* Rebuilds the plan (layout, tables, captured graph) with layer tiles of `tile` x `tile`, tile
 * 128 (the default: the single-matrix kernel's tiles) or 64 (32 x 32 per wave: less padding for
 * small matrices, more LDS traffic per flop). Results differ from the other tile size at most by
 * the order of FP32 sums. Waits for the device first (a launch of the plan may be in flight), then
 * replaces the captured graph; on failure the plan is left empty and its launches fail. */
int fe_batch_plan_retile(fe_batch_plan* plan, int32_t tile);

/* How a plan runs the layers of a pass. FE_BATCH_LAUNCH_QUEUE (the default for batches whose
 * first layer holds at least two 128 x 128 tiles per compute unit; smaller batches, bound by their
 * chain of layers, default to FE_BATCH_LAUNCH_LAYERS): every layer of every matrix in one launch: each matrix's (tile, layer) work items sit in the queue of one XCD in
 * layer-major order; a workgroup takes the next item of its XCD's queue and starts it once the
 * matrix has completed its previous layer (bounded waits; the XCD is read from the hardware, so
 * the L2 that holds the matrix is the one its readers use). It needs the device to deal
 * workgroups to its XCDs round-robin, which a probe launch checks once per device; where that
 * fails, plans fall back to FE_BATCH_LAUNCH_LAYERS: one grouped launch per layer over all upper
 * tiles of all matrices. Both forms run the same per-tile arithmetic in the same order, so they
 * give bitwise equal results. If a wait gives up (it never should: every wait is on earlier items of
 * the same queue, all held by running workgroups), the matrix's outputs are NaN and its status
 * FE_ERR_HIP. The queue launch holds 16 B of device tables per work item (upper tiles x layers,
 * summed over the matrices and both passes), allocated with the plan. */
#define FE_BATCH_LAUNCH_LAYERS 0
#define FE_BATCH_LAUNCH_QUEUE  1
/* Rebuilds the plan with the given launch form (keeping its tile size); waits for the device
 * first, as fe_batch_plan_retile, and likewise leaves the plan empty on failure. FE_ERR_ARG for
 * FE_BATCH_LAUNCH_QUEUE where the device probe failed (the plan is then left as it was). */
int fe_batch_plan_set_launch(fe_batch_plan* plan, int32_t launch);

/* Autotunes the plan's tile size and launch form: builds it with each tile size (128 and 64;
 * FE_PREC_BF16X3 plans have the 128 x 128 tile only) under each launch form (the queue launch
 * where the device allows it, and the per-layer launches), times three replays of each on
 * `stream` (after a warm-up) and keeps the fastest pair. tile (host, may be NULL) receives the
 * chosen tile size, ms (host, 2 entries, may be NULL) the ms per replay for tiles 128 and 64 (the
 * faster launch form of each; NaN for a tile not tried). Waits for the device first and
 * synchronizes; on failure the plan is rebuilt in the default form. fe_batch_plan_get reports
 * the choice. */
int fe_batch_plan_autotune(fe_batch_plan* plan, void* stream, int32_t* tile, double* ms);
/* The plan's current layer tile size and launch form (host outputs, each may be NULL). */
int fe_batch_plan_get(const fe_batch_plan* plan, int32_t* tile, int32_t* launch);
int fe_batch_plan_destroy(fe_batch_plan* plan);

/* One-shot batch: create a plan, launch it on `stream`, wait for the stream, destroy the plan. */
int fe_batched_expand(const fe_batch_item* items, int32_t count, const fe_model* m,
                      const fe_model* mS, double alpha, int32_t prec, int32_t* status,
                      fe_workspace* ws, void* stream);

/* ---- coefficient training (Sec. III.C) ------------------------------------------------- */
#define FE_TARGET_FERMI    0   /* g(y) = 1/(1 + exp(beta0 (mu0 - y))) on the model coordinate */
#define FE_TARGET_ENTROPY  1   /* -g ln g - (1-g) ln(1-g), model 4 ln2 u(1-u) with
                                  u = layers(alpha (y - mu0) + mu0) (Eq. entropy expansion) */
#define FE_SAMPLE_UNIFORM  0   /* sample density on [0, 1]: p ~ 1 */
#define FE_SAMPLE_DERIV    1   /* p ~ 1 + |g'| */
#define FE_SAMPLE_ARCLEN   2   /* p ~ sqrt(1 + g'^2) */

typedef struct {
    int32_t target;       /* FE_TARGET_* */
    int32_t L;            /* layers, 1..96 */
    double beta0, mu0;    /* training point (model coordinate) */
    double alpha;         /* entropy input rescale (ignored for the Fermi target) */
    int32_t n_points;     /* fixed sample points (quantiles of the sampling density), >= 4L */
    int32_t sampling;     /* FE_SAMPLE_* */
    int32_t max_iter;     /* Levenberg-Marquardt iterations */
    double tol;           /* stop when max |model - target| over the points is below tol */
    /* Optional matrix set (Fermi target only; n_mats = 0 for none): after the fit on the points,
     * the coefficients are refined on F = sum_k r_k^2 / 2 + (mat_weight / 2) sum_m
     * ||P(X0_m) - Dref_m||_F^2, P the recursion of the layers evaluated on the matrix by the FP32
     * kernels of fe_matrix_forward / fe_matrix_backward (Sec. III.C trains on numbers; the matrix
     * term trains on the same function at the matrices' own spectra). Each refinement step is a
     * damped Gauss-Newton step whose metric is the points' J^T J and whose gradient holds both
     * terms; it is kept when F decreases. */
    int32_t n_mats;               /* number of training matrices */
    int32_t mat_iters;            /* refinement iterations (>= 1 when n_mats > 0) */
    int64_t mat_n;                /* their size, a multiple of 64 */
    const float* const* X0s;      /* host array of n_mats device pointers: X0 in the model
                                     coordinate (FP32, mat_n x mat_n, symmetric) */
    const double* const* Drefs;   /* host array of n_mats device pointers: the target density in
                                     the same coordinate, g(X0) (FP64, mat_n x mat_n) */
    double mat_weight;            /* weight of the matrix term (> 0) */
} fe_train_spec;

typedef struct {
    int32_t iters;
    double rms;             /* RMS residual over the sample points */
    double max_err_points;  /* max |residual| over the sample points */
    double max_err_grid;    /* max |model - target| on 200001 uniform points of [0, 1], FP64 */
    double lambda;          /* final damping */
    int32_t mat_iters;      /* matrix-set refinement: iterations run, */
    int32_t mat_accepted;   /*   steps kept, */
    double mat_loss_start;  /*   sum_m ||P(X0_m) - Dref_m||_F^2 before and */
    double mat_loss_end;    /*   after the refinement (FP32 kernels, FP64 sums) */
} fe_train_report;

/* Fit the coefficients by Levenberg-Marquardt with geodesic acceleration (Sec. III.C). Starts
 * from theta_init (host L x 4) or, if NULL, from the SP2 embedding at mu0 (Eq. sp2-mu, App. C)
 * over the layer count of Eq. (layer count) followed by identity layers. Residuals and the
 * Jacobian run on the GPU in FP64; the damped normal equations are solved on the host.
 * theta_out (host L x 4) receives the best coefficients. Synchronizes. Allocates its own device
 * scratch for the duration of the call (the workspace argument is reserved, may be NULL).
 * Returns FE_ERR_NO_CONVERGENCE (with theta_out filled) if tol was not reached. */
int fe_train_coeffs(const fe_train_spec* spec, const double* theta_init, double* theta_out,
                    fe_train_report* rep, fe_workspace* ws, void* stream);

/* The scalar model at n device points y (model coordinate), FP64: r = model(y) - tgt (tgt may be
 * NULL), and if JT is not NULL the Jacobian transposed, JT[4i + c][k] = d model(y_k) /
 * d theta_{i,c}. theta is host L x 4 (L <= 96). Asynchronous. */
int fe_scalar_eval(const double* y, int32_t n, const double* theta, int32_t L, int32_t target,
                   double mu0, double alpha, const double* tgt, double* r, double* JT, void* stream);

/* Second directional derivative of the scalar model along a coefficient direction, the input of
 * the trainer's geodesic acceleration (Sec. III.C): r2[k] = d^2/dt^2 model(y_k; theta + t v) at
 * t = 0, exact (forward mode of second order, FP64). y, r2: device, n points; v: device L x 4
 * (the layout of theta); theta: host L x 4 (L <= 96). Asynchronous. */
int fe_scalar_second(const double* y, int32_t n, const double* theta, int32_t L, int32_t target,
                     double mu0, double alpha, const double* v, double* r2, void* stream);

/* FP32 matrix recursion for fitting on matrices: hist is device float32 (L+1) x n x n with
 * hist[0] = X0 (symmetric, model coordinate) on entry; layer i writes X_{i+1} into hist[i+1]
 * (FP32 MFMA); P (device n x n float32) receives A_L + X_L. n must be a multiple of 64. */
int fe_matrix_forward(float* hist, int64_t n, const double* theta, int32_t L, float* P,
                      void* stream);

/* Backward of fe_matrix_forward: given G = dLoss/dP (device n x n float32, symmetric), writes
 * grad (device float64 L x 4) = dLoss/dtheta: per layer one FP32 MFMA product
 * M = Xb_{i+1} X_i and an elementwise pass Xb_i = a_i (M + M^T) + b_i Xb_{i+1} + d_i G with the
 * coefficient gradients <M, X_i>, <Xb_{i+1}, X_i>, Tr Xb_{i+1}, <G, X_i> reduced in FP64.
 * work: device float32 3 n^2; part: device float64 4 * nblocks (nblocks >= 1 reduction blocks). */
int fe_matrix_backward(const float* hist, int64_t n, const double* theta, int32_t L,
                       const float* G, float* work, double* part, int32_t nblocks,
                       double* grad, void* stream);

/* ---- schedule autotuner -------------------------------------------------------------------- */

/* Chooses the tile shape and schedule of the 16-bit layer kernel per matrix size on this device:
 * 0 = 128 x 128 tiles, one workgroup per upper tile; 1 = 256 x 256 tiles, stream-K over one
 * workgroup per CU; 2 = 128 x 128 tiles, stream-K over two workgroups per CU (1 and 2 need a
 * workspace with max_n >= 1536). Each candidate runs a short expansion (1 warm-up + 3 timed, HIP
 * events on the stream) of a device-generated random symmetric matrix of each size; the fastest
 * is recorded process-wide for (device, prec, size). The timing model is a 6-layer SP2 recursion
 * with a small accumulator weight on every layer (the accumulator epilogue runs every second
 * layer, as in trained models). Later expansions of a size within a factor
 * sqrt(2) of a tuned one use its schedule (FE_SCHEDULE still overrides). sizes: host, count
 * entries, each <= ws max_n. choice (host, count, may be NULL) receives the chosen schedules, ms
 * (host, 3 x count, may be NULL) each candidate's time per expansion (NaN if not run). prec:
 * FE_PREC_FP16X2 or FE_PREC_BF16X2. Allocates one n_max x n_max FP64 matrix for the call;
 * synchronizes. */
int fe_autotune(const int64_t* sizes, int32_t count, int32_t prec, int32_t* choice, double* ms,
                fe_workspace* ws, void* stream);

/* The same choice made on the caller's own input: each candidate runs the expansion of H (n x n,
 * leading dimension ldh, device FP64) at (mu, kT) with model m (1 warm-up + 2 timed), and the
 * fastest is recorded for (device, prec, n) as above. The layer kernel's MFMA rate depends on the
 * data (a banded H runs its layers 20-26% faster than a random dense one of the same size, and
 * not equally under every schedule), so this is the tuner to use when the inputs of a run look
 * alike. choice: host, may be NULL. ms: host, 3 entries, may be NULL (NaN where not run).
 * Arguments are checked as for fe_expand_density; allocates nothing; synchronizes. */
int fe_autotune_input(const double* H, int64_t n, int64_t ldh, double mu, double kT,
                      const fe_model* m, int32_t prec, int32_t* choice, double* ms,
                      fe_workspace* ws, void* stream);

/* The schedule an expansion of size n with precision prec on ws would use now (host out). */
int fe_autotune_lookup(int64_t n, int32_t prec, fe_workspace* ws, int32_t* schedule);

/* Forgets every tuned entry (the size policy applies again). */
int fe_autotune_clear(void);

/* ---- Skip-SP2 and Max-SP2 (Sec. III.A) ------------------------------------------------- */

#define FE_ARCH_MAX   1   /* Max-SP2 (Eq. maxsp2, Alg. maxsp2-1d) */
#define FE_ARCH_SKIP  2   /* Skip-SP2 with k skips and K accumulators (Sec. III.A.3) */

/* A Skip-SP2 or Max-SP2 model. x_0 is the rescaled matrix (the model coordinate: the rescale
 * performs the SP2 flip) and every layer squares an affine combination of stored matrices.
 * coef (host, fe_qmodel_coef_count doubles), in this order:
 *  FE_ARCH_MAX, L layers: for i = 0 .. L-1: delta_i, theta_{i,0} .. theta_{i,i}; then
 *    c, gamma_0 .. gamma_L.
 *    x_{i+1} = (delta_i I + sum_{j<=i} theta_{i,j} x_j)^2,  f = c I + sum_{i=0}^{L} gamma_i x_i
 *    (the output carries both printed forms: Eq. maxsp2's gamma_0 x_0 and Alg. maxsp2-1d's
 *    constant).
 *  FE_ARCH_SKIP: for i = 0 .. L-1: alpha_c_i, alpha_{i,0} .. alpha_{i,k-1}, beta_{i,1} ..
 *    beta_{i,K}, gamma_{i,1} .. gamma_{i,K}; then a0_1 .. a0_K, omega.
 *    x_{i+1} = (alpha_c_i I + sum_{j<k, i-j>=0} alpha_{i,j} x_{i-j} + sum_l beta_{i,l} A_{i,l})^2,
 *    A_{i+1,l} = A_{i,l} + gamma_{i,l} x_i,  A_{0,l} = a0_l I,  f = omega x_L + sum_l A_{L,l}
 *    ((1 + k + 2K) L + K + 1 coefficients: the paper's (1 + k + 2K) n + 2 at K = 1; the weight
 *    omega on x_L is what App. C's embedding of MLSP2 needs). */
typedef struct {
    int32_t arch;        /* FE_ARCH_MAX or FE_ARCH_SKIP */
    int32_t L;           /* layers (squarings), 1..64 */
    int32_t k, K;        /* FE_ARCH_SKIP: skips 1..4 and accumulators 1..4 (ignored for Max) */
    double beta0, mu0;   /* training point, as for fe_model (used by the rescale) */
    const double* coef;  /* host coefficients, layout above */
} fe_qmodel;

/* Number of coefficients of a model of this shape in *count (host). */
int fe_qmodel_coef_count(int32_t arch, int32_t L, int32_t k, int32_t K, int64_t* count);

/* Device scratch the expansion of an n x n matrix with model m needs, in *bytes (host):
 * Max-SP2 stores x_0 .. x_L, Skip-SP2 the k most recent x_i and K accumulators (FP32, padded
 * to a multiple of 128), plus the 16-bit hi/lo operand. */
int fe_variant_scratch_bytes(int64_t n, const fe_qmodel* m, int64_t* bytes);

/* D ~ f_FD(H) through a Skip-SP2 or Max-SP2 model: Gershgorin bounds and rescale as for
 * fe_expand_density (Sec. IV.1), then per layer one split-precision MFMA squaring (prec
 * FE_PREC_FP16X2 or FE_PREC_BF16X2, FP32 accumulation, upper tiles) and one pass that forms the
 * next operand from the stored states; the last pass forms f (I - f if the spectrum was
 * flipped), writes D (float32 or, d_is_fp64, float64 values of the FP32 result; may be NULL)
 * and reduces Tr D and sum_ij D_ij^2 in FP64 (trD, trD2: device doubles, may be NULL).
 * scratch: device, at least fe_variant_scratch_bytes; the workspace provides the bounds and
 * trace buffers. Asynchronous unless info is non-NULL (then as fe_expand_density).
 * FE_ERR_RANGE if an operand leaves [-16, 16] on the model coordinate's unit interval. */
int fe_expand_density_variant(const double* H, int64_t n, int64_t ldh, double mu, double kT,
                              const fe_qmodel* m, int32_t prec, void* scratch, int64_t scratch_bytes,
                              void* D, int32_t d_is_fp64, int64_t ldd, double* trD, double* trD2,
                              fe_rescale_info* info, fe_workspace* ws, void* stream);

/* Embedding of an MLSP2 model (Eq. mlsp2) in Skip-SP2 with k = K = 1 (arch FE_ARCH_SKIP) or in
 * Max-SP2 (FE_ARCH_MAX), App. C: with x~_0 = x_0 and x~_{i+1} = (x_i + b_i/(2a_i))^2 the MLSP2
 * state is x_i = a_{i-1} x~_i + c_{i-1} - b_{i-1}^2/(4a_{i-1}); the same function with the
 * same layer count. coef_out (host) receives fe_qmodel_coef_count(arch, src->L, 1, 1) doubles.
 * FE_ERR_ARG if some a_i is 0 (such a layer is not a square of an affine form). */
int fe_embed_mlsp2(const fe_model* src, int32_t arch, double* coef_out);

/* The scalar model at n device points y: r = f(y) - tgt (tgt may be NULL) and, if JT is not
 * NULL, JT[p][k] = d f(y_k) / d coef_p (reverse mode, FP64). m gives the shape; its coef field
 * is ignored: coef is a device array in the same layout. Asynchronous. */
int fe_variant_eval(const double* y, int32_t n, const fe_qmodel* m, const double* coef,
                    const double* tgt, double* r, double* JT, void* stream);

/* Fit a Skip-SP2 or Max-SP2 model to the Fermi target of spec (spec->target must be
 * FE_TARGET_FERMI and spec->n_mats 0; spec->L is ignored) by the same Levenberg-Marquardt iteration as
 * fe_train_coeffs, starting from init (shape and host coefficients; the embedding of a trained
 * MLSP2 model, fe_embed_mlsp2, is the intended start, App. C). coef_out (host) receives the
 * best coefficients. Synchronizes; allocates its own device scratch for the call. */
int fe_train_variant(const fe_train_spec* spec, const fe_qmodel* init, double* coef_out,
                     fe_train_report* rep, void* stream);

/* ---- helpers ---------------------------------------------------------------------------- */

/* SP2 for a known chemical potential embedded in the layer form (Eq. sp2-mu; App. C):
 * theta_out (host, L x 4) receives (1,0,0,0) for X^2 and (-1,2,0,0) for 2X - X^2. */
int fe_sp2_coeffs(double mu_p, int32_t L, double* theta_out);

/* Layer count estimate n_l = ln(beta'/4) / ln(2 phi), phi the inverse golden ratio
 * (Sec. V.B, Eq. layer count). */
double fe_layer_count(double beta_p);

/* ---- diagnostics ------------------------------------------------------------------------ */

/* The stream-K work split of the 16-bit layer kernel (the split of each layer's (tile, K-block)
 * iterations over persistent workgroups that balances the last round of X^2 tiles, Sec. V.A's
 * layer GEMM), evaluated on the host by the same code the kernel runs; no device work.
 * np: padded size, a positive multiple of the schedule's tile (256 for schedule 1, 128 for 2).
 * schedule: 1 (256 x 256 tiles) or 2 (128 x 128 tiles). grid: the workgroups offered (the
 * library offers one per CU for schedule 1, two for schedule 2). geom: host int32[6], receives
 * T (tiles per side), ntiles, nk (K-blocks per tile), dp_tiles (leading tiles computed whole
 * before the stream-K launch), groups and the grid actually launched. w: a workgroup of that
 * grid (outside it: *count = 0). segs: host int32[5 * cap] or NULL, receives w's segments in run
 * order as (pass, tile, kb0, kb1, jlo): pass 0 publishes blocks [kb0, kb1) of the tile as a
 * partial, passes 1 and 2 finish the tile after adding the partials of the group's workgroups
 * jlo .. (w / groups) - 1 (ids w % groups + groups jj). count: host, the number of segments. */
int fe_streamk_segments(int64_t np, int32_t schedule, int32_t grid, int32_t w, int32_t* geom,
                        int32_t* segs, int32_t cap, int32_t* count);

/* Test hook for failure handling (process-wide): while enabled, every stream-K wait of the layer
 * kernel waits for a flag value that no workgroup writes and gives up after a short bounded spin,
 * as a wait that timed out would. Every kernel still exits normally; the tiles finished after a
 * give-up are NaN, the traces NaN, and the rescale info status FE_ERR_HIP. */
int fe_debug_streamk_giveup(int32_t enable);

/* Host-side view of the queue launch's work tables (no device work; for tests of the layout the
 * kernel relies on): matrices of padded sizes np[i] (multiples of tile) running L[i] layers, in
 * that (batch) order, dealt to nq queues as a plan deals them. items: host int32[4 * cap] or
 * NULL, receives {matrix, tile, layer, need} per item, queue after queue, each queue in ticket
 * order; qoff: host int32[nq + 1], queue x = items [qoff[x], qoff[x + 1]); nitems: the total. */
int fe_batch_queue_layout(int32_t count, const int64_t* np, const int32_t* L, int32_t tile,
                          int32_t nq, int32_t* items, int64_t cap, int32_t* qoff, int64_t* nitems);

/* Test hook for failure handling (process-wide), the same for the batch queue launch
 * (FE_BATCH_LAUNCH_QUEUE): batch plans built while it is enabled wait, for every work item, for a
 * completion count that no matrix reaches; the first wait gives up after a short bounded spin and
 * the rest at once. Every kernel still exits normally; every matrix of such a plan gets NaN
 * outputs and status FE_ERR_HIP. */
int fe_debug_batch_queue_giveup(int32_t enable);

/* Per-launch timing of the layer kernel with HIP events on the call's stream (process-wide; for
 * the roofline measurement of Sec. V.A's layer product): while enabled, every expansion on the
 * 16-bit split path records an event before its first layer launch and one after each layer
 * launch. fe_debug_layer_events_read waits for the most recent call's last event and writes the
 * elapsed time of each of its layer launches, in ms, to ms[0 .. min(count, cap) - 1] (host);
 * count (host) receives the number of layers timed. Enabling or disabling clears the record. */
int fe_debug_layer_events(int32_t enable);
int fe_debug_layer_events_read(double* ms, int32_t cap, int32_t* count);

/* Message for the last error on the calling thread (static storage, never NULL). */
const char* fe_last_error(void);

/* Library version string. */
const char* fe_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FE_H */
