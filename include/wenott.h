/*
 * wenott.h - C ABI of the WENO-TT hot path for AMD Instinct MI355X (gfx950).
 *
 * The library advances a compressible-flow state stored as tensor trains (one TT per
 * conserved variable, Sec. 4.1 after eq. euler-system-TT) by the WENO-TT scheme:
 * cross-interpolated Lax-Friedrichs + WENO5-JS numerical fluxes (Sec. 4.2-4.3,
 * Algorithms lf-cross and weno-cross, fused into one cross per direction), the
 * shift-operator flux difference (eqs. shifted-fluxes and euler-system-TT), SSP-RK3
 * stages rounded once each (Sec. 4.4, eq. tt-ssprk3) with the dynamic truncation
 * tolerance of Sec. 4.6 (eq. eps-tt-formula).
 *
 * Conventions that hold for every call:
 *  - Every call returns a wenott_status; nothing throws across the ABI.
 *  - Pointers are plain host or device pointers as stated per argument. "device" means
 *    memory of the HIP device that was current when wenott_init ran.
 *  - All GPU work is enqueued on the hip stream given to wenott_init (NULL = the null
 *    stream). Calls that return host values synchronise that stream before returning.
 *  - A context is used by one host thread at a time.
 *  - Tensor-train cores are (R_{k-1}, N_k, R_k) arrays in C order (R_k fastest),
 *    R_0 = R_d = 1, FP64. Grids are cell-centred: x_i = lo + (i + 1/2) h, h = (hi-lo)/N.
 */
#ifndef WENOTT_H
#define WENOTT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wenott_ctx wenott_ctx; /* opaque */

typedef enum {
    WENOTT_OK = 0,
    WENOTT_EINVAL = -1,   /* bad argument: shapes, ranks, sizes, NULL pointers */
    WENOTT_ENOMEM = -2,   /* device or host allocation failed */
    WENOTT_EHIP = -3,     /* a HIP runtime call failed */
    WENOTT_ENOCONV = -4,  /* a cross did not reach its tolerance within max_sweeps / rank_cap */
    WENOTT_ENONPHYS = -5, /* rho <= 0 or p <= 0 met at an evaluated point */
    WENOTT_ENAN = -6,     /* NaN or Inf met */
    WENOTT_ENOTBUILT = -7 /* feature not available in this library */
} wenott_status;

/* Boundary treatment per grid side (Sec. 4.5), each with three ghost cells. PERIODIC copies
 * core slices (Sec. 4.5.1), on both sides of a dimension or neither. TRANSMISSIVE is zero-order
 * extrapolation (the paper does not describe it). SYMMETRY is a symmetry plane (Sec. 4.5.3): the
 * ghosts mirror the cells next to the face, ghost -1-l taking cell l, with the momentum normal
 * to the face negated (Euler law). INFLOW (Sec. 4.5.2) holds the side's constant inflow state
 * in its ghosts, the full-tensor value of the paper's zeroed ghost slices plus its rank-1
 * boundary TT; the state is given by wenott_set_inflow. All of them are realised in the
 * gathers as index maps and values of the ghost cells, never as stored ghost slices, so no
 * boundary TT is added and no rounding is spent on it. */
typedef enum {
    WENOTT_BC_PERIODIC = 0,
    WENOTT_BC_TRANSMISSIVE = 1,
    WENOTT_BC_SYMMETRY = 2,
    WENOTT_BC_INFLOW = 3
} wenott_bc;

/* The conservation law the state obeys. EULER: the compressible Euler system with the ideal-gas
 * law (Sec. 2.1), ncomp = ndim + 2 (rho, momenta, total energy). The two scalar laws of Sec. 5.1
 * and 5.2, one component, unit velocity along every axis: LINADV u_t + sum_d u_{x_d} = 0
 * (f_d(u) = u, alpha = 1), BURGERS u_t + sum_d (u^2/2)_{x_d} = 0 (f_d(u) = u^2/2, alpha =
 * max |u|). The scalar laws run in scheme 0 without the learned proposal; gamma is not used. */
typedef enum { WENOTT_LAW_EULER = 0, WENOTT_LAW_LINADV = 1, WENOTT_LAW_BURGERS = 2 } wenott_law;

/* Uniform cell-centred grid: ndim in {2, 3}; n[d] interior cells; box [lo, hi]. */
typedef struct {
    int32_t ndim;
    int32_t pad_;
    int64_t n[3];
    double lo[3];
    double hi[3];
} wenott_grid;

/* A list of ncomp tensor trains (one per conserved variable: ncomp = ndim + 2 for the Euler
 * law, 1 for a scalar law).
 * ranks:  host array [ncomp][ndim + 1]; ranks[c][0] = ranks[c][ndim] = 1.
 * cores:  host array of ncomp * ndim pointers; cores[c * ndim + k] points to the
 *         (ranks[c][k], N_k, ranks[c][k+1]) FP64 core, on the host (on_device = 0) or
 *         the device (on_device = 1).
 * In views returned by the library, ranks and cores point into library-owned memory
 * that stays valid until the next call that changes the state; the cores are then
 * device pointers and every component carries the same (padded) ranks. */
typedef struct {
    int32_t ndim;
    int32_t ncomp;
    const int64_t *ranks;
    const void *const *cores;
    int32_t dtype;     /* 0 = FP64 (the only accepted value) */
    int32_t on_device; /* 0 host, 1 device */
} wenott_tt;

/* Options. wenott_default_opts fills the defaults listed in brackets. */
typedef struct {
    double c_eps;       /* C_eps of eq. eps-tt-formula, used when eps_mode = 1 and eps0 <= 0 [0] */
    double eps0;        /* eps_mode 0: the fixed eps_TT; eps_mode 1: eps at t = 0 fixes C_eps [1e-10] */
    int32_t eps_mode;   /* 0 fixed eps_TT, 1 dynamic eps_TT (Sec. 4.6) [0] */
    int32_t precision;  /* 0 FP64 fiber evaluation; 1 FP32 gather + reconstruction [0] */
    int32_t max_sweeps; /* maximum left-to-right cross sweeps per cross [4] */
    int32_t kick_rank;  /* random enrichment indices added to each sampled index set [4] */
    int32_t rank_cap;   /* maximum rank of any bond, cross and rounding [256] */
    int32_t probe_points; /* random points of the sampled cross residual [4096] */
    uint64_t seed;      /* seed of the library's own counter-based generator [12345] */
    int32_t alpha_mode; /* the Lax-Friedrichs alpha of every stage (eq. lax-friedrichs; for the Euler
                           system the maximum of |u| + a, Sec. 4.2): 0 exact maximum over every cell;
                           1 estimated by a search along grid lines that never visits all N^d cells
                           (the role of tt_max_abs in eq. cfl-other), a lower bound of the exact
                           maximum that reaches it whenever a visited line crosses the maximising
                           cell; 2 alpha_given [1] */
    int32_t use_proposal; /* 1: seed stage crosses from the learned proposal (wenott_set_proposal) [0] */
    double alpha_given; /* the Lax-Friedrichs alpha when alpha_mode = 2 */
    int32_t rounds_per_stage; /* 1: one rounding per SSP-RK3 stage, after the whole combination
                                 a U^n + b (X + dt L(X)) [1]. 2: eq. tt-ssprk3 literally (Sec. 4.4):
                                 X + dt L(X) is rounded (the forward Euler step of eq.
                                 tt-forward-euler), and in stages 2 and 3 the combination with U^n
                                 is rounded again. Not available in batched stepping. */
    int32_t graph_mode; /* reserved, must be 0 [0] */
    int32_t scheme;     /* 0: one cross per stage of the stage value a U^n + b (X + dt L(X)) itself;
                           1: one cross of the flux Fhat_d per direction (Algorithms lf-cross and
                              weno-cross fused), shift difference on core d, TT sum of the stage
                              terms;
                           2: the two-stage pipeline of Sec. 4.2-4.3 as written: per direction
                              one LF-cross of the 2 ncomp split fluxes at the cells (Algorithm
                              lf-cross, a last core of 2 ncomp slices), then one WENO-cross per
                              slice on the faces (Algorithm weno-cross: f^+ slices left-biased,
                              f^- slices mirrored), shift differences, TT sum, rounding; FP64,
                              periodic and transmissive sides. [0] */
    double conv_slack;  /* a cross is accepted when its sampled relative residual is <= eps; one whose
                           residual is still above conv_slack * eps after max_sweeps sweeps fails the
                           call with ENOCONV (and the state is left unchanged). >= 1 [1] */
    int32_t law;        /* the conservation law (wenott_law) [WENOTT_LAW_EULER] */
    int32_t pad_;
    double cross_ratio; /* eps_cross / eps_TT, in (0, 1]: the crosses stop their pivot searches and
                           accept their sampled residuals at cross_ratio * eps_TT while the roundings
                           keep eps_TT. 1 is the paper's eps_cross = eps_TT (Sec. 5); below 1 the
                           crosses keep the singular directions just under eps_TT and the rounding
                           truncates them optimally (SVD) instead of the cross's interpolation [1] */
} wenott_opts;

/* Per-call diagnostics, filled by wenott_get_info. */
typedef struct {
    int32_t ndim, ncomp;
    int64_t ranks[4];        /* bond ranks of the state (padded, common to all components) */
    double alpha[3];         /* alpha used by each stage of the last step (or of the last rhs in [0]) */
    double eps;              /* eps_TT used by the last step */
    double c_eps;            /* C_eps in force (dynamic mode) */
    double max_norm;         /* max over components of the Frobenius norm after the last rounding */
    int32_t sweeps[3][3];    /* [stage][direction] left-to-right sweeps of each cross */
    double residual[3][3];   /* [stage][direction] sampled relative residual of the accepted cross */
    int64_t flux_rank[3][3]; /* [stage][direction] largest bond rank of each flux TT */
    int64_t sum_rank[3];     /* largest bond rank of each stage's sum before rounding */
    int64_t fiber_points;    /* flux values evaluated by fiber kernels in the last call */
    double fiber_ms;         /* device time of the fiber kernels in the last call */
    int64_t fiber_launches;  /* number of fiber-kernel launches in the last call */
    double step_ms;          /* host wall time of the last call */
    /* With profiling on: per kernel class of the last call, [0] fiber (fused flux / stage
     * kernel), [1] pivot selection (rank-revealing LU), [2] Householder TSQR, [3] Jacobi SVD:
     * device time from HIP events on the context's stream, launches, and the algorithmic
     * flops and bytes of those launches (counted from the formulas, not measured). */
    double class_ms[4];
    int64_t class_launches[4];
    double class_flops[4];
    double class_bytes[4];
    /* learned proposal: stage crosses seeded by it and those whose first sweep was accepted */
    int64_t proposals_tried, proposals_accepted;
    int64_t pivots_total;    /* rank-revealing LU pivots taken in the last call */
    /* pivot searches of the last call that stopped at their rank limit (min(rank_cap, 128) or the
     * block's size) while their residual was still above the pivot tolerance */
    int64_t rank_capped;
    /* pivot searches of the last call whose single-launch (persistent) form gave up waiting for
     * workgroups that were not resident, and that were redone with one launch per pivot */
    int64_t pivot_fallbacks;
} wenott_info;

/* Fill *o with the defaults. */
void wenott_default_opts(wenott_opts *o);

/*
 * Create a context holding a copy of the state (the caller keeps ownership of its buffers).
 *   out:    receives the context.
 *   state:  the initial TT list (Sec. 4.1: U_TT = {rho_TT, (rho u)_TT, ..., (rho E)_TT}).
 *   grid:   the cell-centred grid; state mode sizes must equal grid.n.
 *   gamma:  ratio of specific heats (Sec. 2.1), > 1 (Euler law; not used by the scalar laws).
 *   The law comes from opts->law; state->ncomp must be its component count.
 *   bc:     6 entries, bc[2*d + side] (side 0 = low, 1 = high), wenott_bc values; a periodic
 *           side needs a periodic opposite side. An INFLOW side needs its state from
 *           wenott_set_inflow before the first step.
 *   opts:   NULL for defaults.
 *   hip_stream: a hipStream_t (NULL = null stream).
 * Errors: EINVAL on inconsistent shapes/ranks/options, ENOMEM, EHIP.
 */
wenott_status wenott_init(wenott_ctx **out, const wenott_tt *state, const wenott_grid *grid, double gamma,
                          const int32_t *bc, const wenott_opts *opts, void *hip_stream);

/*
 * The TT of the semi-discrete right-hand side L(U) = -sum_d (T^d - 1) Fhat_d / h_d
 * (eq. euler-system-TT): one cross of the fused LF + WENO5 flux per direction (Algorithms
 * lf-cross and weno-cross), the shift difference on that direction's core, the sum over
 * directions and one rounding at the context's eps. The state is not changed.
 * alpha: the Lax-Friedrichs alpha to use, or <= 0 for the alpha_mode rule.
 * view:  receives a library-owned view of L(U) (device cores), valid until the next call.
 */
wenott_status wenott_rhs(wenott_ctx *ctx, double alpha, wenott_tt *view);

/*
 * One SSP-RK3 step of size dt (eq. tt-ssprk3, Shu-Osher form) with one rounding per
 * stage. eps <= 0 selects the eps_mode rule (fixed eps0, or eq. eps-tt-formula).
 * alphas: NULL, or 3 host doubles giving the alpha of each stage (used when
 *         alpha_mode = 2 semantics are wanted per stage); the alphas used are reported by
 *         wenott_get_info either way.
 * On error the state is left unchanged.
 */
wenott_status wenott_rk3_step(wenott_ctx *ctx, double dt, double eps, const double *alphas);

/*
 * n independent states (each its own context, all created on the same stream, ndim equal,
 * scheme 0, no proposal) advanced by one SSP-RK3 step each, in lock-step: every phase of a
 * stage (alpha, the pivot searches of each cross sweep, the sampled residuals, the rounding's
 * norms, Jacobi SVDs and truncation ranks) is one batched launch and one host
 * synchronisation for the whole batch. dt[n] per state; eps: NULL or eps[n] (<= 0 selects the
 * state's rule). Results equal n separate wenott_rk3_step calls up to the random enrichment
 * indices. On error no state is changed.
 */
wenott_status wenott_batch_rk3_step(wenott_ctx **ctxs, int32_t n, const double *dt, const double *eps);

/*
 * Tile autotuner of the FP64 contractions (process-wide). Each problem bucket (transposes and
 * the binary orders of magnitude of M, N, K and the batch) is tuned on its first live calls:
 * the candidate shapes (0-3: 64x64, 32x64, 64x32, 32x32 on the vector units; 4: 64x64 on the
 * FP64 matrix cores; 5-7: matrix-core forms with one operand staged once per workgroup, A
 * (M <= 64) or B in groups of 64 or 32 columns, for untransposed products with K <= 64) are
 * timed with events collected without synchronising (three timings each; one in buckets of at
 * least 2^24 outputs), and the fastest is kept. The vector
 * shapes sum every output in the same order; the matrix-core shapes agree with them to
 * rounding. mode 1: tuned (default); 0: the 64x64 vector shape everywhere; 2 + k: shape k
 * everywhere (k = 0..7; a resident-operand shape runs as shape 4 on a product it does not
 * fit). The table call copies up to max rows of {ta, tb, log2 M, log2 N, log2 K, log2 batch,
 * shape (-1 while tuning)} into out (may be NULL) and stores the number of rows in *count.
 */
wenott_status wenott_gemm_autotune(int32_t mode);
wenott_status wenott_gemm_autotune_table(int32_t *out, int32_t max, int32_t *count);

/* TT-rounding of the state (Sec. 3.2): right-to-left orthogonalisation, then left-to-right
 * truncated SVDs, so that ||X - Y||_F <= eps ||X||_F per component. eps > 0. */
wenott_status wenott_round(wenott_ctx *ctx, double eps);

/* Dense values of the state: every cell's value is the product of its core slices,
 * U(i_1..i_d) = G_1(i_1) ... G_d(i_d) (Sec. 3.1, eqs. TT_def and TT_def_2), for every conserved
 * variable of the list U_TT (Sec. 4.1, after eq. euler-system-TT), written to a caller buffer
 * out[ncomp][N_1][N_2][N_3] (C order, FP64, interior cells only; the caller owns it).
 * on_device = 1: out is device memory (written on the stream, no synchronisation); 0: host
 * memory (synchronises). Errors: EINVAL on NULL arguments, EHIP. */
wenott_status wenott_to_dense(wenott_ctx *ctx, double *out, int32_t on_device);

/* Library-owned view of the current state U_TT (Sec. 4.1: one TT per conserved variable, cores
 * as in eq. TT_def): device core pointers and padded common ranks (the zero-padded rows and
 * columns leave every value of eq. TT_def_2 unchanged). Valid until the next call that changes
 * the state; the caller must not free or write it. Errors: EINVAL on NULL arguments. */
wenott_status wenott_get_state(wenott_ctx *ctx, wenott_tt *view);

/* Diagnostics of the last rhs / rk3_step call and the current ranks: the alpha of each stage
 * (eq. lax-friedrichs with the alpha of Sec. 4.2), the eps_TT and C_eps of eq. eps-tt-formula
 * (Sec. 4.6), the sweeps and sampled residuals of each cross (Sec. 3.3 and the eps_cross =
 * eps_TT rule of Sec. 5), the ranks before and after each rounding (Sec. 3.2), and the kernel
 * class timings. Copied into the caller's struct. Synchronises. Errors: EINVAL on NULL. */
wenott_status wenott_get_info(wenott_ctx *ctx, wenott_info *info);

/* max over the grid of |u| + a for the current state (the alpha of eq. lax-friedrichs as
 * defined for the Euler system in Sec. 4.2; max |u| for Burgers, 1 for linear advection), for
 * the caller's dt = lambda h / alpha (eq. cfl-other): exact with alpha_mode 0 or 2, the
 * line-search estimate with alpha_mode 1.
 * The first stage of the next step reuses it. Synchronises. ENONPHYS if rho <= 0 or p <= 0 at
 * an evaluated cell (every cell in mode 0). */
wenott_status wenott_max_wavespeed(wenott_ctx *ctx, double *alpha);

/* wenott_max_wavespeed without any allocation, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * kernels and the same result as wenott_max_wavespeed, with their workspace in a static device
 * array of 1 MiB per GPU (held until the process ends) instead of the context's cache. It calls
 * no hipMalloc, hipFree or allocating library routine. Supported: alpha_mode 1 (any grid; about
 * 16 KB of workspace) and the exact alpha (alpha_mode 0 or 2) of 2D states whose per-workgroup
 * partial maxima fit the array; anything larger is rejected with EINVAL. Every call on one GPU
 * shares that GPU's array, which keeps the last call's contents (every entry a call reads it has
 * written first, so nothing needs clearing): calls that overlap on one GPU, on any contexts or
 * streams, race. Synchronises; the first stage of the next step reuses the value. */
wenott_status wenott_max_wavespeed_noalloc(wenott_ctx *ctx, double *alpha);

/* The inflow state of side `side` (0 low, 1 high) of dimension `dim`, a WENOTT_BC_INFLOW side
 * (Sec. 4.5.2): prim holds the primitive values rho, u_1..u_ndim, p (Euler law; ndim + 2 host
 * doubles, rho > 0, p > 0) or u (scalar law; one double). The ghost cells of the side take the
 * conserved state rho, rho u_d, p / (gamma - 1) + rho |u|^2 / 2 from the next step on; it may be
 * changed between steps. Errors: EINVAL for a side that is not INFLOW or a non-physical state. */
wenott_status wenott_set_inflow(wenott_ctx *ctx, int32_t dim, int32_t side, const double *prim);

/* Current eps_TT of the dynamic rule (eq. eps-tt-formula) or the fixed one. */
wenott_status wenott_current_eps(wenott_ctx *ctx, double *eps);

/* Testing hook (process-wide): the bound on the polls with which the single-launch pivot search
 * waits for its other workgroups. < 0 restores the default bound; 0 makes every such wait give
 * up at once, so that the fallback (the block evaluated again and searched one launch per pivot
 * step, counted in wenott_info.pivot_fallbacks) runs. Every kernel still ends normally. */
wenott_status wenott_set_pivot_wait_limit(int32_t polls);

/* The pivot selection of the cross on its own (Sec. 3.3: the maximum-volume choice of the
 * interpolation rows and columns, taken greedily): full-pivot rank-revealing LU of the m x n
 * row-major device matrix A (not modified; copied to a workspace the call allocates). Each step
 * takes the entry of largest magnitude of the residual (ties to the lowest linear index), records
 * its row and column and eliminates it; the search stops when the residual's squared Frobenius
 * norm is <= rel_tol2 times A's, after rmax pivots (1 <= rmax <= min(m, n)), or at a zero
 * residual, and always takes one pivot of a nonzero block. Outputs (device): rowpiv[rmax] and
 * colpiv[rmax] (the first rank entries are set), L (m x rmax row-major: column t is the residual
 * column of pivot t divided by the pivot, 1 at the pivot row); info (host, 3 doubles) = {rank,
 * final residual squared norm, stopping threshold}. allow_persistent = 0 forces the one-launch-
 * per-step layouts (the fallback of the persistent ones); 1 lets the library choose, as the
 * cross does. Synchronises hip_stream. Errors: EINVAL, ENOMEM, EHIP. */
wenott_status wenott_pivot_search(const double *A, int32_t m, int32_t n, int32_t rmax, double rel_tol2,
                                  int32_t allow_persistent, int32_t *rowpiv, int32_t *colpiv, double *L, double *info,
                                  void *hip_stream);

/* Diagnostic: the layout the pivot search (full-pivot rank-revealing LU, Sec. 3.3 maxvol role)
 * takes for an m x n cross block on the current device, into out[7] = {mode (0 one workgroup,
 * registers; 1 and 3 one launch per pivot step; 2 and 4 one persistent launch), tile shape or
 * rows per thread, rows per workgroup, workgroups, the device's capacity for that persistent
 * launch (0 when stepped), the capacities of the 24-row-per-thread persistent form and of the
 * form that streams further rows}.
 * Errors: EINVAL. */
wenott_status wenott_pivot_layout(int32_t m, int32_t n, int32_t *out);

/* Record device time of the fiber kernels (reported as fiber_ms by wenott_get_info). */
wenott_status wenott_set_profiling(wenott_ctx *ctx, int32_t on);

/* Text of the last error met by this context ("" if none); with ctx = NULL, the last error
 * met by any call on this host thread (e.g. a failed wenott_init). */
const char *wenott_last_error(wenott_ctx *ctx);

void wenott_destroy(wenott_ctx *ctx);
const char *wenott_strerror(wenott_status s);

/* Process-level drain and release: waits for the current device, returns the device blocks the
 * library keeps cached for reuse to the runtime and destroys the GEMM autotuner's events (its
 * chosen tile shapes are kept). Meant to run before the HIP runtime is torn down (the Python
 * binding registers it at interpreter exit), so that no library-owned HIP object outlives the
 * runtime; the library stays usable afterwards. Contexts are not touched: destroy them first.
 * Errors: EHIP. */
wenott_status wenott_finalize(void);

/* ------------------------------------------------------------------------------------
 * Learned cross proposal (an addition to the paper's method). A 3-layer MLP
 * IN -> HID -> HID -> OUT (ReLU) maps per-bond features of the previous stage cross (the
 * histogram of the right indices its pivots used, the normalised singular-value tail of the
 * last rounding, ranks, sweeps, residual, eps, CFL, stage) to logits of the rank change
 * (RANK_CLASSES, change -8..+8) and of where the next right index set should sample
 * (BINS bins along the bond's first right mode). A proposal seeds the first sweep of the
 * stage cross; it is accepted only if that sweep's sampled residual is <= eps, otherwise the
 * plain cross continues from it. Parameters are one FP32 device array (W1[IN][HID], b1, W2,
 * b2, W3[HID][OUT], b3). Inference inside the library rounds weights and activations to
 * BF16 and accumulates in FP32. Training: loss = cross-entropy of the rank class +
 * cross-entropy of the bin distribution against the target histogram, batch mean.
 * ---------------------------------------------------------------------------------- */
#define WENOTT_MLP_IN 96
#define WENOTT_MLP_HID 128
#define WENOTT_MLP_OUT 81
#define WENOTT_MLP_RANK_CLASSES 17
#define WENOTT_MLP_BINS 64

int64_t wenott_mlp_nparams(void);
/* floats of device workspace for a batch (forward and loss_grad) */
int64_t wenott_mlp_workspace(int32_t batch);
/* He-normal weights, zero biases, from a counter-based generator. params: device. */
wenott_status wenott_mlp_init_params(float *params, uint64_t seed, void *hip_stream);
/* y[batch][OUT] = MLP(x[batch][IN]); all device; bf16 != 0: operands rounded to BF16, FP32 sums on
 * the matrix cores (v_mfma_f32_16x16x16bf16_1k). */
wenott_status wenott_mlp_forward(const float *params, const float *x, int32_t batch, float *y, int32_t bf16,
                                 float *work, void *hip_stream);
/* grad[nparams] and loss (device scalar) of a batch; rank_class[batch] in 0..16, hist[batch][BINS]. */
wenott_status wenott_mlp_loss_grad(const float *params, const float *x, const int32_t *rank_class, const float *hist,
                                   int32_t batch, float *grad, float *loss, float *work, void *hip_stream);
/* one Adam step (beta 0.9 / 0.999, eps 1e-8) at step t >= 1 with learning rate lr; m, v: device state. */
wenott_status wenott_mlp_adam_step(float *params, const float *grad, float *m, float *v, int32_t t, float lr,
                                   void *hip_stream);
/* Use (params != NULL, device, kept by the caller) or stop using the learned proposal. */
wenott_status wenott_set_proposal(wenott_ctx *ctx, const float *params);
/* Record one (features, rank class, bin histogram) sample per bond of every stage cross. */
wenott_status wenott_set_cross_logging(wenott_ctx *ctx, int32_t on);
/* Copy up to max logged samples to host arrays x[max][IN], rank_class[max], hist[max][BINS];
 * *n receives the count; the log is cleared. */
wenott_status wenott_get_cross_log(wenott_ctx *ctx, float *x, int32_t *rank_class, float *hist, int32_t max,
                                   int32_t *n);

/* ------------------------------------------------------------------------------------
 * Dense comparator: the same FP64 scheme on the full grid (the paper's "full-tensor"
 * solver of Sec. 2, eq. euler-system-no-for-loop), run on the GPU. It is what WENO-TT's
 * dense-equivalent throughput is compared with; it is not used by the TT path.
 * U and L are device arrays [ncomp][N_1][N_2][N_3] (C order, FP64) owned by the caller.
 * ---------------------------------------------------------------------------------- */
typedef struct wenott_dense wenott_dense;

/* Euler law only; bc as for wenott_init, with periodic, transmissive and symmetry sides. */
wenott_status wenott_dense_init(wenott_dense **out, const wenott_grid *grid, double gamma, const int32_t *bc,
                                void *hip_stream);
/* exact max over the grid of |u| + a; ENONPHYS if rho <= 0 or p <= 0 anywhere. Synchronises. */
wenott_status wenott_dense_max_wavespeed(wenott_dense *ctx, const double *U, double *alpha);
/* L(U) with the given Lax-Friedrichs alpha (> 0). */
wenott_status wenott_dense_rhs(wenott_dense *ctx, const double *U, double alpha, double *L);
/* One SSP-RK3 step in place. alphas: NULL (exact alpha of each stage input, synchronises per
 * stage) or 3 host doubles; alphas_used: NULL or 3 host doubles receiving the alphas. */
wenott_status wenott_dense_rk3_step(wenott_dense *ctx, double *U, double dt, const double *alphas,
                                    double *alphas_used);
void wenott_dense_destroy(wenott_dense *ctx);

#ifdef __cplusplus
}
#endif
#endif /* WENOTT_H */
