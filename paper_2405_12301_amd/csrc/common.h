// Internal declarations shared by the HIP kernels and the host driver of libwenott.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <stdexcept>
#include <string>

#include "wenott.h"

namespace wtt {

struct HipError : std::runtime_error {
    hipError_t code;
    HipError(hipError_t c, const char *file, int line)
        : std::runtime_error(std::string(hipGetErrorString(c)) + " at " + file + ":" + std::to_string(line)), code(c) {}
};
struct StatusError : std::runtime_error {
    wenott_status status;
    StatusError(wenott_status s, const std::string &m) : std::runtime_error(m), status(s) {}
};

#define WTT_HIP(x)                                                     \
    do {                                                               \
        hipError_t e_ = (x);                                           \
        if (e_ != hipSuccess) throw ::wtt::HipError(e_, __FILE__, __LINE__); \
    } while (0)
#define WTT_REQUIRE(cond, status, msg)                                 \
    do {                                                               \
        if (!(cond)) throw ::wtt::StatusError(status, msg);            \
    } while (0)

constexpr int kMaxDim = 3;
constexpr int kMaxComp = 5;
constexpr int kMaxRankLds = 128;  // largest cross rank whose pivot block fits in LDS

// Device flag bits raised by evaluation kernels.
constexpr int kFlagNonPhys = 1;
constexpr int kFlagNaN = 2;

// Ghost-cell map: periodic wraps, transmissive clamps (both sides alike).
// Random probe cells: coordinate j of point i is splitmix64(seed + golden (e + 1)) mod N_j with
// e = i d + j, so any kernel can form a point's cell from (seed, i) alone.
__host__ __device__ inline int probe_coord(unsigned long long seed, long long e, int nj) {
    unsigned long long z = seed + 0x9E3779B97F4A7C15ULL * (unsigned long long)(e + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return (int)(z % (unsigned long long)nj);
}

// Boundary code of one grid dimension: the low side's wenott_bc in bits 0-3, the high side's in
// bits 4-7 (periodic only in pairs).
__host__ __device__ inline int bc_code(int lo, int hi) { return lo | (hi << 4); }
__host__ __device__ inline int bc_side(int bc, int hi) { return hi ? (bc >> 4) & 15 : bc & 15; }

// Interior cell whose values cell i (-3 <= i < n + 3) of a grid line takes (Sec. 4.5): itself
// inside; periodic wraps (Sec. 4.5.1); a symmetry plane mirrors, ghost -1-l <-> cell l at the low
// side and n+l <-> n-1-l at the high side (Sec. 4.5.3); transmissive clamps. An inflow ghost takes
// the side's constant state (Sec. 4.5.2); the clamp returned for it only keeps reads in bounds.
__host__ __device__ inline int ghost_map(int i, int n, int bc) {
    if (i >= 0 && i < n) return i;
    const int b = bc_side(bc, i >= n);
    if (b == WENOTT_BC_PERIODIC) {
        int r = i % n;
        return r < 0 ? r + n : r;
    }
    if (b == WENOTT_BC_SYMMETRY) return i < 0 ? -1 - i : 2 * n - 1 - i;
    return i < 0 ? 0 : n - 1;
}

// What the value of cell i is beyond ghost_map's cell: kGhostPlain (that cell's values),
// kGhostMirror (a symmetry ghost: the momentum normal to the plane negated), kGhostInflow (the
// side's inflow state).
enum { kGhostPlain = 0, kGhostMirror = 1, kGhostInflow = 2 };
// A dimension with a symmetry or inflow side (its ghost values are more than an index map).
__host__ __device__ inline bool bc_special(int bc) {
    return (bc & 15) >= WENOTT_BC_SYMMETRY || ((bc >> 4) & 15) >= WENOTT_BC_SYMMETRY;
}
__host__ __device__ inline int ghost_kind(int i, int n, int bc) {
    if (i >= 0 && i < n) return kGhostPlain;
    const int b = bc_side(bc, i >= n);
    return b == WENOTT_BC_SYMMETRY ? kGhostMirror : (b == WENOTT_BC_INFLOW ? kGhostInflow : kGhostPlain);
}

// ------------------------------------------------------------------ linalg.hip
// Batched C = alpha * op(A) * op(B) + beta * C, row-major FP64. Batch index z = zc * nb2 + zs.
struct GemmBatch {
    int nb1 = 1, nb2 = 1;
    long long sA1 = 0, sA2 = 0, sB1 = 0, sB2 = 0, sC1 = 0, sC2 = 0;
    int ktot = 0;  // > 0: split-K, batch index z2 is the K-chunk of length K, valid up to ktot
};
void gemm_f64(hipStream_t s, bool ta, bool tb, int M, int N, int K, double alpha, const double *A, int lda,
              const double *B, int ldb, double beta, double *C, int ldc, const GemmBatch &bt = GemmBatch());
// The tile shape of gemm_f64 comes from a process-wide table tuned on live calls (mode 1, the
// default); mode 0: the 64 x 64 vector shape everywhere; mode 2 + k: shape k everywhere.
// gemm_tune_table copies up to max_entries rows of {ta, tb, log2 M, log2 N, log2 K, log2 batch,
// shape (-1 while tuning)} and returns the count.
void gemm_tune_enable(int mode);
// Waits for the timings in flight and destroys the tuner's events (the chosen shapes are kept).
void gemm_tune_release();
int gemm_tune_table(int32_t *out, int max_entries);

// C[z] = A[z]^T B[z] (A: K x M, B: K x N) with the long reduction split into chunks summed
// by a second pass; part needs gemm_tn_splitk_part(M, N, K, batch) doubles (falls back to
// one pass when part_cap is smaller).
void gemm_tn_splitk(hipStream_t s, int M, int N, int K, const double *A, int lda, const double *B, int ldb, double *C,
                    int ldc, int batch, long long sA, long long sB, long long sC, double *part, size_t part_cap);
size_t gemm_tn_splitk_part(int M, int N, int K, int batch);

// R factor of a batch of tall matrices by Householder TSQR. Element (i, j) of matrix z is
// A[z * sz + i * rs + j * cs]. Writes the n x n upper-triangular R of each into
// R[z * n * n] (row-major, zeros below the diagonal). Needs scratch of tsqr_scratch_doubles.
size_t tsqr_scratch_doubles(int m, int n, int batch);
void tsqr_r(hipStream_t s, int m, int n, int batch, const double *A, long long sz, long long rs, long long cs,
            double *R, double *scratch);

// Singular values and right singular vectors of tall matrices C_z = Q_z R_z from their n x n
// row-major upper-triangular R factors (R at R[z * n * n]), by one-sided Jacobi on R^T.
// Outputs sigma[z * n + j] sorted descending and V[z * n * n] row-major with column j the right
// singular vector of sigma_j (zero for sigma_j = 0). The matrices live in LDS when n^2 doubles
// fit; otherwise scratch must hold jacobi_scratch_doubles(n, batch) doubles.
// delta (device, one per matrix, may be null): truncation threshold of the singular values;
// rotations whose effect stays far below it are skipped.
// tr (may be null): also form the truncation ranks as trunc_ranks would, in the same launch;
// returns whether it did (false: the caller runs trunc_ranks).
struct TruncArgs {
    const double *delta_abs = nullptr;
    double rel = 0.0;
    int rcap = 0;
    int *ranks = nullptr;
};
bool jacobi_svd(hipStream_t s, int n, int batch, const double *R, double *sigma, double *V, double *scratch,
                const double *delta = nullptr, const TruncArgs *tr = nullptr);
size_t jacobi_scratch_doubles(int n, int batch);

// Full-pivot rank-revealing LU of one m x n row-major matrix (overwritten by its residual).
// Stops when the residual's squared Frobenius norm <= rel_tol2 * (initial squared norm), after
// rmax pivots, or at a zero residual. Writes rank (>= 1), row/col pivots, L columns (m x rmax, row-major) and the final
// residual norm^2 and the stopping threshold into info[0..2] = {rank, resid2, tol2} (as doubles).
// ws: prrlu_ws_doubles(m, n) doubles (double-buffered per-workgroup partials and candidate rows,
// and control, of the multi-workgroup form used when the block does not fit one workgroup's
// registers). That form runs one launch per step, launch t deciding pivot t - 1 and eliminating
// it: this call launches steps t_begin..min(t_end, rmax + 1) and returns the next step; info[0]
// stays negative until the factorisation has stopped, and the caller continues from the
// returned step. The register form and the persistent form finish in one call (t_begin = 0);
// info[0] = -2 reports a persistent launch whose waits for the other workgroups' partials ran
// out (A is then partly eliminated: the caller evaluates it again and calls with
// allow_persistent = false, which takes the one-launch-per-step form). Needs rmax >= 1.
int prrlu(hipStream_t s, int m, int n, double *A, int rmax, double rel_tol2, int *rowpiv, int *colpiv, double *L,
          double *info, double *ws, int t_begin, int t_end, bool allow_persistent = true);
// Bound on the polls of the persistent pivot search's waits for other workgroups (< 0: the
// default bound; 0: the waits give up at once, to exercise the fallback). Process-wide.
void set_coop_spin(int polls);
size_t prrlu_ws_doubles(int m, int n);
// The layout prrlu takes for an m x n block: {mode, shape (tile id or K), rows per workgroup,
// workgroups, device capacity of that persistent form (0 if stepped), capacity of the K = 8 and
// K = 16 persistent forms}.
void prrlu_layout(int m, int n, bool allow_big, int *out);

// X = R^{-1} for the upper Cholesky factor R of each r x r Gram matrix G (batch); ws holds
// batch * r * r doubles. Zero (padding) columns keep a unit diagonal.
void chol_upper_inv(hipStream_t s, int r, int batch, const double *G, double *X, double *ws);
// X = R^{-1} for the upper Cholesky factor of U_z^T U_z, U_z the m x r row-major matrix at
// U + z sU (X_z at X + z r^2), Gram matrix and factorisation in one launch; false (nothing
// launched) when r exceeds 32 or the Gram matrix is too tall for one workgroup (m r^2 > 4e6).
bool gram_chol_inv(hipStream_t s, int m, int r, int batch, const double *U, long long sU, double *X);

// Batched forms: one workgroup per job (and per component for the SVD / Cholesky), the jobs
// read from a device array; used to step many independent states in lock-step.
struct PrrluJob {
    double *A;
    int m, n, rmax;
    double rel_tol2;
    int *rowpiv, *colpiv;
    double *L, *info, *ws;  // ws: prrlu_ws_doubles(m, n) doubles
    // set by prrlu_prepare: 0 single-workgroup register tiles (shape: tile shape id), 1
    // multi-workgroup (rows per workgroup, workgroups) stepped one launch per pivot, 2 the same
    // layout in one persistent launch (when the workgroups can all be resident), 3 stepped with
    // longer stripes, 4 one persistent launch of long stripes (K rows per thread in shape)
    int mode, shape, rows, nblk;
    int spin;  // poll bound of the persistent form's waits (set by prrlu_prepare)
    int kl;    // mode 4: rows per thread held in LDS (set by prrlu_prepare)
};
void prrlu_prepare(PrrluJob &j, bool allow_big = false);
struct SvdJob {
    const double *A;  // R factors, as for jacobi_svd
    double *sigma, *V;
    int n, batch;
    const double *delta;  // per component truncation threshold (device) or null
};
struct CholJob {
    const double *G;
    double *X, *R;
    int r, batch;
};
// Launches the register jobs (t_begin = 0) and steps t_begin..t_end of the multi-workgroup jobs.
void prrlu_batch(hipStream_t s, int njobs, const PrrluJob *host_jobs, const PrrluJob *dev_jobs, int t_begin,
                 int t_end);
bool jacobi_batch_fits(int nmax);
void jacobi_svd_batch(hipStream_t s, int njobs, int ncomp, int nmax, const SvdJob *dev_jobs);
void chol_upper_inv_batch(hipStream_t s, int njobs, int ncomp, int rmax, const CholJob *dev_jobs);  // rmax: largest r

// X (m x r, row-major) = L (m x ldl) * inv(L[rowpiv, :r]), the interpolative basis.
void interp_solve(hipStream_t s, int m, int r, const double *L, int ldl, const int *rowpiv, double *X);

// ------------------------------------------------------------------ fiber.hip
// Conservation laws the fiber kernels evaluate: the Euler system (Sec. 2.1, d + 2 components)
// and the two scalar laws of Sec. 5.1-5.2 with unit velocity along every axis, linear advection
// f_dir(u) = u and Burgers f_dir(u) = u^2 / 2 (one component).
enum { kLawEuler = 0, kLawLinAdv = 1, kLawBurgers = 2 };
template <int ND, int LW>
struct LawNC {
    static constexpr int v = LW == kLawEuler ? ND + 2 : 1;
};

struct FiberGeom {
    int d, ncomp, dir, k;       // dimension, components, flux direction, free core
    int law;                    // kLawEuler / kLawLinAdv / kLawBurgers
    int n[kMaxDim];             // cells per dimension
    int bc[kMaxDim];            // boundary code per dimension
    double gamma, alpha, eps_w; // EOS, LF alpha, WENO epsilon (h_dir^2)
    const double *alpha_dev;    // if set, alpha is read from this device scalar instead
    double qin[kMaxDim][2][5];  // conserved ghost state of each inflow side [dim][low/high][c]
};

__device__ inline double geom_alpha(const FiberGeom &g) { return g.alpha_dev ? *g.alpha_dev : g.alpha; }

// Value of component c at cell `raw` along mode m (maybe a ghost) from the value v read at
// ghost_map's cell: negated for the normal momentum of a symmetry plane (Euler law), the inflow
// state on an inflow side.
template <typename T>
__device__ inline T ghost_fix(const FiberGeom &g, int m, int raw, int c, T v) {
    if (!bc_special(g.bc[m])) return v;  // uniform: periodic and transmissive sides are index maps
    const int kind = ghost_kind(raw, g.n[m], g.bc[m]);
    if (kind == kGhostMirror && g.law == kLawEuler && c == 1 + m) return -v;
    if (kind == kGhostInflow) return T(g.qin[m][raw >= g.n[m]][c]);
    return v;
}

// Lane moves within a wave: a double permuted with a DPP control word (both 32-bit halves moved
// alike).
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// The value of lane `lane` (wave-uniform) in every lane, through scalar registers.
__device__ __forceinline__ double readlane_d(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}

// 1/x, 1/sqrt(x) and sqrt(x) for x > 0 (nr_sqrt(0) = 0) to about 1 ulp: the hardware estimates
// (about 23 correct bits) refined by two Newton-Raphson steps each, for r = 1/x
// (r <- r + r (1 - x r)) and for y = 1/sqrt(x) (y <- y + y (1 - x y^2) / 2), sqrt(x) = x y. They
// take about a third of the instructions of the correctly rounded forms.
__device__ __forceinline__ double nr_rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ double nr_rsqrt(double x) {
    double y = __builtin_amdgcn_rsq(x);
    y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
    return fma(0.5 * y, fma(-x * y, y, 1.0), y);
}
__device__ __forceinline__ double nr_sqrt(double x) { return x > 0.0 ? x * nr_rsqrt(x) : 0.0; }

// Interface matrices of the state cores. Left (side 0): P[c][s][a][R_k] for the p left
// multi-indices idx[a * k + j], j < k. Right (side 1): Q[c][s][R_{k+1}][b] for the q right
// multi-indices idx[b * (d-1-k) + j] (modes k+1..d-1). The entry on mode shift_mode (if it is
// one of the multi-index modes) is shifted: shift slot s = 0..S-1 takes cell v - 3 + s
// (ghost-mapped): S = 6 for a face index (cells m-3..m+2), S = 7 for a cell (i-3..i+3).
void iface(hipStream_t s, const FiberGeom &g, int side, const double *const *cores, const int *ranks, int count,
           const int *idx, int S, int shift_mode, double *out);
// The same for up to 8 interface matrices of one block (same geometry, free core g.k) in one
// launch; each request as the arguments of iface.
struct IfaceReq {
    const double *const *cores;
    const int *ranks;
    int side, count, S, shift_mode;
    const int *idx;
    double *out;
};
void iface_batch(hipStream_t s, const FiberGeom &g, int n, const IfaceReq *req);

// Fused stage kernel: Y = wn Un + wx X + wl L(X) at the block points (a, i, b) of core k,
// L(X) = -sum_d (Fhat_d(+1/2) - Fhat_d(-1/2)) / h_d from the seven cells around each point in
// every direction, computed in T (FP64, or FP32 for the reduced-precision path). X stencil
// values: W0[c][a][cell][b] over the N_k cells of mode k (the neighbours along mode k) and,
// for every direction d != k, Wd[d][c][s][a][i][b] (s = 0..6 for cells -3..+3). The pass-through
// terms use FP64 values: X0[c][a][i][b] (X itself) and WN (Un, read only when wn != 0).
template <typename T>
struct StageArgsT {
    const T *W0;  // X at the block points, [c][a][i][b] with component stride w0_cs
    const T *Wd[kMaxDim];
    const double *X0;  // the same values in FP64 (same layout as W0)
    const double *WN;  // Un at the block points, [c][a][i][b] (component stride p Nk q)
    double wn, wx, wl;
    double inv_h[kMaxDim], eps_w[kMaxDim];
    long long w0_cs;  // p Nk q for a separate gather; 7 p Nk q when W0 is the centre slice of a Wd
};
template <typename T>
void stage_block(hipStream_t s, const FiberGeom &g, int p, int q, const StageArgsT<T> &a, double *out, long long sa,
                 long long si, long long sb, long long sc, int *flags);

// LF-cross (Sec. 4.2): f^+ and f^- of every component at the block's cells from the state there
// (W0[c * cs + (a Nk + i) q + b]); output (a, i, b, c) with c < 2 ncomp, f^+ first, at
// out[a * sa + i * si + b * sb + c * sc]. The sampled residual of such a cross: the state at the
// probe cells pts (ustencil: npts * 6 * ncomp doubles of workspace) against the candidate
// (fcores, franks; last core [R][N][2 ncomp]); acc receives one partial pair per 256 points.
void lf_block(hipStream_t s, const FiberGeom &g, int p, int q, const double *W0, long long cs, double *out,
              long long sa, long long si, long long sb, long long sc, int *flags);
void sample_lf_residual(hipStream_t s, const FiberGeom &g, const double *const *ucores, const int *ranks, int npts,
                        const int *pts, const double *const *fcores, const int *franks, double *ustencil, double *acc,
                        int *flags);

// Writes the conserved inflow state of g.qin into the gathered block W ([c][s][a][i][b], component
// stride cs, shift stride ss, block p x Nk x q) at the cells on an inflow side of mode `mode`:
// `pairs` (device, 3 ints each: shift s, pivot index, side 0 low / 1 high) list the (shift, pivot)
// combinations of the left interface (right = false, pivot a) or the right one (right = true,
// pivot b) whose shifted cell is an inflow ghost; their interface rows are zero (iface).
template <typename T>
void inflow_fill(hipStream_t s, const FiberGeom &g, int mode, int npairs, const int *pairs, bool right, int p, int Nk,
                 int q, long long cs, long long ss, T *W);

// FP32 batched GEMM C = A B (row-major) on the matrix cores (v_mfma_f32_16x16x4f32).
void gemm_f32(hipStream_t s, int M, int N, int K, const float *A, int lda, const float *B, int ldb, float *C, int ldc,
              const GemmBatch &bt = GemmBatch());
void to_f32(hipStream_t s, long long n, const double *x, float *y);

// Workgroups (partial sum pairs written to acc) of sample_stage for d dimensions.
int sample_stage_blocks(int d, int npts);
// Exact stage value at random cells and the sampled residual of a TT of it: X at the 7 d
// star cells (slot d*7 + s), Un at the point, TT approximation (shared cores + last core with
// one slice per component).
void sample_stage(hipStream_t s, const FiberGeom &g, const double *const *xcores, const int *xranks,
                  const double *const *ncores, const int *nranks, int npts, unsigned long long seed,
                  const double *const *fcores, const int *franks, double wn, double wx, double wl,
                  const double *inv_h, const double *eps_w, double *ust, double *acc, int *flags);

// Fused LF + WENO5-JS flux evaluation of a block from the gathered stencil values.
// Wv layout: same_dir (k == dir): W[c][a][cell][b] over N_k cells, the block's middle mode is
// the N_k + 1 faces; otherwise W[c][s][a][i][b] (6 shifts, N_k cells). Output element
// (a, i, b, c) goes to out[a * sa + i * si + b * sb + c * sc]. flags: device int (OR-ed bits).
template <typename T>
void weno_block(hipStream_t s, const FiberGeom &g, int p, int q, const T *W, double *out, long long sa, long long si,
                long long sb, long long sc, int *flags);

// Dense evaluation of a TT list from the left part Lm[c] ((prod of N_0..N_{d-2}) x R) and the
// last cores G[c] (R x N_{d-1}): mode 0 writes out[c][cell]; mode 1 reduces the cell wave speed
// (|u| + a for the Euler law, |u| for Burgers) into partial[block] and raises flags on
// non-physical cells. nblocks must be dense_eval_blocks(mode, nrows, R, nlast), the number of
// partials mode 1 writes. law: kLawEuler or kLawBurgers for mode 1, any law for mode 0.
int dense_eval_blocks(int mode, long long nrows, int R, int nlast);
void dense_eval(hipStream_t s, int mode, int d, int law, long long nrows, int R, int nlast, const double *Lm,
                long long lm_stride, const double *G, long long g_stride, double gamma, double *out, double *partial,
                int nblocks, int *flags);
void reduce_max_dev(hipStream_t s, const double *partial, int n, double *dst);

// ------------------------------------------------------------------ alpha.hip
// Estimated max over the grid of the cell wave speed of a TT state (|u| + a for the Euler law,
// ndim + 2 components; |u| for Burgers, one component; cores[k] the [c][R_k][N_k][R_{k+1}] core
// of every component, ranks common): a search along grid lines
// through kAlphaStartCells seeded cells and the previous best cell (best: device int[d], in/out,
// best[0] < 0 for none), then kAlphaRounds - 1 rounds along every mode through the kAlphaKeep
// best cells. Writes the estimate to the device scalar alpha; raises kFlagNonPhys in flags for a
// non-physical cell on a visited line. Workspace: alpha_search_ints(d, N_1) ints and
// alpha_search_doubles(d, N_1) doubles.
constexpr int kAlphaStartCells = 256, kAlphaKeep = 16, kAlphaMiddleLines = 4, kAlphaRounds = 3;
size_t alpha_search_ints(int d, int n1);
size_t alpha_search_doubles(int d, int n1);
void alpha_search(hipStream_t s, int d, int law, const int *n, const double *const *cores, const int *ranks,
                  double gamma, unsigned long long seed, int *best, int *wsi, double *wsd, double *alpha, int *flags);

// Sampled residual of a flux TT at random points (face index on mode dir).
void sample_residual(hipStream_t s, const FiberGeom &g, const double *const *ucores, const int *ranks, int npts,
                     const int *pts, const double *const *fcores, const int *franks, double *ustencil, double *acc,
                     int *flags);

// ------------------------------------------------------------------ tt.hip
void fill(hipStream_t s, double *p, long long n, double v);
// out[c][o_r + a][i][o_c + b] = w * G[c][a][i][b] (per-component strides given).
void place_block(hipStream_t s, int ncomp, int ra, int n, int rb, const double *G, long long gstride, double w,
                 double *out, int Ra, int Rb, long long ostride, int o_r, int o_c);
// out[c][a][i][b] = scale * (G[c][a][i+1][b] - G[c][a][i][b]), i < n (G has n + 1 faces).
void face_diff(hipStream_t s, int ncomp, int ra, int n, int rb, const double *G, long long gstride, double scale,
               double *out, long long ostride);
// Transposed copy: out[t][i][b] = X[(i * q + b) * r + t] (R->L interpolative core).
void transpose_rows(hipStream_t s, int M, int q, int r, const double *X, double *out);
// Copy the last core's component slices into per-component cores: out[c][a][i][0] = G[a][i][c].
void split_last(hipStream_t s, int ra, int n, int ncomp, const double *G, double *out, long long ostride);
// Broadcast a shared core to every component slot.
void broadcast_core(hipStream_t s, int ncomp, long long len, const double *G, double *out, long long ostride);
// Rounding helpers: per component c, rank r_c from sigma tail vs delta_c, then
// W1[c] = V[:, :r_c] diag(1/sigma) (n x R), W2[c] = diag(sigma) V[:, :r_c]^T (R x n), padded to R.
void trunc_ranks(hipStream_t s, int n, int batch, const double *sigma, const double *delta_abs, double rel, int rcap,
                 int *ranks);
void build_projectors(hipStream_t s, int n, int batch, int R, const double *sigma, const double *V, const int *ranks,
                      double *W1, double *W2);
// npts random cells of an n[0] x ... x n[d-1] grid (int [npts][d]), drawn on the device from seed.
void sample_points(hipStream_t s, int npts, int d, const int *n, unsigned long long seed, int *out);

// out[z] = ||X[z]||_F; if scaled is given, scaled[z] = scale * out[z] as well.
void frob_norms(hipStream_t s, int batch, long long len, const double *X, long long stride, double *out,
                double *scaled = nullptr, double scale = 0.0);

}  // namespace wtt
