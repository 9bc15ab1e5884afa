// Dense FP64 linear algebra for the TT hot path on gfx950:
//  - batched GEMM (LDS-tiled vector shapes, or 64x64 tiles on the FP64 matrix cores), tile
//    shape autotuned per problem bucket;
//  - Householder TSQR returning the R factor of tall unfoldings (one workgroup per row
//    block, leaves held in registers for up to 64 columns, reduction tree of stacked R factors);
//  - one-sided (Hestenes) Jacobi SVD of the small R factors (on R^T), one workgroup per matrix;
//  - full-pivot rank-revealing LU used to choose cross pivots (greedy maximum volume:
//    each step takes the largest residual entry, found by wavefront reductions): one workgroup
//    with the block in registers, a persistent multi-workgroup form, or one launch per step;
//  - the interpolative basis L * inv(L[I, :]) of a cross (Sec. 3.3, CUR / skeleton form);
//  - CholeskyQR factors (Gram matrix on the FP64 matrix cores, Cholesky and inverse in one
//    wave's registers) for re-orthonormalising a basis.
#include <algorithm>
#include <array>
#include <map>
#include <mutex>
#include <vector>
#include <cmath>

#include "common.h"

namespace wtt {

namespace {

constexpr int kWave = 64;


template <int CTRL>
__device__ __forceinline__ long long dpp_ll(long long v) {
    const int lo = __builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), CTRL, 0xF, 0xF, false);
    return ((long long)hi << 32) | (unsigned)lo;
}

__device__ __forceinline__ long long readlane_ll(long long v, int lane) {
    const int lo = __builtin_amdgcn_readlane((int)v, lane);
    const int hi = __builtin_amdgcn_readlane((int)(v >> 32), lane);
    return ((long long)hi << 32) | (unsigned)lo;
}

// (largest magnitude, its linear index) with ties to the lower index, and a running sum.
template <typename I>
__device__ __forceinline__ void amax_merge(double &m, I &i, double om, I oi) {
    const bool take = om > m || (om == m && oi < i);
    m = take ? om : m;
    i = take ? oi : i;
}

template <int CTRL, typename I>
__device__ __forceinline__ void amax_sum_step(double &m, I &i, double &s) {
    const double om = dpp_d<CTRL>(m), os = dpp_d<CTRL>(s);
    I oi;
    if constexpr (sizeof(I) == 8) oi = dpp_ll<CTRL>(i);
    else oi = dpp_i<CTRL>(i);
    amax_merge(m, i, om, oi);
    s += os;
}

// Wave-wide argmax and sum (every lane active); every lane gets the results.
template <typename I>
__device__ __forceinline__ void wave_amax_sum(double &m, I &i, double &s) {
    amax_sum_step<0xB1>(m, i, s);
    amax_sum_step<0x4E>(m, i, s);
    amax_sum_step<0x141>(m, i, s);
    amax_sum_step<0x140>(m, i, s);
    double rm[4], rs[4];
    I ri[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        rm[r] = readlane_d(m, 16 * r);
        rs[r] = readlane_d(s, 16 * r);
        if constexpr (sizeof(I) == 8) ri[r] = readlane_ll(i, 16 * r);
        else ri[r] = __builtin_amdgcn_readlane(i, 16 * r);
    }
    m = rm[0]; i = ri[0];
#pragma unroll
    for (int r = 1; r < 4; ++r) amax_merge(m, i, rm[r], ri[r]);
    s = (rs[0] + rs[1]) + (rs[2] + rs[3]);
}

// Argmax and sum over lanes 0..15 (every lane active); the result of row 0 is returned to all
// lanes. Used to combine up to 16 per-wave partials read from LDS.
template <typename I>
__device__ __forceinline__ void row0_amax_sum(double &m, I &i, double &s) {
    amax_sum_step<0xB1>(m, i, s);
    amax_sum_step<0x4E>(m, i, s);
    amax_sum_step<0x141>(m, i, s);
    amax_sum_step<0x140>(m, i, s);
    m = readlane_d(m, 0);
    s = readlane_d(s, 0);
    if constexpr (sizeof(I) == 8) i = readlane_ll(i, 0);
    else i = __builtin_amdgcn_readlane(i, 0);
}

// Sum over the 64 lanes of a wave (every lane active); every lane gets the result. Within each
// row of 16 lanes: swap neighbours, swap pairs (quad permutations), mirror halves, mirror the
// row; then the four row sums are read from lanes 0, 16, 32, 48.
__device__ inline double wave_sum(double v) {
    v += dpp_d<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_d<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_d<0x141>(v);  // row_half_mirror
    v += dpp_d<0x140>(v);  // row_mirror
    return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

// Sum over the workgroup; every thread gets the result. red must hold >= nwaves doubles.
__device__ inline double block_sum(double v, double *red) {
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave, nw = blockDim.x / kWave;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < nw; ++i) t += red[i];
    return t;
}

// ------------------------------------------------------------------------------ GEMM
constexpr int BK = 16;

// C tile TBM x TBN per 256-thread workgroup; thread (ty, tx) = (t / 16, t % 16) owns rows
// ty * (TBM / 16) + i and columns tx + 16 j. Every output sums over k in the same order for
// every tile shape, so the shape changes the speed, never the result.
template <bool TA, bool TB, int TBM, int TBN>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, double alpha, const double *__restrict__ A,
                                              int lda, const double *__restrict__ B, int ldb, double beta,
                                              double *__restrict__ C, int ldc, GemmBatch bt) {
    constexpr int RI = TBM / 16, RJ = TBN / 16;
    const int z = blockIdx.z, z1 = z / bt.nb2, z2 = z % bt.nb2;
    A += z1 * bt.sA1 + z2 * bt.sA2;
    B += z1 * bt.sB1 + z2 * bt.sB2;
    C += z1 * bt.sC1 + z2 * bt.sC2;
    if (bt.ktot > 0) K = min(K, bt.ktot - z2 * K);  // split-K: chunk z2 of the reduction
    __shared__ double As[BK][TBM + 1];
    __shared__ double Bs[BK][TBN + 1];
    const int t = threadIdx.x, tx = t % 16, ty = t / 16;
    const int m0 = blockIdx.y * TBM, n0 = blockIdx.x * TBN;
    double acc[RI][RJ];
#pragma unroll
    for (int i = 0; i < RI; ++i)
#pragma unroll
        for (int j = 0; j < RJ; ++j) acc[i][j] = 0.0;
    for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
        for (int l = 0; l < (TBM * BK + 255) / 256; ++l) {
            const int e = t + 256 * l;
            if (e < TBM * BK) {
                int r, kk;
                if (!TA) { r = e / BK; kk = e % BK; } else { kk = e / TBM; r = e % TBM; }
                const int gm = m0 + r, gk = k0 + kk;
                double v = 0.0;
                if (gm < M && gk < K) v = TA ? A[(long long)gk * lda + gm] : A[(long long)gm * lda + gk];
                As[kk][r] = v;
            }
        }
#pragma unroll
        for (int l = 0; l < (TBN * BK + 255) / 256; ++l) {
            const int e = t + 256 * l;
            if (e < TBN * BK) {
                int c, kk;
                if (!TB) { kk = e / TBN; c = e % TBN; } else { c = e / BK; kk = e % BK; }
                const int gn = n0 + c, gk = k0 + kk;
                double v = 0.0;
                if (gn < N && gk < K) v = TB ? B[(long long)gn * ldb + gk] : B[(long long)gk * ldb + gn];
                Bs[kk][c] = v;
            }
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < BK; ++kk) {
            double a[RI], b[RJ];
#pragma unroll
            for (int i = 0; i < RI; ++i) a[i] = As[kk][ty * RI + i];
#pragma unroll
            for (int j = 0; j < RJ; ++j) b[j] = Bs[kk][tx + 16 * j];
#pragma unroll
            for (int i = 0; i < RI; ++i)
#pragma unroll
                for (int j = 0; j < RJ; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < RI; ++i) {
        const int gm = m0 + ty * RI + i;
        if (gm >= M) continue;
#pragma unroll
        for (int j = 0; j < RJ; ++j) {
            const int gn = n0 + tx + 16 * j;
            if (gn >= N) continue;
            double *c = C + (long long)gm * ldc + gn;
            *c = beta == 0.0 ? alpha * acc[i][j] : alpha * acc[i][j] + beta * *c;
        }
    }
}

// FP64 matrix-core form: 64 x 64 tile per 256-thread workgroup, each wave a 32 x 32 quarter as
// 2 x 2 v_mfma_f64_16x16x4f64 tiles, operands staged through LDS in depth-16 slices. Operand
// layout of the instruction: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; its four
// accumulators hold D[l / 16 + 4 v][l % 16], v = 0..3 (checked on the device against a host
// product). The matrix core sums each group of four products in its own order, so results
// agree with the vector form to rounding.
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_gemm_mfma(int M, int N, int K, double alpha, const double *__restrict__ A,
                                                   int lda, const double *__restrict__ B, int ldb, double beta,
                                                   double *__restrict__ C, int ldc, GemmBatch bt) {
    constexpr int TBM = 64, TBN = 64;
    const int z = blockIdx.z, z1 = z / bt.nb2, z2 = z % bt.nb2;
    A += z1 * bt.sA1 + z2 * bt.sA2;
    B += z1 * bt.sB1 + z2 * bt.sB2;
    C += z1 * bt.sC1 + z2 * bt.sC2;
    if (bt.ktot > 0) K = min(K, bt.ktot - z2 * K);
    __shared__ double As[BK][TBM + 1];
    __shared__ double Bs[BK][TBN + 1];
    const int t = threadIdx.x, lane = t % 64, wv = t / 64, wr = wv / 2, wc = wv % 2;
    const int m0 = blockIdx.y * TBM, n0 = blockIdx.x * TBN;
    f64x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
        for (int l = 0; l < TBM * BK / 256; ++l) {
            const int e = t + 256 * l;
            int r, kk;
            if (!TA) { r = e / BK; kk = e % BK; } else { kk = e / TBM; r = e % TBM; }
            const int gm = m0 + r, gk = k0 + kk;
            double v = 0.0;
            if (gm < M && gk < K) v = TA ? A[(long long)gk * lda + gm] : A[(long long)gm * lda + gk];
            As[kk][r] = v;
            int c;
            if (!TB) { kk = e / TBN; c = e % TBN; } else { c = e / BK; kk = e % BK; }
            const int gn = n0 + c;
            const int gk2 = k0 + kk;
            v = 0.0;
            if (gn < N && gk2 < K) v = TB ? B[(long long)gn * ldb + gk2] : B[(long long)gk2 * ldb + gn];
            Bs[kk][c] = v;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < BK; ks += 4) {
            double a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = As[ks + lane / 16][wr * 32 + i * 16 + lane % 16];
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = Bs[ks + lane / 16][wc * 32 + j * 16 + lane % 16];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gm = m0 + wr * 32 + i * 16 + lane / 16 + 4 * v;
                const int gn = n0 + wc * 32 + j * 16 + lane % 16;
                if (gm < M && gn < N) {
                    double *c = C + (long long)gm * ldc + gn;
                    *c = beta == 0.0 ? alpha * acc[i][j][v] : alpha * acc[i][j][v] + beta * *c;
                }
            }
}

// Resident-operand forms for products with a short reduction (K <= 4 KSM, no split-K, neither
// operand transposed), the interface contractions of the gathers: one operand is staged once per
// workgroup in LDS, in the lane order of the v_mfma_f64_16x16x4f64 fragments (one conflict-free
// 64-lane read per fragment), and the other streams from memory in 16-wide strips, each wave
// loading its next strip while the matrix cores work on the current one; registers hold only the
// streamed strips and the accumulators, so that several waves share a SIMD. Lane group
// g = l / 16 takes the reduction indices [g KS, (g + 1) KS), KS = ceil(K / 4), one per MFMA step,
// so that a lane reads KS consecutive entries of a row of A and every 16 lanes read 128
// contiguous bytes of a row of B; indices at or beyond K contribute zeros. Accumulator v of lane
// l holds D[l / 16 + 4 v][l % 16].

// s_waitcnt vmcnt(0) with expcnt and lgkmcnt left open (gfx9 encoding: vmcnt in bits 3:0 and
// 15:14, expcnt 6:4, lgkmcnt 11:8). Issued after a strip's products and before its stores, while
// only the next strip's loads are in flight, it lets the copies of those loads at the end of the
// iteration go without waiting on the stores.
constexpr int kWaitLoadsOnly = 0x0F70;
// Load from base + a 32-bit byte offset (the streamed operand of one batch entry spans less
// than 2^31 bytes), so that a load takes one 32-bit offset register beside the scalar base.
__device__ __forceinline__ double ld_at(const double *__restrict__ base, unsigned byte_off) {
    return *reinterpret_cast<const double *>(reinterpret_cast<const char *>(base) + byte_off);
}

// waves per SIMD the resident-operand kernels are compiled for (at most 512 / 3 registers each):
// several waves hide the latency of the streamed loads
constexpr int kResidentWaves = 3;

// A resident (M <= 16 MI; LDS [i][s][lane] = A[16 i + l % 16][g KS + s]): wave w of the grid takes
// the 16-column strips w, w + W, ... of B and C.
template <int MI, int KSM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kResidentWaves))) void k_gemm_mfma_ra(int M, int N, int K, double alpha, const double *__restrict__ A,
                                                      int lda, const double *__restrict__ B, int ldb, double beta,
                                                      double *__restrict__ C, int ldc, GemmBatch bt) {
    __shared__ double As[MI * KSM * kWave];
    const int z = blockIdx.z, z1 = z / bt.nb2, z2 = z % bt.nb2;
    A += z1 * bt.sA1 + z2 * bt.sA2;
    B += z1 * bt.sB1 + z2 * bt.sB2;
    C += z1 * bt.sC1 + z2 * bt.sC2;
    const int lane = threadIdx.x % kWave, g = lane / 16, c = lane % 16;
    const int KS = (K + 3) / 4, k0 = g * KS;
    for (int e = threadIdx.x; e < MI * KSM * kWave; e += blockDim.x) {
        const int l = e % kWave, s = (e / kWave) % KSM, i = e / (kWave * KSM);
        const int row = 16 * i + l % 16, k = (l / 16) * KS + s;
        As[e] = (s < KS && k < K && row < M) ? A[(long long)row * lda + k] : 0.0;
    }
    __syncthreads();
    const int nstrip = (N + 15) / 16, nw = gridDim.x * (blockDim.x / kWave);
    int st = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    // The streamed loads are unconditional, from clamped indices: a row k >= K of B meets a zero
    // of A in LDS, and a column at or beyond N only feeds outputs that are not stored; so no load
    // needs a predicate, and the next strip's loads stay in flight across the products.
    double bn[KSM];
#pragma unroll
    for (int s = 0; s < KSM; ++s) bn[s] = ld_at(B, 8u * (unsigned)(min(k0 + s, K - 1) * ldb + min(16 * st + c, N - 1)));
    while (st < nstrip) {
        double b[KSM];
#pragma unroll
        for (int s = 0; s < KSM; ++s) b[s] = bn[s];
        const int nx = st + nw;
#pragma unroll
        for (int s = 0; s < KSM; ++s)
            bn[s] = ld_at(B, 8u * (unsigned)(min(k0 + s, K - 1) * ldb + min(16 * nx + c, N - 1)));
        f64x4 acc[MI];
#pragma unroll
        for (int i = 0; i < MI; ++i) acc[i] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < KSM; ++s) {
            if (s < KS)
#pragma unroll
                for (int i = 0; i < MI; ++i)
                    acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(As[(i * KSM + s) * kWave + lane], b[s], acc[i], 0, 0, 0);
            if (s % 4 == 3) __builtin_amdgcn_sched_barrier(0);  // fragments read four steps at a time
        }
        __builtin_amdgcn_s_waitcnt(kWaitLoadsOnly);
        const int col = 16 * st + c;
        if (beta == 0.0) {
#pragma unroll
            for (int i = 0; i < MI; ++i)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = 16 * i + g + 4 * v;
                    if (row < M && col < N) C[(long long)row * ldc + col] = alpha * acc[i][v];
                }
        } else {
#pragma unroll
            for (int i = 0; i < MI; ++i)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = 16 * i + g + 4 * v;
                    if (row < M && col < N) {
                        double *o = C + (long long)row * ldc + col;
                        *o = alpha * acc[i][v] + beta * *o;
                    }
                }
        }
        st = nx;
    }
}

// B resident (LDS [j][s][lane] = B[g KS + s][cb + 16 j + l % 16]): blockIdx.y picks the group of NJ
// 16-column blocks starting at column cb; wave w of the x-grid takes the 16-row strips
// w, w + W, ... of A and C.
template <int NJ, int KSM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kResidentWaves))) void k_gemm_mfma_rb(int M, int N, int K, double alpha, const double *__restrict__ A,
                                                      int lda, const double *__restrict__ B, int ldb, double beta,
                                                      double *__restrict__ C, int ldc, GemmBatch bt) {
    __shared__ double Bs[NJ * KSM * kWave];
    const int z = blockIdx.z, z1 = z / bt.nb2, z2 = z % bt.nb2;
    A += z1 * bt.sA1 + z2 * bt.sA2;
    B += z1 * bt.sB1 + z2 * bt.sB2;
    C += z1 * bt.sC1 + z2 * bt.sC2;
    const int lane = threadIdx.x % kWave, g = lane / 16, c = lane % 16;
    const int KS = (K + 3) / 4, k0 = g * KS, cb = 16 * NJ * blockIdx.y;
    for (int e = threadIdx.x; e < NJ * KSM * kWave; e += blockDim.x) {
        const int l = e % kWave, s = (e / kWave) % KSM, j = e / (kWave * KSM);
        const int col = cb + 16 * j + l % 16, k = (l / 16) * KS + s;
        Bs[e] = (s < KS && k < K && col < N) ? B[(long long)k * ldb + col] : 0.0;
    }
    __syncthreads();
    const int nstrip = (M + 15) / 16, nw = gridDim.x * (blockDim.x / kWave);
    int st = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    // unconditional loads from clamped indices, as in k_gemm_mfma_ra: a column k >= K of A meets a
    // zero of B in LDS, and a row at or beyond M only feeds outputs that are not stored
    double an[KSM];
#pragma unroll
    for (int s = 0; s < KSM; ++s) an[s] = ld_at(A, 8u * (unsigned)(min(16 * st + c, M - 1) * lda + min(k0 + s, K - 1)));
    while (st < nstrip) {
        double a[KSM];
#pragma unroll
        for (int s = 0; s < KSM; ++s) a[s] = an[s];
        const int nx = st + nw;
#pragma unroll
        for (int s = 0; s < KSM; ++s)
            an[s] = ld_at(A, 8u * (unsigned)(min(16 * nx + c, M - 1) * lda + min(k0 + s, K - 1)));
        f64x4 acc[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) acc[j] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < KSM; ++s) {
            if (s < KS)
#pragma unroll
                for (int j = 0; j < NJ; ++j)
                    acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], Bs[(j * KSM + s) * kWave + lane], acc[j], 0, 0, 0);
            if (s % 4 == 3) __builtin_amdgcn_sched_barrier(0);  // fragments read four steps at a time
        }
        __builtin_amdgcn_s_waitcnt(kWaitLoadsOnly);
        if (beta == 0.0) {
#pragma unroll
            for (int j = 0; j < NJ; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = 16 * st + g + 4 * v, col = cb + 16 * j + c;
                    if (row < M && col < N) C[(long long)row * ldc + col] = alpha * acc[j][v];
                }
        } else {
#pragma unroll
            for (int j = 0; j < NJ; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = 16 * st + g + 4 * v, col = cb + 16 * j + c;
                    if (row < M && col < N) {
                        double *o = C + (long long)row * ldc + col;
                        *o = alpha * acc[j][v] + beta * *o;
                    }
                }
        }
        st = nx;
    }
}

// --------------------------------------------------------------------------- TSQR
// Householder QR of one row block [r0, r0 + nr) of matrix z, in a column-major scratch copy;
// only R is kept. Step j reflects column j onto its diagonal: every thread derives the
// reflector (beta, tau and the scale of the unnormalised vector) from the squared norm of the
// column below the diagonal, which the wave that updated column j in the previous step left in
// LDS; the waves then apply it to the trailing columns, the wave of column j + 1 also forming
// that column's new norm. One barrier per column.
// LEAF: leaf level (true, one launch per TSQR call) or tree level (false); the two levels get
// distinct kernel names so that profiles can count TSQR calls.
template <int RPL, int NT, bool LEAF>
__global__ __launch_bounds__(NT) void k_hhqr(int m, int n, int bm, int nblk, const double *__restrict__ A,
                                            long long sz, long long rs, long long cs, double *__restrict__ Rout,
                                            double *__restrict__ scratch, int use_lds) {
    extern __shared__ double wlds[];
    __shared__ double red[NT / kWave];
    __shared__ double snorm[2];
    const int blk = blockIdx.x, z = blockIdx.y, tid = threadIdx.x;
    const int lane = tid % kWave, w = tid / kWave, nw = NT / kWave;
    const int r0 = blk * bm;
    const int nr = min(bm, m - r0);
    // LDS copies use a padded leading dimension so that a row of consecutive columns does not
    // fall into one bank
    const int ldw = use_lds ? bm + 1 : bm;
    double *W = use_lds ? wlds : scratch + ((long long)z * nblk + blk) * (long long)bm * n;
    const double *Az = A + (long long)z * sz;
    const long long tot = (long long)nr * n;
    if (cs <= rs) {
        for (long long e = tid; e < tot; e += NT) {
            int i = (int)(e / n), j = (int)(e % n);
            W[(long long)j * ldw + i] = Az[(long long)(r0 + i) * rs + (long long)j * cs];
        }
    } else {
        for (long long e = tid; e < tot; e += NT) {
            int j = (int)(e / nr), i = (int)(e % nr);
            W[(long long)j * ldw + i] = Az[(long long)(r0 + i) * rs + (long long)j * cs];
        }
    }
    __syncthreads();
    {
        double ss = 0.0;
        for (int i = 1 + tid; i < nr; i += NT) ss += W[i] * W[i];
        ss = block_sum(ss, red);
        if (tid == 0) snorm[0] = ss;
    }
    __syncthreads();
    // lane L owns rows L + 64 q, q < RPL (RPL * 64 >= bm); a column's entries at those rows are
    // loaded into registers together, so one LDS latency covers the whole column
    const int kmax = min(nr, n);
    double beta_prev = 0.0;
    for (int j = 0; j < kmax; ++j) {
        const double *col = W + (long long)j * ldw;
        if (tid == 0 && j > 0) W[(long long)(j - 1) * ldw + (j - 1)] = beta_prev;  // nobody reads it any more
        const double a = col[j], xn2 = snorm[j & 1];
        double beta, tau, scale;
        if (xn2 == 0.0) {
            beta = a; tau = 0.0; scale = 0.0;
        } else {
            beta = -copysign(sqrt(a * a + xn2), a);
            tau = (beta - a) / beta;
            scale = 1.0 / (a - beta);
        }
        beta_prev = beta;
        if (j + 1 + w < n) {  // this wave has trailing columns
        double cv[RPL];
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
            const int i = lane + kWave * q;
            cv[q] = (i > j && i < nr) ? col[i] : 0.0;
        }
        // v = [1; scale * col[j+1..]]; each trailing column l: cl -= tau (v . cl) v
        for (int l = j + 1 + w; l < n; l += nw) {
            double *cl = W + (long long)l * ldw;
            double x[RPL];
#pragma unroll
            for (int q = 0; q < RPL; ++q) {
                const int i = lane + kWave * q;
                x[q] = (i > j && i < nr) ? cl[i] : 0.0;
            }
            double ss = 0.0;  // squared norm of the updated column below row j + 1 (for l = j + 1)
            if (tau != 0.0) {
                double dot = 0.0;
#pragma unroll
                for (int q = 0; q < RPL; ++q) dot = fma(cv[q], x[q], dot);
                const double clj = readlane_d(lane == 0 ? cl[j] : 0.0, 0);
                dot = clj + scale * wave_sum(dot);
                const double f = tau * dot, fs = f * scale;
                if (lane == 0) cl[j] = clj - f;
#pragma unroll
                for (int q = 0; q < RPL; ++q) {
                    const int i = lane + kWave * q;
                    const double v = x[q] - fs * cv[q];
                    if (i > j && i < nr) cl[i] = v;
                    if (i >= j + 2 && i < nr) ss = fma(v, v, ss);
                }
            } else {
#pragma unroll
                for (int q = 0; q < RPL; ++q) {
                    const int i = lane + kWave * q;
                    if (i >= j + 2) ss = fma(x[q], x[q], ss);
                }
            }
            if (l == j + 1) {
                ss = wave_sum(ss);
                if (lane == 0) snorm[(j + 1) & 1] = ss;
            }
        }
        }
        __syncthreads();
    }
    if (tid == 0 && kmax > 0) W[(long long)(kmax - 1) * ldw + (kmax - 1)] = beta_prev;
    __syncthreads();
    double *R = Rout + ((long long)z * nblk + blk) * (long long)n * n;
    for (long long e = tid; e < (long long)n * n; e += NT) {
        int i = (int)(e / n), jj = (int)(e % n);
        R[e] = (i <= jj && i < nr) ? W[(long long)jj * ldw + i] : 0.0;
    }
}

// Sum over each row of 16 lanes (all 16 active); every lane of the row gets the same bits.
__device__ __forceinline__ double row_sum16(double v) {
    v += dpp_d<0xB1>(v);
    v += dpp_d<0x4E>(v);
    v += dpp_d<0x141>(v);
    v += dpp_d<0x140>(v);
    return v;
}

// Register-resident Householder QR of a row block with at most 64 columns and 16 RPT rows, one
// 1024-thread workgroup per block. Lane l of wave w holds column c = 4 w + l / 16 at rows
// l % 16 + 16 q, q < RPT, for the whole factorisation; per column step only the Householder
// vector (and tau) passes through LDS, double-buffered by step parity, so one barrier per step.
// Each row of 16 lanes reduces its dot products with DPP alone. At step j every trailing column
// is reflected, then its row j (final, an entry of R) moves to the LDS copy of R and is zeroed in
// the registers, so rows above the current step never enter a sum; the owner of column j + 1
// then forms the next vector from its registers: alpha = its row j + 1, xn2 = the squared norm
// below it, beta = -sign(alpha) sqrt(alpha^2 + xn2), tau = (beta - alpha) / beta,
// v = [1; x / (alpha - beta)]. Rows past the block's end are zeros and stay zeros.
template <int RPT>
__device__ __forceinline__ void qr_reg_prep(double (&a)[RPT], int j, int lane, double *__restrict__ vb,
                                            double *__restrict__ tb, double *__restrict__ Rl) {
    const int rg = lane & 15, qj = j >> 4, src = __builtin_amdgcn_readfirstlane((lane & 48) | (j & 15));
    double x = 0.0;
#pragma unroll
    for (int q = 0; q < RPT; ++q)
        if (q == qj) x = a[q];
    const double alpha = readlane_d(x, src);
    if (rg == (j & 15)) {
#pragma unroll
        for (int q = 0; q < RPT; ++q)
            if (q == qj) a[q] = 0.0;
    }
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;  // four chains for latency
#pragma unroll
    for (int q = 0; q < RPT; q += 4) {
        s0 = fma(a[q], a[q], s0);
        s1 = fma(a[q + 1], a[q + 1], s1);
        s2 = fma(a[q + 2], a[q + 2], s2);
        s3 = fma(a[q + 3], a[q + 3], s3);
    }
    const double xn2 = row_sum16((s0 + s1) + (s2 + s3));
    double beta, tau, scale;
    if (xn2 == 0.0) {
        beta = alpha; tau = 0.0; scale = 0.0;
    } else {
        beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
        tau = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) vb[rg + 16 * q] = a[q] * scale;
    if (rg == (j & 15)) {
        vb[j] = 1.0;
        Rl[j * 64 + j] = beta;
        *tb = tau;
    }
}

template <int RPT, int NT>
__global__ __launch_bounds__(NT) void k_qr_reg(int m, int n, int bm, int nblk, const double *__restrict__ A,
                                               long long sz, long long rs, long long cs, double *__restrict__ Rout) {
    __shared__ double vb[2][16 * RPT];
    __shared__ double tb[2];
    __shared__ double Rl[64 * 64];
    const int blk = blockIdx.x, z = blockIdx.y, tid = threadIdx.x;
    const int lane = tid % kWave, w = tid / kWave;
    const int rg = lane & 15, c = 4 * w + (lane >> 4);
    const int r0 = blk * bm, nr = min(bm, m - r0);
    const double *Az = A + (long long)z * sz;
    double a[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int i = rg + 16 * q;
        a[q] = (c < n && i < nr) ? Az[(long long)(r0 + i) * rs + (long long)c * cs] : 0.0;
    }
    if (c == 0) qr_reg_prep<RPT>(a, 0, lane, vb[0], &tb[0], Rl);
    __syncthreads();
    for (int j = 0; j < n; ++j) {
        if (c > j && c < n) {
            const double *v = vb[j & 1];
            double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;  // four chains for latency
#pragma unroll
            for (int q = 0; q < RPT; q += 4) {
                d0 = fma(v[rg + 16 * q], a[q], d0);
                d1 = fma(v[rg + 16 * (q + 1)], a[q + 1], d1);
                d2 = fma(v[rg + 16 * (q + 2)], a[q + 2], d2);
                d3 = fma(v[rg + 16 * (q + 3)], a[q + 3], d3);
            }
            const double f = tb[j & 1] * row_sum16((d0 + d1) + (d2 + d3));
#pragma unroll
            for (int q = 0; q < RPT; ++q) a[q] = fma(-f, v[rg + 16 * q], a[q]);
            const int qj = j >> 4;
            if (rg == (j & 15)) {
#pragma unroll
                for (int q = 0; q < RPT; ++q)
                    if (q == qj) {
                        Rl[j * 64 + c] = a[q];
                        a[q] = 0.0;
                    }
            }
            if (c == j + 1) qr_reg_prep<RPT>(a, j + 1, lane, vb[(j + 1) & 1], &tb[(j + 1) & 1], Rl);
        }
        __syncthreads();
    }
    double *R = Rout + ((long long)z * nblk + blk) * (long long)n * n;
    for (int e = tid; e < n * n; e += NT) {
        const int i = e / n, l = e % n;
        R[e] = i <= l ? Rl[i * 64 + l] : 0.0;
    }
}

__global__ void k_sum_chunks(long long per, int nchunk, int batch, const double *__restrict__ part, double *__restrict__ C,
                             int M, int N, int ldc, long long sC) {
    long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e >= per * batch) return;
    const int z = (int)(e / per);
    const long long r = e % per;
    const int i = (int)(r / N), j = (int)(r % N);
    double acc = 0.0;
    for (int k = 0; k < nchunk; ++k) acc += part[((long long)z * nchunk + k) * per + r];
    C[z * sC + (long long)i * ldc + j] = acc;
    (void)M;
}

int leaf_rows(int n) {
    int bm = std::max(256, 2 * n);
    return (bm + 63) / 64 * 64;
}

// ---------------------------------------------------------------------- Jacobi SVD
// One-sided (Hestenes) Jacobi on the columns of an n x n matrix. Column pairs follow the
// round-robin "circle" schedule: with np = n rounded up to even, round r pairs player np-1
// with r and (r + k) mod (np-1) with (r - k) mod (np-1) for k = 1 .. np/2 - 1; np - 1 rounds
// meet every pair once. A padded column (odd n) is never rotated.
__device__ inline void circle_pair(int r, int k, int np, int *p, int *q) {
    // 0 <= r < np - 1 and 0 <= k < np / 2: one conditional wrap reduces r + k and r - k mod np - 1
    int a, b;
    if (k == 0) { a = np - 1; b = r; }
    else {
        a = r + k;
        a = a >= np - 1 ? a - (np - 1) : a;
        b = r - k;
        b = b < 0 ? b + (np - 1) : b;
    }
    *p = a < b ? a : b;
    *q = a < b ? b : a;
}

// The SVD of an n x n upper-triangular R (the R factor of a tall matrix C = Q R) is taken by
// one-sided Jacobi on X = R^T, whose columns are the rows of R: the rotations make the columns
// of X V_x orthogonal, R^T V_x = U_x Sigma, so C = (Q V_x) Sigma U_x^T and the right singular
// vectors of C are the normalised final columns of X. The rotations need not be accumulated,
// and Jacobi on R^T needs about half the sweeps of Jacobi on R (the transposed triangular
// factor is the classical preconditioning of one-sided Jacobi).
// X is column-major (column j at j * n), in LDS or global memory. Squared column norms are
// recomputed at the start of every sweep and updated through each rotation (a' = a - t c,
// b' = b + t c), so a pair needs one dot product; nrm holds n doubles. A pair whose cross
// product is at most eta (an absolute threshold, 0 for none) is left alone: with
// eta = 0.01 delta^2 / n, where delta is the truncation threshold of the singular values, the
// skipped rotations move no singular value by more than 1% of delta, and columns far below
// delta are not orthogonalised against each other to full relative precision.
__device__ void jacobi_sweeps(int n, double *X, int *nrot, double *nrm, double eta) {
    const int tid = threadIdx.x, lane = tid % kWave, w = tid / kWave, nw = blockDim.x / kWave;
    const int np = n + (n & 1);
    const double tol = 1e-15;
    for (int sweep = 0; sweep < 60; ++sweep) {
        for (int j = w; j < n; j += nw) {
            const double *xj = X + (long long)j * n;
            double ss = 0.0;
            for (int i = lane; i < n; i += kWave) ss += xj[i] * xj[i];
            ss = wave_sum(ss);
            if (lane == 0) nrm[j] = ss;
        }
        if (tid == 0) *nrot = 0;
        __syncthreads();
        for (int r = 0; r < np - 1; ++r) {
            for (int k = w; k < np / 2; k += nw) {
                int p, q;
                circle_pair(r, k, np, &p, &q);
                if (q >= n) continue;
                double *xp = X + (long long)p * n, *xq = X + (long long)q * n;
                double c = 0.0;
                for (int i = lane; i < n; i += kWave) c += xp[i] * xq[i];
                c = wave_sum(c);
                const double a = nrm[p], b = nrm[q];
                if (c == 0.0 || !(fabs(c) > tol * sqrt(a * b)) || !(fabs(c) > eta)) continue;
                // t = tan of the rotation angle: the root of t^2 c + (b - a) t - c = 0 of smaller
                // magnitude, t = sign(b - a) 2c / (|b - a| + sqrt((b - a)^2 + 4 c^2))
                const double dd = b - a;
                const double t = copysign(1.0, dd) * (2.0 * c) / (fabs(dd) + sqrt(dd * dd + 4.0 * c * c));
                const double cs = rsqrt(1.0 + t * t), sn = cs * t;
                for (int i = lane; i < n; i += kWave) {
                    const double x = xp[i], y = xq[i];
                    xp[i] = cs * x - sn * y;
                    xq[i] = sn * x + cs * y;
                }
                if (lane == 0) {
                    nrm[p] = fmax(a - t * c, 0.0);
                    nrm[q] = b + t * c;
                    *nrot = 1;  // every writer stores the same value
                }
            }
            __syncthreads();
        }
        const int done = *nrot == 0;
        __syncthreads();
        if (done) break;
    }
}

// Sum over each 8-lane segment (every lane active): every lane of a segment gets the same sum,
// so decisions taken on it agree across the segment.
__device__ __forceinline__ double seg8_sum(double v) {
    v += dpp_d<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_d<0x4E>(v);   // quad_perm [2,3,0,1]
    return v + dpp_d<0x141>(v);  // row_half_mirror: the other quad of the segment
}

// The same sweeps for n <= 8 RPL with eight column pairs per wave: pair k of a round goes to the
// 8-lane segment k (the workgroup has at least n / 2 segments), lane l of a segment holding rows
// l, l + 8, ..., l + 8 (RPL - 1) of both columns in registers from the dot product to the
// rotation. Every pair of a round is in flight at once, the rotation angle is formed once per
// eight pairs, and a pair's dot product is one three-step segment sum; the pairs, their order and
// the rotation formulas are those of jacobi_sweeps, with the roots and the reciprocal taken by
// nr_sqrt, nr_rcp and nr_rsqrt.
template <int RPL>
__device__ void jacobi_sweeps_seg(int n, double *X, int *nrot, double *nrm, double eta) {
    const int tid = threadIdx.x, sl = tid & 7, slot = tid >> 3, nslots = (int)(blockDim.x >> 3);
    const int np = n + (n & 1);
    const double tol2 = 1e-30;  // (1e-15)^2: the relative threshold of jacobi_sweeps, squared
    for (int sweep = 0; sweep < 60; ++sweep) {
        for (int j0 = 0; j0 < n; j0 += nslots) {
            const int j = j0 + slot;
            double ss = 0.0;
            if (j < n) {
                const double *xj = X + (long long)j * n;
#pragma unroll
                for (int k = 0; k < RPL; ++k) {
                    const int i = sl + 8 * k;
                    const double u = i < n ? xj[i] : 0.0;
                    ss = fma(u, u, ss);
                }
            }
            ss = seg8_sum(ss);
            if (j < n && sl == 0) nrm[j] = ss;
        }
        if (tid == 0) *nrot = 0;
        __syncthreads();
        for (int r = 0; r < np - 1; ++r) {
            int p = 0, q = n;
            if (slot < np / 2) circle_pair(r, slot, np, &p, &q);
            const bool valid = q < n;
            double *xp = X + (long long)p * n, *xq = X + (long long)(valid ? q : p) * n;
            double x[RPL], y[RPL], a = 0.0, b = 0.0, c = 0.0;
#pragma unroll
            for (int k = 0; k < RPL; ++k) {
                const int i = sl + 8 * k;
                const bool in = valid && i < n;
                x[k] = in ? xp[i] : 0.0;
                y[k] = in ? xq[i] : 0.0;
                c = fma(x[k], y[k], c);
            }
            if (valid) {
                a = nrm[p];
                b = nrm[q];
            }
            c = seg8_sum(c);
            if (valid && c != 0.0 && c * c > tol2 * (a * b) && fabs(c) > eta) {
                const double dd = b - a;
                const double t = copysign(1.0, dd) * (2.0 * c) * nr_rcp(fabs(dd) + nr_sqrt(fma(dd, dd, 4.0 * c * c)));
                const double cs = nr_rsqrt(fma(t, t, 1.0)), sn = cs * t;
#pragma unroll
                for (int k = 0; k < RPL; ++k) {
                    const int i = sl + 8 * k;
                    if (i < n) {
                        xp[i] = cs * x[k] - sn * y[k];
                        xq[i] = sn * x[k] + cs * y[k];
                    }
                }
                if (sl == 0) {
                    nrm[p] = fmax(a - t * c, 0.0);
                    nrm[q] = b + t * c;
                    *nrot = 1;  // every writer stores the same value
                }
            }
            __syncthreads();
        }
        const int done = *nrot == 0;
        __syncthreads();
        if (done) break;
    }
}

__device__ __forceinline__ void jacobi_run(int n, double *X, int *nrot, double *nrm, double eta) {
    // the segment forms need a segment per pair of a round: (n + 1) / 2 <= blockDim.x / 8
    const bool fits = (n + 1) / 2 <= (int)(blockDim.x >> 3);
    if (fits && n <= 32) jacobi_sweeps_seg<4>(n, X, nrot, nrm, eta);
    else if (fits && n <= 64) jacobi_sweeps_seg<8>(n, X, nrot, nrm, eta);
    else if (fits && n <= 128) jacobi_sweeps_seg<16>(n, X, nrot, nrm, eta);
    else jacobi_sweeps(n, X, nrot, nrm, eta);
}

// Singular values = final column norms of X, descending by rank counting (ties to the lower
// column); the right singular vectors of C are the normalised columns (row-major V, column pos
// = singular vector pos; a zero column gives a zero vector, whose singular value 0 is never
// kept by the truncation).
// sorted (LDS, may be null): also receives the singular values in descending order.
__device__ void jacobi_finish(int n, const double *X, double *sig_tmp, double *sigma, double *Vout,
                              double *sorted = nullptr) {
    const int tid = threadIdx.x, lane = tid % kWave, w = tid / kWave, nw = blockDim.x / kWave;
    for (int j = w; j < n; j += nw) {
        double s = 0.0;
        for (int i = lane; i < n; i += kWave) s += X[(long long)j * n + i] * X[(long long)j * n + i];
        s = wave_sum(s);
        if (lane == 0) sig_tmp[j] = sqrt(s);
    }
    __syncthreads();
    for (int j = w; j < n; j += nw) {
        const double sj = sig_tmp[j];
        int pos = 0;
        for (int i = lane; i < n; i += kWave) pos += (sig_tmp[i] > sj) || (sig_tmp[i] == sj && i < j);
        pos = (int)wave_sum((double)pos);
        const double inv = sj > 0.0 ? 1.0 / sj : 0.0;
        if (lane == 0) {
            sigma[pos] = sj;
            if (sorted) sorted[pos] = sj;
        }
        for (int i = lane; i < n; i += kWave) Vout[(long long)i * n + pos] = X[(long long)j * n + i] * inv;
    }
}

__device__ __forceinline__ double jacobi_eta(const double *delta, int z, int n) {
    return delta ? 0.01 * delta[z] * delta[z] / n : 0.0;
}

// One workgroup per matrix; X = R^T is a plain copy of the row-major R (column j = row j).
// With tr.ranks set, the truncation rank of each matrix is formed in the same launch from its
// sorted singular values, by the arithmetic of trunc_ranks (the tail sum of the smallest
// sigma^2 at most delta^2, at least 1, at most rcap).
__global__ __launch_bounds__(1024) void k_jacobi_lds(int n, const double *__restrict__ Rin, double *__restrict__ sigma,
                                                     double *__restrict__ Vout, const double *__restrict__ delta,
                                                     TruncArgs tr) {
    extern __shared__ double X[];
    __shared__ int nrot;
    __shared__ double sig_tmp[512], sorted[512];
    const int z = blockIdx.x, tid = threadIdx.x;
    const double *Rz = Rin + (long long)z * n * n;
    for (int e = tid; e < n * n; e += blockDim.x) X[e] = Rz[e];
    __syncthreads();
    jacobi_run(n, X, &nrot, sig_tmp, jacobi_eta(delta, z, n));
    jacobi_finish(n, X, sig_tmp, sigma + (long long)z * n, Vout + (long long)z * n * n, tr.ranks ? sorted : nullptr);
    if (!tr.ranks) return;
    __syncthreads();
    if (tid == 0) {
        double tot = 0.0;
        for (int j = 0; j < n; ++j) tot += sorted[j] * sorted[j];
        const double dl = tr.delta_abs ? tr.delta_abs[z] : tr.rel * sqrt(tot);
        const double d2 = dl * dl;
        double tail = 0.0;
        int r = n;
        while (r > 0 && tail + sorted[r - 1] * sorted[r - 1] <= d2) {
            tail += sorted[r - 1] * sorted[r - 1];
            --r;
        }
        if (r < 1) r = 1;
        if (r > tr.rcap) r = tr.rcap;
        tr.ranks[z] = r;
    }
}

__global__ __launch_bounds__(1024) void k_jacobi_global(int n, const double *__restrict__ Rin,
                                                        double *__restrict__ sigma, double *__restrict__ Vout,
                                                        double *__restrict__ scratch,
                                                        const double *__restrict__ delta) {
    __shared__ int nrot;
    const int z = blockIdx.x, tid = threadIdx.x;
    double *X = scratch + (long long)z * ((long long)n * n + n);
    double *sig_tmp = X + (long long)n * n;
    const double *Rz = Rin + (long long)z * n * n;
    for (long long e = tid; e < (long long)n * n; e += blockDim.x) X[e] = Rz[e];
    __syncthreads();
    jacobi_run(n, X, &nrot, sig_tmp, jacobi_eta(delta, z, n));
    jacobi_finish(n, X, sig_tmp, sigma + (long long)z * n, Vout + (long long)z * n * n);
}

// ------------------------------------------------------------------- prrLU (pivots)
// Multi-workgroup variant for blocks too large for one workgroup's registers: one launch per
// pivot step. Launch t (t >= 1) first decides pivot t - 1 from the partials the workgroups of
// launch t - 1 left (largest magnitude with ties to the lower linear index, its row, and the
// squared sum, per workgroup): every workgroup combines them in workgroup order, so all take
// the same decision without a fence or an atomic. Each then eliminates that pivot from its own
// rows (writing column t - 1 of L), and leaves its partials of the new residual, including the
// whole row of its largest entry (the next pivot row if it wins). Partials are double-buffered
// by step parity. Workspace (doubles): 2 x [max nblk | sum nblk | index nblk | rows nblk x n],
// then a control block.
// stop_launch is 0 until the launch that decides to stop writes its own index t (>= 1) there;
// launches after it return at once. A workgroup of that same launch may read 0 or t, and both
// let it go on and take the same stop decision itself.
struct PrrluCtl {
    double tol2;
    int stop_launch;
    int fail;  // set by a workgroup of the persistent form whose polls ran out
};

// Per parity c (0, 1): max | sum | index (nblk each, one double apiece) | rows (nblk x n).
// The parity copies are found by arithmetic on c, not by indexing arrays of pointers: a
// run-time index into such an array keeps it in scratch memory, reloaded at every step.
struct PrrluWs {
    double *base;       // parity 0
    long long pstride;  // doubles from parity 0 to parity 1
    int nblk;
    PrrluCtl *ctl;
    __host__ __device__ double *pmax(int c) const { return base + c * pstride; }
    __host__ __device__ double *psum(int c) const { return base + c * pstride + nblk; }
    __host__ __device__ long long *pidx(int c) const { return (long long *)(base + c * pstride + 2 * nblk); }
    __host__ __device__ double *prow(int c) const { return base + c * pstride + 3 * nblk; }
};

__host__ __device__ inline PrrluWs prrlu_ws_split(double *ws, int n, int nblk) {
    PrrluWs w;
    w.base = ws;
    w.pstride = 3LL * nblk + (long long)nblk * n;
    w.nblk = nblk;
    w.ctl = (PrrluCtl *)(ws + 2 * w.pstride);
    return w;
}

constexpr int kMwThreads = 256, kMwTW = 8, kMwK = 2, kMwKBig = 8, kMwBigMinBlk = 128;

// One workgroup per job. The persistent form's exchanged words (both parities) start with the
// tag of step -2, which no word of steps 0..5 carries.
__device__ __forceinline__ void prrlu_mw_init_body(const PrrluJob &J) {
    const PrrluWs w = prrlu_ws_split(J.ws, J.n, J.nblk);
    if (threadIdx.x == 0) {
        w.ctl->stop_launch = 0;
        w.ctl->tol2 = 0.0;
        w.ctl->fail = 0;
        J.info[0] = -1.0;  // not finished: the host launches further steps
    }
    if (J.mode == 2 || J.mode == 4) {  // the persistent forms
        long long *p = (long long *)J.ws;
        for (long long e = threadIdx.x; e < 2 * w.pstride; e += blockDim.x) p[e] = 3;
    }
}

// Workgroup b owns a stripe of J.rows = RS * K rows; thread (tr, tc) holds the kMwTW columns
// [8 tc, 8 tc + 8) of rows r0 + tr + k RS, k < K, with RS = 256 / ceil(n / 8); K = K, or
// KBig for tall blocks (more loads in flight per thread, fewer workgroups per step). The stripe is
// loaded before the decision (it does not depend on it); the candidate row a workgroup leaves
// for the next launch comes from the registers of the threads that hold it.
constexpr int kMwCand = 2048;  // doubles: the widest pivot row (n <= 256 * 8)

template <int K>
__device__ __forceinline__ void prrlu_mw_step_body(const PrrluJob &J, int t) {
    __shared__ double lc[kMwThreads * K];
    __shared__ double u[kMwCand];
    __shared__ double wmax[kMwThreads / kWave], wsum[kMwThreads / kWave];
    __shared__ long long widx[kMwThreads / kWave];
    __shared__ int s_stop, s_wk;
    __shared__ long long s_gi, s_bi;
    const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
    const int m = J.m, n = J.n, rmax = J.rmax;
    const PrrluWs w = prrlu_ws_split(J.ws, n, J.nblk);
    double *__restrict__ A = J.A;
    const int sl = w.ctl->stop_launch;
    if (sl != 0 && sl < t) return;
    const int tpr = (n + kMwTW - 1) / kMwTW, RS = kMwThreads / tpr;
    const int tr = tid / tpr, tc = tid % tpr, c0 = tc * kMwTW;
    const bool active = tr < RS;
    const int r0 = blockIdx.x * J.rows;
    const int cur = t & 1, prev = cur ^ 1;
    double a[K][kMwTW];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int row = r0 + tr + k * RS;
        const bool rv = active && row < m;
#pragma unroll
        for (int j = 0; j < kMwTW; ++j) a[k][j] = (rv && c0 + j < n) ? A[(long long)row * n + c0 + j] : 0.0;
    }
    int pi = -1, pj = -1;
    const double *urow = u;  // the pivot row
    if (t > 0) {
        // decide pivot t - 1 from the previous launch's partials (the same in every workgroup)
        double bm = -1.0, bs = 0.0;
        long long bi = 0x7fffffffffffffffLL;
        for (int b = tid; b < J.nblk; b += kMwThreads) {
            amax_merge(bm, bi, w.pmax(prev)[b], w.pidx(prev)[b]);
            bs += w.psum(prev)[b];
        }
        // the winning workgroup is the owner of the winning index's row stripe
        wave_amax_sum(bm, bi, bs);
        if (lane == 0) { wmax[wv] = bm; widx[wv] = bi; wsum[wv] = bs; }
        __syncthreads();
        if (tid == 0) {
            double gm = wmax[0], gs = 0.0;
            long long gi = widx[0];
            for (int k = 0; k < kMwThreads / kWave; ++k) {
                gs += wsum[k];
                amax_merge(gm, gi, wmax[k], widx[k]);
            }
            const int tp = t - 1;  // the pivot being decided
            const double tol2 = tp == 0 ? J.rel_tol2 * gs : w.ctl->tol2;
            int stop = (tp >= rmax) || (gm <= 0.0) || (gs <= tol2);
            if (tp == 0 && gm <= 0.0) stop = 2;  // all-zero block
            if (tp == 0 && stop == 1) stop = 0;  // always take at least one pivot of a nonzero block
            s_stop = stop;
            s_gi = gi;
            s_wk = gm > 0.0 ? (int)((gi / n) / J.rows) : 0;  // the workgroup whose stripe holds the row
            if (blockIdx.x == 0) {
                if (tp == 0) w.ctl->tol2 = tol2;
                if (stop) {
                    int rank = tp;
                    if (stop == 2) {
                        rank = 1;
                        J.rowpiv[0] = 0; J.colpiv[0] = 0;
                    }
                    J.info[0] = (double)rank;
                    J.info[1] = gs;
                    J.info[2] = tol2;
                    w.ctl->stop_launch = t;
                } else {
                    J.rowpiv[tp] = (int)(gi / n);
                    J.colpiv[tp] = (int)(gi % n);
                }
            }
        }
        __syncthreads();
        if (s_stop) {
            if (s_stop == 2)
                for (int row = r0 + tid; row < min(m, r0 + J.rows); row += kMwThreads)
                    J.L[(long long)row * rmax] = (row == 0) ? 1.0 : 0.0;
            return;
        }
        pi = (int)(s_gi / n);
        pj = (int)(s_gi % n);
        {
            const double *prow = w.prow(prev) + (long long)s_wk * n;
            for (int j = tid; j < n; j += kMwThreads) u[j] = prow[j];
        }
        if (active && pj >= c0 && pj < c0 + kMwTW) {  // the pivot column's owners publish it
#pragma unroll
            for (int j = 0; j < kMwTW; ++j)
                if (c0 + j == pj)
#pragma unroll
                    for (int k = 0; k < K; ++k) lc[tr + k * RS] = a[k][j];
        }
        __syncthreads();
        const double inv = 1.0 / urow[pj];
        if (active) {
            double uu[kMwTW];
#pragma unroll
            for (int j = 0; j < kMwTW; ++j) uu[j] = c0 + j < n ? urow[c0 + j] : 0.0;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int row = r0 + tr + k * RS;
                if (row >= m) continue;
                const double l = row == pi ? 1.0 : lc[tr + k * RS] * inv;
                if (tc == 0) J.L[(long long)row * rmax + (t - 1)] = l;
                if (row == pi) {
#pragma unroll
                    for (int j = 0; j < kMwTW; ++j) a[k][j] = 0.0;
                } else {
#pragma unroll
                    for (int j = 0; j < kMwTW; ++j) a[k][j] = fma(-l, uu[j], a[k][j]);
                }
            }
            if (pj >= c0 && pj < c0 + kMwTW) {
#pragma unroll
                for (int j = 0; j < kMwTW; ++j)
                    if (c0 + j == pj)
#pragma unroll
                        for (int k = 0; k < K; ++k) a[k][j] = 0.0;
            }
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int row = r0 + tr + k * RS;
                if (row >= m) continue;
#pragma unroll
                for (int j = 0; j < kMwTW; ++j)
                    if (c0 + j < n) A[(long long)row * n + c0 + j] = a[k][j];
            }
        }
    }
    double lmax = -1.0, lsum = 0.0;
    long long lidx = 0x7fffffffffffffffLL;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const long long rb = (long long)(r0 + tr + k * RS) * n + c0;
#pragma unroll
        for (int j = 0; j < kMwTW; ++j) {
            const double v = a[k][j], av = fabs(v);
            lsum = fma(v, v, lsum);
            const bool gt = av > lmax;
            lmax = gt ? av : lmax;
            lidx = gt ? rb + j : lidx;
        }
    }
    if (!active) { lmax = -1.0; lsum = 0.0; }
    wave_amax_sum(lmax, lidx, lsum);
    // wmax / widx / wsum were last read by thread 0 before the barriers above
    if (lane == 0) { wmax[wv] = lmax; widx[wv] = lidx; wsum[wv] = lsum; }
    __syncthreads();
    if (tid == 0) {
        double bm = wmax[0], bs = 0.0;
        long long bi = widx[0];
        for (int k = 0; k < kMwThreads / kWave; ++k) {
            bs += wsum[k];
            amax_merge(bm, bi, wmax[k], widx[k]);
        }
        w.pmax(cur)[blockIdx.x] = bm;
        w.psum(cur)[blockIdx.x] = bs;
        w.pidx(cur)[blockIdx.x] = bi;
        s_bi = bi;
    }
    __syncthreads();
    // the candidate pivot row: the whole row of this stripe's largest entry, from the registers
    // of the threads that hold it (a real row: ties go to the lowest index, and the stripe's
    // first entry is real)
    if (s_bi != 0x7fffffffffffffffLL && active) {
        const int local = (int)(s_bi / n) - r0;
        if (local % RS == tr) {
            double *dst = w.prow(cur) + (long long)blockIdx.x * n;
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (k == local / RS)
#pragma unroll
                    for (int j = 0; j < kMwTW; ++j)
                        if (c0 + j < n) dst[c0 + j] = a[k][j];
        }
    }
}

// Persistent form, for blocks of at most kCoopMaxBlk stripes: one launch for the whole
// factorisation, each stripe held in registers throughout (the same layout as above). It is
// launched only when the device holds all its workgroups at once (the grid is at most the
// occupancy times the compute units); a plain launch is used, since the cooperative launch API
// costs about 0.1 ms of host time per call. Workgroups are dispatched in order, so even a grid
// that other work keeps partly waiting makes progress as slots free up.
// Per pivot step t every workgroup publishes its partials (max, index, sum) and candidate row,
// double-buffered by step parity, as 64-bit words that carry the step in their two lowest bits
// (tag (t >> 1) & 3; a double gives up its last two mantissa bits, which every reader clears
// alike), written and read with relaxed device-scope atomics, which are coherent across the
// chip without the L2 write-back and invalidation of release/acquire fences. Every wave of every
// workgroup gathers all slots itself, lane b polling the three partials of slot b until they
// carry step t's tag, and reduces them in slot order, so all waves take the same decision with
// no barrier between workgroups; each thread then polls its columns of the winning row the same
// way, and only the pivot column of the stripe passes through LDS. A slot of one parity is
// rewritten every second step, so a word left from an earlier step differs by its tag for the
// next three rewrites (the slots start with the tag of step -2); the index is range-checked
// before use all the same. The polls are bounded: after J.spin polls (kCoopSpin unless the host
// set another bound) a workgroup marks the job failed (info[0] = -2) and leaves, and the others
// leave at their next poll.
constexpr int kCoopMaxBlk = 64;  // one slot per lane of a wave
constexpr int kCoopBigSlots = 256;  // the persistent form for large blocks: four slots per lane
constexpr int kCoopBigRows = 2048;  // its stripes' rows at most (the pivot-column buffer)
// the LDS buffer of the form that also holds rows in LDS: all of the 160 KB but the wave partials
constexpr int kCoopLdsDoubles = 20464;
constexpr int kCoopSpin = 1 << 22;
constexpr int kCoopGLChunk = 3;  // streamed rows loaded together
constexpr long long kNoRow = 0x7fffffffffffffffLL;

__device__ __forceinline__ int coop_tag(int t) { return (t >> 1) & 3; }
__device__ __forceinline__ long long coop_word_d(double v, int tg) { return (__double_as_longlong(v) & ~3LL) | tg; }
__device__ __forceinline__ double coop_val_d(long long b) { return __longlong_as_double(b & ~3LL); }
__device__ __forceinline__ long long coop_word_i(long long i, int tg) {
    return (i == kNoRow ? (kNoRow & ~3LL) : (i << 2)) | tg;
}
__device__ __forceinline__ long long coop_val_i(long long b) {
    return (b & ~3LL) == (kNoRow & ~3LL) ? kNoRow : (b >> 2);
}
__device__ __forceinline__ void coop_put(long long *p, long long b) {
    __hip_atomic_store(p, b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ long long coop_get(const long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Polls the NW words p[off[q]] until each carries tag tg (the loads of one round are issued
// together); false when the job has failed or the polls ran out (then the job is marked failed).
template <int NW>
__device__ __forceinline__ bool coop_poll(const long long *p, const int (&off)[NW], int tg, PrrluCtl *ctl, int spin,
                                          long long (&out)[NW]) {
    for (int sp = 0; sp < spin; ++sp) {
        bool all = true;
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            out[q] = coop_get(p + off[q]);
            all = all && (int)(out[q] & 3) == tg;
        }
        if (all) return true;
        if (__hip_atomic_load(&ctl->fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
        __builtin_amdgcn_s_sleep(1);
    }
    __hip_atomic_store(&ctl->fail, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return false;
}

// Partials (largest magnitude, its position, squared sum) of the entries one thread holds, in NC
// independent chains (column j goes to chain j mod NC); entries are added in increasing position
// k kMwTW + j, and strict comparisons keep the first (lowest-index) entry of a tie.
template <int NC>
struct CoopAcc {
    double pm[NC], ps[NC];
    int pq[NC];
    __device__ __forceinline__ void reset() {
#pragma unroll
        for (int c = 0; c < NC; ++c) { pm[c] = -1.0; ps[c] = 0.0; pq[c] = 0; }
    }
    __device__ __forceinline__ void add(int j, int k, double v) {
        const int c = j % NC;
        ps[c] = fma(v, v, ps[c]);
        const double av = fabs(v);
        const bool gt = av > pm[c];
        pm[c] = gt ? av : pm[c];
        pq[c] = gt ? k * kMwTW + j : pq[c];
    }
    // position as k kMwTW + j, in the order of the global index
    __device__ __forceinline__ void merge(double &mx, double &sm, int &pos) const {
        mx = pm[0]; sm = ps[0]; pos = pq[0];
#pragma unroll
        for (int c = 1; c < NC; ++c) {
            sm += ps[c];
            const bool take = pm[c] > mx || (pm[c] == mx && pq[c] < pos);
            mx = take ? pm[c] : mx;
            pos = take ? pq[c] : pos;
        }
    }
};

// NT threads per workgroup; NA = RS tpr of them are active (tpr = ceil(n / kMwTW)). Active thread
// (tr, tc) owns the columns tc + j tpr, j < kMwTW (so that the lanes of a wave touch consecutive
// words) of the stripe rows r0 + tr + k RS: rows k < K in registers,
// K <= k < K + kl (kl = J.kl) in LDS and, with GL, rows K + kl <= k < J.shape left in A itself and
// streamed through at every step. Up to 64 SPL workgroups (each polling lane gathers SPL slots).
// One LDS buffer of LB doubles holds the LDS rows (element (k, j) of thread tid at
// ld[((k - K) kMwTW + j) NA + tid]: consecutive threads, consecutive words) and after them the
// pivot column (J.rows doubles, element (tr, k) at lc[tr KT + k]).
// Each step's elimination forms the partials of the next step in the same pass, with no branch
// per row: the holders of the pivot column clear it when they publish it, those of the pivot row
// clear the row before the pass, and both stay zero in it (the pivot row's multiplier is
// published as 0, the pivot row's entry in the pivot column is taken as 0).
template <int NT, int K, bool GL, int SPL, int LB>
__device__ __forceinline__ void prrlu_coop_body_t(const PrrluJob &J) {
    __shared__ double lbuf[LB];
    __shared__ double wmax[NT / kWave], wsum[NT / kWave];
    __shared__ long long widx[NT / kWave];
    __shared__ int s_fail;
    const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
    const int m = J.m, n = J.n, rmax = J.rmax, G = J.nblk, blk = blockIdx.x;
    const PrrluWs w = prrlu_ws_split(J.ws, n, J.nblk);
    const int tpr = (n + kMwTW - 1) / kMwTW, RS = NT / tpr, NA = RS * tpr;
    const int tr = tid / tpr, tc = tid % tpr;  // column j of the thread: tc + j tpr
    const bool active = tr < RS;
    const int r0 = blk * J.rows;
    const int kl = J.kl;  // rows per thread in LDS
    const int KT = GL ? J.shape : K + kl;  // rows per thread
    double *__restrict__ A = J.A;
    double *const ldt = lbuf + tid;  // this thread's LDS rows: element (k, j) at ldt[(k kMwTW + j) NA]
    double *const lc = lbuf + kl * kMwTW * NA;
    CoopAcc<(K >= 14) ? 1 : 4> acc;  // as many chains as the registers allow
    acc.reset();
    double a[K][kMwTW];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int row = r0 + tr + k * RS;
        const bool rv = active && row < m;
#pragma unroll
        for (int j = 0; j < kMwTW; ++j) {
            a[k][j] = (rv && tc + j * tpr < n) ? A[(long long)row * n + tc + j * tpr] : 0.0;
            acc.add(j, k, a[k][j]);
        }
    }
    if (active) {
        for (int k = 0; k < kl; ++k) {
            const int row = r0 + tr + (K + k) * RS;
            const double *src = A + (long long)row * n + tc;
            double v[kMwTW];
#pragma unroll
            for (int j = 0; j < kMwTW; ++j) v[j] = (row < m && tc + j * tpr < n) ? src[j * tpr] : 0.0;
#pragma unroll
            for (int j = 0; j < kMwTW; ++j) {
                ldt[(k * kMwTW + j) * NA] = v[j];
                acc.add(j, K + k, v[j]);
            }
        }
        if (GL)
            for (int k = K + kl; k < KT; ++k) {
                const int row = r0 + tr + k * RS;
                if (row >= m) break;
                const double *src = A + (long long)row * n + tc;
                double v[kMwTW];
#pragma unroll
                for (int j = 0; j < kMwTW; ++j) v[j] = tc + j * tpr < n ? src[j * tpr] : 0.0;
#pragma unroll
                for (int j = 0; j < kMwTW; ++j) acc.add(j, k, v[j]);
            }
    }
    if (tid == 0) s_fail = 0;
    double tol2 = 0.0;  // every workgroup forms the same value from the same partials
    for (int t = 0;; ++t) {
        const int cur = t & 1;
        // partials of the residual after t pivots, and this stripe's candidate row
        double lmax, lsum;
        int lk;  // the thread's best entry as k * kMwTW + j (the global index is formed once)
        acc.merge(lmax, lsum, lk);
        long long lidx = (long long)(r0 + tr + (lk / kMwTW) * RS) * n + tc + (lk % kMwTW) * tpr;
        if (!active) { lmax = -1.0; lsum = 0.0; lidx = kNoRow; }
        wave_amax_sum(lmax, lidx, lsum);
        if (lane == 0) { wmax[wv] = lmax; widx[wv] = lidx; wsum[wv] = lsum; }
        __syncthreads();
        double bm = wmax[0], bs = 0.0;
        long long bi = widx[0];
        for (int k = 0; k < NT / kWave; ++k) {
            bs += wsum[k];
            amax_merge(bm, bi, wmax[k], widx[k]);
        }
        const int tg = coop_tag(t);
        long long *const pmx = (long long *)w.pmax(cur), *const psm = (long long *)w.psum(cur);
        long long *const pix = w.pidx(cur), *const prw = (long long *)w.prow(cur);
        if (tid == 0) {
            coop_put(pmx + blk, coop_word_d(bm, tg));
            coop_put(psm + blk, coop_word_d(bs, tg));
            coop_put(pix + blk, coop_word_i(bi, tg));
        }
        if (bi != kNoRow && active) {  // a real row: ties go to the lowest index
            const int local = (int)(bi / n) - r0;
            if (local % RS == tr) {
                long long *dst = prw + (long long)blk * n;
                const int kk = local / RS;
#pragma unroll
                for (int k = 0; k < K; ++k)
                    if (k == kk)
#pragma unroll
                        for (int j = 0; j < kMwTW; ++j)
                            if (tc + j * tpr < n) coop_put(dst + tc + j * tpr, coop_word_d(a[k][j], tg));
                if (kk >= K && kk < K + kl) {
#pragma unroll
                    for (int j = 0; j < kMwTW; ++j)
                        if (tc + j * tpr < n) coop_put(dst + tc + j * tpr, coop_word_d(ldt[((kk - K) * kMwTW + j) * NA], tg));
                } else if (GL && kk >= K + kl) {
                    const double *src = A + (long long)(r0 + local) * n;
#pragma unroll
                    for (int j = 0; j < kMwTW; ++j)
                        if (tc + j * tpr < n) coop_put(dst + tc + j * tpr, coop_word_d(src[tc + j * tpr], tg));
                }
            }
        }
        // every wave gathers every slot and decides pivot t on its own
        double gm = -1.0, gs = 0.0;
        long long gi = kNoRow;
        bool ok = true;
        long long got[3 * SPL];
        if (lane < G) {  // slots lane, lane + 64, ...; a slot past the grid polls slot lane again
            // (max, sum and index of a slot at offsets 0, G, 2G from pmx)
            int off[3 * SPL];
#pragma unroll
            for (int q = 0; q < SPL; ++q) {
                const int sl = lane + kWave * q < G ? lane + kWave * q : lane;
                off[3 * q] = sl;
                off[3 * q + 1] = G + sl;
                off[3 * q + 2] = 2 * G + sl;
            }
            ok = coop_poll<3 * SPL>(pmx, off, tg, w.ctl, J.spin, got);
        }
        bool wave_ok = __ballot(!ok) == 0;
        if (lane < G && wave_ok) {
#pragma unroll
            for (int q = 0; q < SPL; ++q)
                if (lane + kWave * q < G) {  // slots in workgroup order within the lane
                    gs += coop_val_d(got[3 * q + 1]);
                    amax_merge(gm, gi, coop_val_d(got[3 * q]), coop_val_i(got[3 * q + 2]));
                }
        }
        wave_amax_sum(gm, gi, gs);
        if (t == 0) tol2 = J.rel_tol2 * gs;
        int stop = (t >= rmax) || (gm <= 0.0) || (gs <= tol2);
        if (t == 0 && gm <= 0.0) stop = 2;  // all-zero block
        if (t == 0 && stop == 1) stop = 0;  // always take at least one pivot of a nonzero block
        if (!stop && !(gi >= 0 && gi < (long long)m * n)) wave_ok = false;  // not a pivot of this block
        const int pi = stop ? 0 : (int)(gi / n), pj = stop ? 0 : (int)(gi % n);
        const int wk = stop ? 0 : pi / J.rows;  // the workgroup whose stripe holds the pivot row
        double uu[kMwTW], upj = 1.0;
        if (!wave_ok) {
            if (lane == 0) s_fail = 1;
        } else {
            if (blk == 0 && tid == 0) {
                if (stop) {
                    int rank = t;
                    if (stop == 2) {
                        rank = 1;
                        J.rowpiv[0] = 0; J.colpiv[0] = 0;
                    }
                    J.info[0] = (double)rank;
                    J.info[1] = gs;
                    J.info[2] = tol2;
                } else {
                    J.rowpiv[t] = pi;
                    J.colpiv[t] = pj;
                }
            }
            if (!stop) {
                // the pivot entry and this thread's columns of the winning row, polled together
                // (a column past the block's end polls the pivot entry again)
                const long long *urow = prw + (long long)wk * n;
                int off[kMwTW + 1];
                off[0] = pj;
#pragma unroll
                for (int j = 0; j < kMwTW; ++j) off[1 + j] = (active && tc + j * tpr < n) ? tc + j * tpr : pj;
                long long v[kMwTW + 1];
                if (coop_poll<kMwTW + 1>(urow, off, tg, w.ctl, J.spin, v)) {
                    upj = coop_val_d(v[0]);
#pragma unroll
                    for (int j = 0; j < kMwTW; ++j)  // the pivot column is left out of the update
                        uu[j] = (active && tc + j * tpr < n && tc + j * tpr != pj) ? coop_val_d(v[1 + j]) : 0.0;
                } else {
                    s_fail = 1;
                }
                if (active && pj % tpr == tc) {
                    // the pivot column's owners publish it, with 0 in the pivot row (whose
                    // holders clear it and leave it out of the update), and clear it
                    const int jp = pj / tpr;
#pragma unroll
                    for (int j = 0; j < kMwTW; ++j)
                        if (j == jp) {
#pragma unroll
                            for (int k = 0; k < K; ++k) {
                                lc[tr * KT + k] = r0 + tr + k * RS == pi ? 0.0 : a[k][j];
                                a[k][j] = 0.0;
                            }
                        }
                    for (int k = 0; k < kl; ++k) {
                        const int e = (k * kMwTW + jp) * NA;
                        lc[tr * KT + K + k] = r0 + tr + (K + k) * RS == pi ? 0.0 : ldt[e];
                        ldt[e] = 0.0;
                    }
                    if (GL)  // the streamed rows' entries, four reads issued together
                        for (int k0 = K + kl; k0 < KT; k0 += 4) {
                            double v[4];
#pragma unroll
                            for (int h = 0; h < 4; ++h) {
                                const int row = r0 + tr + (k0 + h) * RS;
                                v[h] = k0 + h < KT && row < m ? A[(long long)row * n + pj] : 0.0;
                            }
                            asm volatile("" : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]));
#pragma unroll
                            for (int h = 0; h < 4; ++h) {
                                const int k = k0 + h, row = r0 + tr + k * RS;
                                if (k < KT) {
                                    lc[tr * KT + k] = row != pi ? v[h] : 0.0;
                                    if (row < m) A[(long long)row * n + pj] = 0.0;
                                }
                            }
                        }
                }
            }
        }
        __syncthreads();
        if (s_fail) {
            if (tid == 0) J.info[0] = -2.0;
            return;
        }
        if (stop) {  // every wave took the same decision
            if (stop == 2)
                for (int row = r0 + tid; row < min(m, r0 + J.rows); row += NT)
                    J.L[(long long)row * rmax] = (row == 0) ? 1.0 : 0.0;
            return;
        }
        const double inv = 1.0 / upj;
        acc.reset();
        if (active) {
            // where the pivot row sits for this workgroup (pk uniform)
            const int pl = pi - r0;
            const int pk = (pl >= 0 && pl < J.rows) ? pl / RS : -1;
            const bool rown = pk >= 0 && pl % RS == tr;
            const double *lcr = lc + tr * KT;  // this thread's rows of the pivot column
            // the pivot row's holders clear it (its multiplier in lc is 0, so it stays 0)
            if (pk >= 0 && pk < K) {
#pragma unroll
                for (int k = 0; k < K; ++k)
                    if (k == pk) {
                        if (rown)
#pragma unroll
                            for (int j = 0; j < kMwTW; ++j) a[k][j] = 0.0;
                    }
            } else if (pk >= K && pk < K + kl) {
                if (rown)
#pragma unroll
                    for (int j = 0; j < kMwTW; ++j) ldt[((pk - K) * kMwTW + j) * NA] = 0.0;
            } else if (GL && pk >= K + kl) {
                if (rown)
#pragma unroll
                    for (int j = 0; j < kMwTW; ++j)
                        if (tc + j * tpr < n) A[(long long)pi * n + tc + j * tpr] = 0.0;
            }
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const double l = lcr[k] * inv;
#pragma unroll
                for (int j = 0; j < kMwTW; ++j) {
                    a[k][j] = fma(-l, uu[j], a[k][j]);
                    acc.add(j, k, a[k][j]);
                }
            }
            for (int k = 0; k < kl; ++k) {
                const double l = lcr[K + k] * inv;
                double v[kMwTW];
#pragma unroll
                for (int j = 0; j < kMwTW; ++j) v[j] = ldt[(k * kMwTW + j) * NA];
                // all the row's reads are issued before the first is used
                static_assert(kMwTW == 8, "one asm operand per column");
                asm volatile("" : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]), "+v"(v[6]),
                             "+v"(v[7]));
#pragma unroll
                for (int j = 0; j < kMwTW; ++j) {
                    v[j] = fma(-l, uu[j], v[j]);
                    ldt[(k * kMwTW + j) * NA] = v[j];
                    acc.add(j, K + k, v[j]);
                }
            }
            if (GL)
                for (int k = K + kl; k < KT; ++k) {
                    const int row = r0 + tr + k * RS;
                    if (row >= m) break;
                    const double l = lcr[k] * inv;
                    double *dst = A + (long long)row * n + tc;
                    double v[kMwTW];
#pragma unroll
                    for (int j = 0; j < kMwTW; ++j) v[j] = tc + j * tpr < n ? dst[j * tpr] : 0.0;
                    asm volatile("" : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]), "+v"(v[6]),
                                 "+v"(v[7]));
#pragma unroll
                    for (int j = 0; j < kMwTW; ++j) {
                        v[j] = fma(-l, uu[j], v[j]);
                        if (tc + j * tpr < n) dst[j * tpr] = v[j];
                        acc.add(j, k, v[j]);
                    }
                }
        }
        // the multipliers (the pivot row's is 1), stripe row q = tr + k RS from lc[tr KT + k]
        for (int q = tid; q < J.rows; q += NT) {
            const int row = r0 + q;
            if (row < m) J.L[(long long)row * rmax + t] = row == pi ? 1.0 : lc[(q % RS) * KT + q / RS] * inv;
        }
        // lc and the wave partials are next written after the next step's first barrier, which
        // every wave reaches only when done with this step's values
    }
}

__device__ __forceinline__ void prrlu_coop_body(const PrrluJob &J) {
    prrlu_coop_body_t<kMwThreads, kMwK, false, 1, kMwThreads * kMwK>(J);
}

__global__ __launch_bounds__(kMwThreads) void k_prrlu_coop(PrrluJob J) { prrlu_coop_body(J); }

// The persistent form for large blocks: K rows per thread in registers (a block of 22528 x 240
// is 176 stripes of 128 rows at K = 16), with LB > kCoopBigRows J.kl more in LDS and with GL the
// rest streamed, up to 256 workgroups, one per CU.
template <int K, bool GL, int LB>
__global__ __launch_bounds__(kMwThreads) void k_prrlu_coop_big(PrrluJob J) {
    prrlu_coop_body_t<kMwThreads, K, GL, kCoopBigSlots / kWave, LB>(J);
}

__global__ __launch_bounds__(kMwThreads) void k_prrlu_coop_batch(const PrrluJob *__restrict__ jobs) {
    const PrrluJob J = jobs[blockIdx.y];
    if (J.mode != 2 || (int)blockIdx.x >= J.nblk) return;
    prrlu_coop_body(J);
}

__global__ void k_prrlu_mw_init(PrrluJob J) { prrlu_mw_init_body(J); }

template <int K>
__global__ __launch_bounds__(kMwThreads) void k_prrlu_mw_step(PrrluJob J, int t) { prrlu_mw_step_body<K>(J, t); }

__global__ void k_prrlu_mw_init_batch(const PrrluJob *__restrict__ jobs) {
    const PrrluJob J = jobs[blockIdx.x];
    if (J.mode >= 1) prrlu_mw_init_body(J);
}

// Steps the jobs of the modes in mode_mask (bit m: mode m) whose stripes hold K rows per thread.
template <int K>
__global__ __launch_bounds__(kMwThreads) void k_prrlu_mw_step_batch(const PrrluJob *__restrict__ jobs, int t,
                                                                     int mode_mask) {
    const PrrluJob J = jobs[blockIdx.y];
    if (!((mode_mask >> J.mode) & 1) || (int)blockIdx.x >= J.nblk) return;
    prrlu_mw_step_body<K>(J, t);
}

// Single-workgroup form: the whole block stays in registers for all pivot steps. Thread tid
// holds the TH x TW tile at rows [TH (tid / tn), +TH), columns [TW (tid % tn), +TW), with
// tn = ceil(n / TW); the launch needs ceil(m / TH) * tn <= 1024. Per pivot step only the pivot
// row and column pass through LDS. Two barriers per step: after the wave partials (every thread
// then reduces the 16 partials itself) and after the pivot row and column are published. The
// eliminated row and column are set to exact zeros.
template <int TH, int TW, int NT>
__device__ __forceinline__ void prrlu_tile_body(int m, int n, const double *__restrict__ A, int rmax,
                                                double rel_tol2, int *__restrict__ rowpiv, int *__restrict__ colpiv,
                                                double *__restrict__ L, double *__restrict__ info) {
    extern __shared__ double sm[];
    double *colv = sm, *rowv = sm + m;
    __shared__ double wmax[NT / kWave], wsum[NT / kWave];
    __shared__ int widx[NT / kWave];
    const int tid = threadIdx.x, lane = tid % kWave, w = tid / kWave, nw = NT / kWave;
    const int tn = (n + TW - 1) / TW, tm = (m + TH - 1) / TH;
    const bool active = tid < tm * tn;
    const int r0 = active ? (tid / tn) * TH : m, c0 = active ? (tid % tn) * TW : n;
    const int base = r0 * n + c0;
    double a[TH][TW];
#pragma unroll
    for (int i = 0; i < TH; ++i)
#pragma unroll
        for (int j = 0; j < TW; ++j) a[i][j] = (r0 + i < m && c0 + j < n) ? A[base + i * n + j] : 0.0;
    double tol2 = 0.0, bs = 0.0;
    int t = 0, stop = 0;
    for (;; ++t) {
        double lmax = -1.0, lsum = 0.0;
        int lidx = 0x7fffffff;
#pragma unroll
        for (int i = 0; i < TH; ++i) {
            const int rb = base + i * n;
#pragma unroll
            for (int j = 0; j < TW; ++j) {
                const double v = a[i][j], av = fabs(v);
                lsum = fma(v, v, lsum);
                const bool gt = av > lmax;
                lmax = gt ? av : lmax;
                lidx = gt ? rb + j : lidx;
            }
        }
        if (!active) lmax = -1.0;
        wave_amax_sum(lmax, lidx, lsum);
        if (lane == 0) { wmax[w] = lmax; widx[w] = lidx; wsum[w] = lsum; }
        __syncthreads();  // barrier A
        double bm = lane < nw ? wmax[lane] : -1.0;
        int bi = lane < nw ? widx[lane] : 0x7fffffff;
        bs = lane < nw ? wsum[lane] : 0.0;
        row0_amax_sum(bm, bi, bs);
        if (t == 0) tol2 = rel_tol2 * bs;
        stop = (t >= rmax) || (bm <= 0.0) || (bs <= tol2);
        if (t == 0 && bm <= 0.0) stop = 2;
        if (t == 0 && stop == 1) stop = 0;
        if (stop) break;
        const int pi = bi / n, pj = bi % n;
        const bool own_r = pi >= r0 && pi < r0 + TH, own_c = pj >= c0 && pj < c0 + TW;
        if (own_r) {  // owners publish the pivot row and column
#pragma unroll
            for (int i = 0; i < TH; ++i)
                if (r0 + i == pi)
#pragma unroll
                    for (int j = 0; j < TW; ++j)
                        if (c0 + j < n) rowv[c0 + j] = a[i][j];
        }
        if (own_c) {
#pragma unroll
            for (int j = 0; j < TW; ++j)
                if (c0 + j == pj)
#pragma unroll
                    for (int i = 0; i < TH; ++i)
                        if (r0 + i < m) colv[r0 + i] = a[i][j];
        }
        __syncthreads();  // barrier B
        const double inv = 1.0 / rowv[pj];
        if (tid == 0) { rowpiv[t] = pi; colpiv[t] = pj; }
        if (active) {
            double u[TW];
#pragma unroll
            for (int j = 0; j < TW; ++j) u[j] = c0 + j < n ? rowv[c0 + j] : 0.0;
#pragma unroll
            for (int i = 0; i < TH; ++i) {
                const double l = r0 + i < m ? colv[r0 + i] * inv : 0.0;
#pragma unroll
                for (int j = 0; j < TW; ++j) a[i][j] = fma(-l, u[j], a[i][j]);
            }
            if (own_r) {
#pragma unroll
                for (int i = 0; i < TH; ++i)
                    if (r0 + i == pi)
#pragma unroll
                        for (int j = 0; j < TW; ++j) a[i][j] = 0.0;
            }
            if (own_c) {
#pragma unroll
                for (int j = 0; j < TW; ++j)
                    if (c0 + j == pj)
#pragma unroll
                        for (int i = 0; i < TH; ++i) a[i][j] = 0.0;
            }
        }
        for (int i = tid; i < m; i += NT) L[(long long)i * rmax + t] = (i == pi) ? 1.0 : colv[i] * inv;
    }
    if (tid == 0) {
        int rank = t;
        if (stop == 2) {
            rank = 1;
            rowpiv[0] = 0; colpiv[0] = 0;
        }
        info[0] = (double)rank;
        info[1] = bs;
        info[2] = tol2;
    }
    if (stop == 2)
        for (int i = tid; i < m; i += NT) L[(long long)i * rmax] = (i == 0) ? 1.0 : 0.0;
}

template <int TH, int TW, int NT>
__global__ __launch_bounds__(NT) void k_prrlu_tile(int m, int n, const double *__restrict__ A, int rmax,
                                                   double rel_tol2, int *__restrict__ rowpiv,
                                                   int *__restrict__ colpiv, double *__restrict__ L,
                                                   double *__restrict__ info) {
    prrlu_tile_body<TH, TW, NT>(m, n, A, rmax, rel_tol2, rowpiv, colpiv, L, info);
}

// One workgroup per job of the given tile shape: the pivot searches of a batch of blocks.
template <int TH, int TW, int NT>
__global__ __launch_bounds__(NT) void k_prrlu_tile_batch(const PrrluJob *__restrict__ jobs, int shape) {
    const PrrluJob j = jobs[blockIdx.x];
    if (j.mode != 0 || j.shape != shape) return;
    prrlu_tile_body<TH, TW, NT>(j.m, j.n, j.A, j.rmax, j.rel_tol2, j.rowpiv, j.colpiv, j.L, j.info);
}

// Tile shapes of the single-workgroup form, smallest register footprint first: 1024 threads
// with up to 36 entries each, then 512 threads (twice the registers per thread) with up to 80.
struct TileShape {
    int th, tw, nt;
};
constexpr TileShape kTileShapes[] = {{1, 4, 1024}, {2, 4, 1024}, {1, 16, 1024}, {4, 4, 1024}, {2, 8, 1024},
                                     {8, 2, 1024}, {4, 8, 1024}, {8, 4, 1024},  {2, 16, 1024}, {4, 9, 1024},
                                     {8, 8, 512},  {8, 10, 512}};
constexpr int kNumTileShapes = sizeof(kTileShapes) / sizeof(kTileShapes[0]);

template <int TH, int TW, int NT>
void launch_tile(hipStream_t s, int nb, size_t lds, const PrrluJob *jobs, int shape, int m, int n, const double *A,
                 int rmax, double rel_tol2, int *rowpiv, int *colpiv, double *L, double *info) {
    if (jobs) k_prrlu_tile_batch<TH, TW, NT><<<nb, NT, lds, s>>>(jobs, shape);
    else k_prrlu_tile<TH, TW, NT><<<1, NT, lds, s>>>(m, n, A, rmax, rel_tol2, rowpiv, colpiv, L, info);
}

void dispatch_tile(hipStream_t s, int shape, int nb, size_t lds, const PrrluJob *jobs, int m, int n, const double *A,
                   int rmax, double rel_tol2, int *rowpiv, int *colpiv, double *L, double *info) {
#define WTT_TILE(ID, TH, TW, NT) \
    case ID: launch_tile<TH, TW, NT>(s, nb, lds, jobs, shape, m, n, A, rmax, rel_tol2, rowpiv, colpiv, L, info); break;
    switch (shape) {
        WTT_TILE(0, 1, 4, 1024) WTT_TILE(1, 2, 4, 1024) WTT_TILE(2, 1, 16, 1024) WTT_TILE(3, 4, 4, 1024)
        WTT_TILE(4, 2, 8, 1024) WTT_TILE(5, 8, 2, 1024) WTT_TILE(6, 4, 8, 1024) WTT_TILE(7, 8, 4, 1024)
        WTT_TILE(8, 2, 16, 1024) WTT_TILE(9, 4, 9, 1024) WTT_TILE(10, 8, 8, 512) WTT_TILE(11, 8, 10, 512)
        default: throw StatusError(WENOTT_EINVAL, "bad pivot tile shape");
    }
#undef WTT_TILE
}

// First tile shape whose tiles cover the m x n block within its thread count, or -1.
int tile_shape_for(int m, int n) {
    if (sizeof(double) * (size_t)(m + n) > 48 * 1024) return -1;
    for (int k = 0; k < kNumTileShapes; ++k) {
        const long long tiles = (long long)((m + kTileShapes[k].th - 1) / kTileShapes[k].th) *
                                ((n + kTileShapes[k].tw - 1) / kTileShapes[k].tw);
        if (tiles <= kTileShapes[k].nt) return k;
    }
    return -1;
}

// Row i of X solves x L_I = L[i, :r] with L_I = L[rowpiv, :r] unit lower triangular in pivot
// order (entry (s, t) is zero for t > s and one for t = s: the pivot rows were eliminated).
__global__ void k_interp(int m, int r, const double *__restrict__ L, int ldl, const int *__restrict__ rowpiv,
                         double *__restrict__ X) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    double *x = X + (long long)i * r;
    const double *l = L + (long long)i * ldl;
    for (int t = r - 1; t >= 0; --t) {
        double acc = l[t];
        for (int s = t + 1; s < r; ++s) acc -= x[s] * L[(long long)rowpiv[s] * ldl + t];
        x[t] = acc;
    }
}

// The same with L_I = L[rowpiv, :r] staged in LDS by every workgroup (LI[s * r + t]).
__global__ __launch_bounds__(256) void k_interp_lds(int m, int r, const double *__restrict__ L, int ldl,
                                                    const int *__restrict__ rowpiv, double *__restrict__ X) {
    extern __shared__ double LI[];
    for (int e = threadIdx.x; e < r * r; e += blockDim.x) {
        const int sr = e / r, t = e % r;
        LI[e] = L[(long long)rowpiv[sr] * ldl + t];
    }
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    double *x = X + (long long)i * r;
    const double *l = L + (long long)i * ldl;
    for (int t = r - 1; t >= 0; --t) {
        double acc = l[t];
        for (int sr = t + 1; sr < r; ++sr) acc -= x[sr] * LI[sr * r + t];
        x[t] = acc;
    }
}

// The same for r <= RMAX with the row held in registers: v starts as L[i, :r]; for s from r - 1
// down, v[s] is final and v[t] -= v[s] L_I[s][t] for t < s (the unrolled loops keep v in
// registers). A pivot row gets its exact unit row (x = e_s for row rowpiv[s]) in the same
// launch.
template <int RMAX>
__global__ __launch_bounds__(128) void k_interp_reg(int m, int r, const double *__restrict__ L, int ldl,
                                                    const int *__restrict__ rowpiv, double *__restrict__ X) {
    extern __shared__ double LI[];
    __shared__ int piv_of[128];  // pivot position of this workgroup's rows, -1 for none
    const int tid = threadIdx.x, i0 = blockIdx.x * 128;
    piv_of[tid] = -1;
    for (int e = tid; e < r * r; e += 128) LI[e] = L[(long long)rowpiv[e / r] * ldl + e % r];
    __syncthreads();
    for (int sp = tid; sp < r; sp += 128) {
        const int pr = rowpiv[sp] - i0;
        if (pr >= 0 && pr < 128) piv_of[pr] = sp;
    }
    __syncthreads();
    const int i = i0 + tid;
    if (i >= m) return;
    double *x = X + (long long)i * r;
    const int ps = piv_of[tid];
    if (ps >= 0) {
        for (int t = 0; t < r; ++t) x[t] = t == ps ? 1.0 : 0.0;
        return;
    }
    const double *l = L + (long long)i * ldl;
    double v[RMAX];
#pragma unroll
    for (int t = 0; t < RMAX; ++t) v[t] = t < r ? l[t] : 0.0;
#pragma unroll
    for (int sp = RMAX - 1; sp > 0; --sp) {
        if (sp < r) {
            const double *li = LI + sp * r;
#pragma unroll
            for (int t = 0; t < sp; ++t) v[t] = fma(-v[sp], li[t], v[t]);
        }
    }
#pragma unroll
    for (int t = 0; t < RMAX; ++t)
        if (t < r) x[t] = v[t];
}

__global__ void k_interp_exact_rows(int r, const int *__restrict__ rowpiv, double *__restrict__ X) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= r * r) return;
    int s = e / r, t = e % r;
    X[(long long)rowpiv[s] * r + t] = (s == t) ? 1.0 : 0.0;
}

// ---------------------------------------------------------------- CholeskyQR helper
// X = R^{-1} with G = R^T R (upper Cholesky factor) of a nearly orthonormal basis's Gram
// matrix, one workgroup per matrix. A column whose squared norm is below 1/2 is a padding
// zero column: it keeps a unit diagonal and no coupling, so it stays zero after U X.
__device__ __forceinline__ void chol_inv_body(int r, const double *__restrict__ G, double *__restrict__ X,
                                              double *__restrict__ R) {
    const int tid = threadIdx.x;
    __shared__ double diag;
    __shared__ int zero_col;
    for (int e = tid; e < r * r; e += blockDim.x) R[e] = 0.0;
    __syncthreads();
    for (int j = 0; j < r; ++j) {
        if (tid == 0) {
            double dd = G[(long long)j * r + j];
            for (int k = 0; k < j; ++k) dd -= R[(long long)k * r + j] * R[(long long)k * r + j];
            zero_col = !(dd > 0.5);
            diag = zero_col ? 1.0 : sqrt(dd);
            R[(long long)j * r + j] = diag;
        }
        __syncthreads();
        for (int i = j + 1 + tid; i < r; i += blockDim.x) {
            double v = 0.0;
            if (!zero_col) {
                v = G[(long long)j * r + i];
                for (int k = 0; k < j; ++k) v -= R[(long long)k * r + j] * R[(long long)k * r + i];
                v /= diag;
            }
            R[(long long)j * r + i] = v;
        }
        __syncthreads();
    }
    // inverse of the upper-triangular R, one column per thread (back substitution)
    for (int i = tid; i < r; i += blockDim.x) {
        for (int j = r - 1; j >= 0; --j) X[(long long)j * r + i] = 0.0;
        for (int j = i; j >= 0; --j) {
            double v = (j == i) ? 1.0 : 0.0;
            for (int k = j + 1; k <= i; ++k) v -= R[(long long)j * r + k] * X[(long long)k * r + i];
            X[(long long)j * r + i] = v / R[(long long)j * r + j];
        }
    }
}

// One workgroup of kCholWaves waves per matrix for r <= 63, everything in LDS (leading
// dimension r + 1): right-looking Cholesky with lane i of every wave owning column i, wave w
// updating the trailing rows k with k % kCholWaves == w; then R^{-1} by back substitution in the
// first wave, lane i forming column i; the loops go four rows at a time so that their LDS loads
// overlap. The same arithmetic as above (a column whose pivot is not above 0.5 is a zero padding
// column with a unit diagonal); the sums run in another order.
constexpr int kCholWaveMax = 63;  // 2 r (r + 1) doubles of LDS stay within 64 KB
constexpr int kCholWaves = 4;

// The factorisation and inverse from A (r x r in LDS, leading dimension r + 1, upper triangle
// read); Xs: LDS of the same size. Every thread of the workgroup calls it (the barriers). At step
// j every thread forms the entries R_jk = A_jk / R_jj it needs from the unscaled row j (the
// products a stored scaled row would hold), so one barrier per step suffices; the first wave
// then stores the scaled row j, which no later step of the factorisation reads.
__device__ __forceinline__ void chol_inv_lds(int r, double *A, double *Xs, double *__restrict__ X) {
    const int ld = r + 1, lane = threadIdx.x % kWave, w = threadIdx.x / kWave, W = blockDim.x / kWave;
    for (int j = 0; j < r; ++j) {
        const double dd = A[j * ld + j];
        const bool zc = !(dd > 0.5);
        const double rjj = zc ? 1.0 : sqrt(dd), inv = 1.0 / rjj;
        double rji = 0.0;
        if (lane > j && lane < r) {
            rji = zc ? 0.0 : A[j * ld + lane] * inv;
            int k = j + 1 + (w - (j + 1) % W + W) % W;  // the first row after j that is this wave's
            for (; k + 3 * W <= lane; k += 4 * W) {
                const double r0 = zc ? 0.0 : A[j * ld + k] * inv, r1 = zc ? 0.0 : A[j * ld + k + W] * inv,
                             r2 = zc ? 0.0 : A[j * ld + k + 2 * W] * inv, r3 = zc ? 0.0 : A[j * ld + k + 3 * W] * inv;
                const double a0 = A[k * ld + lane], a1 = A[(k + W) * ld + lane], a2 = A[(k + 2 * W) * ld + lane],
                             a3 = A[(k + 3 * W) * ld + lane];
                A[k * ld + lane] = fma(-r0, rji, a0);
                A[(k + W) * ld + lane] = fma(-r1, rji, a1);
                A[(k + 2 * W) * ld + lane] = fma(-r2, rji, a2);
                A[(k + 3 * W) * ld + lane] = fma(-r3, rji, a3);
            }
            for (; k <= lane; k += W) A[k * ld + lane] = fma(-(zc ? 0.0 : A[j * ld + k] * inv), rji, A[k * ld + lane]);
        }
        __syncthreads();
        if (w == 0) {
            if (lane > j && lane < r) A[j * ld + lane] = rji;
            if (lane == j) A[j * ld + j] = rjj;
        }
    }
    __syncthreads();
    if (w == 0 && lane < r) {
        const int i = lane;
        for (int j = i; j >= 0; --j) {
            double v0 = (j == i) ? 1.0 : 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;  // four chains
            int k = j + 1;
            for (; k + 3 <= i; k += 4) {
                v0 = fma(-A[j * ld + k], Xs[k * ld + i], v0);
                v1 = fma(-A[j * ld + k + 1], Xs[(k + 1) * ld + i], v1);
                v2 = fma(-A[j * ld + k + 2], Xs[(k + 2) * ld + i], v2);
                v3 = fma(-A[j * ld + k + 3], Xs[(k + 3) * ld + i], v3);
            }
            for (; k <= i; ++k) v0 = fma(-A[j * ld + k], Xs[k * ld + i], v0);
            Xs[j * ld + i] = ((v0 + v1) + (v2 + v3)) / A[j * ld + j];
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < r * r; e += blockDim.x) {
        const int j = e / r, i = e % r;
        X[e] = j <= i ? Xs[j * ld + i] : 0.0;
    }
}

__device__ __forceinline__ void chol_inv_wave_body(int r, const double *__restrict__ G, double *__restrict__ X) {
    extern __shared__ double cw[];
    const int ld = r + 1;
    double *A = cw, *Xs = cw + r * ld;
    for (int e = threadIdx.x; e < r * r; e += blockDim.x) A[(e / r) * ld + e % r] = G[e];
    __syncthreads();
    chol_inv_lds(r, A, Xs, X);
}

// The same factorisation and inverse in one wave's registers, for the fused kernel below (where
// the LDS form's barriers span all its waves): lane i holds column i of the upper triangle
// (a[k] = A_ki, k <= i; zero below); at step j lane j's a[j] is the pivot, lanes i > j scale
// their a[j] into R_ji and update their column with row j of R, R_jk read from lane k
// (readlane). Then R^{-1} in place by back substitution, rows in descending order, lane i
// forming column i from row j of R, read from the other lanes before a[j] is overwritten; the
// sums run in four chains. The loops are unrolled (static register indices); rows at or beyond
// r are skipped by uniform branches.
template <int RM>
__device__ __forceinline__ void chol_inv_reg(int r, double (&a)[RM]) {
    const int i = threadIdx.x % kWave;
#pragma unroll
    for (int j = 0; j < RM; ++j) {
        if (j < r) {
            const double dd = readlane_d(a[j], j);
            const bool zc = !(dd > 0.5);
            const double rjj = zc ? 1.0 : sqrt(dd), inv = 1.0 / rjj;
            const double rji = (i > j && !zc) ? a[j] * inv : 0.0;
            a[j] = i > j ? rji : (i == j ? rjj : a[j]);
#pragma unroll
            for (int k = j + 1; k < RM; ++k)
                if (k < r) a[k] = fma(-readlane_d(a[j], k), rji, a[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < RM; ++k)
        if (k > i) a[k] = 0.0;
#pragma unroll
    for (int j = RM - 1; j >= 0; --j) {
        if (j < r) {
            double v[4] = {i == j ? 1.0 : 0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int k = j + 1; k < RM; ++k)
                if (k < r) v[(k - j - 1) & 3] = fma(-readlane_d(a[j], k), a[k], v[(k - j - 1) & 3]);
            a[j] = ((v[0] + v[1]) + (v[2] + v[3])) / readlane_d(a[j], j);
        }
    }
}

// One CholeskyQR factor per workgroup for r <= kGramMaxR: the Gram matrix U^T U of the tall
// m x r matrix U (row-major) on the matrix cores, then the factorisation and inverse above on
// it (the Gram GEMM, its partial-sum reduction and the factorisation in one launch). Wave w
// takes the groups of four rows g = w, w + 8, ...; per group lane l loads U[4g + l / 16][l % 16]
// and U[4g + l / 16][16 + l % 16], which is at once the A operand (U^T) and the B operand (U) of
// v_mfma_f64_16x16x4f64, so three products per group give the blocks (0,0), (0,1) and (1,1) of
// G (one for r <= 16); the eight waves' partial blocks are summed in wave order through LDS,
// whose space then holds G for the register factorisation of the first wave.
constexpr int kGramMaxR = 32, kGramWaves = 8, kGramQ = 8;

// The first wave's factorisation and inverse of G (Gs: kGramMaxR x kGramMaxR, upper triangle),
// X = R^{-1} row-major r x r.
template <int RM>
__device__ __forceinline__ void gram_chol_finish(int r, const double *Gs, double *__restrict__ X) {
    const int lane = threadIdx.x % kWave;
    double a[RM];
#pragma unroll
    for (int k = 0; k < RM; ++k) a[k] = (k <= lane && lane < r) ? Gs[k * kGramMaxR + lane] : 0.0;
    chol_inv_reg<RM>(r, a);
#pragma unroll
    for (int j = 0; j < RM; ++j)
        if (j < r && lane < r) X[j * r + lane] = a[j];
}

__global__ __launch_bounds__(kGramWaves * 64) void k_gram_chol_inv(int m, int r, const double *__restrict__ Uall,
                                                                   long long sU, double *__restrict__ Xall,
                                                                   long long sX) {
    __shared__ double red[kGramWaves][3][4][kWave];  // then G (kGramMaxR x kGramMaxR)
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave, z = blockIdx.x;
    const int cl = lane % 16, rl = lane / 16;
    const double *U = Uall + (long long)z * sU;
    const bool two = r > 16;
    f64x4 d00 = {0.0, 0.0, 0.0, 0.0}, d01 = d00, d11 = d00;
    for (int gb = w; 4 * gb < m; gb += kGramWaves * kGramQ) {
        double u0[kGramQ], u1[kGramQ];
#pragma unroll
        for (int q = 0; q < kGramQ; ++q) {
            const int t = 4 * (gb + kGramWaves * q) + rl;
            u0[q] = (t < m && cl < r) ? U[(long long)t * r + cl] : 0.0;
            u1[q] = (two && t < m && 16 + cl < r) ? U[(long long)t * r + 16 + cl] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < kGramQ; ++q) {
            d00 = __builtin_amdgcn_mfma_f64_16x16x4f64(u0[q], u0[q], d00, 0, 0, 0);
            if (two) {
                d01 = __builtin_amdgcn_mfma_f64_16x16x4f64(u0[q], u1[q], d01, 0, 0, 0);
                d11 = __builtin_amdgcn_mfma_f64_16x16x4f64(u1[q], u1[q], d11, 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        red[w][0][v][lane] = d00[v];
        red[w][1][v][lane] = d01[v];
        red[w][2][v][lane] = d11[v];
    }
    __syncthreads();
    double g[2];  // this thread's entries of the summed blocks (e = tid, tid + 512)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int e = threadIdx.x + q * kGramWaves * kWave;
        g[q] = 0.0;
        if (e < 3 * 4 * kWave) {
            const int T = e / (4 * kWave), v = (e / kWave) % 4, l = e % kWave;
#pragma unroll
            for (int ww = 0; ww < kGramWaves; ++ww) g[q] += red[ww][T][v][l];
        }
    }
    __syncthreads();  // the partial blocks are consumed; their LDS takes G
    double *Gs = &red[0][0][0][0];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int e = threadIdx.x + q * kGramWaves * kWave;
        if (e < 3 * 4 * kWave) {
            const int T = e / (4 * kWave), v = (e / kWave) % 4, l = e % kWave;
            // accumulator v of lane l holds block entry (l / 16 + 4 v, l % 16)
            const int row = (T == 2 ? 16 : 0) + l / 16 + 4 * v, col = (T == 0 ? 0 : 16) + l % 16;
            Gs[row * kGramMaxR + col] = g[q];
        }
    }
    __syncthreads();
    if (w != 0) return;
    double *X = Xall + (long long)z * sX;
    if (r <= 8) gram_chol_finish<8>(r, Gs, X);  // the unrolled code sized to r
    else if (r <= 16) gram_chol_finish<16>(r, Gs, X);
    else if (r <= 24) gram_chol_finish<24>(r, Gs, X);
    else gram_chol_finish<kGramMaxR>(r, Gs, X);
}

// X = R^{-1} of the upper Cholesky factor of one r x r matrix G (row-major, upper triangle read)
// per workgroup of one wave, r <= RM <= 64, in registers (chol_inv_reg).
template <int RM>
__global__ __launch_bounds__(64) void k_chol_inv_reg(int r, const double *__restrict__ Gin, double *__restrict__ Xout) {
    const int lane = threadIdx.x;
    const long long off = (long long)blockIdx.x * r * r;
    double a[RM];
#pragma unroll
    for (int k = 0; k < RM; ++k) a[k] = (k <= lane && lane < r) ? Gin[off + (long long)k * r + lane] : 0.0;
    chol_inv_reg<RM>(r, a);
#pragma unroll
    for (int j = 0; j < RM; ++j)
        if (j < r && lane < r) Xout[off + (long long)j * r + lane] = a[j];
}

__global__ __launch_bounds__(kCholWaves * kWave) void k_chol_inv_wave(int r, const double *__restrict__ Gin, double *__restrict__ Xout) {
    const long long off = (long long)blockIdx.x * r * r;
    chol_inv_wave_body(r, Gin + off, Xout + off);
}

__global__ __launch_bounds__(kCholWaves * kWave) void k_chol_inv_wave_batch(const CholJob *__restrict__ jobs) {
    const CholJob j = jobs[blockIdx.x];
    if ((int)blockIdx.y >= j.batch) return;
    const long long off = (long long)blockIdx.y * j.r * j.r;
    chol_inv_wave_body(j.r, j.G + off, j.X + off);
}

__global__ __launch_bounds__(256) void k_chol_inv(int r, const double *__restrict__ Gin, double *__restrict__ Xout,
                                                  double *__restrict__ Rws) {
    const long long off = (long long)blockIdx.x * r * r;
    chol_inv_body(r, Gin + off, Xout + off, Rws + off);
}

// grid (jobs, components): job j holds ncomp matrices of size r_j x r_j
__global__ __launch_bounds__(256) void k_chol_inv_batch(const CholJob *__restrict__ jobs) {
    const CholJob j = jobs[blockIdx.x];
    if ((int)blockIdx.y >= j.batch) return;
    const long long off = (long long)blockIdx.y * j.r * j.r;
    chol_inv_body(j.r, j.G + off, j.X + off, j.R + off);
}

// grid (jobs, components): one-sided Jacobi of the n_j x n_j matrices of a batch of jobs in LDS
__global__ __launch_bounds__(1024) void k_jacobi_lds_batch(const SvdJob *__restrict__ jobs) {
    extern __shared__ double X[];
    __shared__ int nrot;
    __shared__ double sig_tmp[512];
    const SvdJob j = jobs[blockIdx.x];
    if ((int)blockIdx.y >= j.batch) return;
    const int n = j.n, z = blockIdx.y, tid = threadIdx.x;
    const double *Rz = j.A + (long long)z * n * n;
    for (int e = tid; e < n * n; e += blockDim.x) X[e] = Rz[e];
    __syncthreads();
    jacobi_run(n, X, &nrot, sig_tmp, jacobi_eta(j.delta, z, n));
    jacobi_finish(n, X, sig_tmp, j.sigma + (long long)z * n, j.V + (long long)z * n * n);
}

inline unsigned cdiv(long long a, long long b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

namespace {

// ------------------------------------------------------------------ GEMM autotuner
// Tile shapes (TBM x TBN) of k_gemm. The table maps a bucket of the problem (transposes and the
// binary orders of magnitude of M, N, K and the batch) to the shape chosen for it. A bucket seen
// for the first time is tuned on the live calls: each call launches the next candidate between
// two events; the timings are collected when the events have completed (no synchronisation),
// and after kTuneSamples timings of every candidate (one for buckets of at least 2^24 outputs,
// whose launches are long enough to time once) the fastest shape is kept.
// Shapes 0-3 run on the vector units and sum every output in the same order; shape 4 is the
// FP64 matrix-core form (64 x 64), whose results agree with them to rounding. Shapes 5-7 are the
// resident-operand matrix-core forms (A resident; B resident in groups of 64 or 32 columns),
// open to products without transposes or split-K whose K is at most 64 (and M at most 64 for
// shape 5); elsewhere they are not tuned, and a forced one runs as shape 4.
constexpr int kGemmShapes[][2] = {{64, 64}, {32, 64}, {64, 32}, {32, 32}, {64, 64}, {64, 64}, {64, 64}, {64, 64}};
constexpr int kNumGemmShapes = 8, kTuneSamples = 3, kTuneOnceLog2 = 24;
constexpr int kResidentMaxK = 64, kStripsPerWave = 8;

// The streamed operand of one batch entry is addressed by 32-bit byte offsets (B: K rows of ldb;
// A: M rows of lda), so it must span less than 2^31 bytes.
bool gemm_shape_fits(int shape, bool ta, bool tb, int M, int N, int K, int lda, int ldb, const GemmBatch &bt) {
    if (shape < 5) return true;
    if (ta || tb || bt.ktot > 0 || K < 1 || K > kResidentMaxK) return false;  // clamped indices need K >= 1
    if (shape == 5) return M <= 64 && 8LL * K * ldb + 8LL * N < (1LL << 31);
    return 8LL * M * lda + 8LL * K < (1LL << 31);
}

struct TuneEntry {
    int choice = -1;  // chosen shape, -1 while tuning
    int next = 0;     // next candidate to time
    int count[kNumGemmShapes] = {};
    float total[kNumGemmShapes] = {};
    struct Pending {
        int cand;
        hipEvent_t e0, e1;
    };
    std::vector<Pending> pending;
};

struct GemmTuner {
    std::mutex mu;
    std::map<std::array<int, 6>, TuneEntry> table;
    std::vector<hipEvent_t> free_events;
    int enabled = 1;
    hipEvent_t get_event() {
        if (!free_events.empty()) {
            hipEvent_t e = free_events.back();
            free_events.pop_back();
            return e;
        }
        hipEvent_t e;
        WTT_HIP(hipEventCreate(&e));
        return e;
    }
};

GemmTuner &tuner() {
    static GemmTuner *t = new GemmTuner();  // lives until the process ends (events may be in flight)
    return *t;
}

int log2_bucket(long long x) {
    int b = 0;
    while ((1LL << b) < x && b < 40) ++b;
    return b;
}

template <int MI>
void launch_gemm_ra(hipStream_t s, int M, int N, int K, double alpha, const double *A, int lda, const double *B,
                    int ldb, double beta, double *C, int ldc, const GemmBatch &bt) {
    const int nstrip = (N + 15) / 16;
    dim3 grid(cdiv(nstrip, 4 * kStripsPerWave), 1, bt.nb1 * bt.nb2), block(256);
    if (K <= 32) k_gemm_mfma_ra<MI, 8><<<grid, block, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, bt);
    else k_gemm_mfma_ra<MI, 16><<<grid, block, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, bt);
}

template <int NJ>
void launch_gemm_rb(hipStream_t s, int M, int N, int K, double alpha, const double *A, int lda, const double *B,
                    int ldb, double beta, double *C, int ldc, const GemmBatch &bt) {
    const int nstrip = (M + 15) / 16;
    dim3 grid(cdiv(nstrip, 4 * kStripsPerWave), cdiv(N, 16 * NJ), bt.nb1 * bt.nb2), block(256);
    if (K <= 32) k_gemm_mfma_rb<NJ, 8><<<grid, block, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, bt);
    else k_gemm_mfma_rb<NJ, 16><<<grid, block, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, bt);
}

template <bool TA, bool TB>
void launch_gemm_shape(int shape, hipStream_t s, int M, int N, int K, double alpha, const double *A, int lda,
                       const double *B, int ldb, double beta, double *C, int ldc, const GemmBatch &bt) {
    if (shape >= 5 && !gemm_shape_fits(shape, TA, TB, M, N, K, lda, ldb, bt)) shape = 4;
    if constexpr (!TA && !TB) {
        if (shape == 5) {
            if (M <= 16) launch_gemm_ra<1>(s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, bt);
            else if (M <= 32) launch_gemm_ra<2>(s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, bt);
            else if (M <= 48) launch_gemm_ra<3>(s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, bt);
            else launch_gemm_ra<4>(s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, bt);
            return;
        }
        if (shape == 6) return launch_gemm_rb<4>(s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, bt);
        if (shape == 7) return launch_gemm_rb<2>(s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, bt);
    }
    const int tbm = kGemmShapes[shape][0], tbn = kGemmShapes[shape][1];
    dim3 grid(cdiv(N, tbn), cdiv(M, tbm), bt.nb1 * bt.nb2), block(256);
    switch (shape) {
        case 0: k_gemm<TA, TB, 64, 64><<<grid, block, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, bt); break;
        case 1: k_gemm<TA, TB, 32, 64><<<grid, block, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, bt); break;
        case 2: k_gemm<TA, TB, 64, 32><<<grid, block, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, bt); break;
        case 3: k_gemm<TA, TB, 32, 32><<<grid, block, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, bt); break;
        default: k_gemm_mfma<TA, TB><<<grid, block, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, bt); break;
    }
}

void launch_gemm(int shape, hipStream_t s, bool ta, bool tb, int M, int N, int K, double alpha, const double *A,
                 int lda, const double *B, int ldb, double beta, double *C, int ldc, const GemmBatch &bt) {
    if (!ta && !tb) launch_gemm_shape<false, false>(shape, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, bt);
    else if (ta && !tb) launch_gemm_shape<true, false>(shape, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, bt);
    else if (!ta && tb) launch_gemm_shape<false, true>(shape, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, bt);
    else launch_gemm_shape<true, true>(shape, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, bt);
}

}  // namespace

void gemm_tune_release() {
    GemmTuner &t = tuner();
    std::lock_guard<std::mutex> lk(t.mu);
    for (auto &kv : t.table) {
        for (auto &p : kv.second.pending) {  // timings still in flight are dropped
            (void)hipEventSynchronize(p.e1);
            (void)hipEventDestroy(p.e0);
            (void)hipEventDestroy(p.e1);
        }
        kv.second.pending.clear();
    }
    for (hipEvent_t e : t.free_events) (void)hipEventDestroy(e);
    t.free_events.clear();
}

void gemm_tune_enable(int mode) {
    GemmTuner &t = tuner();
    std::lock_guard<std::mutex> lk(t.mu);
    t.enabled = mode;
}

int gemm_tune_table(int32_t *out, int max_entries) {
    GemmTuner &t = tuner();
    std::lock_guard<std::mutex> lk(t.mu);
    int n = 0;
    for (auto &kv : t.table) {
        if (out && n < max_entries) {
            for (int q = 0; q < 6; ++q) out[n * 7 + q] = kv.first[q];
            out[n * 7 + 6] = kv.second.choice;
        }
        ++n;
    }
    return n;
}

namespace {

void gemm_f64_tuned(hipStream_t s, bool ta, bool tb, int M, int N, int K, double alpha, const double *A, int lda,
                    const double *B, int ldb, double beta, double *C, int ldc, const GemmBatch &bt) {
    GemmTuner &t = tuner();
    int shape = 0;
    TuneEntry::Pending timed{-1, nullptr, nullptr};
    {
        std::lock_guard<std::mutex> lk(t.mu);
        if (t.enabled >= 2) {
            shape = std::min(t.enabled - 2, kNumGemmShapes - 1);  // one shape forced everywhere
        } else if (t.enabled) {
            const std::array<int, 6> key{(int)ta, (int)tb, log2_bucket(M), log2_bucket(N), log2_bucket(K),
                                         log2_bucket((long long)bt.nb1 * bt.nb2)};
            TuneEntry &e = t.table[key];
            if (e.choice >= 0) {
                shape = e.choice;
            } else {
                // collect the timings that have arrived
                for (size_t q = 0; q < e.pending.size();) {
                    auto &pd = e.pending[q];
                    if (hipEventQuery(pd.e1) == hipSuccess) {
                        float ms = 0.f;
                        if (hipEventElapsedTime(&ms, pd.e0, pd.e1) == hipSuccess) {
                            e.total[pd.cand] += ms;
                            e.count[pd.cand] += 1;
                        }
                        t.free_events.push_back(pd.e0);
                        t.free_events.push_back(pd.e1);
                        e.pending.erase(e.pending.begin() + q);
                    } else {
                        ++q;
                    }
                }
                const int need = key[2] + key[3] + key[5] >= kTuneOnceLog2 ? 1 : kTuneSamples;
                bool fits[kNumGemmShapes], done = true;
                for (int c = 0; c < kNumGemmShapes; ++c) {
                    fits[c] = gemm_shape_fits(c, ta, tb, M, N, K, lda, ldb, bt);
                    done = done && (!fits[c] || e.count[c] >= need);
                }
                if (done) {
                    int best = 0;
                    for (int c = 1; c < kNumGemmShapes; ++c)
                        if (fits[c] && e.total[c] / e.count[c] < e.total[best] / e.count[best]) best = c;
                    e.choice = best;
                    shape = best;
                } else {
                    while (!fits[e.next]) e.next = (e.next + 1) % kNumGemmShapes;  // shape 0 always fits
                    shape = e.next;
                    e.next = (e.next + 1) % kNumGemmShapes;
                    timed.cand = shape;
                    timed.e0 = t.get_event();
                    timed.e1 = t.get_event();
                }
            }
        }
    }
    if (timed.cand >= 0) WTT_HIP(hipEventRecord(timed.e0, s));
    launch_gemm(shape, s, ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, bt);
    WTT_HIP(hipGetLastError());
    if (timed.cand >= 0) {
        WTT_HIP(hipEventRecord(timed.e1, s));
        std::lock_guard<std::mutex> lk(t.mu);
        const std::array<int, 6> key{(int)ta, (int)tb, log2_bucket(M), log2_bucket(N), log2_bucket(K),
                                     log2_bucket((long long)bt.nb1 * bt.nb2)};
        t.table[key].pending.push_back(timed);
    }
}

}  // namespace

void gemm_f64(hipStream_t s, bool ta, bool tb, int M, int N, int K, double alpha, const double *A, int lda,
              const double *B, int ldb, double beta, double *C, int ldc, const GemmBatch &bt) {
    if (M <= 0 || N <= 0) return;
    gemm_f64_tuned(s, ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, bt);
}

// Row blocks of the TSQR: a leaf holds bm rows (all of them when they fit in LDS), a tree node
// stacks `group` R factors.
struct TsqrPlan {
    int bm, nblk, group;
    bool leaf_lds;
};

int lds_limit_bytes();

size_t tsqr_lds_bytes(int rows, int n) { return sizeof(double) * (size_t)(rows + 1) * n; }

TsqrPlan tsqr_plan(int m, int n) {
    const long long budget = (long long)lds_limit_bytes() - 2048;  // static LDS of k_hhqr stays below 2 KB
    const long long fit = budget / (8LL * n) - 1;                 // rows with the padded leading dimension
    TsqrPlan p;
    const int want = leaf_rows(n);  // max(256, 2n) rows: two leaves of 256 beat one of 512
    if (m <= want && m <= fit) p.bm = m;
    else p.bm = want;
    p.nblk = (m + p.bm - 1) / p.bm;
    p.leaf_lds = (long long)tsqr_lds_bytes(p.bm, n) <= budget;
    p.group = (int)std::max<long long>(2, std::min<long long>(std::max<long long>(fit, p.bm), 2048) / n);
    return p;
}

size_t tsqr_scratch_doubles(int m, int n, int batch) {
    // the global-memory Householder work area is reused by every level: size it for the largest
    const TsqrPlan p = tsqr_plan(m, n);
    long long w = (long long)p.nblk * p.bm * n;
    const long long r = (long long)p.nblk * n * n;
    for (long long nb = p.nblk; nb > 1;) {
        const long long nb2 = (nb + p.group - 1) / p.group;
        w = std::max(w, nb2 * p.group * (long long)n * n);
        nb = nb2;
    }
    return (size_t)batch * (size_t)(w + 2 * r);
}

int lds_limit_bytes() {
    static int lim = -1;
    if (lim < 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            v = 65536;
        lim = v;
    }
    return lim;
}

template <bool LEAF>
void launch_hhqr(hipStream_t s, int nblk, int batch, bool lds, int m, int n, int bm, const double *A, long long sz,
                 long long rs, long long cs, double *Rout, double *W) {
    const size_t lb = lds ? tsqr_lds_bytes(bm, n) : 0;
    const dim3 grid(nblk, batch);
    if (bm <= 4 * kWave) k_hhqr<4, 1024, LEAF><<<grid, 1024, lb, s>>>(m, n, bm, nblk, A, sz, rs, cs, Rout, W, lds);
    else if (bm <= 8 * kWave) k_hhqr<8, 1024, LEAF><<<grid, 1024, lb, s>>>(m, n, bm, nblk, A, sz, rs, cs, Rout, W, lds);
    else if (bm <= 16 * kWave) k_hhqr<16, 1024, LEAF><<<grid, 1024, lb, s>>>(m, n, bm, nblk, A, sz, rs, cs, Rout, W, lds);
    else if (bm <= 32 * kWave) k_hhqr<32, 512, LEAF><<<grid, 512, lb, s>>>(m, n, bm, nblk, A, sz, rs, cs, Rout, W, lds);
    else throw StatusError(WENOTT_EINVAL, "TSQR row block too tall");
    WTT_HIP(hipGetLastError());
}

// 1024 threads (64 columns) hold up to 16 rows per lane without spilling; 512 threads (32
// columns, twice the registers per lane) hold 32.
constexpr int kQrRegCols = 64;
inline int qr_reg_rows(int n) { return n <= 32 ? 512 : 256; }

void launch_qr_reg(hipStream_t s, int nblk, int batch, int m, int n, int bm, const double *A, long long sz,
                   long long rs, long long cs, double *Rout) {
    const int rows = std::max(bm, n);
    const dim3 grid(nblk, batch);
    WTT_REQUIRE(n <= kQrRegCols && rows <= qr_reg_rows(n), WENOTT_EINVAL, "register QR block too large");
    if (rows <= 64) k_qr_reg<4, 1024><<<grid, 1024, 0, s>>>(m, n, bm, nblk, A, sz, rs, cs, Rout);
    else if (rows <= 128) k_qr_reg<8, 1024><<<grid, 1024, 0, s>>>(m, n, bm, nblk, A, sz, rs, cs, Rout);
    else if (rows <= 256) k_qr_reg<16, 1024><<<grid, 1024, 0, s>>>(m, n, bm, nblk, A, sz, rs, cs, Rout);
    else k_qr_reg<32, 512><<<grid, 512, 0, s>>>(m, n, bm, nblk, A, sz, rs, cs, Rout);
    WTT_HIP(hipGetLastError());
}

void tsqr_r(hipStream_t s, int m, int n, int batch, const double *A, long long sz, long long rs, long long cs,
            double *R, double *scratch) {
    if (n <= kQrRegCols) {
        // register-resident leaves of up to qr_reg_rows(n) rows, then nodes of as many stacked
        // rows; the two R buffers fit in what tsqr_scratch_doubles reserves for the general
        // plan's R buffers (whose leaves are never taller)
        const int maxrows = qr_reg_rows(n);
        int nblk = (m + maxrows - 1) / maxrows;
        const int bm = std::min(m, maxrows);
        double *cur = scratch, *nxt = scratch + (long long)batch * nblk * n * n;
        launch_qr_reg(s, nblk, batch, m, n, bm, A, sz, rs, cs, nblk == 1 ? R : cur);
        const int group = std::max(2, maxrows / n);
        while (nblk > 1) {
            const int nb2 = (nblk + group - 1) / group;
            const int bm2 = std::min(group, nblk) * n;
            launch_qr_reg(s, nb2, batch, nblk * n, n, bm2, cur, (long long)nblk * n * n, n, 1, nb2 == 1 ? R : nxt);
            std::swap(cur, nxt);
            nblk = nb2;
        }
        return;
    }
    const TsqrPlan p = tsqr_plan(m, n);
    int nblk = p.nblk;
    double *W = scratch;
    long long wsize = (long long)nblk * p.bm * n;
    for (long long nb = nblk; nb > 1;) {
        const long long nb2 = (nb + p.group - 1) / p.group;
        wsize = std::max(wsize, nb2 * p.group * (long long)n * n);
        nb = nb2;
    }
    double *R0 = W + (long long)batch * wsize;
    double *R1 = R0 + (long long)batch * nblk * n * n;
    const size_t lds_budget = (size_t)lds_limit_bytes() - 2048;
    launch_hhqr<true>(s, nblk, batch, p.leaf_lds, m, n, p.bm, A, sz, rs, cs, nblk == 1 ? R : R0, W);
    double *cur = R0, *nxt = R1;
    while (nblk > 1) {
        const int mm = nblk * n;  // stacked R factors
        const int nb2 = (nblk + p.group - 1) / p.group;
        const int bm2 = std::min(p.group, nblk) * n;  // rows of a node
        const bool lds2 = tsqr_lds_bytes(bm2, n) <= lds_budget;
        double *out = nb2 == 1 ? R : nxt;
        launch_hhqr<false>(s, nb2, batch, lds2, mm, n, bm2, cur, (long long)nblk * n * n, n, 1, out, W);
        std::swap(cur, nxt);
        nblk = nb2;
    }
}

// Threads of a Jacobi workgroup: for n <= 128 as few waves as give every column pair of a round
// its own 8-lane segment (fewer waves at each round's barrier), else 1024.
int jacobi_threads(int n) {
    if (n > 128) return 1024;
    const int waves = std::max(1, ((n + 1) / 2 + 7) / 8);
    return 64 * waves;
}

bool jacobi_svd(hipStream_t s, int n, int batch, const double *R, double *sigma, double *V, double *scratch,
                const double *delta, const TruncArgs *tr) {
    // static LDS of the kernel: the column-norm and sorted buffers (2 x 512 doubles), a counter
    const size_t lds = sizeof(double) * (size_t)n * n;
    if (n <= 512 && lds + 2 * 512 * sizeof(double) + 64 <= (size_t)lds_limit_bytes()) {
        k_jacobi_lds<<<batch, jacobi_threads(n), lds, s>>>(n, R, sigma, V, delta, tr ? *tr : TruncArgs{});
        WTT_HIP(hipGetLastError());
        return tr != nullptr;
    }
    k_jacobi_global<<<batch, 1024, 0, s>>>(n, R, sigma, V, scratch, delta);
    WTT_HIP(hipGetLastError());
    return false;
}

size_t jacobi_scratch_doubles(int n, int batch) { return (size_t)batch * ((size_t)n * n + n); }

// Workgroups of the persistent pivot kernel that the device holds at once (0: unknown, and the
// persistent form is not used).
int coop_capacity() {
    static int cap = -1;
    if (cap < 0) {
        int dev = 0, ncu = 0, nb = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_prrlu_coop_batch, kMwThreads, 0) != hipSuccess)
            cap = 0;
        else
            cap = nb * ncu;
    }
    return cap;
}

// mode 0: one workgroup, register tiles; 1: multi-workgroup stripes of kMwK rows per thread,
// one launch per step; 2: as 1, small enough for the persistent single launch (stepped as 1
// when the device cannot hold the grid); 3: stripes of kMwKBig rows per thread, one launch per
// step, for blocks tall enough to fill the device with them (measured on 20480 x 180: 23 us per
// step against 25; on 4096 x 180 the longer stripes leave too few workgroups: 17 against 10).
namespace {
int g_coop_spin = kCoopSpin;
}

void set_coop_spin(int polls) { g_coop_spin = polls > 0 ? polls : (polls == 0 ? 0 : kCoopSpin); }

// Workgroups of the large persistent form with K register rows and KL LDS rows per thread that
// the device holds at once.
template <int K, bool GL, int LB>
int coop_big_capacity() {
    static int cap = -1;
    if (cap < 0) {
        int dev = 0, ncu = 0, nb = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_prrlu_coop_big<K, GL, LB>, kMwThreads, 0) != hipSuccess)
            cap = 0;
        else
            cap = nb * ncu;
    }
    return cap;
}

// mode 4 (allow_big): a block whose kMwK-row stripes would need more workgroups than the small
// persistent form takes is split into stripes of 8 or 16 rows per thread held in registers, the
// first whose grid fits kCoopBigSlots and the device at once, or else over as many workgroups as
// the device holds at once into stripes of more rows per thread: 16 in registers, as many more as
// fit in LDS, the rest streamed from the block; all factorised in one persistent launch (shape:
// rows per thread, kl: rows per thread in LDS).
void prrlu_prepare(PrrluJob &j, bool allow_big) {
    j.spin = g_coop_spin;
    j.kl = 0;
    j.shape = tile_shape_for(j.m, j.n);
    const int tpr = (j.n + kMwTW - 1) / kMwTW;
    WTT_REQUIRE(tpr <= kMwThreads && j.n <= kMwCand, WENOTT_EINVAL,
                "pivot block wider than the multi-workgroup form supports");
    j.rows = (kMwThreads / tpr) * kMwK;
    j.nblk = (j.m + j.rows - 1) / j.rows;
    if (j.shape >= 0) {
        j.mode = 0;
        return;
    }
    if (j.nblk <= kCoopMaxBlk) {
        j.mode = 2;
        return;
    }
    if (allow_big) {
        // more than 16 rows per thread in registers would spill to scratch memory
        const int ks[2] = {8, 16};
        const int caps[2] = {coop_big_capacity<8, false, kCoopBigRows>(), coop_big_capacity<16, false, kCoopBigRows>()};
        const int RS = kMwThreads / tpr, NA = RS * tpr;
        for (int q = 0; q < 2; ++q) {
            const int rows = RS * ks[q];
            const int nblk = (j.m + rows - 1) / rows;
            if (rows <= kCoopBigRows && nblk <= kCoopBigSlots && nblk <= caps[q]) {
                j.mode = 4;
                j.shape = ks[q];
                j.rows = rows;
                j.nblk = nblk;
                return;
            }
        }
        const int gmax = std::min(kCoopBigSlots, std::min(coop_big_capacity<16, false, kCoopLdsDoubles>(),
                                                          coop_big_capacity<16, true, kCoopLdsDoubles>()));
        if (gmax > 0) {
            const int per = (j.m + gmax - 1) / gmax;           // rows per workgroup
            const int kt = std::max(17, (per + RS - 1) / RS);  // rows per thread
            const int rows = RS * kt;
            const int kl = std::min(kt - 16, (kCoopLdsDoubles - rows) / (kMwTW * NA));
            if (rows <= kCoopBigRows && kl >= 0) {
                j.mode = 4;
                j.shape = kt;
                j.kl = kl;
                j.rows = rows;
                j.nblk = (j.m + rows - 1) / rows;
                return;
            }
        }
    }
    if (j.nblk < 4 * kMwBigMinBlk) {
        j.mode = 1;
    } else {  // tall enough that the longer stripes still give kMwBigMinBlk workgroups or more
        j.mode = 3;
        j.rows = (kMwThreads / tpr) * kMwKBig;
        j.nblk = (j.m + j.rows - 1) / j.rows;
    }
}

void prrlu_layout(int m, int n, bool allow_big, int *out) {
    PrrluJob j{};
    j.m = m; j.n = n;
    prrlu_prepare(j, allow_big);
    out[0] = j.mode;
    out[1] = j.shape;
    out[2] = j.rows;
    out[3] = j.nblk;
    out[4] = j.mode == 2 ? coop_capacity()
                         : (j.mode == 4 ? (j.shape == 8    ? coop_big_capacity<8, false, kCoopBigRows>()
                                           : j.shape == 16 ? coop_big_capacity<16, false, kCoopBigRows>()
                                           : j.shape == 16 + j.kl ? coop_big_capacity<16, false, kCoopLdsDoubles>()
                                                                  : coop_big_capacity<16, true, kCoopLdsDoubles>())
                                        : 0);
    out[5] = j.kl;
    out[6] = j.mode == 4 && j.shape > 16 ? j.shape - 16 - j.kl : 0;
}

// Enough for every layout prrlu may take for this block (the persistent one and its stepped
// fallback).
size_t prrlu_ws_doubles(int m, int n) {
    size_t best = 0;
    for (int big = 0; big < 2; ++big) {
        PrrluJob j{};
        j.m = m; j.n = n;
        prrlu_prepare(j, big != 0);
        best = std::max(best, 2 * (3 * (size_t)j.nblk + (size_t)j.nblk * n) + sizeof(PrrluCtl) / sizeof(double) + 1);
    }
    return best;
}

int prrlu(hipStream_t s, int m, int n, double *A, int rmax, double rel_tol2, int *rowpiv, int *colpiv, double *L,
          double *info, double *ws, int t_begin, int t_end, bool allow_persistent) {
    PrrluJob j{};
    j.A = A; j.m = m; j.n = n; j.rmax = rmax; j.rel_tol2 = rel_tol2;
    j.rowpiv = rowpiv; j.colpiv = colpiv; j.L = L; j.info = info; j.ws = ws;
    WTT_REQUIRE(rmax >= 1 && m >= 1 && n >= 1, WENOTT_EINVAL, "pivot search needs a nonempty block and rmax >= 1");
    prrlu_prepare(j, allow_persistent);
    if (j.mode == 4) {  // large blocks: the whole factorisation in one launch, stripes in registers
        if (t_begin > 0) return rmax + 2;
        k_prrlu_mw_init<<<1, kMwThreads, 0, s>>>(j);
        if (j.shape == 8) k_prrlu_coop_big<8, false, kCoopBigRows><<<j.nblk, kMwThreads, 0, s>>>(j);
        else if (j.shape == 16) k_prrlu_coop_big<16, false, kCoopBigRows><<<j.nblk, kMwThreads, 0, s>>>(j);
        else if (j.shape == 16 + j.kl) k_prrlu_coop_big<16, false, kCoopLdsDoubles><<<j.nblk, kMwThreads, 0, s>>>(j);
        else k_prrlu_coop_big<16, true, kCoopLdsDoubles><<<j.nblk, kMwThreads, 0, s>>>(j);
        WTT_HIP(hipGetLastError());
        return rmax + 2;
    }
    if (j.mode == 0) {
        if (t_begin > 0) return rmax + 1;
        dispatch_tile(s, j.shape, 1, sizeof(double) * (size_t)(m + n), nullptr, m, n, A, rmax, rel_tol2, rowpiv,
                      colpiv, L, info);
        WTT_HIP(hipGetLastError());
        return rmax + 1;
    }
    if (j.mode == 2 && allow_persistent && j.nblk <= coop_capacity()) {  // the whole factorisation in one launch
        if (t_begin > 0) return rmax + 2;
        k_prrlu_mw_init<<<1, kMwThreads, 0, s>>>(j);
        k_prrlu_coop<<<j.nblk, kMwThreads, 0, s>>>(j);
        WTT_HIP(hipGetLastError());
        return rmax + 2;
    }
    // launch t decides pivot t - 1, so the last possible decision (stop at rmax) is launch rmax + 1
    if (t_begin == 0) k_prrlu_mw_init<<<1, kMwThreads, 0, s>>>(j);
    const int last = std::min(t_end, rmax + 1);
    for (int t = t_begin; t <= last; ++t) {
        if (j.mode == 3) k_prrlu_mw_step<kMwKBig><<<j.nblk, kMwThreads, 0, s>>>(j, t);
        else k_prrlu_mw_step<kMwK><<<j.nblk, kMwThreads, 0, s>>>(j, t);
    }
    WTT_HIP(hipGetLastError());
    return last + 1;
}

void interp_solve(hipStream_t s, int m, int r, const double *L, int ldl, const int *rowpiv, double *X) {
    const size_t lds = sizeof(double) * (size_t)r * r;
    if (r > 0 && r <= 64) {  // registers; the exact pivot rows in the same launch
        if (r <= 16) k_interp_reg<16><<<cdiv(m, 128), 128, lds, s>>>(m, r, L, ldl, rowpiv, X);
        else if (r <= 32) k_interp_reg<32><<<cdiv(m, 128), 128, lds, s>>>(m, r, L, ldl, rowpiv, X);
        else k_interp_reg<64><<<cdiv(m, 128), 128, lds, s>>>(m, r, L, ldl, rowpiv, X);
        WTT_HIP(hipGetLastError());
        return;
    }
    if (r > 0 && lds <= (size_t)lds_limit_bytes() - 1024)
        k_interp_lds<<<cdiv(m, 256), 256, lds, s>>>(m, r, L, ldl, rowpiv, X);
    else
        k_interp<<<cdiv(m, 256), 256, 0, s>>>(m, r, L, ldl, rowpiv, X);
    k_interp_exact_rows<<<cdiv((long long)r * r, 256), 256, 0, s>>>(r, rowpiv, X);
    WTT_HIP(hipGetLastError());
}

bool gram_chol_inv(hipStream_t s, int m, int r, int batch, const double *U, long long sU, double *X) {
    // one workgroup forms each Gram matrix: only while that is a few tens of microseconds of one
    // CU's matrix-core rate (m r^2 <= 4e6); taller bases take the split-K GEMM over the device
    if (r < 1 || r > kGramMaxR || (double)m * r * r > 4e6) return false;
    k_gram_chol_inv<<<batch, kGramWaves * kWave, 0, s>>>(m, r, U, sU, X, (long long)r * r);
    WTT_HIP(hipGetLastError());
    return true;
}

void chol_upper_inv(hipStream_t s, int r, int batch, const double *G, double *X, double *ws) {
    // one wave with column i of the factor in lane i's registers up to 32 columns (the unrolled
    // code of wider forms outgrows the instruction cache: 147 us at r = 57 against 106 us in LDS)
    if (r <= 32) {
        if (r <= 16) k_chol_inv_reg<16><<<batch, kWave, 0, s>>>(r, G, X);
        else k_chol_inv_reg<32><<<batch, kWave, 0, s>>>(r, G, X);
    } else if (r <= kCholWaveMax)
        k_chol_inv_wave<<<batch, kCholWaves * kWave, sizeof(double) * 2 * (size_t)r * (r + 1), s>>>(r, G, X);
    else
        k_chol_inv<<<batch, 256, 0, s>>>(r, G, X, ws);
    WTT_HIP(hipGetLastError());
}

// Rows of K per split-K chunk: a multiple of 64 such that the chunks of the batch number about
// 512 (a few per CU) rather than K / 64 each, whose partial sums would cost more to add than
// the products.
int splitk_chunk(int K, int batch) {
    const long long want = ((long long)K * batch + 511) / 512;
    return (int)std::max(64LL, (want + 63) / 64 * 64);
}

void gemm_tn_splitk(hipStream_t s, int M, int N, int K, const double *A, int lda, const double *B, int ldb, double *C,
                    int ldc, int batch, long long sA, long long sB, long long sC, double *part, size_t part_cap) {
    const int chunk = splitk_chunk(K, batch);
    const int nchunk = (K + chunk - 1) / chunk;
    const long long per = (long long)M * N;
    if (nchunk <= 1 || (size_t)per * nchunk * batch > part_cap) {
        GemmBatch bt;
        bt.nb1 = batch; bt.sA1 = sA; bt.sB1 = sB; bt.sC1 = sC;
        gemm_f64(s, true, false, M, N, K, 1.0, A, lda, B, ldb, 0.0, C, ldc, bt);
        return;
    }
    GemmBatch bt;
    bt.nb1 = batch; bt.nb2 = nchunk;
    bt.sA1 = sA; bt.sA2 = (long long)chunk * lda;
    bt.sB1 = sB; bt.sB2 = (long long)chunk * ldb;
    bt.sC1 = per * nchunk; bt.sC2 = per;
    bt.ktot = K;
    gemm_f64(s, true, false, M, N, chunk, 1.0, A, lda, B, ldb, 0.0, part, N, bt);
    k_sum_chunks<<<cdiv(per * batch, 256), 256, 0, s>>>(per, nchunk, batch, part, C, M, N, ldc, sC);
    WTT_HIP(hipGetLastError());
}

size_t gemm_tn_splitk_part(int M, int N, int K, int batch) {
    const int chunk = splitk_chunk(K, batch);
    return (size_t)M * N * ((K + chunk - 1) / chunk) * batch;
}

void prrlu_batch(hipStream_t s, int njobs, const PrrluJob *host_jobs, const PrrluJob *dev_jobs, int t_begin,
                 int t_end) {
    if (njobs <= 0) return;
    int maxblk = 0, nmw = 0, maxcoop = 0, ncoop = 0, maxbig = 0, nbig = 0;
    int lds_shape[kNumTileShapes] = {};  // LDS bytes per tile shape in use (0: unused)
    for (int i = 0; i < njobs; ++i) {
        const PrrluJob &j = host_jobs[i];
        if (j.mode == 0) {
            lds_shape[j.shape] = std::max(lds_shape[j.shape], (int)(sizeof(double) * (size_t)(j.m + j.n)));
        } else if (j.mode == 3) {
            maxbig = std::max(maxbig, j.nblk);
            ++nbig;
            ++nmw;
        } else {
            maxblk = std::max(maxblk, j.nblk);
            ++nmw;
            if (j.mode == 2) {
                maxcoop = std::max(maxcoop, j.nblk);
                ++ncoop;
            }
        }
    }
    // the persistent launch finishes its jobs (or marks them failed) at the first chunk; jobs
    // still open at later chunks are stepped one launch per step
    const bool coop = t_begin == 0 && ncoop > 0 && (long long)maxcoop * njobs <= coop_capacity();
    if (t_begin == 0)
        for (int k = 0; k < kNumTileShapes; ++k)
            if (lds_shape[k] > 0)
                dispatch_tile(s, k, njobs, (size_t)lds_shape[k], dev_jobs, 0, 0, nullptr, 0, 0.0, nullptr, nullptr,
                              nullptr, nullptr);
    if (nmw) {
        if (t_begin == 0) k_prrlu_mw_init_batch<<<njobs, kMwThreads, 0, s>>>(dev_jobs);
        if (coop) k_prrlu_coop_batch<<<dim3(maxcoop, njobs), kMwThreads, 0, s>>>(dev_jobs);
        const bool small = maxblk > 0 && (!coop || nmw - nbig > ncoop);  // mode 1, or mode 2 stepped
        for (int t = t_begin; t <= t_end; ++t) {
            if (small)
                k_prrlu_mw_step_batch<kMwK><<<dim3(maxblk, njobs), kMwThreads, 0, s>>>(dev_jobs, t, coop ? 2 : 6);
            if (nbig) k_prrlu_mw_step_batch<kMwKBig><<<dim3(maxbig, njobs), kMwThreads, 0, s>>>(dev_jobs, t, 8);
        }
    }
    WTT_HIP(hipGetLastError());
}

bool jacobi_batch_fits(int nmax) {
    const size_t lds = sizeof(double) * (size_t)nmax * nmax;
    return nmax <= 512 && lds + 512 * sizeof(double) + 64 <= (size_t)lds_limit_bytes();
}

void jacobi_svd_batch(hipStream_t s, int njobs, int ncomp, int nmax, const SvdJob *dev_jobs) {
    if (njobs <= 0) return;
    const size_t lds = sizeof(double) * (size_t)nmax * nmax;
    k_jacobi_lds_batch<<<dim3(njobs, ncomp), jacobi_threads(nmax), lds, s>>>(dev_jobs);
    WTT_HIP(hipGetLastError());
}

void chol_upper_inv_batch(hipStream_t s, int njobs, int ncomp, int rmax, const CholJob *dev_jobs) {
    if (njobs <= 0) return;
    if (rmax <= kCholWaveMax)
        k_chol_inv_wave_batch<<<dim3(njobs, ncomp), kCholWaves * kWave, sizeof(double) * 2 * (size_t)rmax * (rmax + 1), s>>>(
            dev_jobs);
    else
        k_chol_inv_batch<<<dim3(njobs, ncomp), 256, 0, s>>>(dev_jobs);
    WTT_HIP(hipGetLastError());
}

}  // namespace wtt
