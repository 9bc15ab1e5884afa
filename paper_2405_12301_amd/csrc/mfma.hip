// FP32 contractions on the CDNA matrix cores for the reduced-precision fiber path.
//
// C = A B (row-major, FP32, batched) with v_mfma_f32_16x16x4f32: a 256-thread workgroup
// computes a 64 x 64 tile, each wave a 32 x 32 quarter as 2 x 2 MFMA 16 x 16 tiles; A and B
// tiles of depth 16 are staged through LDS. Operand layout of the 16x16x4 instruction: lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16]; the four accumulator registers of lane l
// hold D[4 (l / 16) + v][l % 16], v = 0..3.
#include "common.h"

namespace wtt {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int TM = 64, TN = 64, TK = 16;

__global__ __launch_bounds__(256) void k_gemm_f32_mfma(int M, int N, int K, const float *__restrict__ A, int lda,
                                                       const float *__restrict__ B, int ldb, float *__restrict__ C,
                                                       int ldc, GemmBatch bt) {
    const int z = blockIdx.z, z1 = z / bt.nb2, z2 = z % bt.nb2;
    A += z1 * bt.sA1 + z2 * bt.sA2;
    B += z1 * bt.sB1 + z2 * bt.sB2;
    C += z1 * bt.sC1 + z2 * bt.sC2;
    __shared__ float As[TK][TM + 4];
    __shared__ float Bs[TK][TN + 4];
    const int t = threadIdx.x, lane = t % 64, w = t / 64;
    const int wr = w / 2, wc = w % 2;
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += TK) {
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            const int e = t + 256 * l;
            int r = e / TK, kk = e % TK;
            int gm = m0 + r, gk = k0 + kk;
            As[kk][r] = (gm < M && gk < K) ? A[(long long)gm * lda + gk] : 0.f;
            kk = e / TN;
            const int c = e % TN;
            const int gn = n0 + c;
            gk = k0 + kk;
            Bs[kk][c] = (gn < N && gk < K) ? B[(long long)gk * ldb + gn] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < TK; ks += 4) {
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const float a = As[ks + lane / 16][wr * 32 + i * 16 + lane % 16];
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const float b = Bs[ks + lane / 16][wc * 32 + j * 16 + lane % 16];
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[i][j], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gm = m0 + wr * 32 + i * 16 + 4 * (lane / 16) + v;
                const int gn = n0 + wc * 32 + j * 16 + lane % 16;
                if (gm < M && gn < N) C[(long long)gm * ldc + gn] = acc[i][j][v];
            }
}

__global__ void k_to_f32(long long n, const double *__restrict__ x, float *__restrict__ y) {
    long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i < n) y[i] = (float)x[i];
}

inline unsigned cdiv(long long a, long long b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

void gemm_f32(hipStream_t s, int M, int N, int K, const float *A, int lda, const float *B, int ldb, float *C, int ldc,
              const GemmBatch &bt) {
    if (M <= 0 || N <= 0) return;
    dim3 grid(cdiv(N, TN), cdiv(M, TM), bt.nb1 * bt.nb2);
    k_gemm_f32_mfma<<<grid, 256, 0, s>>>(M, N, K, A, lda, B, ldb, C, ldc, bt);
    WTT_HIP(hipGetLastError());
}

void to_f32(hipStream_t s, long long n, const double *x, float *y) {
    if (n <= 0) return;
    k_to_f32<<<cdiv(n, 256), 256, 0, s>>>(n, x, y);
    WTT_HIP(hipGetLastError());
}

}  // namespace wtt
