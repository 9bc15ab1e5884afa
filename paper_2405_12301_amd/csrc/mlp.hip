// Learned cross proposal (not part of the paper's method): a 3-layer MLP
// IN -> HID -> HID -> OUT with ReLU, trained on the pivot logs of the plain cross.
// Parameters (FP32, one flat array): W1[IN][HID], b1[HID], W2[HID][HID], b2[HID],
// W3[HID][OUT], b3[OUT]. Outputs: RANK logits of the rank change, then BINS logits of where
// the next right index set should sample. Loss: cross-entropy of the rank class plus
// cross-entropy of the bin distribution against the target histogram, averaged over the batch.
// Training kernels run in FP32; inference can use BF16 weights and activations with FP32
// accumulation on the matrix cores.
#include <cmath>
#include <cstdint>
#include <functional>

#include "common.h"

namespace wtt {
namespace {

constexpr int IN = WENOTT_MLP_IN, HID = WENOTT_MLP_HID, OUT = WENOTT_MLP_OUT;
constexpr int NR = WENOTT_MLP_RANK_CLASSES, NB = WENOTT_MLP_BINS;
constexpr long long OFF_W1 = 0, OFF_B1 = OFF_W1 + (long long)IN * HID, OFF_W2 = OFF_B1 + HID,
                    OFF_B2 = OFF_W2 + (long long)HID * HID, OFF_W3 = OFF_B2 + HID,
                    OFF_B3 = OFF_W3 + (long long)HID * OUT, NPARAM = OFF_B3 + OUT;

__device__ inline float bf16_round(float x) {
    // round to nearest even on the upper 16 bits of the FP32 encoding
    unsigned u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return x;  // inf / nan unchanged
    u += 0x7fffu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xffff0000u);
}

// out[b][o] = act(sum_i in[b][i] W[i][o] + bias[o]); bf16: operands rounded to BF16, FP32 sums
__global__ void k_dense(int B, int nin, int nout, const float *__restrict__ in, const float *__restrict__ W,
                        const float *__restrict__ bias, float *__restrict__ out, int relu, int bf16) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= B * nout) return;
    const int b = e / nout, o = e % nout;
    float acc = 0.f;
    for (int i = 0; i < nin; ++i) {
        float a = in[b * nin + i], w = W[i * nout + o];
        if (bf16) { a = bf16_round(a); w = bf16_round(w); }
        acc = fmaf(a, w, acc);
    }
    acc += bf16 ? bf16_round(bias[o]) : bias[o];
    out[e] = relu ? fmaxf(acc, 0.f) : acc;
}

// The BF16 encoding of x rounded to nearest even (the upper 16 bits of bf16_round(x)).
__device__ inline short bf16_bits(float x) { return (short)(__float_as_uint(bf16_round(x)) >> 16); }

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// The BF16 form of k_dense on the matrix cores: one wave per 16 x 16 tile of out (16 samples x
// 16 outputs), v_mfma_f32_16x16x16bf16_1k over K in steps of 16. Operand layout of the
// instruction: lane l supplies A[l % 16][4 (l / 16) + j] and B[4 (l / 16) + j][l % 16], j < 4,
// and holds D[4 (l / 16) + v][l % 16], v < 4. The products of BF16 operands are exact in FP32,
// so the result differs from k_dense's BF16 form only by the order of the FP32 sums.
__global__ __launch_bounds__(64) void k_dense_bf16_mfma(int B, int nin, int nout, const float *__restrict__ in,
                                                        const float *__restrict__ W, const float *__restrict__ bias,
                                                        float *__restrict__ out, int relu) {
    const int l = threadIdx.x, o0 = blockIdx.x * 16, b0 = blockIdx.y * 16;
    const int r = l % 16, kg = 4 * (l / 16);
    const int b = b0 + r, o = o0 + r;  // this lane's row of A and column of B
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < nin; k0 += 16) {
        bf16x4 av, bv;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = k0 + kg + j;
            av[j] = (b < B && k < nin) ? bf16_bits(in[(long long)b * nin + k]) : (short)0;
            bv[j] = (o < nout && k < nin) ? bf16_bits(W[(long long)k * nout + o]) : (short)0;
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int bo = b0 + kg + v;
        if (bo < B && o < nout) {
            const float y = acc[v] + bf16_round(bias[o]);
            out[(long long)bo * nout + o] = relu ? fmaxf(y, 0.f) : y;
        }
    }
}

// dy = (softmax - target) / B for both heads; per-sample loss into lossb[b]
__global__ void k_head(int B, const float *__restrict__ y, const int *__restrict__ cls, const float *__restrict__ hist,
                       float *__restrict__ dy, float *__restrict__ lossb) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const float *yb = y + b * OUT;
    float *d = dy + b * OUT;
    float m = -1e30f, s = 0.f;
    for (int j = 0; j < NR; ++j) m = fmaxf(m, yb[j]);
    for (int j = 0; j < NR; ++j) s += expf(yb[j] - m);
    const float lse_r = m + logf(s);
    const int cb = min(max(cls[b], 0), NR - 1);
    float loss = lse_r - yb[cb];
    for (int j = 0; j < NR; ++j) d[j] = (expf(yb[j] - lse_r) - (j == cb ? 1.f : 0.f)) / B;
    m = -1e30f; s = 0.f;
    for (int j = 0; j < NB; ++j) m = fmaxf(m, yb[NR + j]);
    for (int j = 0; j < NB; ++j) s += expf(yb[NR + j] - m);
    const float lse_h = m + logf(s);
    float tsum = 0.f;
    for (int j = 0; j < NB; ++j) tsum += hist[b * NB + j];
    for (int j = 0; j < NB; ++j) {
        const float t = hist[b * NB + j];
        loss += t * (lse_h - yb[NR + j]);
        d[NR + j] = (tsum * expf(yb[NR + j] - lse_h) - t) / B;
    }
    lossb[b] = loss / B;
}

// dW[i][o] = sum_b A[b][i] dZ[b][o]
__global__ void k_wgrad(int B, int nin, int nout, const float *__restrict__ A, const float *__restrict__ dZ,
                        float *__restrict__ dW) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nin * nout) return;
    const int i = e / nout, o = e % nout;
    float acc = 0.f;
    for (int b = 0; b < B; ++b) acc = fmaf(A[b * nin + i], dZ[b * nout + o], acc);
    dW[e] = acc;
}

__global__ void k_bgrad(int B, int nout, const float *__restrict__ dZ, float *__restrict__ db) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= nout) return;
    float acc = 0.f;
    for (int b = 0; b < B; ++b) acc += dZ[b * nout + o];
    db[o] = acc;
}

// dH[b][i] = (sum_o dZ[b][o] W[i][o]) * [H[b][i] > 0]
__global__ void k_back(int B, int nin, int nout, const float *__restrict__ dZ, const float *__restrict__ W,
                       const float *__restrict__ H, float *__restrict__ dH) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= B * nin) return;
    const int b = e / nin, i = e % nin;
    float acc = 0.f;
    for (int o = 0; o < nout; ++o) acc = fmaf(dZ[b * nout + o], W[i * nout + o], acc);
    dH[e] = H[e] > 0.f ? acc : 0.f;
}

__global__ void k_sum(int n, const float *__restrict__ x, float *__restrict__ out) {
    __shared__ float red[256];
    float s = 0.f;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += x[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

__global__ void k_adam(long long n, float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, float lr, float b1, float b2, float c1, float c2, float eps) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// He-normal initialisation from a counter-based generator (splitmix64 + Box-Muller).
__device__ inline unsigned long long mix64(unsigned long long z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
__global__ void k_init(float *__restrict__ p, unsigned long long seed) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= NPARAM) return;
    int fan_in;
    if (i < OFF_B1) fan_in = IN;
    else if (i < OFF_W2) { p[i] = 0.f; return; }
    else if (i < OFF_B2) fan_in = HID;
    else if (i < OFF_W3) { p[i] = 0.f; return; }
    else if (i < OFF_B3) fan_in = HID;
    else { p[i] = 0.f; return; }
    const unsigned long long a = mix64(seed + 0x9E3779B97F4A7C15ULL * (2 * (unsigned long long)i + 1));
    const unsigned long long b = mix64(seed + 0x9E3779B97F4A7C15ULL * (2 * (unsigned long long)i + 2));
    const float u1 = ((a >> 40) + 1.0f) / 16777217.0f, u2 = (b >> 40) / 16777216.0f;
    const float z = sqrtf(-2.f * logf(u1)) * cosf(6.28318530718f * u2);
    p[i] = z * sqrtf(2.f / fan_in);
}

inline unsigned cdiv(long long a, long long b) { return (unsigned)((a + b - 1) / b); }

struct Acts {  // activations of one batch (device, FP32)
    float *h1, *h2, *y;
};

// bf16: BF16 operands with FP32 sums on the matrix cores; else FP32 on the vector units
void forward(hipStream_t s, const float *P, const float *x, int B, Acts a, int bf16) {
    if (bf16) {
        const int bt = (B + 15) / 16;
        k_dense_bf16_mfma<<<dim3((HID + 15) / 16, bt), 64, 0, s>>>(B, IN, HID, x, P + OFF_W1, P + OFF_B1, a.h1, 1);
        k_dense_bf16_mfma<<<dim3((HID + 15) / 16, bt), 64, 0, s>>>(B, HID, HID, a.h1, P + OFF_W2, P + OFF_B2, a.h2, 1);
        k_dense_bf16_mfma<<<dim3((OUT + 15) / 16, bt), 64, 0, s>>>(B, HID, OUT, a.h2, P + OFF_W3, P + OFF_B3, a.y, 0);
    } else {
        k_dense<<<cdiv((long long)B * HID, 256), 256, 0, s>>>(B, IN, HID, x, P + OFF_W1, P + OFF_B1, a.h1, 1, 0);
        k_dense<<<cdiv((long long)B * HID, 256), 256, 0, s>>>(B, HID, HID, a.h1, P + OFF_W2, P + OFF_B2, a.h2, 1, 0);
        k_dense<<<cdiv((long long)B * OUT, 256), 256, 0, s>>>(B, HID, OUT, a.h2, P + OFF_W3, P + OFF_B3, a.y, 0, 0);
    }
    WTT_HIP(hipGetLastError());
}

}  // namespace
}  // namespace wtt

using namespace wtt;

namespace {
wenott_status mlp_guard(const std::function<void()> &f) {
    try {
        f();
        return WENOTT_OK;
    } catch (const StatusError &e) {
        return e.status;
    } catch (const HipError &e) {
        return e.code == hipErrorOutOfMemory ? WENOTT_ENOMEM : WENOTT_EHIP;
    } catch (...) {
        return WENOTT_EINVAL;
    }
}
}  // namespace

extern "C" {

int64_t wenott_mlp_nparams(void) { return NPARAM; }

int64_t wenott_mlp_workspace(int32_t batch) {
    // h1, h2, y, dy, dh2, dh1, per-sample loss
    return (int64_t)batch * (2 * HID + 2 * OUT + 2 * HID + 1);
}

wenott_status wenott_mlp_init_params(float *params, uint64_t seed, void *stream) {
    if (!params) return WENOTT_EINVAL;
    return mlp_guard([&] {
        k_init<<<cdiv(NPARAM, 256), 256, 0, (hipStream_t)stream>>>(params, seed);
        WTT_HIP(hipGetLastError());
    });
}

wenott_status wenott_mlp_forward(const float *params, const float *x, int32_t batch, float *y, int32_t bf16,
                                 float *work, void *stream) {
    if (!params || !x || !y || !work || batch <= 0) return WENOTT_EINVAL;
    return mlp_guard([&] {
        Acts a{work, work + (long long)batch * HID, y};
        forward((hipStream_t)stream, params, x, batch, a, bf16 ? 1 : 0);
    });
}

wenott_status wenott_mlp_loss_grad(const float *params, const float *x, const int32_t *rank_class, const float *hist,
                                   int32_t batch, float *grad, float *loss, float *work, void *stream) {
    if (!params || !x || !rank_class || !hist || !grad || !loss || !work || batch <= 0) return WENOTT_EINVAL;
    return mlp_guard([&] {
        hipStream_t s = (hipStream_t)stream;
        const long long B = batch;
        float *h1 = work, *h2 = h1 + B * HID, *y = h2 + B * HID, *dy = y + B * OUT, *dh2 = dy + B * OUT,
              *dh1 = dh2 + B * HID, *lb = dh1 + B * HID;
        Acts a{h1, h2, y};
        forward(s, params, x, batch, a, 0);
        k_head<<<cdiv(B, 256), 256, 0, s>>>(batch, y, rank_class, hist, dy, lb);
        k_sum<<<1, 256, 0, s>>>(batch, lb, loss);
        k_wgrad<<<cdiv((long long)HID * OUT, 256), 256, 0, s>>>(batch, HID, OUT, h2, dy, grad + OFF_W3);
        k_bgrad<<<cdiv(OUT, 256), 256, 0, s>>>(batch, OUT, dy, grad + OFF_B3);
        k_back<<<cdiv(B * HID, 256), 256, 0, s>>>(batch, HID, OUT, dy, params + OFF_W3, h2, dh2);
        k_wgrad<<<cdiv((long long)HID * HID, 256), 256, 0, s>>>(batch, HID, HID, h1, dh2, grad + OFF_W2);
        k_bgrad<<<cdiv(HID, 256), 256, 0, s>>>(batch, HID, dh2, grad + OFF_B2);
        k_back<<<cdiv(B * HID, 256), 256, 0, s>>>(batch, HID, HID, dh2, params + OFF_W2, h1, dh1);
        k_wgrad<<<cdiv((long long)IN * HID, 256), 256, 0, s>>>(batch, IN, HID, x, dh1, grad + OFF_W1);
        k_bgrad<<<cdiv(HID, 256), 256, 0, s>>>(batch, HID, dh1, grad + OFF_B1);
        WTT_HIP(hipGetLastError());
    });
}

wenott_status wenott_mlp_adam_step(float *params, const float *grad, float *m, float *v, int32_t t, float lr,
                                   void *stream) {
    if (!params || !grad || !m || !v || t < 1) return WENOTT_EINVAL;
    return mlp_guard([&] {
        const float b1 = 0.9f, b2 = 0.999f;
        const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
        k_adam<<<cdiv(NPARAM, 256), 256, 0, (hipStream_t)stream>>>(NPARAM, params, grad, m, v, lr, b1, b2, c1, c2,
                                                                   1e-8f);
        WTT_HIP(hipGetLastError());
    });
}

}  // extern "C"
