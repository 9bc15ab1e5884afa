// Tensor-train algebra on cores (gfx950): sums by core concatenation, the shift-operator
// difference on one core (eqs. shifted-fluxes and euler-system-TT: (T - 1)/h acts on the
// core of its direction only), component splitting of the flux TT's last core (Sec. 4.2:
// the last core carries one slice per component), and the truncation bookkeeping of
// TT-rounding (Sec. 3.2).
#include <cmath>

#include "common.h"

namespace wtt {

namespace {

constexpr int kWave = 64;

__global__ void k_fill(double *p, long long n, double v) {
    long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_place(int ncomp, int ra, int n, int rb, const double *__restrict__ G, long long gstride, double w,
                        double *__restrict__ out, int Ra, int Rb, long long ostride, int o_r, int o_c) {
    const long long per = (long long)ra * n * rb;
    long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e >= per * ncomp) return;
    const int c = (int)(e / per);
    long long r = e % per;
    const int b = (int)(r % rb);
    r /= rb;
    const int i = (int)(r % n);
    const int a = (int)(r / n);
    out[c * ostride + ((long long)(o_r + a) * n + i) * Rb + o_c + b] = w * G[c * gstride + r * rb + b];
    (void)Ra;
}

__global__ void k_face_diff(int ncomp, int ra, int n, int rb, const double *__restrict__ G, long long gstride,
                            double scale, double *__restrict__ out, long long ostride) {
    const long long per = (long long)ra * n * rb;
    long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e >= per * ncomp) return;
    const int c = (int)(e / per);
    long long r = e % per;
    const int b = (int)(r % rb);
    r /= rb;
    const int i = (int)(r % n);
    const int a = (int)(r / n);
    const double *g = G + c * gstride + (long long)a * (n + 1) * rb + b;
    out[c * ostride + ((long long)a * n + i) * rb + b] = scale * (g[(long long)(i + 1) * rb] - g[(long long)i * rb]);
}

__global__ void k_transpose_rows(int M, int q, int r, const double *__restrict__ X, double *__restrict__ out) {
    long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long tot = (long long)r * M * q;
    if (e >= tot) return;
    const int b = (int)(e % q);
    const int i = (int)((e / q) % M);
    const int t = (int)(e / ((long long)q * M));
    out[e] = X[((long long)i * q + b) * r + t];
}

__global__ void k_split_last(int ra, int n, int ncomp, const double *__restrict__ G, double *__restrict__ out,
                             long long ostride) {
    long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long per = (long long)ra * n;
    if (e >= per * ncomp) return;
    const int c = (int)(e / per);
    const long long r = e % per;
    out[c * ostride + r] = G[r * ncomp + c];
}

__global__ void k_broadcast(int ncomp, long long len, const double *__restrict__ G, double *__restrict__ out,
                            long long ostride) {
    long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e >= len * ncomp) return;
    out[(e / len) * ostride + e % len] = G[e % len];
}

// rank of component z: the smallest r with sqrt(sum_{j >= r} sigma_j^2) <= delta_z, at least 1,
// at most rcap and n. delta_z = delta_abs[z] if given, else rel * ||sigma_z||.
__global__ void k_trunc(int n, int batch, const double *__restrict__ sigma, const double *__restrict__ delta_abs,
                        double rel, int rcap, int *__restrict__ ranks) {
    int z = blockIdx.x * blockDim.x + threadIdx.x;
    if (z >= batch) return;
    const double *sg = sigma + (long long)z * n;
    double tot = 0.0;
    for (int j = 0; j < n; ++j) tot += sg[j] * sg[j];
    double delta = delta_abs ? delta_abs[z] : rel * sqrt(tot);
    double d2 = delta * delta, tail = 0.0;
    int r = n;
    while (r > 0 && tail + sg[r - 1] * sg[r - 1] <= d2) {
        tail += sg[r - 1] * sg[r - 1];
        --r;
    }
    if (r < 1) r = 1;
    if (r > rcap) r = rcap;
    ranks[z] = r;
}

__global__ void k_projectors(int n, int batch, int R, const double *__restrict__ sigma, const double *__restrict__ V,
                             const int *__restrict__ ranks, double *__restrict__ W1, double *__restrict__ W2) {
    long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long per = (long long)n * R;
    if (e >= per * batch) return;
    const int z = (int)(e / per);
    const int i = (int)((e % per) / R);
    const int t = (int)(e % R);
    const double sg = sigma[(long long)z * n + (t < n ? t : 0)];
    const bool keep = t < ranks[z] && t < n && sg > 0.0;
    const double v = keep ? V[(long long)z * n * n + (long long)i * n + t] : 0.0;
    W1[(long long)z * per + (long long)i * R + t] = keep ? v / sg : 0.0;        // n x R
    W2[(long long)z * per + (long long)t * n + i] = keep ? v * sg : 0.0;        // R x n
}

__global__ void k_frob(long long len, const double *__restrict__ X, long long stride, double *__restrict__ out,
                       double *__restrict__ scaled, double scale) {
    __shared__ double red[16];
    const double *x = X + blockIdx.x * stride;
    double s = 0.0;
    for (long long i = threadIdx.x; i < len; i += blockDim.x) s += x[i] * x[i];
    for (int off = kWave / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, kWave);
    if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < (int)(blockDim.x / kWave); ++i) t += red[i];
        out[blockIdx.x] = sqrt(t);
        if (scaled) scaled[blockIdx.x] = scale * sqrt(t);
    }
}

inline unsigned cdiv(long long a, long long b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

void fill(hipStream_t s, double *p, long long n, double v) {
    if (n <= 0) return;
    k_fill<<<cdiv(n, 256), 256, 0, s>>>(p, n, v);
    WTT_HIP(hipGetLastError());
}

void place_block(hipStream_t s, int ncomp, int ra, int n, int rb, const double *G, long long gstride, double w,
                 double *out, int Ra, int Rb, long long ostride, int o_r, int o_c) {
    long long tot = (long long)ra * n * rb * ncomp;
    if (tot == 0) return;
    WTT_REQUIRE(o_r + ra <= Ra && o_c + rb <= Rb, WENOTT_EINVAL, "place_block out of range");
    k_place<<<cdiv(tot, 256), 256, 0, s>>>(ncomp, ra, n, rb, G, gstride, w, out, Ra, Rb, ostride, o_r, o_c);
    WTT_HIP(hipGetLastError());
}

void face_diff(hipStream_t s, int ncomp, int ra, int n, int rb, const double *G, long long gstride, double scale,
               double *out, long long ostride) {
    long long tot = (long long)ra * n * rb * ncomp;
    if (tot == 0) return;
    k_face_diff<<<cdiv(tot, 256), 256, 0, s>>>(ncomp, ra, n, rb, G, gstride, scale, out, ostride);
    WTT_HIP(hipGetLastError());
}

void transpose_rows(hipStream_t s, int M, int q, int r, const double *X, double *out) {
    long long tot = (long long)r * M * q;
    if (tot == 0) return;
    k_transpose_rows<<<cdiv(tot, 256), 256, 0, s>>>(M, q, r, X, out);
    WTT_HIP(hipGetLastError());
}

void split_last(hipStream_t s, int ra, int n, int ncomp, const double *G, double *out, long long ostride) {
    long long tot = (long long)ra * n * ncomp;
    k_split_last<<<cdiv(tot, 256), 256, 0, s>>>(ra, n, ncomp, G, out, ostride);
    WTT_HIP(hipGetLastError());
}

void broadcast_core(hipStream_t s, int ncomp, long long len, const double *G, double *out, long long ostride) {
    long long tot = len * ncomp;
    k_broadcast<<<cdiv(tot, 256), 256, 0, s>>>(ncomp, len, G, out, ostride);
    WTT_HIP(hipGetLastError());
}

void trunc_ranks(hipStream_t s, int n, int batch, const double *sigma, const double *delta_abs, double rel, int rcap,
                 int *ranks) {
    k_trunc<<<cdiv(batch, 64), 64, 0, s>>>(n, batch, sigma, delta_abs, rel, rcap, ranks);
    WTT_HIP(hipGetLastError());
}

void build_projectors(hipStream_t s, int n, int batch, int R, const double *sigma, const double *V, const int *ranks,
                      double *W1, double *W2) {
    long long tot = (long long)n * R * batch;
    k_projectors<<<cdiv(tot, 256), 256, 0, s>>>(n, batch, R, sigma, V, ranks, W1, W2);
    WTT_HIP(hipGetLastError());
}

__global__ void k_sample_points(int npts, int d, int n0, int n1, int n2, unsigned long long seed, int *__restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= npts * d) return;
    const int j = e % d;
    out[e] = probe_coord(seed, e, j == 0 ? n0 : (j == 1 ? n1 : n2));
}

void sample_points(hipStream_t s, int npts, int d, const int *n, unsigned long long seed, int *out) {
    k_sample_points<<<cdiv((long long)npts * d, 256), 256, 0, s>>>(npts, d, n[0], d > 1 ? n[1] : 1, d > 2 ? n[2] : 1,
                                                                     seed, out);
    WTT_HIP(hipGetLastError());
}

void frob_norms(hipStream_t s, int batch, long long len, const double *X, long long stride, double *out,
                double *scaled, double scale) {
    k_frob<<<batch, 1024, 0, s>>>(len, X, stride, out, scaled, scale);
    WTT_HIP(hipGetLastError());
}

}  // namespace wtt
