// Dense-grid FP64 WENO5-JS + global Lax-Friedrichs + SSP-RK3 on gfx950: the comparator
// that WENO-TT is measured against (the paper's "full-tensor" scheme of Sec. 2, run on the
// same GPU). One thread per face computes the split flux at the six cells around its face
// and both reconstructions; a second pass takes the face difference along that direction.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <new>
#include <string>

#include "common.h"

namespace wtt {
namespace {

constexpr int kWave = 64;

template <typename T>
__device__ inline T weno5d(T vm2, T vm1, T v0, T vp1, T vp2, T eps) {
    const T c13 = T(13.0 / 12.0), c14 = T(0.25), c16 = T(1.0 / 6.0);
    T q0 = (T(2) * v0 + T(5) * vp1 - vp2) * c16;
    T q1 = (-vm1 + T(5) * v0 + T(2) * vp1) * c16;
    T q2 = (T(2) * vm2 - T(7) * vm1 + T(11) * v0) * c16;
    T a = v0 - T(2) * vp1 + vp2, b = T(3) * v0 - T(4) * vp1 + vp2;
    T b0 = c13 * a * a + c14 * b * b;
    a = vm1 - T(2) * v0 + vp1;
    b = vm1 - vp1;
    T b1 = c13 * a * a + c14 * b * b;
    a = vm2 - T(2) * vm1 + v0;
    b = vm2 - T(4) * vm1 + T(3) * v0;
    T b2 = c13 * a * a + c14 * b * b;
    T t0 = (b0 + eps) * (b0 + eps), t1 = (b1 + eps) * (b1 + eps), t2 = (b2 + eps) * (b2 + eps);
    T a0 = T(0.3) * t1 * t2, a1 = T(0.6) * t0 * t2, a2 = T(0.1) * t0 * t1;
    return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2);
}

struct DenseGeom {
    int d;
    int n[kMaxDim];
    int bc[kMaxDim];
    long long stride[kMaxDim];  // C-order strides of the interior grid
    long long ncell;
};

// F-hat along dir at every face: faces indexed like cells but with extent n[dir] + 1.
template <int ND>
__global__ __launch_bounds__(256) void k_face_flux(DenseGeom g, int dir, double gamma, double alpha, double eps,
                                                   const double *__restrict__ U, double *__restrict__ F,
                                                   long long nface, int *__restrict__ flags) {
    constexpr int NC = ND + 2;
    long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e >= nface) return;
    // decode face coordinates (extent n[dir] + 1 along dir)
    int coord[ND];
    long long r = e;
#pragma unroll
    for (int d = ND - 1; d >= 0; --d) {
        int ext = g.n[d] + (d == dir ? 1 : 0);
        coord[d] = (int)(r % ext);
        r /= ext;
    }
    long long base = 0;
#pragma unroll
    for (int d = 0; d < ND; ++d)
        if (d != dir) base += coord[d] * g.stride[d];
    const int m = coord[dir];
    double fp[NC][6], fm[NC][6];
    bool ok = true;
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        const int cell = ghost_map(m - 3 + s, g.n[dir], g.bc[dir]);
        const long long idx = base + cell * g.stride[dir];
        double q[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) q[c] = U[c * g.ncell + idx];
        if (bc_special(g.bc[dir]) && ghost_kind(m - 3 + s, g.n[dir], g.bc[dir]) == kGhostMirror) q[1 + dir] = -q[1 + dir];
        const double inv = 1.0 / q[0];
        double ke = 0.0;
#pragma unroll
        for (int j = 0; j < ND; ++j) ke += q[1 + j] * q[1 + j];
        ke *= 0.5 * inv;
        const double p = (gamma - 1.0) * (q[NC - 1] - ke);
        const double un = q[1 + dir] * inv;
        ok &= q[0] > 0.0 && p > 0.0;
        double f[NC];
        f[0] = q[1 + dir];
#pragma unroll
        for (int j = 0; j < ND; ++j) f[1 + j] = q[1 + j] * un + (j == dir ? p : 0.0);
        f[NC - 1] = un * (q[NC - 1] + p);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            fp[c][s] = 0.5 * (f[c] + alpha * q[c]);
            fm[c][s] = 0.5 * (f[c] - alpha * q[c]);
        }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
        F[c * nface + e] = weno5d<double>(fp[c][0], fp[c][1], fp[c][2], fp[c][3], fp[c][4], eps) +
                           weno5d<double>(fm[c][5], fm[c][4], fm[c][3], fm[c][2], fm[c][1], eps);
    if (!ok) atomicOr(flags, kFlagNonPhys);
}

// L[cell] (+)= -(F[face m+1] - F[face m]) / h along dir.
template <int ND>
__global__ void k_face_diff_acc(DenseGeom g, int dir, double inv_h, const double *__restrict__ F, long long nface,
                                double *__restrict__ L, int accumulate) {
    constexpr int NC = ND + 2;
    long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e >= g.ncell) return;
    // face index of the cell's left face in the face grid
    long long r = e, fidx = 0, fstride = 1;
    int coord[ND];
#pragma unroll
    for (int d = ND - 1; d >= 0; --d) {
        coord[d] = (int)(r % g.n[d]);
        r /= g.n[d];
    }
    long long fst[ND];
#pragma unroll
    for (int d = ND - 1; d >= 0; --d) {
        fst[d] = fstride;
        fstride *= g.n[d] + (d == dir ? 1 : 0);
    }
#pragma unroll
    for (int d = 0; d < ND; ++d) fidx += coord[d] * fst[d];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const double v = -(F[c * nface + fidx + fst[dir]] - F[c * nface + fidx]) * inv_h;
        L[c * g.ncell + e] = accumulate ? L[c * g.ncell + e] + v : v;
    }
}

template <int ND>
__global__ __launch_bounds__(256) void k_speed(DenseGeom g, double gamma, const double *__restrict__ U,
                                               double *__restrict__ partial, int *__restrict__ flags) {
    constexpr int NC = ND + 2;
    __shared__ double red[4];
    long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    double sp = 0.0;
    bool ok = true;
    if (e < g.ncell) {
        double q[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) q[c] = U[c * g.ncell + e];
        const double inv = 1.0 / q[0];
        double u2 = 0.0;
#pragma unroll
        for (int j = 0; j < ND; ++j) u2 += q[1 + j] * q[1 + j];
        u2 *= inv * inv;
        const double p = (gamma - 1.0) * (q[NC - 1] - 0.5 * q[0] * u2);
        ok = q[0] > 0.0 && p > 0.0;
        sp = ok ? sqrt(u2) + sqrt(gamma * p * inv) : 0.0;
    }
    for (int off = kWave / 2; off > 0; off >>= 1) sp = fmax(sp, __shfl_xor(sp, off, kWave));
    if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = sp;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    if (!ok) atomicOr(flags, kFlagNonPhys);
}

__global__ void k_reduce_max_d(const double *__restrict__ partial, int n, double *__restrict__ out) {
    __shared__ double red[16];
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) v = fmax(v, partial[i]);
    for (int off = kWave / 2; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
    if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int i = 0; i < (int)(blockDim.x / kWave); ++i) m = fmax(m, red[i]);
        out[0] = m;
    }
}

// out = a x + b y + c z (z may alias out)
__global__ void k_axpby(long long n, double a, const double *x, double b, const double *y, double c, const double *z,
                        double *out) {
    long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v = b * y[i] + c * z[i];
    if (a != 0.0) v += a * x[i];
    out[i] = v;
}

inline unsigned cdiv(long long a, long long b) { return (unsigned)((a + b - 1) / b); }

}  // namespace
}  // namespace wtt

using namespace wtt;

struct wenott_dense {
    DenseGeom g{};
    int nc = 0;
    double h[kMaxDim] = {};
    double gamma = 1.4;
    hipStream_t s = nullptr;
    double *F = nullptr, *L = nullptr, *U1 = nullptr, *part = nullptr, *scal = nullptr;
    int *flags = nullptr, *hflag = nullptr;
    double *hscal = nullptr;
    long long maxface = 0;
    int nblk = 0;
    std::string err;
};

namespace {

double dense_alpha(wenott_dense *c, const double *U) {
    if (c->g.d == 2) k_speed<2><<<c->nblk, 256, 0, c->s>>>(c->g, c->gamma, U, c->part, c->flags);
    else k_speed<3><<<c->nblk, 256, 0, c->s>>>(c->g, c->gamma, U, c->part, c->flags);
    k_reduce_max_d<<<1, 1024, 0, c->s>>>(c->part, c->nblk, c->scal);
    WTT_HIP(hipGetLastError());
    WTT_HIP(hipMemcpyAsync(c->hscal, c->scal, sizeof(double), hipMemcpyDeviceToHost, c->s));
    WTT_HIP(hipMemcpyAsync(c->hflag, c->flags, sizeof(int), hipMemcpyDeviceToHost, c->s));
    WTT_HIP(hipStreamSynchronize(c->s));
    if (*c->hflag) {
        WTT_HIP(hipMemsetAsync(c->flags, 0, sizeof(int), c->s));
        throw StatusError(WENOTT_ENONPHYS, "rho <= 0 or p <= 0");
    }
    return *c->hscal;
}

void dense_rhs(wenott_dense *c, const double *U, double alpha, double *L) {
    for (int dir = 0; dir < c->g.d; ++dir) {
        long long nface = c->g.ncell / c->g.n[dir] * (c->g.n[dir] + 1);
        double eps = c->h[dir] * c->h[dir];
        if (c->g.d == 2) {
            k_face_flux<2><<<cdiv(nface, 256), 256, 0, c->s>>>(c->g, dir, c->gamma, alpha, eps, U, c->F, nface, c->flags);
            k_face_diff_acc<2><<<cdiv(c->g.ncell, 256), 256, 0, c->s>>>(c->g, dir, 1.0 / c->h[dir], c->F, nface, L, dir > 0);
        } else {
            k_face_flux<3><<<cdiv(nface, 256), 256, 0, c->s>>>(c->g, dir, c->gamma, alpha, eps, U, c->F, nface, c->flags);
            k_face_diff_acc<3><<<cdiv(c->g.ncell, 256), 256, 0, c->s>>>(c->g, dir, 1.0 / c->h[dir], c->F, nface, L, dir > 0);
        }
        WTT_HIP(hipGetLastError());
    }
}

wenott_status guarded(wenott_dense *c, const std::function<void()> &f) {
    try {
        f();
        return WENOTT_OK;
    } catch (const StatusError &e) {
        if (c) c->err = e.what();
        return e.status;
    } catch (const HipError &e) {
        if (c) c->err = e.what();
        return e.code == hipErrorOutOfMemory ? WENOTT_ENOMEM : WENOTT_EHIP;
    } catch (...) {
        return WENOTT_EINVAL;
    }
}

}  // namespace

extern "C" {

wenott_status wenott_dense_init(wenott_dense **out, const wenott_grid *grid, double gamma, const int32_t *bc,
                                void *hip_stream) {
    if (!out || !grid || !bc) return WENOTT_EINVAL;
    *out = nullptr;
    wenott_dense *c = new (std::nothrow) wenott_dense();
    if (!c) return WENOTT_ENOMEM;
    wenott_status st = guarded(c, [&] {
        const int d = grid->ndim;
        WTT_REQUIRE(d == 2 || d == 3, WENOTT_EINVAL, "ndim must be 2 or 3");
        WTT_REQUIRE(gamma > 1.0, WENOTT_EINVAL, "gamma must exceed 1");
        c->g.d = d;
        c->nc = d + 2;
        c->gamma = gamma;
        c->s = (hipStream_t)hip_stream;
        long long ncell = 1;
        for (int k = 0; k < d; ++k) {
            WTT_REQUIRE(grid->n[k] >= 3 && grid->hi[k] > grid->lo[k], WENOTT_EINVAL, "bad grid");
            for (int side = 0; side < 2; ++side)
                WTT_REQUIRE(bc[2 * k + side] >= WENOTT_BC_PERIODIC && bc[2 * k + side] <= WENOTT_BC_SYMMETRY,
                            WENOTT_EINVAL, "the dense comparator takes periodic, transmissive and symmetry sides");
            WTT_REQUIRE((bc[2 * k] == WENOTT_BC_PERIODIC) == (bc[2 * k + 1] == WENOTT_BC_PERIODIC), WENOTT_EINVAL,
                        "a periodic side needs a periodic opposite side");
            c->g.n[k] = (int)grid->n[k];
            c->g.bc[k] = bc_code(bc[2 * k], bc[2 * k + 1]);
            c->h[k] = (grid->hi[k] - grid->lo[k]) / grid->n[k];
            ncell *= grid->n[k];
        }
        long long st2 = 1;
        for (int k = d - 1; k >= 0; --k) { c->g.stride[k] = st2; st2 *= c->g.n[k]; }
        c->g.ncell = ncell;
        for (int k = 0; k < d; ++k) c->maxface = std::max(c->maxface, ncell / c->g.n[k] * (c->g.n[k] + 1));
        c->nblk = (int)((ncell + 255) / 256);
        WTT_HIP(hipMalloc((void **)&c->F, sizeof(double) * c->maxface * c->nc));
        WTT_HIP(hipMalloc((void **)&c->L, sizeof(double) * ncell * c->nc));
        WTT_HIP(hipMalloc((void **)&c->U1, sizeof(double) * ncell * c->nc));
        WTT_HIP(hipMalloc((void **)&c->part, sizeof(double) * c->nblk));
        WTT_HIP(hipMalloc((void **)&c->scal, sizeof(double) * 4));
        WTT_HIP(hipMalloc((void **)&c->flags, sizeof(int)));
        WTT_HIP(hipMemset(c->flags, 0, sizeof(int)));
        WTT_HIP(hipHostMalloc((void **)&c->hscal, sizeof(double) * 4, hipHostMallocDefault));
        WTT_HIP(hipHostMalloc((void **)&c->hflag, sizeof(int) * 4, hipHostMallocDefault));
    });
    if (st != WENOTT_OK) {
        wenott_dense_destroy(c);
        return st;
    }
    *out = c;
    return WENOTT_OK;
}

void wenott_dense_destroy(wenott_dense *c) {
    if (!c) return;
    // teardown: errors are not reportable here
    (void)hipStreamSynchronize(c->s);
    (void)hipFree(c->F);
    (void)hipFree(c->L);
    (void)hipFree(c->U1);
    (void)hipFree(c->part);
    (void)hipFree(c->scal);
    (void)hipFree(c->flags);
    if (c->hscal) (void)hipHostFree(c->hscal);
    if (c->hflag) (void)hipHostFree(c->hflag);
    delete c;
}

wenott_status wenott_dense_max_wavespeed(wenott_dense *c, const double *U, double *alpha) {
    if (!c || !U || !alpha) return WENOTT_EINVAL;
    return guarded(c, [&] { *alpha = dense_alpha(c, U); });
}

wenott_status wenott_dense_rhs(wenott_dense *c, const double *U, double alpha, double *L) {
    if (!c || !U || !L || !(alpha > 0.0)) return WENOTT_EINVAL;
    return guarded(c, [&] { dense_rhs(c, U, alpha, L); });
}

wenott_status wenott_dense_rk3_step(wenott_dense *c, double *U, double dt, const double *alphas, double *alphas_used) {
    if (!c || !U || !(dt > 0.0)) return WENOTT_EINVAL;
    return guarded(c, [&] {
        const long long n = c->g.ncell * c->nc;
        const unsigned nb = cdiv(n, 256);
        const double aw[3] = {0.0, 0.75, 1.0 / 3.0}, bw[3] = {1.0, 0.25, 2.0 / 3.0};
        const double *X = U;
        for (int st = 0; st < 3; ++st) {
            double a = alphas ? alphas[st] : dense_alpha(c, X);
            if (alphas_used) alphas_used[st] = a;
            dense_rhs(c, X, a, c->L);
            // U1 = a_s U + b_s (X + dt L); the last stage writes U
            double *dst = st == 2 ? U : c->U1;
            k_axpby<<<nb, 256, 0, c->s>>>(n, aw[st], U, bw[st], X, bw[st] * dt, c->L, dst);
            WTT_HIP(hipGetLastError());
            X = c->U1;
        }
        if (alphas) {
            WTT_HIP(hipMemcpyAsync(c->hflag, c->flags, sizeof(int), hipMemcpyDeviceToHost, c->s));
            WTT_HIP(hipStreamSynchronize(c->s));
            if (*c->hflag) {
                WTT_HIP(hipMemsetAsync(c->flags, 0, sizeof(int), c->s));
                throw StatusError(WENOTT_ENONPHYS, "rho <= 0 or p <= 0");
            }
        }
    });
}

}  // extern "C"
