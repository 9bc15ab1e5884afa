// Fiber evaluation of the fused LF + WENO5-JS flux on TT cores (gfx950).
//
// A cross over the flux tensor Fhat_dir(i_1..i_d, c) needs the flux on blocks
// (I_<k, i_k, J_>k). The state value at one point is the chain product of its cores
// (Sec. 3.1, eq. TT_def_2), so a block of state values is P . G_k . Q with P, Q the left
// and right interface matrices at the pivots. The flux needs the state at the six cells
// m-3 .. m+2 around face m along dir (Sec. 2.2 stencils S_0..S_2 for f^+ and their mirror
// for f^-), realised as six shifted interface matrices or, when the free mode is dir
// itself, as six neighbouring cells of the same block.
#include <cmath>

#include "common.h"

namespace wtt {

namespace {

constexpr int kWave = 64;

struct CoreSet {
    const double *c[kMaxDim];
    long long cstride[kMaxDim];
    int R[kMaxDim + 1];
    int N[kMaxDim];
};

inline CoreSet make_coreset(const FiberGeom &g, const double *const *cores, const int *ranks, const int *modes) {
    CoreSet cs{};
    for (int k = 0; k <= g.d; ++k) cs.R[k] = ranks[k];
    for (int k = 0; k < g.d; ++k) {
        cs.c[k] = cores[k];
        cs.N[k] = modes[k];
        cs.cstride[k] = (long long)ranks[k] * modes[k] * ranks[k + 1];
    }
    return cs;
}

// Entry v of mode `mode` of a multi-index. On the shifted mode it is a face index m (S = 6,
// cells m-3 .. m+2) or a cell index i (S = 7, cells i-3 .. i+3); shift slot s gives cell v - 3 + s.
__device__ inline int mode_index(const FiberGeom &g, int mode, int v, int s, int shift_mode) {
    if (mode == shift_mode) return ghost_map(v - 3 + s, g.n[mode], g.bc[mode]);
    return v;
}

// Factor of an interface entry whose shifted mode m sits at cell `raw` (maybe a ghost): -1 for
// the normal momentum at a symmetry plane, 0 on an inflow side (whose constant state is written
// into the gathered block afterwards, inflow_fill), else 1.
__device__ inline double ghost_factor(const FiberGeom &g, int m, int raw, int c) {
    if (!bc_special(g.bc[m])) return 1.0;
    const int kind = ghost_kind(raw, g.n[m], g.bc[m]);
    if (kind == kGhostInflow) return 0.0;
    return kind == kGhostMirror && g.law == kLawEuler && c == 1 + m ? -1.0 : 1.0;
}

__device__ inline void iface_entry(const FiberGeom &g, const CoreSet &cs, int side, int count,
                                   const int *__restrict__ idx, int S, int shift_mode, double *__restrict__ out,
                                   long long e) {
    const int k = g.k;
    const int Rout = side == 0 ? cs.R[k] : cs.R[k + 1];
    const long long tot = (long long)g.ncomp * S * count * Rout;
    if (e >= tot) return;
    const int beta = (int)(e % Rout);
    long long r = e / Rout;
    const int a = (int)(r % count);
    r /= count;
    const int s = (int)(r % S);
    const int c = (int)(r / S);
    double val;
    if (side == 0) {
        const int *mi = idx + (long long)a * k;
        const int i0 = mode_index(g, 0, mi[0], s, shift_mode);
        const double *G0 = cs.c[0] + c * cs.cstride[0];
        if (k == 1) {
            val = G0[(long long)i0 * cs.R[1] + beta];
        } else {  // k == 2
            const int i1 = mode_index(g, 1, mi[1], s, shift_mode);
            const double *G1 = cs.c[1] + c * cs.cstride[1];
            double acc = 0.0;
            for (int al = 0; al < cs.R[1]; ++al)
                acc += G0[(long long)i0 * cs.R[1] + al] * G1[((long long)al * cs.N[1] + i1) * cs.R[2] + beta];
            val = acc;
        }
        if (shift_mode >= 0) val *= ghost_factor(g, shift_mode, mi[shift_mode] - 3 + s, c);
        out[(((long long)c * S + s) * count + a) * Rout + beta] = val;
    } else {
        const int len = g.d - 1 - k;
        const int *mi = idx + (long long)a * len;
        const int last = g.d - 1;
        if (len == 1) {
            const int j = mode_index(g, last, mi[0], s, shift_mode);
            const double *G = cs.c[last] + c * cs.cstride[last];
            val = G[(long long)beta * cs.N[last] + j];
        } else {  // k == 0, d == 3
            const int j1 = mode_index(g, 1, mi[0], s, shift_mode), j2 = mode_index(g, 2, mi[1], s, shift_mode);
            const double *G1 = cs.c[1] + c * cs.cstride[1];
            const double *G2 = cs.c[2] + c * cs.cstride[2];
            double acc = 0.0;
            for (int b2 = 0; b2 < cs.R[2]; ++b2)
                acc += G1[((long long)beta * cs.N[1] + j1) * cs.R[2] + b2] * G2[(long long)b2 * cs.N[2] + j2];
            val = acc;
        }
        if (shift_mode >= 0) val *= ghost_factor(g, shift_mode, mi[shift_mode - k - 1] - 3 + s, c);
        out[(((long long)c * S + s) * Rout + beta) * count + a] = val;
    }
}

__global__ void k_iface(FiberGeom g, CoreSet cs, int side, int count, const int *__restrict__ idx, int S,
                        int shift_mode, double *__restrict__ out) {
    iface_entry(g, cs, side, count, idx, S, shift_mode, out, blockIdx.x * (long long)blockDim.x + threadIdx.x);
}

// Several interface matrices of one block (the left and right ones of every gather) in one
// launch: job q owns workgroups [first[q], first[q + 1]).
constexpr int kMaxIfaceJobs = 8;
struct IfaceJob {
    CoreSet cs;
    const int *idx;
    double *out;
    int side, count, S, shift_mode;
};
struct IfaceBatch {
    IfaceJob job[kMaxIfaceJobs];
    int first[kMaxIfaceJobs + 1];
    int n;
};

__global__ void k_iface_batch(FiberGeom g, IfaceBatch b) {
    int q = 0;
    while (q + 1 < b.n && (int)blockIdx.x >= b.first[q + 1]) ++q;
    const IfaceJob &J = b.job[q];
    iface_entry(g, J.cs, J.side, J.count, J.idx, J.S, J.shift_mode, J.out,
                (long long)((int)blockIdx.x - b.first[q]) * blockDim.x + threadIdx.x);
}

// Left-biased WENO5-JS value at x_{i+1/2} from v_{i-2..i+2} (Sec. 2.2): candidate values,
// smoothness indicators beta_r, weights d_r / (beta_r + eps)^2 normalised, written with one
// reciprocal: w_r = d_r prod_{s != r} t_s / sum_s d_s prod_{u != s} t_u, t_r = (beta_r + eps)^2.
template <typename T>
__device__ inline T weno5(T vm2, T vm1, T v0, T vp1, T vp2, T eps) {
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

// f^{+-} = (f_dir(q) +- alpha q) / 2 for one stencil cell (eq. lax-friedrichs) with the Euler
// fluxes of Sec. 2.1, or the scalar fluxes of Sec. 5.1 (f = u) and Sec. 5.2 (f = u^2 / 2).
template <int ND, int LW, typename T>
__device__ inline bool split_flux(const T *q, int dir, T gm1, T alpha, T *fp, T *fm) {
    if (LW != kLawEuler) {
        const T f = LW == kLawLinAdv ? q[0] : T(0.5) * q[0] * q[0];
        fp[0] = T(0.5) * (f + alpha * q[0]);
        fm[0] = T(0.5) * (f - alpha * q[0]);
        return true;
    }
    constexpr int NC = ND + 2;
    T rho = q[0];
    T inv = T(1) / rho;
    T ke = T(0);
#pragma unroll
    for (int j = 0; j < ND; ++j) ke += q[1 + j] * q[1 + j];
    ke *= T(0.5) * inv;
    T p = gm1 * (q[NC - 1] - ke);
    T un = q[1 + dir] * inv;
    T f[NC];
    f[0] = q[1 + dir];
#pragma unroll
    for (int j = 0; j < ND; ++j) f[1 + j] = q[1 + j] * un + (j == dir ? p : T(0));
    f[NC - 1] = un * (q[NC - 1] + p);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        fp[c] = T(0.5) * (f[c] + alpha * q[c]);
        fm[c] = T(0.5) * (f[c] - alpha * q[c]);
    }
    return rho > T(0) && p > T(0);
}

template <int ND, int LW, typename T>
__global__ __launch_bounds__(256) void k_weno(FiberGeom g, int p, int M, int q, const T *__restrict__ W,
                                              double *__restrict__ out, long long sa, long long si, long long sb,
                                              long long sc, int *__restrict__ flags) {
    constexpr int NC = LawNC<ND, LW>::v;
    const long long tot = (long long)p * M * q;
    long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e >= tot) return;
    const int b = (int)(e % q);
    const long long r = e / q;
    const int i = (int)(r % M);
    const int a = (int)(r / M);
    const int Nk = g.n[g.k];
    const bool same = g.k == g.dir;
    T fp[NC][6], fm[NC][6];
    bool ok = true;
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        T qv[NC];
        if (same) {
            const int cell = ghost_map(i - 3 + s, Nk, g.bc[g.k]);
#pragma unroll
            for (int c = 0; c < NC; ++c)
                qv[c] = ghost_fix<T>(g, g.k, i - 3 + s, c, W[(((long long)c * p + a) * Nk + cell) * q + b]);
        } else {
#pragma unroll
            for (int c = 0; c < NC; ++c) qv[c] = W[((((long long)c * 6 + s) * p + a) * Nk + i) * q + b];
        }
        T fpt[NC], fmt[NC];
        ok &= split_flux<ND, LW, T>(qv, g.dir, T(g.gamma - 1.0), T(geom_alpha(g)), fpt, fmt);
#pragma unroll
        for (int c = 0; c < NC; ++c) { fp[c][s] = fpt[c]; fm[c][s] = fmt[c]; }
    }
    const T eps = T(g.eps_w);
    bool finite = true;
    double *o = out + a * sa + i * si + b * sb;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        // face m sits between cells m-1 and m: f^+ from cells m-3..m+1 (slots 0..4),
        // f^- mirrored from cells m+2..m-2 (slots 5..1)
        T hp = weno5<T>(fp[c][0], fp[c][1], fp[c][2], fp[c][3], fp[c][4], eps);
        T hm = weno5<T>(fm[c][5], fm[c][4], fm[c][3], fm[c][2], fm[c][1], eps);
        double v = (double)hp + (double)hm;
        finite &= (v == v) && fabs(v) < 1e300;
        o[c * sc] = v;
    }
    if (!ok) atomicOr(flags, kFlagNonPhys);
    if (!finite) atomicOr(flags, kFlagNaN);
}

// LF-cross evaluation (Sec. 4.2, Algorithm lf-cross): the split fluxes f^+ and f^- of every
// component at the block's cells, 2 ncomp values per point (f^+ in slots 0..ncomp-1, f^- after
// them). W0 holds the state at the block points, W0[c * cs + (a Nk + i) q + b].
template <int ND, int LW>
__global__ __launch_bounds__(256) void k_lf(FiberGeom g, int p, int q, const double *__restrict__ W0, long long cs,
                                            double *__restrict__ out, long long sa, long long si, long long sb,
                                            long long sc, int *__restrict__ flags) {
    constexpr int NC = LawNC<ND, LW>::v;
    const int Nk = g.n[g.k];
    const long long tot = (long long)p * Nk * q;
    const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e >= tot) return;
    const int b = (int)(e % q);
    const long long r = e / q;
    const int i = (int)(r % Nk);
    const int a = (int)(r / Nk);
    double qv[NC], fp[NC], fm[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) qv[c] = W0[c * cs + e];
    const bool ok = split_flux<ND, LW, double>(qv, g.dir, g.gamma - 1.0, geom_alpha(g), fp, fm);
    bool finite = true;
    double *o = out + a * sa + i * si + b * sb;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        finite &= (fp[c] == fp[c]) && (fm[c] == fm[c]) && fabs(fp[c]) < 1e300 && fabs(fm[c]) < 1e300;
        o[c * sc] = fp[c];
        o[(NC + c) * sc] = fm[c];
    }
    if (!ok) atomicOr(flags, kFlagNonPhys);
    if (!finite) atomicOr(flags, kFlagNaN);
}

// Sampled residual of an LF-cross: the split fluxes at each probe cell (from the state value in
// slot 3 of the k_sample_state layout) against the candidate TT with 2 ncomp slices on its last
// core; one partial pair (|diff|^2, |exact|^2) per workgroup.
template <int ND, int LW>
__global__ __launch_bounds__(256) void k_sample_lf(FiberGeom g, CoreSet fs, int npts, const int *__restrict__ pts,
                                                   const double *__restrict__ ust, double *__restrict__ acc,
                                                   int *__restrict__ flags) {
    constexpr int NC = LawNC<ND, LW>::v, NO = 2 * NC;
    __shared__ double red[2][4];
    const int pt = blockIdx.x * blockDim.x + threadIdx.x;
    double d2 = 0.0, n2 = 0.0;
    bool ok = true;
    if (pt < npts) {
        double qv[NC], ex[NO];
#pragma unroll
        for (int c = 0; c < NC; ++c) qv[c] = ust[((long long)pt * 6 + 3) * NC + c];
        ok = split_flux<ND, LW, double>(qv, g.dir, g.gamma - 1.0, geom_alpha(g), ex, ex + NC);
        const int *m = pts + pt * ND;
        double approx[NO];
#pragma unroll
        for (int c = 0; c < NO; ++c) approx[c] = 0.0;
        if (ND == 2) {
            const double *g0 = fs.c[0] + (long long)m[0] * fs.R[1];
            const double *g1 = fs.c[1] + (long long)m[1] * NO;
            for (int al = 0; al < fs.R[1]; ++al)
#pragma unroll
                for (int c = 0; c < NO; ++c) approx[c] = fma(g0[al], g1[al * (long long)fs.N[1] * NO + c], approx[c]);
        } else {
            for (int be = 0; be < fs.R[2]; ++be) {
                double v = 0.0;
                for (int al = 0; al < fs.R[1]; ++al)
                    v += fs.c[0][(long long)m[0] * fs.R[1] + al] * fs.c[1][((long long)al * fs.N[1] + m[1]) * fs.R[2] + be];
                const double *last = fs.c[2] + ((long long)be * fs.N[2] + m[2]) * NO;
#pragma unroll
                for (int c = 0; c < NO; ++c) approx[c] = fma(v, last[c], approx[c]);
            }
        }
#pragma unroll
        for (int c = 0; c < NO; ++c) {
            d2 += (ex[c] - approx[c]) * (ex[c] - approx[c]);
            n2 += ex[c] * ex[c];
        }
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
        d2 += __shfl_xor(d2, off, kWave);
        n2 += __shfl_xor(n2, off, kWave);
    }
    if (threadIdx.x % kWave == 0) { red[0][threadIdx.x / kWave] = d2; red[1][threadIdx.x / kWave] = n2; }
    __syncthreads();
    if (threadIdx.x == 0) {
        acc[2 * blockIdx.x] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        acc[2 * blockIdx.x + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    }
    if (!ok) atomicOr(flags, kFlagNonPhys);
}

// sum_t x[t sx] y[t sy], t < n, in four interleaved chains so that the loads of several terms
// are in flight at once (the operands come from L2)
__device__ inline double dot4(const double *__restrict__ x, long long sx, const double *__restrict__ y, long long sy,
                              int n) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int t = 0;
    for (; t + 3 < n; t += 4) {
        a0 = fma(x[t * sx], y[t * sy], a0);
        a1 = fma(x[(t + 1) * sx], y[(t + 1) * sy], a1);
        a2 = fma(x[(t + 2) * sx], y[(t + 2) * sy], a2);
        a3 = fma(x[(t + 3) * sx], y[(t + 3) * sy], a3);
    }
    for (; t < n; ++t) a0 = fma(x[t * sx], y[t * sy], a0);
    return (a0 + a1) + (a2 + a3);
}

template <int ND, int LW>
__global__ __launch_bounds__(256) void k_dense_eval(int mode, long long nrows, int R, int nlast,
                                                    const double *__restrict__ Lm, long long lm_stride,
                                                    const double *__restrict__ G, long long g_stride, double gamma,
                                                    double *__restrict__ out, double *__restrict__ partial,
                                                    int *__restrict__ flags) {
    constexpr int NC = LawNC<ND, LW>::v;
    __shared__ double red[4];
    const long long ncell = nrows * nlast;
    long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    double speed = 0.0;
    bool ok = true;
    if (e < ncell) {
        // (row, j) of this cell without a 64-bit division per thread: the block's first cell is
        // split once (uniform values), the thread's offset by at most one 32-bit division
        const long long e0 = (long long)blockIdx.x * blockDim.x;
        long long row = e0 / nlast;
        int j = (int)(e0 - row * nlast) + (int)threadIdx.x;
        if (j >= nlast) {
            const int q = (int)((unsigned)j / (unsigned)nlast);
            row += q;
            j -= q * nlast;
        }
        double qv[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) qv[c] = dot4(Lm + c * lm_stride + row * R, 1, G + c * g_stride + j, nlast, R);
        if (mode == 0) {
#pragma unroll
            for (int c = 0; c < NC; ++c) out[c * ncell + e] = qv[c];
        } else if (LW == kLawBurgers) {
            speed = fabs(qv[0]);
        } else {
            double inv = 1.0 / qv[0], u2 = 0.0;
#pragma unroll
            for (int d = 0; d < ND; ++d) u2 += qv[1 + d] * qv[1 + d];
            u2 *= inv * inv;
            double pr = (gamma - 1.0) * (qv[NC - 1] - 0.5 * qv[0] * u2);
            ok = qv[0] > 0.0 && pr > 0.0;
            speed = ok ? sqrt(u2) + sqrt(gamma * pr * inv) : 0.0;
        }
    }
    if (mode == 1) {
        for (int off = kWave / 2; off > 0; off >>= 1) speed = fmax(speed, __shfl_xor(speed, off, kWave));
        if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = speed;
        __syncthreads();
        if (threadIdx.x == 0) partial[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
        if (!ok) atomicOr(flags, kFlagNonPhys);
    }
}

// Mode 1 (the exact alpha) with the last core's column held in registers: thread j of a
// workgroup keeps G[c][:, j] (NC x R values) and sweeps RB rows of the left part, staged in LDS
// first by one coalesced load of the chunk (NC x RB x R values, read back as broadcasts); per
// cell it forms NC dot products of length R from registers. The form above re-reads the column
// for every cell, and at N^3 cells that L2 traffic, not the arithmetic, sets its time; loading
// the rows one by one inside the sweep would instead wait a memory round trip per row. The cell
// speeds only feed a maximum; their reciprocal and square roots are the Newton-refined ones.
// RM: the register columns' length; EXACT: R == RM, so that no term needs a rank check.
template <int ND, int LW, int RM, bool EXACT>
__global__ __launch_bounds__(256) void k_alpha_eval(long long nrows, int R, int nlast, int RB,
                                                    const double *__restrict__ Lm, long long lm_stride,
                                                    const double *__restrict__ G, long long g_stride, double gamma,
                                                    double *__restrict__ partial, int *__restrict__ flags) {
    constexpr int NC = LawNC<ND, LW>::v;
    if (EXACT) R = RM;
    __shared__ double red[4];
    extern __shared__ double lrows[];  // [c][row - r0][b], NC x RB x R
    const int j = blockIdx.x * 256 + threadIdx.x;
    const bool jv = j < nlast;
    const long long r0 = (long long)blockIdx.y * RB, r1 = min(nrows, r0 + RB);
    const int chunk = RB * R;
    for (int e = threadIdx.x; e < NC * chunk; e += 256) {
        const int c = e / chunk, q = e - c * chunk;
        lrows[e] = r0 * R + q < r1 * R ? Lm[c * lm_stride + r0 * R + q] : 0.0;
    }
    double g[NC][RM];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int b = 0; b < RM; ++b) g[c][b] = (jv && b < R) ? G[c * g_stride + (long long)b * nlast + j] : 0.0;
    __syncthreads();
    double speed = 0.0;
    bool ok = true;
    for (long long row = r0; row < r1; ++row) {
        double qv[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double *l = lrows + c * chunk + (row - r0) * R;
            double s0 = 0.0, s1 = 0.0;
#pragma unroll
            for (int b = 0; b < RM; b += 2) {
                if (EXACT || b < R) s0 = fma(l[b], g[c][b], s0);
                if (b + 1 < RM && (EXACT || b + 1 < R)) s1 = fma(l[b + 1], g[c][b + 1], s1);
            }
            qv[c] = s0 + s1;
        }
        if (jv && LW == kLawBurgers) {
            speed = fmax(speed, fabs(qv[0]));
        } else if (jv) {
            const double inv = nr_rcp(qv[0]);
            double m2 = 0.0;
#pragma unroll
            for (int d = 0; d < ND; ++d) m2 = fma(qv[1 + d], qv[1 + d], m2);
            const double u2 = m2 * inv * inv;
            const double pr = (gamma - 1.0) * (qv[NC - 1] - 0.5 * qv[0] * u2);
            const bool cell_ok = qv[0] > 0.0 && pr > 0.0;
            ok = ok && cell_ok;
            speed = fmax(speed, cell_ok ? nr_sqrt(u2) + nr_sqrt(gamma * pr * inv) : 0.0);
        }
    }
    for (int off = kWave / 2; off > 0; off >>= 1) speed = fmax(speed, __shfl_xor(speed, off, kWave));
    if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = speed;
    __syncthreads();
    if (threadIdx.x == 0)
        partial[(long long)blockIdx.y * gridDim.x + blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    if (!ok) atomicOr(flags, kFlagNonPhys);
}

__global__ void k_reduce_max(const double *__restrict__ partial, int n, double *__restrict__ out) {
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

// State value of component c at a cell multi-index (chain product over the cores).
template <int ND>
__device__ inline double tt_point(const CoreSet &cs, int c, const int *cell) {
    const double *G0 = cs.c[0] + c * cs.cstride[0];
    const double *G1 = cs.c[1] + c * cs.cstride[1];
    if (ND == 2) {
        return dot4(G0 + (long long)cell[0] * cs.R[1], 1, G1 + cell[1], cs.N[1], cs.R[1]);
    } else {
        // four right indices at a time: per left index one contiguous run of G1(a, i1, be..be+3),
        // so the loads of a run are issued together rather than one dependent dot product per be
        const double *G2 = cs.c[2] + c * cs.cstride[2];
        const int R1 = cs.R[1], R2 = cs.R[2];
        const long long s1 = (long long)cs.N[1] * R2;
        const double *g0 = G0 + (long long)cell[0] * R1, *g1 = G1 + (long long)cell[1] * R2;
        double acc = 0.0;
        for (int b0 = 0; b0 < R2; b0 += 4) {
            const int nb = min(4, R2 - b0);
            double v[4] = {0.0, 0.0, 0.0, 0.0};
            for (int a = 0; a < R1; ++a) {
                const double x = g0[a];
                const double *r = g1 + a * s1 + b0;
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    if (t < nb) v[t] = fma(x, r[t], v[t]);
            }
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (t < nb) acc = fma(v[t], G2[(long long)(b0 + t) * cs.N[2] + cell[2]], acc);
        }
        return acc;
    }
}

template <int ND>
__global__ void k_sample_state(FiberGeom g, CoreSet cs, int npts, const int *__restrict__ pts,
                               double *__restrict__ ust) {
    const int NC = g.ncomp;
    long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e >= (long long)npts * 6 * NC) return;
    const int c = (int)(e % NC);
    const int s = (int)((e / NC) % 6);
    const int pt = (int)(e / (NC * 6));
    int cell[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        int v = pts[pt * ND + d];
        cell[d] = d == g.dir ? ghost_map(v - 3 + s, g.n[d], g.bc[d]) : v;
    }
    ust[e] = ghost_fix<double>(g, g.dir, pts[pt * ND + g.dir] - 3 + s, c, tt_point<ND>(cs, c, cell));
}

template <int ND, int LW>
__global__ __launch_bounds__(256) void k_sample_flux(FiberGeom g, CoreSet fs, int npts, const int *__restrict__ pts,
                                                     const double *__restrict__ ust, double *__restrict__ acc,
                                                     int *__restrict__ flags) {
    constexpr int NC = LawNC<ND, LW>::v;
    __shared__ double red[2][4];
    const int pt = blockIdx.x * blockDim.x + threadIdx.x;
    double d2 = 0.0, n2 = 0.0;
    bool ok = true;
    if (pt < npts) {
        double fp[NC][6], fm[NC][6];
        for (int s = 0; s < 6; ++s) {
            double qv[NC], a[NC], b[NC];
            for (int c = 0; c < NC; ++c) qv[c] = ust[((long long)pt * 6 + s) * NC + c];
            ok &= split_flux<ND, LW, double>(qv, g.dir, g.gamma - 1.0, geom_alpha(g), a, b);
            for (int c = 0; c < NC; ++c) { fp[c][s] = a[c]; fm[c][s] = b[c]; }
        }
        // approximation: shared cores 0..d-2, last core (R, M, NC)
        const int *m = pts + pt * ND;
        double approx[NC];
        for (int c = 0; c < NC; ++c) approx[c] = 0.0;
        if (ND == 2) {  // two rank terms per pass, each with its own accumulators
            const double *g0 = fs.c[0] + (long long)m[0] * fs.R[1];
            const double *g1 = fs.c[1] + (long long)m[1] * NC;
            const long long st1 = (long long)fs.N[1] * NC;
            double ap2[NC];
            for (int c = 0; c < NC; ++c) ap2[c] = 0.0;
            int al = 0;
            for (; al + 1 < fs.R[1]; al += 2) {
                const double l0 = g0[al], l1 = g0[al + 1];
                const double *a0 = g1 + al * st1, *a1 = a0 + st1;
                for (int c = 0; c < NC; ++c) {
                    approx[c] = fma(l0, a0[c], approx[c]);
                    ap2[c] = fma(l1, a1[c], ap2[c]);
                }
            }
            if (al < fs.R[1])
                for (int c = 0; c < NC; ++c) approx[c] = fma(g0[al], g1[al * st1 + c], approx[c]);
            for (int c = 0; c < NC; ++c) approx[c] += ap2[c];
        } else {
            for (int be = 0; be < fs.R[2]; ++be) {
                double v = 0.0;
                for (int al = 0; al < fs.R[1]; ++al)
                    v += fs.c[0][(long long)m[0] * fs.R[1] + al] * fs.c[1][((long long)al * fs.N[1] + m[1]) * fs.R[2] + be];
                const double *last = fs.c[2] + ((long long)be * fs.N[2] + m[2]) * NC;
                for (int c = 0; c < NC; ++c) approx[c] += v * last[c];
            }
        }
        const double eps = g.eps_w;
        for (int c = 0; c < NC; ++c) {
            double ex = weno5<double>(fp[c][0], fp[c][1], fp[c][2], fp[c][3], fp[c][4], eps) +
                        weno5<double>(fm[c][5], fm[c][4], fm[c][3], fm[c][2], fm[c][1], eps);
            d2 += (ex - approx[c]) * (ex - approx[c]);
            n2 += ex * ex;
        }
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
        d2 += __shfl_xor(d2, off, kWave);
        n2 += __shfl_xor(n2, off, kWave);
    }
    if (threadIdx.x % kWave == 0) { red[0][threadIdx.x / kWave] = d2; red[1][threadIdx.x / kWave] = n2; }
    __syncthreads();
    if (threadIdx.x == 0) {
        acc[2 * blockIdx.x] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        acc[2 * blockIdx.x + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    }
    if (!ok) atomicOr(flags, kFlagNonPhys);
}

// ---------------------------------------------------------------------------- stage
// -(Fhat(+1/2) - Fhat(-1/2)) / h along one direction from the state at cells -3..+3
// (slots 0..6) of every component. Face +1/2: f^+ from slots 1..5, f^- mirrored from 6..2;
// face -1/2: f^+ from slots 0..4, f^- mirrored from 5..1.
template <int ND, int LW, typename T>
__device__ inline bool stage_dir(const T (&v)[LawNC<ND, LW>::v][7], int dir, T gm1, T alpha, T eps, T inv_h,
                                 T *acc) {
    constexpr int NC = LawNC<ND, LW>::v;
    T fp[NC][7], fm[NC][7];
    bool ok = true;
#pragma unroll
    for (int s = 0; s < 7; ++s) {
        T qv[NC], a[NC], b[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) qv[c] = v[c][s];
        ok &= split_flux<ND, LW, T>(qv, dir, gm1, alpha, a, b);
#pragma unroll
        for (int c = 0; c < NC; ++c) { fp[c][s] = a[c]; fm[c][s] = b[c]; }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        T fr = weno5<T>(fp[c][1], fp[c][2], fp[c][3], fp[c][4], fp[c][5], eps) +
               weno5<T>(fm[c][6], fm[c][5], fm[c][4], fm[c][3], fm[c][2], eps);
        T fl = weno5<T>(fp[c][0], fp[c][1], fp[c][2], fp[c][3], fp[c][4], eps) +
               weno5<T>(fm[c][5], fm[c][4], fm[c][3], fm[c][2], fm[c][1], eps);
        acc[c] -= (fr - fl) * inv_h;
    }
    return ok;
}

// DG lanes per point. With DG > 1 the points of a small block (a 3D block has ~10^4, a few dozen
// workgroups at one point per thread) are split over the directions (DG = 2 in 2D; 4 in 3D, one
// idle): lane d forms the flux difference along direction d from its own gathered cells, the
// group's sum is taken by shuffles (the lanes of a group are consecutive and all alive or all
// gone) and the group's first lane forms the stage combination; more and shorter threads
// shorten the dependent chain each one runs. A large block fills the device at one point per
// thread (DG = 1, every direction in one lane). The direction-dependent operands are chosen by
// comparisons (a per-lane index into the argument arrays would send them to scratch memory).
template <int ND, int LW, int DG, typename T>
__global__ __launch_bounds__(256) void k_stage(FiberGeom g, int p, int q, StageArgsT<T> sa_, double *__restrict__ out,
                                               long long sa, long long si, long long sb, long long sc,
                                               int *__restrict__ flags) {
    constexpr int NC = LawNC<ND, LW>::v;
    const int Nk = g.n[g.k];
    const long long tot = (long long)p * Nk * q;
    const long long et = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long e = et / DG;
    const int d = (int)(et % DG);
    if (e >= tot) return;
    const int b = (int)(e % q);
    const long long r = e / q;
    const int i = (int)(r % Nk);
    const int a = (int)(r / Nk);
    const T gm1 = T(g.gamma - 1.0), alpha = T(geom_alpha(g));
    T acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = T(0);
    bool ok = true;
#pragma unroll
    for (int dd = d; dd < ND; dd += DG) {
        T v[NC][7];
        if (dd == g.k) {
#pragma unroll
            for (int s = 0; s < 7; ++s) {
                const int cell = ghost_map(i - 3 + s, Nk, g.bc[g.k]);
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    v[c][s] = ghost_fix<T>(g, g.k, i - 3 + s, c,
                                           sa_.W0[c * sa_.w0_cs + ((long long)a * Nk + cell) * q + b]);
            }
        } else {
            const T *W = dd == 0 ? sa_.Wd[0] : (dd == 1 ? sa_.Wd[1] : sa_.Wd[ND - 1]);
#pragma unroll
            for (int s = 0; s < 7; ++s)
#pragma unroll
                for (int c = 0; c < NC; ++c) v[c][s] = W[((((long long)c * 7 + s) * p + a) * Nk + i) * q + b];
        }
        const T eps = T(dd == 0 ? sa_.eps_w[0] : (dd == 1 ? sa_.eps_w[1] : sa_.eps_w[ND - 1]));
        const T ih = T(dd == 0 ? sa_.inv_h[0] : (dd == 1 ? sa_.inv_h[1] : sa_.inv_h[ND - 1]));
        ok &= stage_dir<ND, LW, T>(v, dd, gm1, alpha, eps, ih, acc);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int off = 1; off < DG; off <<= 1) acc[c] += __shfl_xor(acc[c], off, kWave);
    if (!ok) atomicOr(flags, kFlagNonPhys);
    if (d != 0) return;
    bool finite = true;
    double *o = out + a * sa + i * si + b * sb;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const long long idx = (((long long)c * p + a) * Nk + i) * q + b;
        double y = sa_.wx * sa_.X0[c * sa_.w0_cs + ((long long)a * Nk + i) * q + b] + sa_.wl * (double)acc[c];
        if (sa_.wn != 0.0) y += sa_.wn * sa_.WN[idx];
        finite &= (y == y) && fabs(y) < 1e300;
        o[c * sc] = y;
    }
    if (!finite) atomicOr(flags, kFlagNaN);
}

// X at the 7 d star cells (slot d * 7 + s) of every point; cs2 (Un) at slot 7 d when given.
// Layout ust[(slot * NC + c) * npts + pt]: the point is the fastest index, so that the stage
// kernel (one point per thread) reads it coalesced.
template <int ND>
__global__ void k_sample_star(FiberGeom g, CoreSet cs, CoreSet un, int use_un, int npts, unsigned long long seed,
                              double *__restrict__ ust) {
    const int NC = g.ncomp;
    constexpr int SL = 7 * ND + 1;
    long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e >= (long long)npts * SL * NC) return;
    const int pt = (int)(e % npts);
    const int c = (int)((e / npts) % NC);
    const int slot = (int)(e / ((long long)npts * NC));
    int cell[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) cell[d] = probe_coord(seed, (long long)pt * ND + d, g.n[d]);
    if (slot == 7 * ND) {
        ust[e] = use_un ? tt_point<ND>(un, c, cell) : 0.0;
        return;
    }
    const int d = slot / 7, s = slot % 7;
    const int raw = cell[d] - 3 + s;
    cell[d] = ghost_map(raw, g.n[d], g.bc[d]);
    ust[e] = ghost_fix<double>(g, d, raw, c, tt_point<ND>(cs, c, cell));
}

// 3D star samples by slices of the middle core: workgroup j owns slice j of mode 1 and serves
// every (probe point, shift) whose mode-1 cell maps to j, so each slice G1(:, j, :) of every
// component is read once, staged in LDS, instead of by every point that needs it (a point needs 7
// slices; at R = 60 a slice is 28 KB and 4096 points would read ~4 GB). The pairs of the slice
// are collected from all points into an LDS list; per component the slice is staged and one wave
// serves a pair, its lanes over the right rank index be:
//   t(be) = sum_al G0(i0, al) S(al, be); slot 7 + s (mode-1 line) = sum_be t(be) G2(be, i2).
// The pair whose shift is 0 (j = i1) also forms the mode-2 line from v = t (slots 14 + q:
// sum_be t(be) G2(be, i2 + q - 3)) and the mode-0 line from w1(al) = sum_be S(al, be) G2(be, i2)
// (slots q: sum_al G0(i0 + q - 3, al) w1(al), lanes over al); then U^n's slice H1(:, j, :) takes
// the LDS and those pairs form U^n at the point (slot 21) by the same contraction as t.
// A slice larger than the LDS budget is read from global memory in place.
__device__ inline double wave_sum_d(double v) {
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}


constexpr int kSlicePairs = 2048;      // pairs held at once (a slice gets ~7 npts / N1 of them)
constexpr int kSliceLdsDoubles = 8192;  // staged slice (R1 R2 <= 8192)
// threads of k_sample_slices3 (one workgroup per slice): eight waves share a slice's pairs, two
// workgroups per CU
constexpr int kSliceThreads = 512;

// Dynamic LDS of k_sample_slices3: room for each of the two slices it stages (state and U^n),
// which it does for a slice of at most kSliceLdsDoubles (a larger one is read in place); sized
// to the ranks, so that several workgroups share a CU.
size_t slice_lds_bytes(long long r1r2, long long s1s2) {
    const long long a = r1r2 <= kSliceLdsDoubles ? r1r2 : 0, b = s1s2 <= kSliceLdsDoubles ? s1s2 : 0;
    return (size_t)std::max(a, b) * sizeof(double);
}

__global__ __launch_bounds__(kSliceThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_sample_slices3(FiberGeom g, CoreSet cs, CoreSet un, int use_un, int npts,
                                                        unsigned long long seed, double *__restrict__ ust) {
    const int NC = g.ncomp;
    __shared__ int pair_pt[kSlicePairs];
    __shared__ unsigned char pair_s[kSlicePairs];
    __shared__ int npairs;
    extern __shared__ double S_lds[];  // slice_lds_bytes
    const int j = blockIdx.x, tid = threadIdx.x, lane = tid % kWave, w = tid / kWave;
    const int N0 = g.n[0], N1 = g.n[1], N2 = g.n[2];
    const int R1 = cs.R[1], R2 = cs.R[2];
    const long long s1 = (long long)N1 * R2;
    const bool staged = (long long)R1 * R2 <= kSliceLdsDoubles;
    int scan = 0;  // next point to scan
    while (scan < npts) {
        // collect pairs until the list could overflow with the next 256 points (7 pairs each),
        // 256 points a round
        if (tid == 0) npairs = 0;
        __syncthreads();
        while (scan < npts && npairs + 7 * 256 <= kSlicePairs) {
            const int pt = scan + tid;
            if (tid < 256 && pt < npts) {
                const int i1 = probe_coord(seed, (long long)pt * 3 + 1, N1);
                for (int sh = 0; sh < 7; ++sh)
                    if (ghost_map(i1 + sh - 3, N1, g.bc[1]) == j) {
                        const int q = atomicAdd(&npairs, 1);
                        pair_pt[q] = pt;
                        pair_s[q] = (unsigned char)sh;
                    }
            }
            scan += 256;
            __syncthreads();
        }
        const int np = npairs;
        for (int c = 0; c < NC && np > 0; ++c) {
            const double *G1c = cs.c[1] + c * cs.cstride[1] + (long long)j * R2;  // S(al, be) = G1c[al s1 + be]
            if (staged) {
                for (int e = tid; e < R1 * R2; e += kSliceThreads) {
                    const int al = e / R2, be = e - al * R2;
                    S_lds[e] = G1c[al * s1 + be];
                }
            }
            __syncthreads();
            const double *S = staged ? S_lds : G1c;
            const long long sS = staged ? R2 : s1;
            const double *G0 = cs.c[0] + c * cs.cstride[0];
            const double *G2 = cs.c[2] + c * cs.cstride[2];
            for (int q = w; q < np; q += kSliceThreads / kWave) {
                const int p = pair_pt[q], sh = pair_s[q];
                const int i0 = probe_coord(seed, (long long)p * 3, N0), i2 = probe_coord(seed, (long long)p * 3 + 2, N2);
                const int i1 = probe_coord(seed, (long long)p * 3 + 1, N1);
                const double *g0 = G0 + (long long)i0 * R1;
                const bool centre = sh == 3;
                double val = 0.0, l2[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                int k2[7];
#pragma unroll
                for (int qq = 0; qq < 7; ++qq) k2[qq] = ghost_map(i2 + qq - 3, N2, g.bc[2]);
                double g2c = 0.0;  // G2(be, i2) of this lane's be (R2 <= 64: every be has its lane)
                for (int be0 = 0; be0 < R2; be0 += kWave) {
                    const int be = be0 + lane;
                    double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
                    for (int al0 = 0; al0 < R1; al0 += kWave) {
                        const double gv = al0 + lane < R1 ? g0[al0 + lane] : 0.0;
                        const int na = min(kWave, R1 - al0);
                        int a = 0;
#pragma unroll 4
                        for (; a + 3 < na; a += 4) {
                            const double x0 = readlane_d(gv, a), x1 = readlane_d(gv, a + 1);
                            const double x2 = readlane_d(gv, a + 2), x3 = readlane_d(gv, a + 3);
                            if (be < R2) {
                                t0 = fma(x0, S[(al0 + a) * sS + be], t0);
                                t1 = fma(x1, S[(al0 + a + 1) * sS + be], t1);
                                t2 = fma(x2, S[(al0 + a + 2) * sS + be], t2);
                                t3 = fma(x3, S[(al0 + a + 3) * sS + be], t3);
                            }
                        }
                        for (; a < na; ++a) {
                            const double x0 = readlane_d(gv, a);
                            if (be < R2) t0 = fma(x0, S[(al0 + a) * sS + be], t0);
                        }
                    }
                    if (be >= R2) continue;
                    const double t = (t0 + t1) + (t2 + t3);
                    const double *g2 = G2 + (long long)be * N2;
                    const double g2v = g2[i2];
                    if (be0 == 0) g2c = g2v;
                    val = fma(t, g2v, val);
                    if (centre)
#pragma unroll
                        for (int qq = 0; qq < 7; ++qq) l2[qq] = fma(t, g2[k2[qq]], l2[qq]);
                }
                val = wave_sum_d(val);
                if (lane == 0) ust[((long long)(7 + sh) * NC + c) * npts + p] = ghost_fix<double>(g, 1, i1 + sh - 3, c, val);
                if (!centre) continue;
#pragma unroll
                for (int qq = 0; qq < 7; ++qq) {
                    const double v2 = wave_sum_d(l2[qq]);
                    if (lane == 0) ust[((long long)(14 + qq) * NC + c) * npts + p] = ghost_fix<double>(g, 2, i2 + qq - 3, c, v2);
                }
                // mode-0 line: w1(al) = S(al, :) . G2(:, i2), lanes over al; G2(:, i2) comes from the
                // lanes that loaded it above when R2 <= 64 (by shuffles), else from memory
                double l0[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                for (int al0 = 0; al0 < R1; al0 += kWave) {
                    const int al = al0 + lane;
                    const double *row = S + (al < R1 ? al : 0) * sS;
                    double w0 = 0.0, w1 = 0.0;
                    if (R2 <= kWave) {
                        int be = 0;
                        for (; be + 1 < R2; be += 2) {
                            const double x0 = readlane_d(g2c, be), x1 = readlane_d(g2c, be + 1);
                            w0 = fma(row[be], x0, w0);
                            w1 = fma(row[be + 1], x1, w1);
                        }
                        if (be < R2) w0 = fma(row[be], readlane_d(g2c, be), w0);
                    } else {
                        for (int be = 0; be < R2; ++be) w0 = fma(row[be], G2[(long long)be * N2 + i2], w0);
                    }
                    if (al >= R1) continue;
                    const double wv = w0 + w1;
#pragma unroll
                    for (int qq = 0; qq < 7; ++qq)
                        l0[qq] = fma(G0[(long long)ghost_map(i0 + qq - 3, N0, g.bc[0]) * R1 + al], wv, l0[qq]);
                }
#pragma unroll
                for (int qq = 0; qq < 7; ++qq) {
                    const double v0 = wave_sum_d(l0[qq]);
                    if (lane == 0) ust[((long long)qq * NC + c) * npts + p] = ghost_fix<double>(g, 0, i0 + qq - 3, c, v0);
                }
            }
            __syncthreads();  // the staged slice is replaced by U^n's, then by the next component's
            // U^n at the centre points (slot 21), its slice H1(:, j, :) staged in the same LDS
            const int S1 = un.R[1], S2 = un.R[2];
            const bool staged_un = use_un && (long long)S1 * S2 <= kSliceLdsDoubles;
            const long long t1g = (long long)N1 * S2;
            const double *H1g = use_un ? un.c[1] + c * un.cstride[1] + (long long)j * S2 : nullptr;
            if (staged_un) {
                for (int e = tid; e < S1 * S2; e += kSliceThreads) {
                    const int al = e / S2, be = e - al * S2;
                    S_lds[e] = H1g[al * t1g + be];
                }
            }
            __syncthreads();
            const double *H1 = staged_un ? S_lds : H1g;
            const long long t1s = staged_un ? S2 : t1g;
            for (int q = w; q < np; q += kSliceThreads / kWave) {
                if (pair_s[q] != 3) continue;
                const int p = pair_pt[q];
                double unv = 0.0;
                if (use_un) {
                    const int i0 = probe_coord(seed, (long long)p * 3, N0), i2 = probe_coord(seed, (long long)p * 3 + 2, N2);
                    const double *H0 = un.c[0] + c * un.cstride[0] + (long long)i0 * S1;
                    const double *H2 = un.c[2] + c * un.cstride[2];
                    for (int be0 = 0; be0 < S2; be0 += kWave) {
                        const int be = be0 + lane, bq = be < S2 ? be : 0;
                        double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
                        for (int al0 = 0; al0 < S1; al0 += kWave) {
                            const double hv = al0 + lane < S1 ? H0[al0 + lane] : 0.0;
                            const int na = min(kWave, S1 - al0);
                            int a = 0;
                            for (; a + 3 < na; a += 4) {
                                t0 = fma(readlane_d(hv, a), H1[(al0 + a) * t1s + bq], t0);
                                t1 = fma(readlane_d(hv, a + 1), H1[(al0 + a + 1) * t1s + bq], t1);
                                t2 = fma(readlane_d(hv, a + 2), H1[(al0 + a + 2) * t1s + bq], t2);
                                t3 = fma(readlane_d(hv, a + 3), H1[(al0 + a + 3) * t1s + bq], t3);
                            }
                            for (; a < na; ++a) t0 = fma(readlane_d(hv, a), H1[(al0 + a) * t1s + bq], t0);
                        }
                        if (be < S2) unv = fma((t0 + t1) + (t2 + t3), H2[(long long)be * N2 + i2], unv);
                    }
                    unv = wave_sum_d(unv);
                }
                if (lane == 0) ust[((long long)21 * NC + c) * npts + p] = unv;
            }
            __syncthreads();
        }
    }
}

// One point per DG lanes (2 in 2D; 4 in 3D, one idle), 256 / DG points per workgroup: lane d
// forms the flux difference along direction d and a share of the flux TT's rank sum at the
// point; the group adds both by shuffles and its first lane forms the residual terms. One
// partial pair per workgroup (sample_stage_blocks of them). Launched for 2D states; 3D states
// take k_sample_stage3 below, one wave per point.
template <int ND, int LW>
__global__ __launch_bounds__(256) void k_sample_stage(FiberGeom g, CoreSet fs, int npts, unsigned long long seed,
                                                       const double *__restrict__ ust, double wn, double wx, double wl,
                                                       StageArgsT<double> hs, double *__restrict__ acc,
                                                       int *__restrict__ flags) {
    constexpr int NC = LawNC<ND, LW>::v, DG = ND == 2 ? 2 : 4;
    __shared__ double red[2][4];
    const int pt = blockIdx.x * (256 / DG) + threadIdx.x / DG, d = threadIdx.x % DG;
    double d2 = 0.0, n2 = 0.0;
    bool ok = true;
    if (pt < npts) {  // the lanes of a point are alive together
        const double *u = ust + pt;  // slot q, component c at u[(q * NC + c) * npts]
        double L[NC], approx[NC];
        for (int c = 0; c < NC; ++c) L[c] = approx[c] = 0.0;
        if (d < ND) {
            double v[NC][7];
            for (int s = 0; s < 7; ++s)
                for (int c = 0; c < NC; ++c) v[c][s] = u[((long long)(d * 7 + s) * NC + c) * npts];
            const double eps = d == 0 ? hs.eps_w[0] : (d == 1 ? hs.eps_w[1] : hs.eps_w[ND - 1]);
            const double ih = d == 0 ? hs.inv_h[0] : (d == 1 ? hs.inv_h[1] : hs.inv_h[ND - 1]);
            ok = stage_dir<ND, LW, double>(v, d, g.gamma - 1.0, geom_alpha(g), eps, ih, L);
        }
        int m[ND];
        for (int dd = 0; dd < ND; ++dd) m[dd] = probe_coord(seed, (long long)pt * ND + dd, g.n[dd]);
        if (ND == 2) {  // rank terms al = d, d + DG, ...
            const double *g0 = fs.c[0] + (long long)m[0] * fs.R[1];
            const double *g1 = fs.c[1] + (long long)m[1] * NC;
            const long long st1 = (long long)fs.N[1] * NC;
            for (int al = d; al < fs.R[1]; al += DG) {
                const double l0 = g0[al];
                const double *a0 = g1 + al * st1;
                for (int c = 0; c < NC; ++c) approx[c] = fma(l0, a0[c], approx[c]);
            }
        } else {  // right rank terms be = d, d + DG, ...
            for (int be = d; be < fs.R[2]; be += DG) {
                double v = 0.0;
                for (int al = 0; al < fs.R[1]; ++al)
                    v += fs.c[0][(long long)m[0] * fs.R[1] + al] * fs.c[1][((long long)al * fs.N[1] + m[1]) * fs.R[2] + be];
                const double *last = fs.c[2] + ((long long)be * fs.N[2] + m[2]) * NC;
                for (int c = 0; c < NC; ++c) approx[c] += v * last[c];
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int off = 1; off < DG; off <<= 1) {
                L[c] += __shfl_xor(L[c], off, kWave);
                approx[c] += __shfl_xor(approx[c], off, kWave);
            }
        if (d == 0)
            for (int c = 0; c < NC; ++c) {
                double ex = wx * u[((long long)3 * NC + c) * npts] + wl * L[c] +
                            (wn != 0.0 ? wn * u[((long long)7 * ND * NC + c) * npts] : 0.0);
                d2 += (ex - approx[c]) * (ex - approx[c]);
                n2 += ex * ex;
            }
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
        d2 += __shfl_xor(d2, off, kWave);
        n2 += __shfl_xor(n2, off, kWave);
    }
    if (threadIdx.x % kWave == 0) { red[0][threadIdx.x / kWave] = d2; red[1][threadIdx.x / kWave] = n2; }
    __syncthreads();
    if (threadIdx.x == 0) {
        acc[2 * blockIdx.x] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        acc[2 * blockIdx.x + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    }
    if (!ok) atomicOr(flags, kFlagNonPhys);
}

// The same residual partials in 3D with one wave per point (the waves of at most
// kStageSampleBlocks workgroups take the points in grid-stride order): its lanes run over the
// right rank index be of the candidate's value sum_be (sum_al G0(m0, al) G1(al, m1, be))
// G2(be, m2, :), so that the rows of G1 are read coalesced and 4096 points keep the device busy;
// lanes 0-2 form the flux differences along the three directions from the point's star samples
// and sum them in the order of the four-lane form. Each be-sum is formed as there; the sums over
// be and over the points are grouped differently.
template <int LW>
__global__ __launch_bounds__(256) void k_sample_stage3(FiberGeom g, CoreSet fs, int npts, unsigned long long seed,
                                                       const double *__restrict__ ust, double wn, double wx, double wl,
                                                       StageArgsT<double> hs, double *__restrict__ acc,
                                                       int *__restrict__ flags) {
    constexpr int NC = LawNC<3, LW>::v;
    __shared__ double red[2][4];
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave, nw = gridDim.x * (256 / kWave);
    const int R1 = fs.R[1], R2 = fs.R[2], N1 = fs.N[1], N2 = fs.N[2];
    double d2 = 0.0, n2 = 0.0;  // lane 0 of each wave
    bool ok = true;
    for (int pt = blockIdx.x * (256 / kWave) + w; pt < npts; pt += nw) {
        const double *u = ust + pt;  // slot q, component c at u[(q * NC + c) * npts]
        double L[NC], approx[NC];
        for (int c = 0; c < NC; ++c) L[c] = approx[c] = 0.0;
        if (lane < 3) {
            double v[NC][7];
            for (int s = 0; s < 7; ++s)
                for (int c = 0; c < NC; ++c) v[c][s] = u[((long long)(lane * 7 + s) * NC + c) * npts];
            // the direction's operands by comparisons (a per-lane index would go through scratch)
            const double eps = lane == 0 ? hs.eps_w[0] : (lane == 1 ? hs.eps_w[1] : hs.eps_w[2]);
            const double ih = lane == 0 ? hs.inv_h[0] : (lane == 1 ? hs.inv_h[1] : hs.inv_h[2]);
            const bool okd = stage_dir<3, LW, double>(v, lane, g.gamma - 1.0, geom_alpha(g), eps, ih, L);
            ok = ok && okd;
        }
        const int m0 = probe_coord(seed, (long long)pt * 3, g.n[0]), m1 = probe_coord(seed, (long long)pt * 3 + 1, g.n[1]),
                  m2 = probe_coord(seed, (long long)pt * 3 + 2, g.n[2]);
        const double *g0 = fs.c[0] + (long long)m0 * R1;
        for (int be0 = 0; be0 < R2; be0 += kWave) {
            const int be = be0 + lane;
            if (be >= R2) continue;
            double v = 0.0;
            for (int al = 0; al < R1; ++al) v += g0[al] * fs.c[1][((long long)al * N1 + m1) * R2 + be];
            const double *last = fs.c[2] + ((long long)be * N2 + m2) * NC;
            for (int c = 0; c < NC; ++c) approx[c] += v * last[c];
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            for (int off = 1; off < 4; off <<= 1) L[c] += __shfl_xor(L[c], off, kWave);
            approx[c] = wave_sum_d(approx[c]);
        }
        if (lane == 0)
            for (int c = 0; c < NC; ++c) {
                double ex = wx * u[((long long)3 * NC + c) * npts] + wl * L[c] +
                            (wn != 0.0 ? wn * u[((long long)7 * 3 * NC + c) * npts] : 0.0);
                d2 += (ex - approx[c]) * (ex - approx[c]);
                n2 += ex * ex;
            }
    }
    if (lane == 0) { red[0][w] = d2; red[1][w] = n2; }
    __syncthreads();
    if (threadIdx.x == 0) {
        acc[2 * blockIdx.x] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        acc[2 * blockIdx.x + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    }
    if (!ok) atomicOr(flags, kFlagNonPhys);
}

inline unsigned cdiv(long long a, long long b) { return (unsigned)((a + b - 1) / b); }

// Gathered block values of the cells on an inflow side (Sec. 4.5.2): for every listed pair
// (shift s, pivot t, side) of the left (right = 0: t indexes a) or right (right = 1: t indexes b)
// interface, W[c][s][a][i][b] = the side's conserved inflow state for all i and the other pivot.
// Component stride cs, shift stride ss, block p x Nk x q.
template <typename T>
__global__ void k_inflow_fill(FiberGeom g, int mode, int npairs, const int *__restrict__ pairs, int right, int p,
                              int Nk, int q, long long cs, long long ss, T *__restrict__ W) {
    const long long per = right ? (long long)p * Nk : (long long)Nk * q;
    const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e >= (long long)npairs * g.ncomp * per) return;
    const long long r = e % per;
    const int c = (int)((e / per) % g.ncomp);
    const int pr = (int)(e / (per * g.ncomp));
    const int s = pairs[3 * pr], t = pairs[3 * pr + 1], side = pairs[3 * pr + 2];
    long long off;
    if (right) off = r * q + t;                          // r = a Nk + i
    else off = ((long long)t * Nk + r / q) * q + r % q;  // r = i q + b
    W[c * cs + s * ss + off] = T(g.qin[mode][side][c]);
}

}  // namespace

template <typename T>
void inflow_fill(hipStream_t s, const FiberGeom &g, int mode, int npairs, const int *pairs, bool right, int p, int Nk,
                 int q, long long cs, long long ss, T *W) {
    const long long per = right ? (long long)p * Nk : (long long)Nk * q;
    const long long tot = (long long)npairs * g.ncomp * per;
    if (tot == 0) return;
    k_inflow_fill<T><<<cdiv(tot, 256), 256, 0, s>>>(g, mode, npairs, pairs, right ? 1 : 0, p, Nk, q, cs, ss, W);
    WTT_HIP(hipGetLastError());
}
template void inflow_fill<double>(hipStream_t, const FiberGeom &, int, int, const int *, bool, int, int, int,
                                  long long, long long, double *);
template void inflow_fill<float>(hipStream_t, const FiberGeom &, int, int, const int *, bool, int, int, int,
                                 long long, long long, float *);

void iface(hipStream_t s, const FiberGeom &g, int side, const double *const *cores, const int *ranks, int count,
           const int *idx, int S, int shift_mode, double *out) {
    int modes[kMaxDim];
    for (int k = 0; k < g.d; ++k) modes[k] = g.n[k];
    CoreSet cs = make_coreset(g, cores, ranks, modes);
    int Rout = side == 0 ? ranks[g.k] : ranks[g.k + 1];
    long long tot = (long long)g.ncomp * S * count * Rout;
    if (tot == 0) return;
    k_iface<<<cdiv(tot, 256), 256, 0, s>>>(g, cs, side, count, idx, S, shift_mode, out);
    WTT_HIP(hipGetLastError());
}

void iface_batch(hipStream_t s, const FiberGeom &g, int n, const IfaceReq *req) {
    WTT_REQUIRE(n >= 0 && n <= kMaxIfaceJobs, WENOTT_EINVAL, "too many interface matrices in one launch");
    int modes[kMaxDim];
    for (int k = 0; k < g.d; ++k) modes[k] = g.n[k];
    IfaceBatch b{};
    long long blocks = 0;
    for (int q = 0; q < n; ++q) {
        const IfaceReq &r = req[q];
        IfaceJob &J = b.job[b.n];
        J.cs = make_coreset(g, r.cores, r.ranks, modes);
        J.idx = r.idx; J.out = r.out; J.side = r.side; J.count = r.count; J.S = r.S; J.shift_mode = r.shift_mode;
        const int Rout = r.side == 0 ? r.ranks[g.k] : r.ranks[g.k + 1];
        const long long tot = (long long)g.ncomp * r.S * r.count * Rout;
        if (tot == 0) continue;
        b.first[b.n] = (int)blocks;
        blocks += cdiv(tot, 256);
        ++b.n;
    }
    if (b.n == 0) return;
    WTT_REQUIRE(blocks < (1LL << 31), WENOTT_EINVAL, "interface matrices too large");
    b.first[b.n] = (int)blocks;
    k_iface_batch<<<(unsigned)blocks, 256, 0, s>>>(g, b);
    WTT_HIP(hipGetLastError());
}

template <typename T>
void weno_block(hipStream_t s, const FiberGeom &g, int p, int q, const T *W, double *out, long long sa, long long si,
                long long sb, long long sc, int *flags) {
    const int M = g.k == g.dir ? g.n[g.k] + 1 : g.n[g.k];
    long long tot = (long long)p * M * q;
    if (tot == 0) return;
#define WTT_WENO(ND_, LW_) k_weno<ND_, LW_, T><<<cdiv(tot, 256), 256, 0, s>>>(g, p, M, q, W, out, sa, si, sb, sc, flags)
    if (g.law == kLawEuler) {
        if (g.d == 2) WTT_WENO(2, kLawEuler); else WTT_WENO(3, kLawEuler);
    } else if (g.law == kLawLinAdv) {
        if (g.d == 2) WTT_WENO(2, kLawLinAdv); else WTT_WENO(3, kLawLinAdv);
    } else {
        if (g.d == 2) WTT_WENO(2, kLawBurgers); else WTT_WENO(3, kLawBurgers);
    }
#undef WTT_WENO
    WTT_HIP(hipGetLastError());
}
template void weno_block<double>(hipStream_t, const FiberGeom &, int, int, const double *, double *, long long,
                                 long long, long long, long long, int *);
template void weno_block<float>(hipStream_t, const FiberGeom &, int, int, const float *, double *, long long,
                                long long, long long, long long, int *);

// Rows per workgroup of k_alpha_eval: enough workgroups (about 2048) to fill the device, at most
// 64 rows each and at most 48 KB of staged rows (5 components x R doubles a row).
int alpha_rows_per_block(long long nrows, int R, int nlast) {
    const long long gx = (long long)cdiv(nlast, 256);
    const long long cap = std::min(64LL, 6144LL / (5LL * std::max(R, 1)));
    return (int)std::max(1LL, std::min(cap, nrows * gx / 2048));
}

// k_alpha_eval serves mode 1 when the rank fits its registers and each thread sweeps rows
// enough (four or more) to repay holding the column.
bool alpha_reg_path(int mode, long long nrows, int R, int nlast) {
    return mode == 1 && R <= 32 && alpha_rows_per_block(nrows, R, nlast) >= 4;
}

int dense_eval_blocks(int mode, long long nrows, int R, int nlast) {
    if (alpha_reg_path(mode, nrows, R, nlast))
        return (int)((long long)cdiv(nlast, 256) * (long long)cdiv(nrows, alpha_rows_per_block(nrows, R, nlast)));
    return (int)cdiv(nrows * nlast, 256);
}

template <int ND, int LW>
void launch_alpha_eval(hipStream_t s, long long nrows, int R, int nlast, const double *Lm, long long lm_stride,
                       const double *G, long long g_stride, double gamma, double *partial, int *flags) {
    const int RB = alpha_rows_per_block(nrows, R, nlast);
    const dim3 grid((unsigned)cdiv(nlast, 256), (unsigned)cdiv(nrows, RB));
    const size_t lds = sizeof(double) * (size_t)LawNC<ND, LW>::v * RB * R;  // <= 48 KB
#define WTT_ALPHA(RM_, EX_) \
    k_alpha_eval<ND, LW, RM_, EX_><<<grid, 256, lds, s>>>(nrows, R, nlast, RB, Lm, lm_stride, G, g_stride, gamma, partial, flags)
    switch (R) {
    case 1: WTT_ALPHA(1, true); break;
    case 2: WTT_ALPHA(2, true); break;
    case 3: WTT_ALPHA(3, true); break;
    case 4: WTT_ALPHA(4, true); break;
    case 5: WTT_ALPHA(5, true); break;
    case 6: WTT_ALPHA(6, true); break;
    case 7: WTT_ALPHA(7, true); break;
    case 8: WTT_ALPHA(8, true); break;
    default:
        if (R <= 16) WTT_ALPHA(16, false);
        else WTT_ALPHA(32, false);
    }
#undef WTT_ALPHA
}

template <int LW>
void dense_eval_t(hipStream_t s, int mode, int d, long long nrows, int R, int nlast, const double *Lm,
                  long long lm_stride, const double *G, long long g_stride, double gamma, double *out, double *partial,
                  int nblocks, int *flags) {
    if (alpha_reg_path(mode, nrows, R, nlast)) {
        if (d == 2) launch_alpha_eval<2, LW>(s, nrows, R, nlast, Lm, lm_stride, G, g_stride, gamma, partial, flags);
        else launch_alpha_eval<3, LW>(s, nrows, R, nlast, Lm, lm_stride, G, g_stride, gamma, partial, flags);
        WTT_HIP(hipGetLastError());
        return;
    }
    if (d == 2)
        k_dense_eval<2, LW><<<nblocks, 256, 0, s>>>(mode, nrows, R, nlast, Lm, lm_stride, G, g_stride, gamma, out,
                                                    partial, flags);
    else
        k_dense_eval<3, LW><<<nblocks, 256, 0, s>>>(mode, nrows, R, nlast, Lm, lm_stride, G, g_stride, gamma, out,
                                                    partial, flags);
    WTT_HIP(hipGetLastError());
}

void dense_eval(hipStream_t s, int mode, int d, int law, long long nrows, int R, int nlast, const double *Lm,
                long long lm_stride, const double *G, long long g_stride, double gamma, double *out, double *partial,
                int nblocks, int *flags) {
    WTT_REQUIRE(dense_eval_blocks(mode, nrows, R, nlast) == nblocks, WENOTT_EINVAL, "dense_eval block count");
    WTT_REQUIRE(mode == 0 || law != kLawLinAdv, WENOTT_EINVAL, "linear advection has no wave-speed evaluation");
    // the scalar laws share the one-component evaluation (the speed of mode 1 is Burgers')
    if (law == kLawEuler)
        dense_eval_t<kLawEuler>(s, mode, d, nrows, R, nlast, Lm, lm_stride, G, g_stride, gamma, out, partial, nblocks,
                                flags);
    else
        dense_eval_t<kLawBurgers>(s, mode, d, nrows, R, nlast, Lm, lm_stride, G, g_stride, gamma, out, partial,
                                  nblocks, flags);
}

void reduce_max_dev(hipStream_t s, const double *partial, int n, double *dst) {
    k_reduce_max<<<1, 1024, 0, s>>>(partial, n, dst);
    WTT_HIP(hipGetLastError());
}

void sample_residual(hipStream_t s, const FiberGeom &g, const double *const *ucores, const int *ranks, int npts,
                     const int *pts, const double *const *fcores, const int *franks, double *ustencil, double *acc,
                     int *flags) {
    int modes[kMaxDim], fmodes[kMaxDim];
    for (int k = 0; k < g.d; ++k) {
        modes[k] = g.n[k];
        fmodes[k] = g.n[k] + (k == g.dir ? 1 : 0);
    }
    CoreSet us = make_coreset(g, ucores, ranks, modes);
    CoreSet fs{};
    for (int k = 0; k <= g.d; ++k) fs.R[k] = franks[k];
    for (int k = 0; k < g.d; ++k) {
        fs.c[k] = fcores[k];
        fs.N[k] = fmodes[k];
        fs.cstride[k] = 0;
    }
    long long n1 = (long long)npts * 6 * g.ncomp;
    if (g.d == 2) k_sample_state<2><<<cdiv(n1, 256), 256, 0, s>>>(g, us, npts, pts, ustencil);
    else k_sample_state<3><<<cdiv(n1, 256), 256, 0, s>>>(g, us, npts, pts, ustencil);
#define WTT_SFLUX(ND_, LW_) \
    k_sample_flux<ND_, LW_><<<cdiv(npts, 256), 256, 0, s>>>(g, fs, npts, pts, ustencil, acc, flags)
    if (g.law == kLawEuler) {
        if (g.d == 2) WTT_SFLUX(2, kLawEuler); else WTT_SFLUX(3, kLawEuler);
    } else if (g.law == kLawLinAdv) {
        if (g.d == 2) WTT_SFLUX(2, kLawLinAdv); else WTT_SFLUX(3, kLawLinAdv);
    } else {
        if (g.d == 2) WTT_SFLUX(2, kLawBurgers); else WTT_SFLUX(3, kLawBurgers);
    }
#undef WTT_SFLUX
    WTT_HIP(hipGetLastError());
}


void lf_block(hipStream_t s, const FiberGeom &g, int p, int q, const double *W0, long long cs, double *out,
              long long sa, long long si, long long sb, long long sc, int *flags) {
    const long long tot = (long long)p * g.n[g.k] * q;
    if (tot == 0) return;
#define WTT_LF(ND_, LW_) k_lf<ND_, LW_><<<cdiv(tot, 256), 256, 0, s>>>(g, p, q, W0, cs, out, sa, si, sb, sc, flags)
    if (g.law == kLawEuler) {
        if (g.d == 2) WTT_LF(2, kLawEuler); else WTT_LF(3, kLawEuler);
    } else if (g.law == kLawLinAdv) {
        if (g.d == 2) WTT_LF(2, kLawLinAdv); else WTT_LF(3, kLawLinAdv);
    } else {
        if (g.d == 2) WTT_LF(2, kLawBurgers); else WTT_LF(3, kLawBurgers);
    }
#undef WTT_LF
    WTT_HIP(hipGetLastError());
}

void sample_lf_residual(hipStream_t s, const FiberGeom &g, const double *const *ucores, const int *ranks, int npts,
                        const int *pts, const double *const *fcores, const int *franks, double *ustencil, double *acc,
                        int *flags) {
    int modes[kMaxDim];
    for (int k = 0; k < g.d; ++k) modes[k] = g.n[k];
    CoreSet us = make_coreset(g, ucores, ranks, modes);
    CoreSet fs{};
    for (int k = 0; k <= g.d; ++k) fs.R[k] = franks[k];
    for (int k = 0; k < g.d; ++k) {
        fs.c[k] = fcores[k];
        fs.N[k] = modes[k];
        fs.cstride[k] = 0;
    }
    const long long n1 = (long long)npts * 6 * g.ncomp;
    if (g.d == 2) k_sample_state<2><<<cdiv(n1, 256), 256, 0, s>>>(g, us, npts, pts, ustencil);
    else k_sample_state<3><<<cdiv(n1, 256), 256, 0, s>>>(g, us, npts, pts, ustencil);
#define WTT_SLF(ND_, LW_) k_sample_lf<ND_, LW_><<<cdiv(npts, 256), 256, 0, s>>>(g, fs, npts, pts, ustencil, acc, flags)
    if (g.law == kLawEuler) {
        if (g.d == 2) WTT_SLF(2, kLawEuler); else WTT_SLF(3, kLawEuler);
    } else if (g.law == kLawLinAdv) {
        if (g.d == 2) WTT_SLF(2, kLawLinAdv); else WTT_SLF(3, kLawLinAdv);
    } else {
        if (g.d == 2) WTT_SLF(2, kLawBurgers); else WTT_SLF(3, kLawBurgers);
    }
#undef WTT_SLF
    WTT_HIP(hipGetLastError());
}

template <typename T>
void stage_block(hipStream_t s, const FiberGeom &g, int p, int q, const StageArgsT<T> &a, double *out, long long sa,
                 long long si, long long sb, long long sc, int *flags) {
    long long tot = (long long)p * g.n[g.k] * q;
    if (tot == 0) return;
    const bool split = tot < (1LL << 17);  // fewer points than ~512 workgroups of one point per thread
#define WTT_STAGE(ND_, LW_)                                                                                    \
    if (split) k_stage<ND_, LW_, ND_ == 2 ? 2 : 4, T><<<cdiv((ND_ == 2 ? 2 : 4) * tot, 256), 256, 0, s>>>(      \
                   g, p, q, a, out, sa, si, sb, sc, flags);                                                    \
    else k_stage<ND_, LW_, 1, T><<<cdiv(tot, 256), 256, 0, s>>>(g, p, q, a, out, sa, si, sb, sc, flags)
    if (g.law == kLawEuler) {
        if (g.d == 2) { WTT_STAGE(2, kLawEuler); } else { WTT_STAGE(3, kLawEuler); }
    } else if (g.law == kLawLinAdv) {
        if (g.d == 2) { WTT_STAGE(2, kLawLinAdv); } else { WTT_STAGE(3, kLawLinAdv); }
    } else {
        if (g.d == 2) { WTT_STAGE(2, kLawBurgers); } else { WTT_STAGE(3, kLawBurgers); }
    }
#undef WTT_STAGE
    WTT_HIP(hipGetLastError());
}
template void stage_block<double>(hipStream_t, const FiberGeom &, int, int, const StageArgsT<double> &, double *,
                                  long long, long long, long long, long long, int *);
template void stage_block<float>(hipStream_t, const FiberGeom &, int, int, const StageArgsT<float> &, double *,
                                 long long, long long, long long, long long, int *);

// partials of the sampled stage residual: 2D, one workgroup per 128 points (two lanes each);
// 3D, one wave per point over at most kStageSampleBlocks workgroups of four waves
constexpr int kStageSampleBlocks = 256;
int sample_stage_blocks(int d, int npts) {
    if (d == 2) return (int)cdiv((long long)npts * 2, 256);
    return (int)std::min<long long>(kStageSampleBlocks, cdiv(npts, 256 / kWave));
}

void sample_stage(hipStream_t s, const FiberGeom &g, const double *const *xcores, const int *xranks,
                  const double *const *ncores, const int *nranks, int npts, unsigned long long seed,
                  const double *const *fcores, const int *franks, double wn, double wx, double wl,
                  const double *inv_h, const double *eps_w, double *ust, double *acc, int *flags) {
    int modes[kMaxDim];
    for (int k = 0; k < g.d; ++k) modes[k] = g.n[k];
    CoreSet xs = make_coreset(g, xcores, xranks, modes);
    CoreSet us = ncores ? make_coreset(g, ncores, nranks, modes) : xs;
    CoreSet fs{};
    for (int k = 0; k <= g.d; ++k) fs.R[k] = franks[k];
    for (int k = 0; k < g.d; ++k) {
        fs.c[k] = fcores[k];
        fs.N[k] = modes[k];
        fs.cstride[k] = 0;
    }
    StageArgsT<double> hs{};
    for (int k = 0; k < g.d; ++k) { hs.inv_h[k] = inv_h[k]; hs.eps_w[k] = eps_w[k]; }
    const int SL = 7 * g.d + 1;
    long long n1 = (long long)npts * SL * g.ncomp;
    if (g.d == 2) {
        k_sample_star<2><<<cdiv(n1, 256), 256, 0, s>>>(g, xs, us, ncores != nullptr, npts, seed, ust);
    } else {
        // the slice form pays off once a cell costs more than a few hundred multiply-adds
        // (R1 R2); below that one thread per sample value is faster
        if ((long long)xs.R[1] * xs.R[2] > 512)
            k_sample_slices3<<<g.n[1], kSliceThreads,
                               slice_lds_bytes((long long)xs.R[1] * xs.R[2],
                                               ncores ? (long long)us.R[1] * us.R[2] : 0),
                               s>>>(g, xs, us, ncores != nullptr, npts, seed, ust);
        else
            k_sample_star<3><<<cdiv(n1, 256), 256, 0, s>>>(g, xs, us, ncores != nullptr, npts, seed, ust);
    }
    const unsigned nb = sample_stage_blocks(g.d, npts);
#define WTT_SSTAGE2(LW_) k_sample_stage<2, LW_><<<nb, 256, 0, s>>>(g, fs, npts, seed, ust, wn, wx, wl, hs, acc, flags)
#define WTT_SSTAGE3(LW_) k_sample_stage3<LW_><<<nb, 256, 0, s>>>(g, fs, npts, seed, ust, wn, wx, wl, hs, acc, flags)
    if (g.law == kLawEuler) {
        if (g.d == 2) WTT_SSTAGE2(kLawEuler); else WTT_SSTAGE3(kLawEuler);
    } else if (g.law == kLawLinAdv) {
        if (g.d == 2) WTT_SSTAGE2(kLawLinAdv); else WTT_SSTAGE3(kLawLinAdv);
    } else {
        if (g.d == 2) WTT_SSTAGE2(kLawBurgers); else WTT_SSTAGE3(kLawBurgers);
    }
#undef WTT_SSTAGE2
#undef WTT_SSTAGE3
    WTT_HIP(hipGetLastError());
}

}  // namespace wtt
