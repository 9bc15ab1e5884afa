// Estimated Lax-Friedrichs alpha of a TT state (gfx950).
//
// The scheme needs one global alpha = max over the grid of |u| + a (eq. lax-friedrichs with the
// alpha of Sec. 4.2). The paper does not form it cell by cell: it cross-interpolates the field
// |u| + a and estimates its maximum with the TT-Toolbox's tt_max_abs (Sec. 5.5, eq. cfl-other),
// a search that only visits entries of the tensor. The search here is of that kind and never
// touches all N^d cells: it evaluates |u| + a on whole grid lines (all cells along one mode, the
// other indices fixed) through a set of start cells and climbs coordinate-wise:
//   round 0: lines along the first and the last mode through M random cells and the best cell of
//            the previous search (in 3D also the middle mode through the first few of them);
//   rounds 1, 2: lines along every mode through the K best cells found so far.
// A line costs one vector of partial products (the cores on either side of its mode, taken at the
// start cell) and one contraction per cell, so a search costs O(M N R) instead of O(N^d R). The
// result is a lower bound of the exact maximum and equals it whenever a visited line crosses the
// maximising cell; wenott_info reports the alpha used, so any comparison can use the same value.
// Non-physical cells met on the lines raise the context's flag word like the exact evaluation.
#include "common.h"

namespace wtt {

namespace {

constexpr int kWave = 64;
// threads of the line kernels: one cell of a 512-cell outer line per thread; sixteen waves share a
// middle-line chunk's (cell, component) tasks
constexpr int kOuterThreads = 512, kMidThreads = 1024;

struct LineCores {
    const double *c[kMaxDim];
    long long cs[kMaxDim];  // component stride of core k
    int R[kMaxDim + 1];
    int N[kMaxDim];
};

// max with the smallest index among equal values
__device__ inline void amax_pair(double &v, int &i, double ov, int oi) {
    if (ov > v || (ov == v && oi < i)) { v = ov; i = oi; }
}

// Wave speed of a cell from its conserved values: |u| + a for the Euler law, 0 (and ok = false)
// for a non-physical cell; |u| for Burgers (|f'(u)| of f = u^2 / 2).
template <int ND, int LW>
__device__ inline double cell_speed(const double *q, double gamma, bool &ok) {
    if (LW == kLawBurgers) return fabs(q[0]);
    constexpr int NC = ND + 2;
    const double rho = q[0];
    double u2 = 0.0;
#pragma unroll
    for (int d = 0; d < ND; ++d) u2 += q[1 + d] * q[1 + d];
    u2 /= rho * rho;
    const double p = (gamma - 1.0) * (q[NC - 1] - 0.5 * rho * u2);
    const bool phys = rho > 0.0 && p > 0.0;
    ok = ok && phys;
    return phys ? sqrt(u2) + sqrt(gamma * p / rho) : 0.0;
}

// One workgroup per (start cell, outer mode dd = 0 or d - 1): |u| + a along the line through the
// cell. The other cores at the start cell reduce to one vector per component (R_1 values for
// mode 0, R_{d-1} for the last mode), so each cell of the line is one dot product with a row
// (mode 0) or a column (last mode) of its core. Candidate pt * ND + dd receives the line's largest
// value and its cell; a mode outside mode_mask (or the middle mode) writes -1.
template <int ND, int LW>
__global__ __launch_bounds__(kOuterThreads) void k_alpha_outer(LineCores T, double gamma, int npts,
                                                              const int *__restrict__ pts, int mode_mask,
                                                              double *__restrict__ cval, int *__restrict__ ccell,
                                                              int *__restrict__ flags) {
    constexpr int NC = LawNC<ND, LW>::v;
    extern __shared__ double vec[];  // [NC][R] partial products of the other cores
    __shared__ double wv[kOuterThreads / kWave];
    __shared__ int wi[kOuterThreads / kWave];
    const int pt = blockIdx.x, dd = blockIdx.y, tid = threadIdx.x;
    if (pt >= npts) return;
    const int out = pt * ND + dd;
    int m[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) m[d] = pts[pt * ND + d];
    if (!((mode_mask >> dd) & 1) || (dd != 0 && dd != ND - 1)) {
        if (tid == 0) {
            cval[out] = -1.0;
#pragma unroll
            for (int d = 0; d < ND; ++d) ccell[out * ND + d] = m[d];
        }
        return;
    }
    const bool first = dd == 0;
    const int R = first ? T.R[1] : T.R[ND - 1], Nd = T.N[dd];
    for (int e = tid; e < NC * R; e += kOuterThreads) {
        const int c = e / R, a = e - c * R;
        double v;
        if (first) {  // right part at (m_1, ..., m_{d-1}): G_1(a, m_1, :) [G_2(:, m_2)], R_1 values
            if (ND == 2) {
                v = T.c[1][c * T.cs[1] + (long long)a * T.N[1] + m[1]];
            } else {
                const double *g1 = T.c[1] + c * T.cs[1] + ((long long)a * T.N[1] + m[1]) * T.R[2];
                const double *g2 = T.c[2] + c * T.cs[2] + m[2];
                v = 0.0;
                for (int be = 0; be < T.R[2]; ++be) v = fma(g1[be], g2[(long long)be * T.N[2]], v);
            }
        } else {  // left part at (m_0, ..., m_{d-2}): [G_0(m_0, :)] G_{d-2}(:, m_{d-2}, a)
            if (ND == 2) {
                v = T.c[0][c * T.cs[0] + (long long)m[0] * T.R[1] + a];
            } else {
                const double *g0 = T.c[0] + c * T.cs[0] + (long long)m[0] * T.R[1];
                const double *g1 = T.c[1] + c * T.cs[1] + (long long)m[1] * T.R[2] + a;
                const long long st = (long long)T.N[1] * T.R[2];
                v = 0.0;
                for (int al = 0; al < T.R[1]; ++al) v = fma(g0[al], g1[al * st], v);
            }
        }
        vec[e] = v;
    }
    __syncthreads();
    double best = -1.0;
    int bi = 0;
    bool ok = true;
    for (int i = tid; i < Nd; i += kOuterThreads) {
        double q[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double *vv = vec + c * R;
            double acc0 = 0.0, acc1 = 0.0;
            if (first) {  // row i of G_0: contiguous
                const double *row = T.c[0] + c * T.cs[0] + (long long)i * R;
                int a = 0;
                for (; a + 1 < R; a += 2) {
                    acc0 = fma(row[a], vv[a], acc0);
                    acc1 = fma(row[a + 1], vv[a + 1], acc1);
                }
                if (a < R) acc0 = fma(row[a], vv[a], acc0);
            } else {  // column i of G_{d-1}: consecutive threads read consecutive cells
                const double *col = T.c[ND - 1] + c * T.cs[ND - 1] + i;
                int a = 0;
                for (; a + 1 < R; a += 2) {
                    acc0 = fma(col[(long long)a * Nd], vv[a], acc0);
                    acc1 = fma(col[(long long)(a + 1) * Nd], vv[a + 1], acc1);
                }
                if (a < R) acc0 = fma(col[(long long)a * Nd], vv[a], acc0);
            }
            q[c] = acc0 + acc1;
        }
        const double sp = cell_speed<ND, LW>(q, gamma, ok);
        if (sp > best) { best = sp; bi = i; }
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const double ov = __shfl_xor(best, off, kWave);
        const int oi = __shfl_xor(bi, off, kWave);
        amax_pair(best, bi, ov, oi);
    }
    if (tid % kWave == 0) { wv[tid / kWave] = best; wi[tid / kWave] = bi; }
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < kOuterThreads / kWave; ++w) amax_pair(best, bi, wv[w], wi[w]);
        cval[out] = best;
        m[dd] = bi;
#pragma unroll
        for (int d = 0; d < ND; ++d) ccell[out * ND + d] = m[d];
    }
    if (!ok) atomicOr(flags, kFlagNonPhys);
}

// Lines along the middle mode of a 3D state, in chunks of kMidCells cells: workgroup (pt, chunk).
// A cell's value is l^T G_1(:, j, :) r with l = G_0(m_0, :) and r = G_2(:, m_2): one wave per
// (cell, component), its lanes over the right rank index so that the row reads of the slice are
// contiguous; the chunk's maximum and its cell are candidate pt * nchunk + chunk.
constexpr int kMidCells = 16;
template <int LW>
__global__ __launch_bounds__(kMidThreads) void k_alpha_mid(LineCores T, double gamma, int npts,
                                                            const int *__restrict__ pts, int nchunk,
                                                            double *__restrict__ cval, int *__restrict__ ccell,
                                                            int *__restrict__ flags) {
    constexpr int NC = LawNC<3, LW>::v;
    extern __shared__ double sm[];  // l [NC][R1], r [NC][R2]
    __shared__ double qv[kMidCells][NC];
    const int pt = blockIdx.x, chunk = blockIdx.y, tid = threadIdx.x, lane = tid % kWave, w = tid / kWave;
    const int R1 = T.R[1], R2 = T.R[2], N1 = T.N[1];
    const int m0 = pts[pt * 3], m2 = pts[pt * 3 + 2];
    double *lv = sm, *rv = sm + NC * R1;
    for (int e = tid; e < NC * R1; e += kMidThreads) {
        const int c = e / R1, a = e - c * R1;
        lv[e] = T.c[0][c * T.cs[0] + (long long)m0 * R1 + a];
    }
    for (int e = tid; e < NC * R2; e += kMidThreads) {
        const int c = e / R2, b = e - c * R2;
        rv[e] = T.c[2][c * T.cs[2] + (long long)b * T.N[2] + m2];
    }
    __syncthreads();
    const int j0 = chunk * kMidCells;
    const long long s1 = (long long)N1 * R2;
    for (int task = w; task < kMidCells * NC; task += kMidThreads / kWave) {
        const int jj = task / NC, c = task - jj * NC, j = j0 + jj;
        double acc = 0.0;
        if (j < N1) {
            const double *G = T.c[1] + c * T.cs[1] + (long long)j * R2;
            const double *l = lv + c * R1, *r = rv + c * R2;
            for (int b0 = 0; b0 < R2; b0 += kWave) {
                const int b = b0 + lane;
                if (b >= R2) continue;
                double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
                int a = 0;
                for (; a + 3 < R1; a += 4) {
                    t0 = fma(l[a], G[a * s1 + b], t0);
                    t1 = fma(l[a + 1], G[(a + 1) * s1 + b], t1);
                    t2 = fma(l[a + 2], G[(a + 2) * s1 + b], t2);
                    t3 = fma(l[a + 3], G[(a + 3) * s1 + b], t3);
                }
                for (; a < R1; ++a) t0 = fma(l[a], G[a * s1 + b], t0);
                acc = fma((t0 + t1) + (t2 + t3), r[b], acc);
            }
        }
        for (int off = kWave / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
        if (lane == 0) qv[jj][c] = acc;
    }
    __syncthreads();
    if (tid < kWave) {
        double best = -1.0;
        int bi = j0;
        bool ok = true;
        if (tid < kMidCells && j0 + tid < N1) {
            double q[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) q[c] = qv[tid][c];
            best = cell_speed<3, LW>(q, gamma, ok);
            bi = j0 + tid;
        }
        for (int off = kWave / 2; off > 0; off >>= 1) {
            const double ov = __shfl_xor(best, off, kWave);
            const int oi = __shfl_xor(bi, off, kWave);
            amax_pair(best, bi, ov, oi);
        }
        if (tid == 0) {
            const int out = pt * nchunk + chunk;
            cval[out] = best;
            ccell[out * 3] = m0;
            ccell[out * 3 + 1] = bi;
            ccell[out * 3 + 2] = m2;
        }
        if (!ok) atomicOr(flags, kFlagNonPhys);
    }
}

// Start cells of round 0: cell i is the probe cell (seed, i) of every mode, cell 0 the best cell
// of the previous search when there is one (best[0] >= 0).
template <int ND>
__global__ void k_alpha_seed(int npts, int n0, int n1, int n2, unsigned long long seed, const int *__restrict__ best,
                             int *__restrict__ pts) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= npts * ND) return;
    const int i = e / ND, d = e - i * ND;
    const int nd = d == 0 ? n0 : (d == 1 ? n1 : n2);
    pts[e] = (i == 0 && best[0] >= 0) ? best[d] : probe_coord(seed, e, nd);
}

// Wave argmax under amax_pair's order (the largest value, the smallest index among equal ones),
// a total order, so the result does not depend on the order of the comparisons: DPP steps within
// each row of 16 lanes, then the four rows' results through scalar registers; every lane gets
// the result.
__device__ inline void wave_amax(double &v, int &i) {
    amax_pair(v, i, dpp_d<0xB1>(v), dpp_i<0xB1>(i));    // quad_perm [1,0,3,2]
    amax_pair(v, i, dpp_d<0x4E>(v), dpp_i<0x4E>(i));    // quad_perm [2,3,0,1]
    amax_pair(v, i, dpp_d<0x141>(v), dpp_i<0x141>(i));  // row_half_mirror
    amax_pair(v, i, dpp_d<0x140>(v), dpp_i<0x140>(i));  // row_mirror
    double bv = readlane_d(v, 0);
    int bi = __builtin_amdgcn_readlane(i, 0);
#pragma unroll
    for (int r = 16; r < kWave; r += 16) amax_pair(bv, bi, readlane_d(v, r), __builtin_amdgcn_readlane(i, r));
    v = bv;
    i = bi;
}

// One wave: alpha (out[0]) = the largest candidate value (combined with the value already there
// when accumulate), its cell into best[], and the cells of the K largest candidates into
// next[K][ND]. Lane l keeps the largest of its candidates l, l + 64, ... (amax_pair's order); a
// round takes the wave's largest, marks it taken (-3) and lets its owner lane rescan.
template <int ND>
__global__ __launch_bounds__(kWave) void k_alpha_select(int ncand, const double *__restrict__ cval,
                                                        const int *__restrict__ ccell, int K,
                                                        int *__restrict__ next, int *__restrict__ best,
                                                        double *__restrict__ alpha, int accumulate) {
    extern __shared__ double vs[];  // ncand values
    const int lane = threadIdx.x;
    for (int e = lane; e < ncand; e += kWave) vs[e] = cval[e];
    __syncthreads();
    double lv = -2.0;
    int li = 0x7fffffff;
    for (int e = lane; e < ncand; e += kWave) amax_pair(lv, li, vs[e], e);
    for (int k = 0; k < K; ++k) {
        double v = lv;
        int i = li;
        wave_amax(v, i);
        if (i < 0 || i >= ncand) i = 0;
        if (lane == 0) {
#pragma unroll
            for (int d = 0; d < ND; ++d) next[k * ND + d] = ccell[i * ND + d];
            if (k == 0) {
                const double a = fmax(vs[i], 0.0);
                const bool better = !accumulate || a >= alpha[0];
                alpha[0] = accumulate ? fmax(alpha[0], a) : a;
                if (better)
#pragma unroll
                    for (int d = 0; d < ND; ++d) best[d] = ccell[i * ND + d];
            }
        }
        if (lane == i % kWave) {  // the owner of candidate i marks it taken and rescans
            vs[i] = -3.0;
            lv = -2.0;
            li = 0x7fffffff;
            for (int e = lane; e < ncand; e += kWave) amax_pair(lv, li, vs[e], e);
        }
    }
}

inline unsigned cdiv(long long a, long long b) { return (unsigned)((a + b - 1) / b); }

int alpha_mid_chunks(int n1) { return (int)cdiv(n1, kMidCells); }

// candidates of a round: ND per start cell (outer lines) and, in 3D, the middle-line chunks
size_t alpha_cands(int d, int npts, int n1) {
    return (size_t)npts * d + (d == 3 ? (size_t)kAlphaMiddleLines * alpha_mid_chunks(n1) : 0);
}

}  // namespace

size_t alpha_search_ints(int d, int n1) {
    // start cells of round 0 and of the later rounds, candidate cells
    return (size_t)kAlphaStartCells * d + (size_t)kAlphaKeep * d * 2 + alpha_cands(d, kAlphaStartCells, n1) * d + 64;
}
size_t alpha_search_doubles(int d, int n1) { return alpha_cands(d, kAlphaStartCells, n1) + 64; }

namespace {

template <int LW>
void alpha_search_t(hipStream_t s, int d, const int *n, const double *const *cores, const int *ranks, double gamma,
                    unsigned long long seed, int *best, int *wsi, double *wsd, double *alpha, int *flags) {
    LineCores T{};
    for (int k = 0; k <= d; ++k) T.R[k] = ranks[k];
    for (int k = 0; k < d; ++k) {
        T.c[k] = cores[k];
        T.N[k] = n[k];
        T.cs[k] = (long long)ranks[k] * n[k] * ranks[k + 1];
    }
    const size_t nc = d == 2 ? LawNC<2, LW>::v : LawNC<3, LW>::v;
    const size_t lds_outer = sizeof(double) * nc * std::max(ranks[1], ranks[d - 1]);
    const size_t lds_mid = d == 3 ? sizeof(double) * nc * (size_t)(ranks[1] + ranks[2]) : 0;
    WTT_REQUIRE(lds_outer <= 60 * 1024 && lds_mid <= 60 * 1024, WENOTT_EINVAL, "ranks too large for the alpha search");
    const int M = kAlphaStartCells, K = kAlphaKeep, KM = kAlphaMiddleLines;
    const int nchunk = d == 3 ? alpha_mid_chunks(n[1]) : 0;
    int *pts0 = wsi, *pts1 = pts0 + M * d, *pts2 = pts1 + K * d, *ccell = pts2 + K * d;
    double *cval = wsd;
    const int outer = 1 | (1 << (d - 1));
    if (d == 2) k_alpha_seed<2><<<cdiv(M * 2, 256), 256, 0, s>>>(M, n[0], n[1], 1, seed, best, pts0);
    else k_alpha_seed<3><<<cdiv(M * 3, 256), 256, 0, s>>>(M, n[0], n[1], n[2], seed, best, pts0);
    int npts = M;
    int *cur = pts0;
    for (int round = 0; round < kAlphaRounds; ++round) {
        int *nxt = round % 2 == 0 ? pts1 : pts2;
        const int nmid = std::min(npts, KM);
        const int ncand = npts * d + (d == 3 ? nmid * nchunk : 0);
        if (d == 2) {
            k_alpha_outer<2, LW><<<dim3(npts, 2), kOuterThreads, lds_outer, s>>>(T, gamma, npts, cur, outer, cval,
                                                                              ccell, flags);
            k_alpha_select<2><<<1, kWave, sizeof(double) * (size_t)ncand, s>>>(ncand, cval, ccell, K, nxt, best,
                                                                            alpha, round > 0);
        } else {
            k_alpha_outer<3, LW><<<dim3(npts, 3), kOuterThreads, lds_outer, s>>>(T, gamma, npts, cur, outer, cval,
                                                                              ccell, flags);
            k_alpha_mid<LW><<<dim3(nmid, nchunk), kMidThreads, lds_mid, s>>>(T, gamma, nmid, cur, nchunk,
                                                                             cval + npts * 3, ccell + npts * 9, flags);
            k_alpha_select<3><<<1, kWave, sizeof(double) * (size_t)ncand, s>>>(ncand, cval, ccell, K, nxt, best,
                                                                            alpha, round > 0);
        }
        npts = K;
        cur = nxt;
    }
    WTT_HIP(hipGetLastError());
}

}  // namespace

void alpha_search(hipStream_t s, int d, int law, const int *n, const double *const *cores, const int *ranks,
                  double gamma, unsigned long long seed, int *best, int *wsi, double *wsd, double *alpha, int *flags) {
    WTT_REQUIRE(d == 2 || d == 3, WENOTT_EINVAL, "alpha search needs 2 or 3 dimensions");
    WTT_REQUIRE(law == kLawEuler || law == kLawBurgers, WENOTT_EINVAL, "alpha search: no search for this law");
    if (law == kLawEuler) alpha_search_t<kLawEuler>(s, d, n, cores, ranks, gamma, seed, best, wsi, wsd, alpha, flags);
    else alpha_search_t<kLawBurgers>(s, d, n, cores, ranks, gamma, seed, best, wsi, wsd, alpha, flags);
}

}  // namespace wtt
