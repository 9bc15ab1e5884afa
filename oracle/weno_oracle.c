/*
 * Dense finite-difference WENO5-JS + global Lax-Friedrichs + SSP-RK3 solver.
 *
 * TEST INFRASTRUCTURE ONLY. This is the oracle that the tensor-train GPU path is
 * checked against; it shares no code with that path and no product code may call it.
 * It is the paper's "full-tensor" scheme written out plainly in FP64:
 *
 *   - Euler system, physical fluxes F, G, H and the ideal-gas pressure
 *     (Sec. 2.1, eqs. euler-system and physical-fluxes, gamma-law EOS);
 *   - conservative semi-discretisation du_i/dt + (f_{i+1/2} - f_{i-1/2})/dx = 0
 *     (Sec. 2.2, eq. 1d-scalar-h-pde-fd), applied dimension by dimension and
 *     component by component (end of Sec. 2.2);
 *   - Lax-Friedrichs splitting f^{+-} = (f +- alpha u)/2 (eq. lax-friedrichs) with one
 *     global alpha = max(|u| + a) per stage (Sec. 4.2 defines alpha_TT = max(|u|+a));
 *   - WENO5-JS candidate polynomials, smoothness indicators, linear weights
 *     d = (3/10, 3/5, 1/10) and eps = dx^2 (Sec. 2.2); the f^- side is the mirror image
 *     of the f^+ side (the paper defers it to Shu 1998);
 *   - SSP-RK3 in Shu-Osher form (Sec. 2.2 and Sec. 4.4, eq. tt-ssprk3 without rounding);
 *   - ghost layers of three cells per side (Sec. 4.5): periodic copies (Sec. 4.5.1); a
 *     symmetry plane mirrors the interior cells with the momentum normal to it negated
 *     (Sec. 4.5.3); an inflow side holds a constant state in its ghost cells, the full-tensor
 *     value of the paper's zeroed ghost slices plus the rank-1 boundary TT (Sec. 4.5.2); for
 *     the transmissive boundaries the paper does not describe, zero-order extrapolation.
 *
 * Two scalar laws are included for the paper's Tables 1 and 2: 3D linear advection
 * u_t + u_x + u_y + u_z = 0 and 3D Burgers u_t + u u_x + u u_y + u u_z = 0 (Sec. 5.1, 5.2).
 *
 * Storage: U[c][i0][i1][i2] in C order over the ndim grid dimensions (last fastest),
 * interior cells only; ghosts are index maps.
 *
 * Built with -O3 -ffp-contract=off so that every run is reproducible to the bit.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OR_OK = 0, OR_EINVAL = -1, OR_ENOMEM = -2, OR_ENONPHYS = -5 };
enum { OR_BC_PERIODIC = 0, OR_BC_TRANSMISSIVE = 1, OR_BC_SYMMETRY = 2, OR_BC_INFLOW = 3 };
enum { OR_EULER = 0, OR_LINADV = 1, OR_BURGERS = 2 };

/* Problem description passed from Python (ctypes) as flat arrays. */
typedef struct {
    int model;      /* OR_EULER / OR_LINADV / OR_BURGERS */
    int ndim;       /* 1, 2 or 3 */
    int64_t n[3];   /* interior cells per dimension */
    double h[3];    /* grid spacing per dimension */
    double gamma;   /* ratio of specific heats (Euler only) */
    int bc[3][2];   /* boundary type per dimension and side (0 low, 1 high) */
    double inflow[3][2][5]; /* conserved state of the ghost cells of an inflow side */
} or_problem;

static int ncomp_of(const or_problem *p) { return p->model == OR_EULER ? p->ndim + 2 : 1; }

static int64_t ncell_of(const or_problem *p) {
    int64_t c = 1;
    for (int d = 0; d < p->ndim; ++d) c *= p->n[d];
    return c;
}

/* Interior cell whose values a cell i (-3 <= i < n + 3) of a grid line takes (Sec. 4.5):
 * itself inside; periodic wraps; a symmetry plane mirrors (ghost -1-l <-> interior l at the
 * low side, n+l <-> n-1-l at the high side); transmissive clamps. An inflow ghost takes no
 * interior cell (its state is the side's inflow state); the clamp is returned for it. */
static int64_t ghost_map(int64_t i, int64_t n, const int bc[2]) {
    if (i >= 0 && i < n) return i;
    int b = bc[i >= n];
    if (b == OR_BC_PERIODIC) {
        int64_t r = i % n;
        return r < 0 ? r + n : r;
    }
    if (b == OR_BC_SYMMETRY) return i < 0 ? -1 - i : 2 * n - 1 - i;
    return i < 0 ? 0 : n - 1;
}

/* Conserved state q of cell i along direction dir of the line starting at interior offset
 * base (stride st): the interior values of ghost_map's cell, with the momentum normal to a
 * symmetry plane negated, or the inflow state of an inflow side. */
static void line_state(const or_problem *p, const double *U, int64_t base, int64_t st, int dir, int64_t i,
                       double *q) {
    int ncomp = ncomp_of(p);
    int64_t nc = ncell_of(p), n = p->n[dir];
    int ghost = i < 0 || i >= n, side = i >= n;
    int b = p->bc[dir][side];
    if (ghost && b == OR_BC_INFLOW) {
        for (int c = 0; c < ncomp; ++c) q[c] = p->inflow[dir][side][c];
        return;
    }
    int64_t j = ghost_map(i, n, p->bc[dir]);
    for (int c = 0; c < ncomp; ++c) q[c] = U[(int64_t)c * nc + base + j * st];
    if (ghost && b == OR_BC_SYMMETRY && p->model == OR_EULER) q[1 + dir] = -q[1 + dir];
}

/* Conserved inflow state from the primitive one (rho, u_1..u_ndim, p) by the boundary
 * relations of Sec. 4.5.2: rho u_d = rho_in u_d,in and rho E = p_in / (gamma - 1) +
 * rho_in |u_in|^2 / 2; the scalar laws take u itself. */
void or_inflow_conserved(const or_problem *p, const double *prim, double *q) {
    if (p->model != OR_EULER) { q[0] = prim[0]; return; }
    int nd = p->ndim;
    double rho = prim[0], ke = 0.0;
    q[0] = rho;
    for (int d = 0; d < nd; ++d) {
        q[1 + d] = rho * prim[1 + d];
        ke += rho * prim[1 + d] * prim[1 + d];
    }
    q[nd + 1] = prim[nd + 1] / (p->gamma - 1.0) + 0.5 * ke;
}

/* Pressure from the ideal-gas law p = (gamma-1)(rhoE - |m|^2/(2 rho)) (Sec. 2.1). */
static double pressure(const double *q, int ndim, double gamma) {
    double rho = q[0], m2 = 0.0;
    for (int d = 0; d < ndim; ++d) m2 += q[1 + d] * q[1 + d];
    return (gamma - 1.0) * (q[ndim + 1] - 0.5 * m2 / rho);
}

/* Physical flux along direction dir (eq. physical-fluxes), for one cell state q. */
static void physical_flux(const or_problem *p, const double *q, int dir, double *f) {
    if (p->model == OR_LINADV) { f[0] = q[0]; return; }
    if (p->model == OR_BURGERS) { f[0] = 0.5 * q[0] * q[0]; return; }
    int nd = p->ndim;
    double rho = q[0];
    double un = q[1 + dir] / rho;
    double pr = pressure(q, nd, p->gamma);
    f[0] = q[1 + dir];
    for (int d = 0; d < nd; ++d) f[1 + d] = q[1 + d] * un + (d == dir ? pr : 0.0);
    f[nd + 1] = un * (q[nd + 1] + pr);
}

/* One WENO5-JS reconstruction at x_{i+1/2} from v_{i-2..i+2} (left-biased), Sec. 2.2. */
static double weno5_left(double vm2, double vm1, double v0, double vp1, double vp2, double eps) {
    double q0 = (2.0 * v0 + 5.0 * vp1 - vp2) / 6.0;
    double q1 = (-vm1 + 5.0 * v0 + 2.0 * vp1) / 6.0;
    double q2 = (2.0 * vm2 - 7.0 * vm1 + 11.0 * v0) / 6.0;
    double t;
    t = v0 - 2.0 * vp1 + vp2;
    double s = 3.0 * v0 - 4.0 * vp1 + vp2;
    double b0 = 13.0 / 12.0 * t * t + 0.25 * s * s;
    t = vm1 - 2.0 * v0 + vp1;
    s = vm1 - vp1;
    double b1 = 13.0 / 12.0 * t * t + 0.25 * s * s;
    t = vm2 - 2.0 * vm1 + v0;
    s = vm2 - 4.0 * vm1 + 3.0 * v0;
    double b2 = 13.0 / 12.0 * t * t + 0.25 * s * s;
    double a0 = 0.3 / ((b0 + eps) * (b0 + eps));
    double a1 = 0.6 / ((b1 + eps) * (b1 + eps));
    double a2 = 0.1 / ((b2 + eps) * (b2 + eps));
    double sum = a0 + a1 + a2;
    return (a0 / sum) * q0 + (a1 / sum) * q1 + (a2 / sum) * q2;
}

int or_ncomp(const or_problem *p) { return ncomp_of(p); }

/* Exact global wave speed of a state: max over interior cells of |u| + a (Euler),
 * |f'(u)| = |u| (Burgers) or 1 (linear advection, unit velocity per axis).
 * Returns OR_ENONPHYS when rho <= 0 or p <= 0 is met (Euler). */
int or_alpha(const or_problem *p, const double *U, double *alpha_out) {
    int64_t nc = ncell_of(p);
    if (p->model == OR_LINADV) { *alpha_out = 1.0; return OR_OK; }
    if (p->model == OR_BURGERS) {
        double a = 0.0;
        for (int64_t i = 0; i < nc; ++i) a = fmax(a, fabs(U[i]));
        *alpha_out = a;
        return OR_OK;
    }
    int nd = p->ndim, ncomp = nd + 2;
    double amax = 0.0;
    int bad = 0;
    for (int64_t i = 0; i < nc; ++i) {
        double q[5];
        for (int c = 0; c < ncomp; ++c) q[c] = U[(int64_t)c * nc + i];
        double pr = pressure(q, nd, p->gamma);
        if (!(q[0] > 0.0) || !(pr > 0.0)) { bad = 1; continue; }
        double u2 = 0.0;
        for (int d = 0; d < nd; ++d) { double u = q[1 + d] / q[0]; u2 += u * u; }
        double a = sqrt(u2) + sqrt(p->gamma * pr / q[0]);
        if (a > amax) amax = a;
    }
    *alpha_out = amax;
    return bad ? OR_ENONPHYS : OR_OK;
}

/* Strides of the C-order interior array. */
static void strides_of(const or_problem *p, int64_t st[3]) {
    int64_t s = 1;
    for (int d = p->ndim - 1; d >= 0; --d) { st[d] = s; s *= p->n[d]; }
}

/*
 * Numerical flux along direction dir at every interface of every grid line:
 * Fhat[c][...][m][...] with the dir-extent N_dir + 1, interface m between interior cells
 * m-1 and m (m = 0 is the left boundary face). f^+ uses cells m-3..m+1, f^- uses m-2..m+2
 * (0-based), i.e. the mirror of the f^+ stencil about the face.
 */
int or_interface_flux(const or_problem *p, double alpha, const double *U, int dir, double *Fhat) {
    if (dir < 0 || dir >= p->ndim) return OR_EINVAL;
    int ncomp = ncomp_of(p), nd = p->ndim;
    int64_t nc = ncell_of(p), st[3];
    strides_of(p, st);
    int64_t N = p->n[dir];
    int64_t nlines = nc / N;
    double eps = p->h[dir] * p->h[dir];
    /* output strides: same shape but extent N+1 along dir */
    int64_t ost[3], osz = 1;
    for (int d = nd - 1; d >= 0; --d) { ost[d] = osz; osz *= (d == dir ? N + 1 : p->n[d]); }
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t line = 0; line < nlines; ++line) {
        /* decode the line's base index (all coordinates except dir) */
        int64_t rem = line, coord[3] = {0, 0, 0};
        for (int d = nd - 1; d >= 0; --d) {
            if (d == dir) continue;
            coord[d] = rem % p->n[d];
            rem /= p->n[d];
        }
        int64_t base = 0, obase = 0;
        for (int d = 0; d < nd; ++d) if (d != dir) { base += coord[d] * st[d]; obase += coord[d] * ost[d]; }
        double *fp = (double *)malloc(sizeof(double) * (size_t)(N + 6) * ncomp);
        double *fm = (double *)malloc(sizeof(double) * (size_t)(N + 6) * ncomp);
        if (!fp || !fm) { free(fp); free(fm); bad |= 2; continue; }
        for (int64_t g = -3; g < N + 3; ++g) {
            double q[5], f[5];
            line_state(p, U, base, st[dir], dir, g, q);
            if (p->model == OR_EULER) {
                if (!(q[0] > 0.0) || !(pressure(q, nd, p->gamma) > 0.0)) bad |= 1;
            }
            physical_flux(p, q, dir, f);
            for (int c = 0; c < ncomp; ++c) {
                fp[(g + 3) * ncomp + c] = 0.5 * (f[c] + alpha * q[c]);
                fm[(g + 3) * ncomp + c] = 0.5 * (f[c] - alpha * q[c]);
            }
        }
        for (int64_t m = 0; m <= N; ++m) {
            /* face m sits between cells m-1 and m; f^+ reconstructs from cell i = m-1 */
            int64_t i = m - 1 + 3; /* shifted index into the ghost-extended line */
            for (int c = 0; c < ncomp; ++c) {
                double hp = weno5_left(fp[(i - 2) * ncomp + c], fp[(i - 1) * ncomp + c], fp[i * ncomp + c],
                                       fp[(i + 1) * ncomp + c], fp[(i + 2) * ncomp + c], eps);
                double hm = weno5_left(fm[(i + 3) * ncomp + c], fm[(i + 2) * ncomp + c], fm[(i + 1) * ncomp + c],
                                       fm[i * ncomp + c], fm[(i - 1) * ncomp + c], eps);
                Fhat[(int64_t)c * osz + obase + m * ost[dir]] = hp + hm;
            }
        }
        free(fp);
        free(fm);
    }
    if (bad & 2) return OR_ENOMEM;
    return (bad & 1) ? OR_ENONPHYS : OR_OK;
}

/* L(U) = -sum_d (Fhat_{i+1/2} - Fhat_{i-1/2}) / h_d, directions summed in the order x, y, z
 * (eq. euler-system-for-loop). */
int or_rhs(const or_problem *p, double alpha, const double *U, double *L) {
    int ncomp = ncomp_of(p), nd = p->ndim;
    int64_t nc = ncell_of(p), st[3];
    strides_of(p, st);
    memset(L, 0, sizeof(double) * (size_t)nc * ncomp);
    int status = OR_OK;
    for (int dir = 0; dir < nd; ++dir) {
        int64_t N = p->n[dir];
        int64_t osz = nc / N * (N + 1);
        double *F = (double *)malloc(sizeof(double) * (size_t)osz * ncomp);
        if (!F) return OR_ENOMEM;
        int s = or_interface_flux(p, alpha, U, dir, F);
        if (s != OR_OK) status = s;
        int64_t ost[3], sz = 1;
        for (int d = nd - 1; d >= 0; --d) { ost[d] = sz; sz *= (d == dir ? N + 1 : p->n[d]); }
        double inv_h = 1.0 / p->h[dir];
#pragma omp parallel for schedule(static)
        for (int64_t cell = 0; cell < nc; ++cell) {
            int64_t rem = cell, o = 0;
            for (int d = nd - 1; d >= 0; --d) {
                int64_t cd = rem % p->n[d];
                rem /= p->n[d];
                o += cd * ost[d];
            }
            for (int c = 0; c < ncomp; ++c) {
                double fr = F[(int64_t)c * osz + o + ost[dir]];
                double fl = F[(int64_t)c * osz + o];
                L[(int64_t)c * nc + cell] -= (fr - fl) * inv_h;
            }
        }
        free(F);
        if (status == OR_ENONPHYS) return status;
    }
    return status;
}

/*
 * One SSP-RK3 step (Shu-Osher form) of size dt, in place on U.
 * alpha_mode 0: compute the exact alpha of each stage input and write it to alphas[s];
 * alpha_mode 1: use alphas[0..2] as given (so a TT run can be replayed exactly).
 */
int or_ssprk3(const or_problem *p, double dt, int alpha_mode, double *alphas, double *U) {
    int ncomp = ncomp_of(p);
    int64_t tot = ncell_of(p) * ncomp;
    double *u1 = (double *)malloc(sizeof(double) * (size_t)tot);
    double *L = (double *)malloc(sizeof(double) * (size_t)tot);
    if (!u1 || !L) { free(u1); free(L); return OR_ENOMEM; }
    int s;
    double a;
    /* stage 1: u1 = u + dt L(u) */
    if (alpha_mode == 0) { s = or_alpha(p, U, &a); if (s) goto out; alphas[0] = a; } else a = alphas[0];
    s = or_rhs(p, a, U, L); if (s) goto out;
    for (int64_t i = 0; i < tot; ++i) u1[i] = U[i] + dt * L[i];
    /* stage 2: u2 = 3/4 u + 1/4 (u1 + dt L(u1)), stored in u1 */
    if (alpha_mode == 0) { s = or_alpha(p, u1, &a); if (s) goto out; alphas[1] = a; } else a = alphas[1];
    s = or_rhs(p, a, u1, L); if (s) goto out;
    for (int64_t i = 0; i < tot; ++i) u1[i] = 0.75 * U[i] + 0.25 * (u1[i] + dt * L[i]);
    /* stage 3: u = 1/3 u + 2/3 (u2 + dt L(u2)) */
    if (alpha_mode == 0) { s = or_alpha(p, u1, &a); if (s) goto out; alphas[2] = a; } else a = alphas[2];
    s = or_rhs(p, a, u1, L); if (s) goto out;
    for (int64_t i = 0; i < tot; ++i) U[i] = U[i] / 3.0 + 2.0 / 3.0 * (u1[i] + dt * L[i]);
out:
    free(u1);
    free(L);
    return s;
}

/* Advance to t_end with dt = cfl * min_d h_d / alpha(U^n) (eq. cfl-other), the last step
 * clipped to land on t_end, or with a fixed dt when fixed_dt > 0. Returns the step count
 * in *nsteps. */
int or_run(const or_problem *p, double t_end, double cfl, double fixed_dt, double *U, int64_t *nsteps) {
    double t = 0.0, hmin = p->h[0];
    for (int d = 1; d < p->ndim; ++d) hmin = fmin(hmin, p->h[d]);
    int64_t k = 0;
    while (t < t_end * (1.0 - 1e-14)) {
        double dt, al[3];
        if (fixed_dt > 0.0) dt = fixed_dt;
        else {
            double a;
            int s = or_alpha(p, U, &a);
            if (s) { *nsteps = k; return s; }
            dt = cfl * hmin / a;
        }
        if (t + dt > t_end) dt = t_end - t;
        int s = or_ssprk3(p, dt, 0, al, U);
        if (s) { *nsteps = k; return s; }
        t += dt;
        ++k;
    }
    *nsteps = k;
    return OR_OK;
}

/* ---------------------------------------------------------------------------------
 * Naive per-point twin of or_rhs, written directly from the formulas with no line
 * buffers: every face flux is recomputed from the seven cells around it. Used on tiny
 * grids to cross-check the line-sweep implementation above.
 * --------------------------------------------------------------------------------- */
static void cell_state(const or_problem *p, const double *U, const int64_t idx[3], int dir, int64_t off,
                       double *q) {
    int64_t st[3], base = 0;
    strides_of(p, st);
    for (int d = 0; d < p->ndim; ++d)
        if (d != dir) base += idx[d] * st[d];
    line_state(p, U, base, st[dir], dir, idx[dir] + off, q);
}

static double face_flux_naive(const or_problem *p, double alpha, const double *U, const int64_t idx[3], int dir,
                              int c, int64_t face_left_cell) {
    /* face between cells face_left_cell and face_left_cell+1 along dir */
    double vp[5], vm[5];
    for (int k = 0; k < 5; ++k) {
        double q[5], f[5];
        cell_state(p, U, idx, dir, face_left_cell - idx[dir] + (k - 2), q);
        physical_flux(p, q, dir, f);
        vp[k] = 0.5 * (f[c] + alpha * q[c]);
        cell_state(p, U, idx, dir, face_left_cell - idx[dir] + (3 - k), q);
        physical_flux(p, q, dir, f);
        vm[k] = 0.5 * (f[c] - alpha * q[c]);
    }
    double eps = p->h[dir] * p->h[dir];
    return weno5_left(vp[0], vp[1], vp[2], vp[3], vp[4], eps) + weno5_left(vm[0], vm[1], vm[2], vm[3], vm[4], eps);
}

int or_rhs_naive(const or_problem *p, double alpha, const double *U, double *L) {
    int ncomp = ncomp_of(p), nd = p->ndim;
    int64_t nc = ncell_of(p);
    for (int64_t cell = 0; cell < nc; ++cell) {
        int64_t idx[3] = {0, 0, 0}, rem = cell;
        for (int d = nd - 1; d >= 0; --d) { idx[d] = rem % p->n[d]; rem /= p->n[d]; }
        for (int c = 0; c < ncomp; ++c) {
            double acc = 0.0;
            for (int dir = 0; dir < nd; ++dir) {
                double fr = face_flux_naive(p, alpha, U, idx, dir, c, idx[dir]);
                double fl = face_flux_naive(p, alpha, U, idx, dir, c, idx[dir] - 1);
                acc -= (fr - fl) / p->h[dir];
            }
            L[(int64_t)c * nc + cell] = acc;
        }
    }
    return OR_OK;
}
