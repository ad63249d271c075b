/*
 * FP64 CPU reference ("oracle") for the TTI and elastic propagators.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg do.  It shares no code with the HIP library.
 *
 * Plain, slow, obviously-correct loops in double precision, parallelised with
 * OpenMP over independent output points only (no blocking, fusion or
 * reordering of the arithmetic).  Layout: arrays of shape (nz, ny, nx), x
 * fastest.  2D grids use ny = 1 and the x and z axes only.
 *
 * Truncation semantics: every array value at an index outside [0, n) reads as
 * zero, wavefields and every intermediate alike; no value is ever computed in a
 * halo.  Under this rule the truncated centred first-derivative matrix D
 * satisfies D^T = -D and the staggered pair satisfies (D+)^T = -D-, which is
 * what makes the rotated operators of the TTI section self-adjoint
 * (Eq. "rot", G = D^T D) and the adjoint tests exact.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int ndim;      /* 2: axes x and z (ny must be 1); 3: x, y, z */
    long n[3];     /* nx, ny, nz */
    double h[3];   /* hx, hy, hz (metres) */
} orc_grid;

static long npts(const orc_grid *g) { return g->n[0] * g->n[1] * g->n[2]; }

static long axis_stride(const orc_grid *g, int axis)
{
    return axis == 0 ? 1 : (axis == 1 ? g->n[0] : g->n[0] * g->n[1]);
}

/* Coordinate of flat index idx along an axis. */
static long coord(const orc_grid *g, long idx, int axis)
{
    if (axis == 0) return idx % g->n[0];
    if (axis == 1) return (idx / g->n[0]) % g->n[1];
    return idx / (g->n[0] * g->n[1]);
}

/* f at (idx shifted by off along axis), zero outside [0, n). */
static double at(const orc_grid *g, const double *f, long idx, int axis, long c, long off)
{
    long cc = c + off;
    if (cc < 0 || cc >= g->n[axis]) return 0.0;
    return f[idx + off * axis_stride(g, axis)];
}

/* ---------------------------------------------------------------------------
 * Centred first derivative of accuracy order so = 2r (weights a_1..a_r):
 *   (D f)_i = sum_j a_j (f_{i+j} - f_{i-j}) / h
 * and its transpose, obtained by re-indexing the matrix entries of D
 * (D has +a_j/h at (i, i+j) and -a_j/h at (i, i-j)):
 *   (D^T g)_i = sum_j a_j (g_{i-j} - g_{i+j}) / h
 * ------------------------------------------------------------------------- */
void orc_dcen(const orc_grid *g, int axis, int r, const double *a, const double *f, double *out)
{
    long N = npts(g);
    double h = g->h[axis];
#pragma omp parallel for schedule(static)
    for (long idx = 0; idx < N; idx++) {
        long c = coord(g, idx, axis);
        double s = 0.0;
        for (int j = 1; j <= r; j++)
            s += a[j - 1] * (at(g, f, idx, axis, c, j) - at(g, f, idx, axis, c, -j));
        out[idx] = s / h;
    }
}

void orc_dcen_T(const orc_grid *g, int axis, int r, const double *a, const double *f, double *out)
{
    long N = npts(g);
    double h = g->h[axis];
#pragma omp parallel for schedule(static)
    for (long idx = 0; idx < N; idx++) {
        long c = coord(g, idx, axis);
        double s = 0.0;
        for (int j = 1; j <= r; j++)
            s += a[j - 1] * (at(g, f, idx, axis, c, -j) - at(g, f, idx, axis, c, j));
        out[idx] = s / h;
    }
}

/* ---------------------------------------------------------------------------
 * Staggered first derivatives (weights c_1..c_r).  Storage index i of a
 * half-node array holds the value at position i + 1/2.
 *   plus : (D+ f)[i] = sum_j c_j (f[i+j]   - f[i+1-j]) / h   (node -> half node)
 *   minus: (D- g)[i] = sum_j c_j (g[i+j-1] - g[i-j])   / h   (half node -> node)
 * Transposes by re-indexing the matrix entries:
 *   (D+^T g)[i] = sum_j c_j (g[i-j]   - g[i+j-1]) / h
 *   (D-^T g)[i] = sum_j c_j (g[i-j+1] - g[i+j])   / h
 * ------------------------------------------------------------------------- */
void orc_dstag(const orc_grid *g, int axis, int plus, int r, const double *cw, const double *f, double *out)
{
    long N = npts(g);
    double h = g->h[axis];
#pragma omp parallel for schedule(static)
    for (long idx = 0; idx < N; idx++) {
        long c = coord(g, idx, axis);
        double s = 0.0;
        for (int j = 1; j <= r; j++) {
            if (plus) s += cw[j - 1] * (at(g, f, idx, axis, c, j) - at(g, f, idx, axis, c, 1 - j));
            else      s += cw[j - 1] * (at(g, f, idx, axis, c, j - 1) - at(g, f, idx, axis, c, -j));
        }
        out[idx] = s / h;
    }
}

void orc_dstag_T(const orc_grid *g, int axis, int plus, int r, const double *cw, const double *f, double *out)
{
    long N = npts(g);
    double h = g->h[axis];
#pragma omp parallel for schedule(static)
    for (long idx = 0; idx < N; idx++) {
        long c = coord(g, idx, axis);
        double s = 0.0;
        for (int j = 1; j <= r; j++) {
            if (plus) s += cw[j - 1] * (at(g, f, idx, axis, c, -j) - at(g, f, idx, axis, c, j - 1));
            else      s += cw[j - 1] * (at(g, f, idx, axis, c, 1 - j) - at(g, f, idx, axis, c, j));
        }
        out[idx] = s / h;
    }
}

/* ---------------------------------------------------------------------------
 * Rotated second derivatives of the TTI section (Eq. "rot" and the listing of
 * rotated derivatives):
 *   D_xbar = cos(th)cos(ph) d/dx + cos(th)sin(ph) d/dy - sin(th) d/dz
 *   D_ybar = -sin(ph) d/dx + cos(ph) d/dy                (orthonormal completion)
 *   D_zbar = sin(th)cos(ph) d/dx + sin(th)sin(ph) d/dy + cos(th) d/dz
 *   G_ii   = D_ibar^T D_ibar,  with the angle factors inside the second
 *            (transposed) derivative pass,  H = -G.
 *   H0 = H_xbar + H_ybar (horizontal), Hz = H_zbar (along the symmetry axis).
 * In 2D (x, z) phi is zero and the ybar term is absent.
 * ------------------------------------------------------------------------- */
static void rot_row(int which, double th, double ph, double R[3])
{
    if (which == 0) { R[0] = cos(th) * cos(ph); R[1] = cos(th) * sin(ph); R[2] = -sin(th); }
    else if (which == 1) { R[0] = -sin(ph); R[1] = cos(ph); R[2] = 0.0; }
    else { R[0] = sin(th) * cos(ph); R[1] = sin(th) * sin(ph); R[2] = cos(th); }
}

/* out = H_{which-group} f.  group 0: H0 = H_xbar + H_ybar; group 1: Hz = H_zbar. */
void orc_tti_H(const orc_grid *g, int r, const double *a, const double *th, const double *ph,
               const double *f, int group, double *out)
{
    long N = npts(g);
    int axes[3], na = 0;
    axes[na++] = 0;
    if (g->ndim == 3) axes[na++] = 1;
    axes[na++] = 2;
    double *d[3], *w = malloc(sizeof(double) * N), *tmp = malloc(sizeof(double) * N);
    double *gi = malloc(sizeof(double) * N);
    for (int k = 0; k < na; k++) {
        d[k] = malloc(sizeof(double) * N);
        orc_dcen(g, axes[k], r, a, f, d[k]);
    }
    memset(out, 0, sizeof(double) * N);
    int rows[2], nrows = 0;
    if (group == 0) { rows[nrows++] = 0; if (g->ndim == 3) rows[nrows++] = 1; }
    else rows[nrows++] = 2;
    for (int ir = 0; ir < nrows; ir++) {
        int row = rows[ir];
        /* gi = D_ibar f = sum_a R_ia D_a f */
#pragma omp parallel for schedule(static)
        for (long idx = 0; idx < N; idx++) {
            double R[3];
            rot_row(row, th[idx], g->ndim == 3 ? ph[idx] : 0.0, R);
            double s = 0.0;
            for (int k = 0; k < na; k++) s += R[axes[k]] * d[k][idx];
            gi[idx] = s;
        }
        /* out -= D_ibar^T gi = sum_a D_a^T (R_ia gi) */
        for (int k = 0; k < na; k++) {
#pragma omp parallel for schedule(static)
            for (long idx = 0; idx < N; idx++) {
                double R[3];
                rot_row(row, th[idx], g->ndim == 3 ? ph[idx] : 0.0, R);
                w[idx] = R[axes[k]] * gi[idx];
            }
            orc_dcen_T(g, axes[k], r, a, w, tmp);
#pragma omp parallel for schedule(static)
            for (long idx = 0; idx < N; idx++) out[idx] -= tmp[idx];
        }
    }
    for (int k = 0; k < na; k++) free(d[k]);
    free(w); free(tmp); free(gi);
}

/* ---------------------------------------------------------------------------
 * One explicit time step of the pseudo-acoustic TTI system
 *     m p_tt + eta p_t = (1+2 eps) H0 p + sqrt(1+2 delta) Hz q
 *     m q_tt + eta q_t = sqrt(1+2 delta) H0 p + Hz q
 * discretised with second-order centred time differences:
 *     a f+ = b f - c f- + L_f,   a = m/dt^2 + eta/(2dt), b = 2m/dt^2, c = m/dt^2 - eta/(2dt).
 * adjoint = 0: L = C (H0 p, Hz q)               (forward operator)
 * adjoint = 1: L = (H0 w_p, Hz w_q), w = C (p, q)  (its transpose: mix first)
 * with the pointwise symmetric C = [[1+2eps, sqrt(1+2delta)], [sqrt(1+2delta), 1]].
 * Sources and receivers are handled by the caller.
 * ------------------------------------------------------------------------- */
void orc_tti_step(const orc_grid *g, int r, const double *a, const double *m, const double *eps,
                  const double *delta, const double *th, const double *ph, const double *eta,
                  double dt, int adjoint, const double *p, const double *q, const double *pm,
                  const double *qm, double *pn, double *qn)
{
    long N = npts(g);
    double *h0 = malloc(sizeof(double) * N), *hz = malloc(sizeof(double) * N);
    if (!adjoint) {
        orc_tti_H(g, r, a, th, ph, p, 0, h0);
        orc_tti_H(g, r, a, th, ph, q, 1, hz);
    } else {
        double *wp = malloc(sizeof(double) * N), *wq = malloc(sizeof(double) * N);
#pragma omp parallel for schedule(static)
        for (long i = 0; i < N; i++) {
            double A = 1.0 + 2.0 * eps[i], B = sqrt(1.0 + 2.0 * delta[i]);
            wp[i] = A * p[i] + B * q[i];
            wq[i] = B * p[i] + q[i];
        }
        orc_tti_H(g, r, a, th, ph, wp, 0, h0);
        orc_tti_H(g, r, a, th, ph, wq, 1, hz);
        free(wp); free(wq);
    }
#pragma omp parallel for schedule(static)
    for (long i = 0; i < N; i++) {
        double Lp, Lq;
        if (!adjoint) {
            double A = 1.0 + 2.0 * eps[i], B = sqrt(1.0 + 2.0 * delta[i]);
            Lp = A * h0[i] + B * hz[i];
            Lq = B * h0[i] + hz[i];
        } else {
            Lp = h0[i];
            Lq = hz[i];
        }
        double ca = m[i] / (dt * dt) + eta[i] / (2.0 * dt);
        double cb = 2.0 * m[i] / (dt * dt);
        double cc = m[i] / (dt * dt) - eta[i] / (2.0 * dt);
        pn[i] = (cb * p[i] - cc * pm[i] + Lp) / ca;
        qn[i] = (cb * q[i] - cc * qm[i] + Lq) / ca;
    }
    free(h0); free(hz);
}

/* ---------------------------------------------------------------------------
 * Isotropic elastic velocity-stress on a staggered grid (Eq. "elas1" with the
 * listing's reading dv/dt = (1/rho) div tau, and the listing's update order:
 * velocities first, then stresses from the new velocities, both multiplied by
 * the damping factor).
 *
 * Field positions (storage index i holds the listed position):
 *   txx, tyy, tzz (i, j, k)     vx (i+1/2, j, k)   vy (i, j+1/2, k)   vz (i, j, k+1/2)
 *   txy (i+1/2, j+1/2, k)       txz (i+1/2, j, k+1/2)               tyz (i, j+1/2, k+1/2)
 * Half-node parameters are arithmetic means of the surrounding nodes, with the
 * last index clamped: bx = (b_i + b_{i+1})/2 etc., mu_xy = mean of 4 nodes etc.
 * Field order in the v[3] / t[6] arrays: vx, vy, vz; txx, tyy, tzz, txy, txz, tyz.
 * ------------------------------------------------------------------------- */
static long clampi(long i, long n) { return i < n ? i : n - 1; }

static double avg2(const orc_grid *g, const double *f, long idx, int ax)
{
    long c = coord(g, idx, ax);
    long c1 = clampi(c + 1, g->n[ax]);
    return 0.5 * (f[idx] + f[idx + (c1 - c) * axis_stride(g, ax)]);
}

static double avg4(const orc_grid *g, const double *f, long idx, int a1, int a2)
{
    long c1 = coord(g, idx, a1), c2 = coord(g, idx, a2);
    long d1 = (clampi(c1 + 1, g->n[a1]) - c1) * axis_stride(g, a1);
    long d2 = (clampi(c2 + 1, g->n[a2]) - c2) * axis_stride(g, a2);
    return 0.25 * (f[idx] + f[idx + d1] + f[idx + d2] + f[idx + d1 + d2]);
}

/* D_tau: the force (div tau) at the three velocity positions. */
static void el_force(const orc_grid *g, int r, const double *cw, double *const *t, double **fo, double *tmp)
{
    long N = npts(g);
    /* (axis, plus, tau component) contributing to each velocity component */
    static const int plan[3][3][3] = {
        {{0, 1, 0}, {1, 0, 3}, {2, 0, 4}},   /* vx: D+x txx + D-y txy + D-z txz */
        {{0, 0, 3}, {1, 1, 1}, {2, 0, 5}},   /* vy: D-x txy + D+y tyy + D-z tyz */
        {{0, 0, 4}, {1, 0, 5}, {2, 1, 2}},   /* vz: D-x txz + D-y tyz + D+z tzz */
    };
    for (int c = 0; c < 3; c++) {
        memset(fo[c], 0, sizeof(double) * N);
        for (int k = 0; k < 3; k++) {
            int ax = plan[c][k][0];
            if (ax == 1 && g->ndim == 2) continue;
            orc_dstag(g, ax, plan[c][k][1], r, cw, t[plan[c][k][2]], tmp);
            for (long i = 0; i < N; i++) fo[c][i] += tmp[i];
        }
    }
}

/* E: strains (exx, eyy, ezz, gxy, gxz, gyz) of a velocity field. */
static void el_strain(const orc_grid *g, int r, const double *cw, double *const *v, double **e, double *tmp)
{
    long N = npts(g);
    static const int plan[6][2][3] = {
        {{0, 0, 0}, {-1, 0, 0}},            /* exx = D-x vx */
        {{1, 0, 1}, {-1, 0, 0}},            /* eyy = D-y vy */
        {{2, 0, 2}, {-1, 0, 0}},            /* ezz = D-z vz */
        {{1, 1, 0}, {0, 1, 1}},             /* gxy = D+y vx + D+x vy */
        {{2, 1, 0}, {0, 1, 2}},             /* gxz = D+z vx + D+x vz */
        {{2, 1, 1}, {1, 1, 2}},             /* gyz = D+z vy + D+y vz */
    };
    for (int c = 0; c < 6; c++) {
        memset(e[c], 0, sizeof(double) * N);
        for (int k = 0; k < 2; k++) {
            int ax = plan[c][k][0];
            if (ax < 0 || (ax == 1 && g->ndim == 2)) continue;
            orc_dstag(g, ax, plan[c][k][1], r, cw, v[plan[c][k][2]], tmp);
            for (long i = 0; i < N; i++) e[c][i] += tmp[i];
        }
    }
}

/* Transpose of el_strain: out_v = E^T s  (s has 6 components). */
static void el_strain_T(const orc_grid *g, int r, const double *cw, double *const *s, double **ov, double *tmp)
{
    long N = npts(g);
    /* (axis, plus, stress component) for each velocity row of E^T */
    static const int plan[3][3][3] = {
        {{0, 0, 0}, {1, 1, 3}, {2, 1, 4}},   /* vx: (D-x)^T s_xx + (D+y)^T s_xy + (D+z)^T s_xz */
        {{1, 0, 1}, {0, 1, 3}, {2, 1, 5}},   /* vy: (D-y)^T s_yy + (D+x)^T s_xy + (D+z)^T s_yz */
        {{2, 0, 2}, {0, 1, 4}, {1, 1, 5}},   /* vz: (D-z)^T s_zz + (D+x)^T s_xz + (D+y)^T s_yz */
    };
    for (int c = 0; c < 3; c++) {
        memset(ov[c], 0, sizeof(double) * N);
        for (int k = 0; k < 3; k++) {
            int ax = plan[c][k][0];
            if (ax == 1 && g->ndim == 2) continue;
            orc_dstag_T(g, ax, plan[c][k][1], r, cw, s[plan[c][k][2]], tmp);
            for (long i = 0; i < N; i++) ov[c][i] += tmp[i];
        }
    }
}

/* Transpose of el_force: out_t = D_tau^T f  (f has 3 components). */
static void el_force_T(const orc_grid *g, int r, const double *cw, double *const *f, double **ot, double *tmp)
{
    long N = npts(g);
    for (int c = 0; c < 6; c++) memset(ot[c], 0, sizeof(double) * N);
    /* same plan as el_force: rows are velocity comps, entries (axis, plus, tau comp) */
    static const int plan[3][3][3] = {
        {{0, 1, 0}, {1, 0, 3}, {2, 0, 4}},
        {{0, 0, 3}, {1, 1, 1}, {2, 0, 5}},
        {{0, 0, 4}, {1, 0, 5}, {2, 1, 2}},
    };
    for (int c = 0; c < 3; c++) {
        for (int k = 0; k < 3; k++) {
            int ax = plan[c][k][0];
            if (ax == 1 && g->ndim == 2) continue;
            orc_dstag_T(g, ax, plan[c][k][1], r, cw, f[c], tmp);
            double *o = ot[plan[c][k][2]];
            for (long i = 0; i < N; i++) o[i] += tmp[i];
        }
    }
}

/* Stiffness C applied pointwise to strain-like s (6 comps) -> stress-like out. */
static void el_stiff(const orc_grid *g, const double *lam, const double *mu, double *const *s, double **out)
{
    long N = npts(g);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < N; i++) {
        double tr = s[0][i] + s[1][i] + s[2][i];
        for (int c = 0; c < 3; c++) out[c][i] = lam[i] * tr + 2.0 * mu[i] * s[c][i];
        out[3][i] = avg4(g, mu, i, 0, 1) * s[3][i];
        out[4][i] = avg4(g, mu, i, 0, 2) * s[4][i];
        out[5][i] = avg4(g, mu, i, 1, 2) * s[5][i];
    }
}

/* The force D_tau tau at the velocity positions (3 outputs) and the strains E v (6 outputs), as
 * used by the step below; exported for the adjoint-state gradient. */
void orc_el_force(const orc_grid *g, int r, const double *cw, double **t, double **out)
{
    double *tmp = malloc(sizeof(double) * npts(g));
    el_force(g, r, cw, t, out, tmp);
    free(tmp);
}

void orc_el_strain(const orc_grid *g, int r, const double *cw, double **v, double **out)
{
    double *tmp = malloc(sizeof(double) * npts(g));
    el_strain(g, r, cw, v, out, tmp);
    free(tmp);
}

/* Forward step, in place:  v <- g (v + dt b D_tau tau);  tau <- g (tau + dt C E v). */
void orc_el_step(const orc_grid *g, int r, const double *cw, const double *lam, const double *mu,
                 const double *b, const double *damp, double dt, double **v, double **t)
{
    long N = npts(g);
    double *tmp = malloc(sizeof(double) * N), *buf[6], *buf2[6];
    for (int c = 0; c < 6; c++) { buf[c] = malloc(sizeof(double) * N); buf2[c] = malloc(sizeof(double) * N); }
    el_force(g, r, cw, t, buf, tmp);
    for (int c = 0; c < 3; c++) {
#pragma omp parallel for schedule(static)
        for (long i = 0; i < N; i++)
            v[c][i] = damp[i] * (v[c][i] + dt * avg2(g, b, i, c) * buf[c][i]);
    }
    el_strain(g, r, cw, v, buf, tmp);
    el_stiff(g, lam, mu, buf, buf2);
    for (int c = 0; c < 6; c++) {
#pragma omp parallel for schedule(static)
        for (long i = 0; i < N; i++) t[c][i] = damp[i] * (t[c][i] + dt * buf2[c][i]);
    }
    for (int c = 0; c < 6; c++) { free(buf[c]); free(buf2[c]); }
    free(tmp);
}

/* Transpose of orc_el_step (without sources/receivers), in place on (vt, tt):
 *   vt += dt E^T C (g tt);  tt <- g tt;     (transpose of the stress update)
 *   tt += dt D_tau^T (b (g vt)); vt <- g vt (transpose of the velocity update) */
void orc_el_step_T(const orc_grid *g, int r, const double *cw, const double *lam, const double *mu,
                   const double *b, const double *damp, double dt, double **vt, double **tt)
{
    long N = npts(g);
    double *tmp = malloc(sizeof(double) * N), *buf[6], *buf2[6];
    for (int c = 0; c < 6; c++) { buf[c] = malloc(sizeof(double) * N); buf2[c] = malloc(sizeof(double) * N); }
    for (int c = 0; c < 6; c++) {
#pragma omp parallel for schedule(static)
        for (long i = 0; i < N; i++) { tt[c][i] *= damp[i]; buf[c][i] = tt[c][i]; }
    }
    el_stiff(g, lam, mu, buf, buf2);
    el_strain_T(g, r, cw, buf2, buf, tmp);
    for (int c = 0; c < 3; c++) {
#pragma omp parallel for schedule(static)
        for (long i = 0; i < N; i++) vt[c][i] += dt * buf[c][i];
    }
    for (int c = 0; c < 3; c++) {
#pragma omp parallel for schedule(static)
        for (long i = 0; i < N; i++) { vt[c][i] *= damp[i]; buf[c][i] = avg2(g, b, i, c) * vt[c][i]; }
    }
    el_force_T(g, r, cw, buf, buf2, tmp);
    for (int c = 0; c < 6; c++) {
#pragma omp parallel for schedule(static)
        for (long i = 0; i < N; i++) tt[c][i] += dt * buf2[c][i];
    }
    for (int c = 0; c < 6; c++) { free(buf[c]); free(buf2[c]); }
    free(tmp);
}
