/*
 * rpy_oracle.c -- plain, slow FP64 CPU oracle for the Ewald-summed
 * Rotne-Prager-Yamakawa (RPY) Brownian-dynamics step of
 * Jain, Sunthar, Duenweg & Prakash, "Optimisation of a Brownian dynamics
 * algorithm for semidilute polymer solutions" (arXiv:1203.6208).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load or call this library.  It shares no
 * code, header, table or constant with the HIP library, and the HIP library
 * must never fall back to it.
 *
 * Every routine is the textbook definition written out: brute-force loops
 * over beads, periodic images and the full +-k lattice, dense matrices, a
 * plain triple-loop matrix-vector product.  No blocking, fusion or
 * reordering beyond what the paper's formulas state.  Where FP64 would
 * cancel catastrophically (the n=0 overlap term, where M1 and M* each grow
 * like 1/r^3 and cancel), the same printed formula is evaluated in IEEE
 * binary128 (libquadmath) and rounded once.
 *
 * Layout conventions: positions [N][3]; vectors [m][N][3]; the dense
 * diffusion matrix is 3N x 3N row-major with row index 3*nu + i (the block
 * matrix of the section "Governing equation").
 *
 * Readings of the paper that this file takes (the GPU library takes the same):
 *  - reciprocal sum uses cos(k.(r_nu - r_mu)) (the printed minus sign in the
 *    Beenakker sum breaks translation invariance);
 *  - the rr coefficient of M* is (3/(2x^3))(x^2/4-1)^2, i.e. M* equals the
 *    branch-B minus branch-A RPY difference (the printed coefficient makes D
 *    jump at r = 2a);
 *  - the overlap correction applies to every image (nu,mu,n) != (nu,nu,0)
 *    with |r| < 2a, so that D stays periodic in each bead;
 *  - coincident distinct beads take the r -> 0 limit of M1 + M*, which is
 *    the self coefficient times the identity;
 *  - Chebyshev coefficients are those of the interpolant of sqrt at the
 *    N_Ch Chebyshev-Gauss nodes mapped onto [d_min, d_max].
 */
#include <math.h>
#include <omp.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------
 * RPY tensor branches (section "Governing equation", eq. b1 and eq. b2).
 * Omega(r) = Omega1 * I + Omega2 * rhat rhat.
 * ---------------------------------------------------------------------- */
void orc_rpy_branch_a(double r, double a, double *o1, double *o2)
{
    /* branch A, r >= 2a */
    *o1 = 3.0 * a / (4.0 * r) * (1.0 + 2.0 * a * a / (3.0 * r * r));
    *o2 = 3.0 * a / (4.0 * r) * (1.0 - 2.0 * a * a / (r * r));
}

void orc_rpy_branch_b(double r, double a, double *o1, double *o2)
{
    /* branch B, 0 < r <= 2a */
    *o1 = 1.0 - 9.0 * r / (32.0 * a);
    *o2 = 3.0 * r / (32.0 * a);
}

/* ------------------------------------------------------------------------
 * Real-space Ewald kernel M1(r) (section "Evaluation of sum D.F as an Ewald
 * sum", eq. M1): returns the coefficients of I and of rhat rhat.
 * ---------------------------------------------------------------------- */
void orc_m1_coeffs(double r, double a, double al, double *c1, double *c2)
{
    double a3 = a * a * a;
    double e = erfc(al * r);
    double g = exp(-al * al * r * r) / sqrt(ORC_PI);
    double r2 = r * r, r3 = r2 * r, r4 = r2 * r2;
    double al3 = al * al * al, al5 = al3 * al * al, al7 = al5 * al * al;
    *c1 = e * (3.0 * a / (4.0 * r) + a3 / (2.0 * r3))
        + g * (3.0 * a * al3 * r2 - 9.0 * a * al / 2.0 + 4.0 * a3 * al7 * r4
               - 20.0 * a3 * al5 * r2 + 14.0 * a3 * al3 + a3 * al / r2);
    *c2 = e * (3.0 * a / (4.0 * r) - 3.0 * a3 / (2.0 * r3))
        + g * (3.0 * a * al / 2.0 - 3.0 * a * al3 * r2 - 4.0 * a3 * al7 * r4
               + 16.0 * a3 * al5 * r2 - 2.0 * a3 * al3 - 3.0 * a3 * al / r2);
}

/* Same formula in binary128. */
static void m1_coeffs_q(__float128 r, __float128 a, __float128 al,
                        __float128 *c1, __float128 *c2)
{
    __float128 a3 = a * a * a;
    __float128 e = erfcq(al * r);
    __float128 g = expq(-al * al * r * r) / sqrtq(M_PIq);
    __float128 r2 = r * r, r3 = r2 * r, r4 = r2 * r2;
    __float128 al3 = al * al * al, al5 = al3 * al * al, al7 = al5 * al * al;
    *c1 = e * (3 * a / (4 * r) + a3 / (2 * r3))
        + g * (3 * a * al3 * r2 - 9 * a * al / 2 + 4 * a3 * al7 * r4
               - 20 * a3 * al5 * r2 + 14 * a3 * al3 + a3 * al / r2);
    *c2 = e * (3 * a / (4 * r) - 3 * a3 / (2 * r3))
        + g * (3 * a * al / 2 - 3 * a * al3 * r2 - 4 * a3 * al7 * r4
               + 16 * a3 * al5 * r2 - 2 * a3 * al3 - 3 * a3 * al / r2);
}

/* ------------------------------------------------------------------------
 * Overlap correction M*(x), x = r/a (section "Modification of the Ewald
 * sum to account for overlapping beads", eq. cor5), with the rr
 * coefficient read as (3/(2x^3))(x^2/4 - 1)^2 so that M* = Omega_B - Omega_A.
 * ---------------------------------------------------------------------- */
void orc_mstar_coeffs(double x, double *c1, double *c2)
{
    double x3 = x * x * x;
    double t1 = 3.0 * x * x / 4.0 + 1.0;
    double t2 = x * x / 4.0 - 1.0;
    *c1 = 1.0 - t1 * t1 / (2.0 * x3);
    *c2 = 3.0 * t2 * t2 / (2.0 * x3);
}

static void mstar_coeffs_q(__float128 x, __float128 *c1, __float128 *c2)
{
    __float128 x3 = x * x * x;
    __float128 t1 = 3 * x * x / 4 + 1;
    __float128 t2 = x * x / 4 - 1;
    *c1 = 1 - t1 * t1 / (2 * x3);
    *c2 = 3 * t2 * t2 / (2 * x3);
}

/* Self coefficient of the Ewald sum (eq. DF, first term). */
double orc_self_coeff(double a, double al)
{
    return 1.0 - 6.0 * a * al / sqrt(ORC_PI)
               + 40.0 * a * a * a * al * al * al / (3.0 * sqrt(ORC_PI));
}

/* Reciprocal-space scalar m(k) of M2(k) = m(k) (I - khat khat) (eq. M2). */
double orc_m2_scalar(double k, double a, double al, double vol)
{
    double k2 = k * k;
    return (a - a * a * a * k2 / 3.0)
         * (1.0 + k2 / (4.0 * al * al) + k2 * k2 / (8.0 * al * al * al * al))
         * (6.0 * ORC_PI / (k2 * vol))
         * exp(-k2 / (4.0 * al * al));
}

/* ------------------------------------------------------------------------
 * Wrapping into the primary box: rt = L * (r/L - floor(r/L)).
 * ---------------------------------------------------------------------- */
void orc_wrap(int n, const double *r, double L, double *rt)
{
    for (int i = 0; i < 3 * n; ++i) {
        double s = r[i] / L;
        s = s - floor(s);
        rt[i] = L * s;
    }
}

/* Pair contribution of one image d (|d|^2 = r2) to the real-space sum,
 * including the overlap correction.  Adds c1 I + c2 dhat dhat into blk. */
static void pair_image(const double d[3], double r2, int in_rc, int overlap,
                       double a, double al, double blk[9])
{
    double c1 = 0.0, c2 = 0.0;
    double r = sqrt(r2);
    if (overlap) {
        if (r2 == 0.0) {
            /* coincident distinct beads (r = 0 <= rc always): the limit of
             * M1 + M* as r -> 0 is the self coefficient times I */
            c1 = orc_self_coeff(a, al);
            c2 = 0.0;
        } else if (in_rc && r / a < 1e-6) {
            /* M1 + M* = Omega_B - S with S smooth and even in r; below
             * r/a = 1e-6 the O(r^2) change of S is < 1e-13 */
            double o1, o2;
            orc_rpy_branch_b(r, a, &o1, &o2);
            c1 = o1 - (1.0 - orc_self_coeff(a, al));
            c2 = o2;
        } else {
            __float128 q1 = 0, q2 = 0, s1, s2;
            __float128 rq = sqrtq((__float128)d[0] * d[0]
                                  + (__float128)d[1] * d[1]
                                  + (__float128)d[2] * d[2]);
            if (in_rc) m1_coeffs_q(rq, a, al, &q1, &q2);
            mstar_coeffs_q(rq / a, &s1, &s2);
            c1 = (double)(q1 + s1);
            c2 = (double)(q2 + s2);
        }
    } else {
        orc_m1_coeffs(r, a, al, &c1, &c2);
    }
    for (int i = 0; i < 3; ++i) {
        blk[3 * i + i] += c1;
        if (r2 > 0.0)
            for (int j = 0; j < 3; ++j)
                blk[3 * i + j] += c2 * d[i] * d[j] / r2;
    }
}

/* ------------------------------------------------------------------------
 * Real-space part of D (eq. DFmodified: second and last sums), brute force
 * (rows variant: only the block rows of the listed beads, stored densely in
 * list order as D[3*nrows][3N])
 * over every pair and every periodic image n in [-ni, ni]^3 with
 * ni = ceil(rc/L) + 1.  The image (nu, nu, 0) is omitted (the prime on the
 * lattice sum).  Images with |d| <= rc take M1; images with |d| < 2a add M*.
 * D is accumulated (+=); rt are wrapped positions.
 * ---------------------------------------------------------------------- */
void orc_real_space_rows(int n, const double *rt, double L, double a, double al,
                         double rc, int nrows, const int *rows, double *D)
{
    int ni = (int)ceil(rc / L) + 1;
    double rc2 = rc * rc, a2x4 = 4.0 * a * a;
    long n3 = 3L * n;
#pragma omp parallel for schedule(dynamic)
    for (int ir = 0; ir < nrows; ++ir) {
        int nu = rows[ir];
        for (int mu = 0; mu < n; ++mu) {
            double blk[9] = {0};
            for (int nx = -ni; nx <= ni; ++nx)
                for (int ny = -ni; ny <= ni; ++ny)
                    for (int nz = -ni; nz <= ni; ++nz) {
                        if (nu == mu && nx == 0 && ny == 0 && nz == 0) continue;
                        double d[3];
                        d[0] = (rt[3 * nu + 0] - rt[3 * mu + 0]) + nx * L;
                        d[1] = (rt[3 * nu + 1] - rt[3 * mu + 1]) + ny * L;
                        d[2] = (rt[3 * nu + 2] - rt[3 * mu + 2]) + nz * L;
                        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                        int in_rc = r2 <= rc2;
                        int overlap = r2 < a2x4;
                        if (!in_rc && !overlap) continue;
                        pair_image(d, r2, in_rc, overlap, a, al, blk);
                    }
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j)
                    D[(3L * ir + i) * n3 + 3L * mu + j] += blk[3 * i + j];
        }
    }
}

void orc_real_space(int n, const double *rt, double L, double a, double al,
                    double rc, double *D)
{
    int *rows = (int *)malloc(sizeof(int) * n);
    for (int i = 0; i < n; ++i) rows[i] = i;
    orc_real_space_rows(n, rt, L, a, al, rc, n, rows, D);
    free(rows);
}

/* Self term on a row subset: D[ir] row block of bead rows[ir]. */
void orc_self_term_rows(int n, double a, double al, int nrows, const int *rows, double *D)
{
    double s = orc_self_coeff(a, al);
    long n3 = 3L * n;
    for (int ir = 0; ir < nrows; ++ir)
        for (int i = 0; i < 3; ++i) D[(3L * ir + i) * n3 + 3L * rows[ir] + i] += s;
}

/* Self term (eq. DF, first term): D_nu,nu += s(alpha) I. */
void orc_self_term(int n, double a, double al, double *D)
{
    double s = orc_self_coeff(a, al);
    long n3 = 3L * n;
    for (long i = 0; i < n3; ++i) D[i * n3 + i] += s;
}

/* ------------------------------------------------------------------------
 * Reciprocal-space part of D (eq. DFmodified, third sum) over the FULL set
 * of wave vectors k = 2 pi nvec / L, nvec != 0, |nvec|^2 <= n2max, with a
 * direct cosine per pair: D_nu,mu += m(k) (I - khat khat) cos(k.(r_nu - r_mu)).
 * ---------------------------------------------------------------------- */
void orc_recip_space_rows(int n, const double *rt, double L, double a, double al,
                          int n2max, int nrows, const int *rows, double *D)
{
    double vol = L * L * L;
    int nm = (int)floor(sqrt((double)n2max)) + 1;
    long n3 = 3L * n;
#pragma omp parallel for schedule(dynamic)
    for (int ir = 0; ir < nrows; ++ir) {
        int nu = rows[ir];
        for (int nx = -nm; nx <= nm; ++nx)
            for (int ny = -nm; ny <= nm; ++ny)
                for (int nz = -nm; nz <= nm; ++nz) {
                    int n2 = nx * nx + ny * ny + nz * nz;
                    if (n2 == 0 || n2 > n2max) continue;
                    double k[3] = {2.0 * ORC_PI * nx / L, 2.0 * ORC_PI * ny / L,
                                   2.0 * ORC_PI * nz / L};
                    double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
                    double mk = orc_m2_scalar(sqrt(k2), a, al, vol);
                    double P[9];
                    for (int i = 0; i < 3; ++i)
                        for (int j = 0; j < 3; ++j)
                            P[3 * i + j] = (i == j ? 1.0 : 0.0) - k[i] * k[j] / k2;
                    for (int mu = 0; mu < n; ++mu) {
                        double ph = k[0] * (rt[3 * nu + 0] - rt[3 * mu + 0])
                                  + k[1] * (rt[3 * nu + 1] - rt[3 * mu + 1])
                                  + k[2] * (rt[3 * nu + 2] - rt[3 * mu + 2]);
                        double w = mk * cos(ph);
                        for (int i = 0; i < 3; ++i)
                            for (int j = 0; j < 3; ++j)
                                D[(3L * ir + i) * n3 + 3L * mu + j] += w * P[3 * i + j];
                    }
                }
    }
}

void orc_recip_space(int n, const double *rt, double L, double a, double al,
                     int n2max, double *D)
{
    int *rows = (int *)malloc(sizeof(int) * n);
    for (int i = 0; i < n; ++i) rows[i] = i;
    orc_recip_space_rows(n, rt, L, a, al, n2max, n, rows, D);
    free(rows);
}

/* Number of wave vectors in the full set (both signs). */
int orc_count_kvectors(int n2max)
{
    int nm = (int)floor(sqrt((double)n2max)) + 1, c = 0;
    for (int nx = -nm; nx <= nm; ++nx)
        for (int ny = -nm; ny <= nm; ++ny)
            for (int nz = -nm; nz <= nm; ++nz) {
                int n2 = nx * nx + ny * ny + nz * nz;
                if (n2 != 0 && n2 <= n2max) ++c;
            }
    return c;
}

/* ------------------------------------------------------------------------
 * out[j] = D . V[j] for j < m (plain loop in ascending column order).
 * ---------------------------------------------------------------------- */
void orc_matvec(int n3, const double *D, int m, const double *V, double *out)
{
#pragma omp parallel for
    for (int i = 0; i < n3; ++i)
        for (int j = 0; j < m; ++j) {
            double s = 0.0;
            for (int k = 0; k < n3; ++k) s += D[(long)i * n3 + k] * V[(long)j * n3 + k];
            out[(long)j * n3 + i] = s;
        }
}

/* Thread control for timing the oracle (no arithmetic): the OpenMP team size
 * of later parallel loops, and the size they would use now. */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_max_threads(void) { return omp_get_max_threads(); }

/* out = R . v for a block of rows R [nrows][ncols] (same plain loop). */
void orc_rows_matvec(int nrows, int ncols, const double *R, const double *v, double *out)
{
#pragma omp parallel for
    for (int i = 0; i < nrows; ++i) {
        double s = 0.0;
        for (int k = 0; k < ncols; ++k) s += R[(long)i * ncols + k] * v[k];
        out[i] = s;
    }
}

/* ------------------------------------------------------------------------
 * Chebyshev coefficients (section "Decomposition of the diffusion tensor",
 * eq. cheb1): c_p = (2/N) sum_{j=1..N} f(cos th_j) cos(p th_j),
 * th_j = pi (j - 1/2)/N, f(x) = sqrt(((dmax-dmin)/2) x + (dmax+dmin)/2).
 * ---------------------------------------------------------------------- */
void orc_cheb_coeffs(int nch, double dmin, double dmax, double *c)
{
    for (int p = 0; p < nch; ++p) {
        double s = 0.0;
        for (int j = 1; j <= nch; ++j) {
            double th = ORC_PI * (j - 0.5) / nch;
            double x = cos(th);
            double f = sqrt(0.5 * (dmax - dmin) * x + 0.5 * (dmax + dmin));
            s += f * cos(p * th);
        }
        c[p] = 2.0 * s / nch;
    }
}

/* y = Y . v with Y = (2/(dmax-dmin)) D - ((dmax+dmin)/(dmax-dmin)) I (eq. cheb3) */
static void apply_Y(int n3, const double *D, double dmin, double dmax,
                    const double *v, double *y)
{
    orc_matvec(n3, D, 1, v, y);
    double s = 2.0 / (dmax - dmin), t = (dmax + dmin) / (dmax - dmin);
    for (int i = 0; i < n3; ++i) y[i] = s * y[i] - t * v[i];
}

/* dS = sum_{p<N_Ch} c_p V_p - (c_0/2) dW with V_0 = dW, V_1 = Y V_0,
 * V_p = 2 Y V_{p-1} - V_{p-2} (eq. cheb1, cheb2).  m right-hand sides. */
void orc_cheb_sqrt(int n3, const double *D, int m, const double *dw, int nch,
                   double dmin, double dmax, double *out)
{
    double *c = (double *)malloc(sizeof(double) * nch);
    double *v0 = (double *)malloc(sizeof(double) * n3);
    double *v1 = (double *)malloc(sizeof(double) * n3);
    double *v2 = (double *)malloc(sizeof(double) * n3);
    orc_cheb_coeffs(nch, dmin, dmax, c);
    for (int j = 0; j < m; ++j) {
        const double *w = dw + (long)j * n3;
        double *o = out + (long)j * n3;
        for (int i = 0; i < n3; ++i) { v0[i] = w[i]; o[i] = c[0] * w[i] - 0.5 * c[0] * w[i]; }
        if (nch > 1) {
            apply_Y(n3, D, dmin, dmax, v0, v1);
            for (int i = 0; i < n3; ++i) o[i] += c[1] * v1[i];
        }
        for (int p = 2; p < nch; ++p) {
            apply_Y(n3, D, dmin, dmax, v1, v2);
            for (int i = 0; i < n3; ++i) {
                v2[i] = 2.0 * v2[i] - v0[i];
                o[i] += c[p] * v2[i];
            }
            double *t = v0; v0 = v1; v1 = v2; v2 = t;
        }
    }
    free(c); free(v0); free(v1); free(v2);
}

/* E_f = sqrt(|dS.dS - dW.D.dW| / (dW.D.dW)) (section "Decomposition of the
 * diffusion tensor", error estimate). */
double orc_sqrt_error(int n3, const double *D, const double *dw, const double *ds)
{
    double *y = (double *)malloc(sizeof(double) * n3);
    orc_matvec(n3, D, 1, dw, y);
    double wdw = 0.0, ss = 0.0;
    for (int i = 0; i < n3; ++i) { wdw += dw[i] * y[i]; ss += ds[i] * ds[i]; }
    free(y);
    return sqrt(fabs(ss - wdw) / wdw);
}

/* Adaptive order (section "Decomposition of the diffusion tensor",
 * eq. nint and the E_f criterion): start from
 *   N_Ch = nint(sqrt(dmax / dmin)) + 1   (nint: round half away from zero)
 * (or from nch0 when nch0 >= 2) and increase N_Ch by one until E_f < tol
 * for every right-hand side, or N_Ch = nmax.  Each trial recomputes the
 * whole recurrence from scratch.  Returns the final N_Ch; out holds its dS. */
int orc_cheb_adaptive(int n3, const double *D, int m, const double *dw, int nch0, int nmax,
                      double dmin, double dmax, double tol, double *out)
{
    int n = nch0 >= 2 ? nch0 : (int)lround(sqrt(dmax / dmin)) + 1;
    if (n < 2) n = 2;
    if (n > nmax) n = nmax;
    for (;;) {
        orc_cheb_sqrt(n3, D, m, dw, n, dmin, dmax, out);
        double worst = 0.0;
        for (int j = 0; j < m; ++j) {
            double e = orc_sqrt_error(n3, D, dw + (long)j * n3, out + (long)j * n3);
            if (e > worst) worst = e;
        }
        if (worst < tol || n >= nmax) return n;
        ++n;
    }
}

/* Lanczos tridiagonalisation of the symmetric D from the start vector
 * (Lanczos 1950): q_1 = start/|start|, and for j = 1..k
 *   w = D q_j - beta_{j-1} q_{j-1},  alpha_j = q_j . w,
 *   w = w - alpha_j q_j,  beta_j = |w|,  q_{j+1} = w / beta_j
 * (no reorthogonalisation).  alpha, beta: [k]. */
void orc_lanczos(int n3, const double *D, const double *start, int k, double *alpha,
                 double *beta)
{
    double *qp = (double *)calloc(n3, sizeof(double));
    double *q = (double *)malloc(sizeof(double) * n3);
    double *w = (double *)malloc(sizeof(double) * n3);
    double nrm = 0.0;
    for (int i = 0; i < n3; ++i) nrm += start[i] * start[i];
    nrm = sqrt(nrm);
    for (int i = 0; i < n3; ++i) q[i] = start[i] / nrm;
    double bprev = 0.0;
    for (int j = 0; j < k; ++j) {
        orc_matvec(n3, D, 1, q, w);
        for (int i = 0; i < n3; ++i) w[i] -= bprev * qp[i];
        double a = 0.0;
        for (int i = 0; i < n3; ++i) a += q[i] * w[i];
        for (int i = 0; i < n3; ++i) w[i] -= a * q[i];
        double b = 0.0;
        for (int i = 0; i < n3; ++i) b += w[i] * w[i];
        b = sqrt(b);
        alpha[j] = a;
        beta[j] = b;
        for (int i = 0; i < n3; ++i) {
            qp[i] = q[i];
            q[i] = w[i] / b;
        }
        bprev = b;
    }
    free(qp); free(q); free(w);
}

/* Paper's semidilute bound rule: lmax_F = U+.D.U+/(3N) (eq. lmax-lmin-dilute),
 * lmax = 0.35 N^0.6 lmax_F (eq. fmax), lmin = lmax/(C N^0.6) (eq. fmin),
 * with d_max = lmax, d_min = lmin. */
void orc_bounds_rule(int nbeads, const double *D, double C, double *dmin, double *dmax)
{
    int n3 = 3 * nbeads;
    double s = 0.0;
    for (long i = 0; i < n3; ++i)
        for (long k = 0; k < n3; ++k) s += D[i * n3 + k];
    double lf = s / n3;
    double lmax = 0.35 * pow((double)nbeads, 0.6) * lf;
    *dmax = lmax;
    *dmin = lmax / (C * pow((double)nbeads, 0.6));
}

/* Dilute bound rule (eq. lmax-lmin-dilute): lmax_F = U+.D.U+/(3N) and
 * lmin_F = U-.D.U-/(3N), U+ all ones, U- alternating 1, -1 over the
 * flattened index 3 nu + i starting with +1, and the bounds the paper quotes
 * with it: d_max = 2 lmax_F, d_min = lmin_F / 2. */
void orc_bounds_dilute(int nbeads, const double *D, double *dmin, double *dmax)
{
    int n3 = 3 * nbeads;
    double sp = 0.0, sm = 0.0;
    for (long i = 0; i < n3; ++i)
        for (long k = 0; k < n3; ++k) {
            double ui = (i % 2 == 0) ? 1.0 : -1.0, uk = (k % 2 == 0) ? 1.0 : -1.0;
            sp += D[i * n3 + k];
            sm += ui * D[i * n3 + k] * uk;
        }
    *dmax = 2.0 * sp / n3;
    *dmin = 0.5 * sm / n3;
}

/* Hookean spring forces (section "Governing equation"): beads are stored
 * chain after chain, bpc beads each; Q_mu = r_{mu+1} - r_mu (unwrapped);
 * F_mu = Q_mu - Q_{mu-1}.  F is overwritten. */
void orc_spring_forces(int nchains, int bpc, const double *r, double *F)
{
    for (int c = 0; c < nchains; ++c)
        for (int b = 0; b < bpc; ++b) {
            int mu = c * bpc + b;
            for (int i = 0; i < 3; ++i) {
                double f = 0.0;
                if (b + 1 < bpc) f += r[3 * (mu + 1) + i] - r[3 * mu + i];
                if (b > 0) f -= r[3 * mu + i] - r[3 * (mu - 1) + i];
                F[3 * mu + i] = f;
            }
        }
}

/* Narrow-Gaussian excluded volume between all beads and all periodic images
 * within rcut: U = zs ds^-3 exp(-r^2/(2 ds^2)) (zs = z-star, ds = d-star),
 * so F_nu += zs ds^-5 d exp(-r^2/(2 ds^2)) with d = r_nu - r_mu + n L.
 * F is accumulated. */
void orc_ev_forces(int n, const double *rt, double L, double zs, double ds,
                   double rcut, double *F)
{
    int ni = (int)ceil(rcut / L) + 1;
    double pref = zs / (ds * ds * ds * ds * ds);
#pragma omp parallel for
    for (int nu = 0; nu < n; ++nu) {
        double f[3] = {0, 0, 0};
        for (int mu = 0; mu < n; ++mu)
            for (int nx = -ni; nx <= ni; ++nx)
                for (int ny = -ni; ny <= ni; ++ny)
                    for (int nz = -ni; nz <= ni; ++nz) {
                        if (nu == mu && nx == 0 && ny == 0 && nz == 0) continue;
                        double d[3];
                        d[0] = (rt[3 * nu + 0] - rt[3 * mu + 0]) + nx * L;
                        d[1] = (rt[3 * nu + 1] - rt[3 * mu + 1]) + ny * L;
                        d[2] = (rt[3 * nu + 2] - rt[3 * mu + 2]) + nz * L;
                        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                        if (r2 > rcut * rcut) continue;
                        double w = pref * exp(-r2 / (2.0 * ds * ds));
                        for (int i = 0; i < 3; ++i) f[i] += w * d[i];
                    }
        for (int i = 0; i < 3; ++i) F[3 * nu + i] += f[i];
    }
}

/* Euler-Maruyama update (eq. sde with kappa = 0):
 * r_out = r + (dt/4) u_d + dS / sqrt(2). */
void orc_euler(int n3, const double *r, double dt, const double *ud,
               const double *ds, double *rout)
{
    for (int i = 0; i < n3; ++i)
        rout[i] = r[i] + dt / 4.0 * ud[i] + ds[i] / sqrt(2.0);
}

/* Per-chain R_e^2 = |r_Nb - r_1|^2 and R_g^2 = (1/(2 Nb^2)) sum_mu sum_nu
 * |r_nu - r_mu|^2 (section "Testing and verification"). */
void orc_chain_observables(int nchains, int bpc, const double *r, double *re2,
                           double *rg2)
{
    for (int c = 0; c < nchains; ++c) {
        const double *x = r + 3L * c * bpc;
        double e = 0.0;
        for (int i = 0; i < 3; ++i) {
            double d = x[3 * (bpc - 1) + i] - x[i];
            e += d * d;
        }
        re2[c] = e;
        double g = 0.0;
        for (int mu = 0; mu < bpc; ++mu)
            for (int nu = 0; nu < bpc; ++nu)
                for (int i = 0; i < 3; ++i) {
                    double d = x[3 * nu + i] - x[3 * mu + i];
                    g += d * d;
                }
        rg2[c] = g / (2.0 * bpc * bpc);
    }
}

/* ------------------------------------------------------------------------
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11): 10 rounds of the 4x32 Philox S-box with
 * multipliers 0xD2511F53, 0xCD9E8D57 and Weyl key increments 0x9E3779B9,
 * 0xBB67AE85.
 * ---------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                       uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Gaussian noise dW ~ N(0, dt) per component.  Element e of the flattened
 * [m][3N] array uses Philox block g = e / 4 with counter
 * (g, step_lo, step_hi, 0x52505942) and key (seed_lo, seed_hi); the four
 * outputs x_j map to u_j = (x_j + 0.5) 2^-32 and Box-Muller gives
 * z0 = rho cos(2 pi u1), z1 = rho sin(2 pi u1) with rho = sqrt(-2 ln u0), and
 * z2, z3 likewise from (u2, u3).  e takes z_{e mod 4} * sqrt(dt). */
void orc_gaussian_noise(long count, uint64_t seed, uint64_t step, double dt,
                        double *out)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    double sdt = sqrt(dt);
    for (long g = 0; 4 * g < count; ++g) {
        uint32_t ctr[4] = {(uint32_t)g, (uint32_t)step, (uint32_t)(step >> 32),
                           0x52505942u};
        uint32_t x[4];
        orc_philox4x32_10(ctr, key, x);
        double u[4], z[4];
        for (int j = 0; j < 4; ++j) u[j] = ((double)x[j] + 0.5) * (1.0 / 4294967296.0);
        double rho0 = sqrt(-2.0 * log(u[0])), rho1 = sqrt(-2.0 * log(u[2]));
        z[0] = rho0 * cos(2.0 * ORC_PI * u[1]);
        z[1] = rho0 * sin(2.0 * ORC_PI * u[1]);
        z[2] = rho1 * cos(2.0 * ORC_PI * u[3]);
        z[3] = rho1 * sin(2.0 * ORC_PI * u[3]);
        for (int j = 0; j < 4 && 4 * g + j < count; ++j) out[4 * g + j] = z[j] * sdt;
    }
}

/* ========================================================================
 * Reverse mode of u = D(R) F + p(D(R)) dW, where p(D) dW is the Chebyshev
 * sum dS of orc_cheb_sqrt with a fixed interval [dmin, dmax] (no
 * dependence of the interval on R).  The derivatives of the pair terms are
 * not printed in the paper; they are the r-derivatives of the coefficients
 * of eq. M1, eq. b1/b2 and eq. cor5 as printed (with reading R2), and of
 * the cosine of eq. M2, written out below.
 *
 * Given g = dL/du, dL/dF = D g (D symmetric) and, with the adjoint
 * vectors of the recurrence
 *   mu_p = c_p g + 2 Y mu_{p+1} - mu_{p+2}   (p = N_Ch-1 .. 1, mu_{N_Ch} = mu_{N_Ch+1} = 0),
 * dL = sum_q x_q^T dD y_q over the pairs (x_q, y_q) = (g, F),
 * (s mu_1, V_0), (2 s mu_p, V_{p-1}) for p >= 2, s = 2/(dmax - dmin).
 * The pair block D_lm depends on d = r_l - r_m only and is even in d, so
 *   dL/dr_l = sum_{m != l} grad_d [ W_lm : D(d) ] at d = r_l - r_m,
 *   W_lm = sum_q (x_q,l y_q,m^T + x_q,m y_q,l^T)   (3 x 3).
 * For D(d) = c1(r) I + c2(r) dhat dhat and symmetric Ws = (W + W^T)/2:
 *   grad_k = c1' dhat_k tr(Ws) + c2' dhat_k (dhat.Ws.dhat)
 *          + (c2 / r) (2 (Ws dhat)_k - 2 dhat_k (dhat.Ws.dhat)),
 * and for the reciprocal part m(k) (I - khat khat) cos(k.d):
 *   grad = - sum_{+-k} m(k) ((I - khat khat) : Ws) sin(k.d) k.
 * The self term and the images of a bead with itself do not move with r_l.
 * At r = 0 (coincident distinct beads) the pair term is not differentiable;
 * it contributes nothing.
 * ====================================================================== */

/* d/dr of the M1 coefficients (eq. M1), binary128:
 * c1 = e A + g B, c2 = e A2 + g B2 with e = erfc(al r), g = exp(-al^2 r^2)/sqrt(pi),
 * de/dr = -2 al g, dg/dr = -2 al^2 r g. */
static void m1_dcoeffs_q(__float128 r, __float128 a, __float128 al,
                         __float128 *d1, __float128 *d2)
{
    __float128 a3 = a * a * a;
    __float128 e = erfcq(al * r);
    __float128 g = expq(-al * al * r * r) / sqrtq(M_PIq);
    __float128 r2 = r * r, r3 = r2 * r, r4 = r2 * r2, r5 = r4 * r;
    __float128 al3 = al * al * al, al5 = al3 * al * al, al7 = al5 * al * al;
    __float128 A = 3 * a / (4 * r) + a3 / (2 * r3);
    __float128 Ap = -3 * a / (4 * r2) - 3 * a3 / (2 * r4);
    __float128 B = 3 * a * al3 * r2 - 9 * a * al / 2 + 4 * a3 * al7 * r4
                 - 20 * a3 * al5 * r2 + 14 * a3 * al3 + a3 * al / r2;
    __float128 Bp = 6 * a * al3 * r + 16 * a3 * al7 * r3 - 40 * a3 * al5 * r - 2 * a3 * al / r3;
    __float128 A2 = 3 * a / (4 * r) - 3 * a3 / (2 * r3);
    __float128 A2p = -3 * a / (4 * r2) + 9 * a3 / (2 * r4);
    __float128 B2 = 3 * a * al / 2 - 3 * a * al3 * r2 - 4 * a3 * al7 * r4
                  + 16 * a3 * al5 * r2 - 2 * a3 * al3 - 3 * a3 * al / r2;
    __float128 B2p = -6 * a * al3 * r - 16 * a3 * al7 * r3 + 32 * a3 * al5 * r + 6 * a3 * al / r3;
    (void)r5;
    *d1 = -2 * al * g * A + e * Ap - 2 * al * al * r * g * B + g * Bp;
    *d2 = -2 * al * g * A2 + e * A2p - 2 * al * al * r * g * B2 + g * B2p;
}

/* d/dx of the M* coefficients (eq. cor5 with reading R2), x = r/a:
 * c1 = 1 - t1^2/(2x^3), t1 = 3x^2/4 + 1;  c2 = 3 t2^2/(2x^3), t2 = x^2/4 - 1. */
static void mstar_dcoeffs_q(__float128 x, __float128 *d1, __float128 *d2)
{
    __float128 x2 = x * x, x3 = x2 * x, x4 = x2 * x2;
    __float128 t1 = 3 * x2 / 4 + 1, t2 = x2 / 4 - 1;
    *d1 = -t1 * (3 * x / 2) / x3 + 3 * t1 * t1 / (2 * x4);
    *d2 = 3 * t2 / (2 * x2) - 9 * t2 * t2 / (2 * x4);
}

/* Gradient with respect to the image separation d of Ws : (c1 I + c2 dhat dhat)
 * for one image (same branches as pair_image); added into gk. */
static void pair_image_grad(const double d[3], double r2, int in_rc, int overlap,
                            double a, double al, const double Ws[9], double gk[3])
{
    if (r2 == 0.0) return;
    double r = sqrt(r2);
    double c2 = 0.0, d1 = 0.0, d2 = 0.0;
    if (overlap) {
        if (in_rc && r / a < 1e-6) {
            /* Omega_B - S with S even and smooth: S' = O(r) */
            c2 = 3.0 * r / (32.0 * a);
            d1 = -9.0 / (32.0 * a);
            d2 = 3.0 / (32.0 * a);
        } else {
            __float128 rq = sqrtq((__float128)d[0] * d[0] + (__float128)d[1] * d[1]
                                  + (__float128)d[2] * d[2]);
            __float128 q1 = 0, q2 = 0, p1 = 0, p2 = 0, s1, s2, t1, t2;
            if (in_rc) {
                m1_coeffs_q(rq, a, al, &q1, &q2);
                m1_dcoeffs_q(rq, a, al, &p1, &p2);
            }
            mstar_coeffs_q(rq / a, &s1, &s2);
            mstar_dcoeffs_q(rq / a, &t1, &t2);
            c2 = (double)(q2 + s2);
            d1 = (double)(p1 + t1 / a);
            d2 = (double)(p2 + t2 / a);
        }
    } else {
        double c1v;
        orc_m1_coeffs(r, a, al, &c1v, &c2);
        __float128 p1, p2;
        m1_dcoeffs_q(r, a, al, &p1, &p2);
        d1 = (double)p1;
        d2 = (double)p2;
    }
    double h[3] = {d[0] / r, d[1] / r, d[2] / r};
    double tr = Ws[0] + Ws[4] + Ws[8];
    double Wh[3], hWh = 0.0;
    for (int i = 0; i < 3; ++i) {
        Wh[i] = Ws[3 * i] * h[0] + Ws[3 * i + 1] * h[1] + Ws[3 * i + 2] * h[2];
        hWh += h[i] * Wh[i];
    }
    for (int k = 0; k < 3; ++k)
        gk[k] += d1 * h[k] * tr + d2 * h[k] * hWh + (c2 / r) * (2.0 * Wh[k] - 2.0 * h[k] * hWh);
}

/* Reverse mode of u = D F + p(D) dW (see above) for the listed beads:
 * gpos[ir][3] = dL/dr of bead rows[ir]; gF[3N] = D g (NULL: skipped).
 * pos are unwrapped positions (the derivative of the wrap is 1). */
void orc_u_vjp_rows(int n, const double *pos, double L, double a, double al, double rc,
                    int n2max, const double *F, const double *dw, const double *g, int nch,
                    double dmin, double dmax, int nrows, const int *rows, double *gpos,
                    double *gF)
{
    long n3 = 3L * n;
    double *rt = (double *)malloc(sizeof(double) * n3);
    double *D = (double *)calloc((size_t)n3 * n3, sizeof(double));
    orc_wrap(n, pos, L, rt);
    orc_real_space(n, rt, L, a, al, rc, D);
    orc_self_term(n, a, al, D);
    orc_recip_space(n, rt, L, a, al, n2max, D);
    if (gF) orc_matvec((int)n3, D, 1, g, gF);
    /* forward recurrence, all V_p kept */
    double *V = (double *)malloc(sizeof(double) * n3 * nch);
    double *c = (double *)malloc(sizeof(double) * nch);
    orc_cheb_coeffs(nch, dmin, dmax, c);
    for (long i = 0; i < n3; ++i) V[i] = dw[i];
    if (nch > 1) apply_Y((int)n3, D, dmin, dmax, V, V + n3);
    for (int p = 2; p < nch; ++p) {
        apply_Y((int)n3, D, dmin, dmax, V + (p - 1) * n3, V + p * n3);
        for (long i = 0; i < n3; ++i) V[p * n3 + i] = 2.0 * V[p * n3 + i] - V[(p - 2) * n3 + i];
    }
    /* adjoint recurrence: mu[p], p = 1 .. nch-1 (mu[nch], mu[nch+1] = 0) */
    double *mu = (double *)calloc((size_t)n3 * (nch + 2), sizeof(double));
    double *t = (double *)malloc(sizeof(double) * n3);
    for (int p = nch - 1; p >= 1; --p) {
        double *m = mu + p * n3;
        apply_Y((int)n3, D, dmin, dmax, mu + (p + 1) * n3, t);
        for (long i = 0; i < n3; ++i)
            m[i] = c[p] * g[i] + 2.0 * t[i] - mu[(p + 2) * n3 + i];
    }
    /* pairs (x_q, y_q), q = 0 .. nch-1 */
    double s = 2.0 / (dmax - dmin);
    int nq = nch;
    double *X = (double *)malloc(sizeof(double) * n3 * nq);
    double *Yv = (double *)malloc(sizeof(double) * n3 * nq);
    for (long i = 0; i < n3; ++i) { X[i] = g[i]; Yv[i] = F[i]; }
    for (int q = 1; q < nq; ++q) {
        double f = q == 1 ? s : 2.0 * s;
        for (long i = 0; i < n3; ++i) {
            X[q * n3 + i] = f * mu[q * n3 + i];
            Yv[q * n3 + i] = V[(q - 1) * n3 + i];
        }
    }
    double vol = L * L * L;
    int nm = (int)floor(sqrt((double)n2max)) + 1;
    int ni = (int)ceil(rc / L) + 1;
    double rc2 = rc * rc, a2x4 = 4.0 * a * a;
#pragma omp parallel for schedule(dynamic)
    for (int ir = 0; ir < nrows; ++ir) {
        int l = rows[ir];
        double acc[3] = {0, 0, 0};
        for (int m = 0; m < n; ++m) {
            if (m == l) continue;
            double W[9] = {0};
            for (int q = 0; q < nq; ++q)
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j)
                        W[3 * i + j] += X[q * n3 + 3 * l + i] * Yv[q * n3 + 3 * m + j]
                                      + X[q * n3 + 3 * m + i] * Yv[q * n3 + 3 * l + j];
            double Ws[9];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) Ws[3 * i + j] = 0.5 * (W[3 * i + j] + W[3 * j + i]);
            double d0[3] = {rt[3 * l] - rt[3 * m], rt[3 * l + 1] - rt[3 * m + 1],
                            rt[3 * l + 2] - rt[3 * m + 2]};
            /* real space: every image within rc or closer than 2a */
            for (int nx = -ni; nx <= ni; ++nx)
                for (int ny = -ni; ny <= ni; ++ny)
                    for (int nz = -ni; nz <= ni; ++nz) {
                        double d[3] = {d0[0] + nx * L, d0[1] + ny * L, d0[2] + nz * L};
                        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                        int in_rc = r2 <= rc2, overlap = r2 < a2x4;
                        if (!in_rc && !overlap) continue;
                        pair_image_grad(d, r2, in_rc, overlap, a, al, Ws, acc);
                    }
            /* reciprocal space: full +-k set */
            for (int kx = -nm; kx <= nm; ++kx)
                for (int ky = -nm; ky <= nm; ++ky)
                    for (int kz = -nm; kz <= nm; ++kz) {
                        int n2 = kx * kx + ky * ky + kz * kz;
                        if (n2 == 0 || n2 > n2max) continue;
                        double k[3] = {2.0 * ORC_PI * kx / L, 2.0 * ORC_PI * ky / L,
                                       2.0 * ORC_PI * kz / L};
                        double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
                        double mk = orc_m2_scalar(sqrt(k2), a, al, vol);
                        double PW = 0.0;
                        for (int i = 0; i < 3; ++i)
                            for (int j = 0; j < 3; ++j)
                                PW += ((i == j ? 1.0 : 0.0) - k[i] * k[j] / k2) * Ws[3 * i + j];
                        double sn = sin(k[0] * d0[0] + k[1] * d0[1] + k[2] * d0[2]);
                        for (int i = 0; i < 3; ++i) acc[i] -= mk * PW * sn * k[i];
                    }
        }
        for (int i = 0; i < 3; ++i) gpos[3 * ir + i] = acc[i];
    }
    free(rt); free(D); free(V); free(c); free(mu); free(t); free(X); free(Yv);
}
