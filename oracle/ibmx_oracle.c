/*
 * ibmx_oracle.c -- plain, sequential FP64 CPU oracle of the direct-forcing
 * IBM outer forcing loop and of the collision pair pass of Yao et al.,
 * "Particle-resolved simulations of four-way coupled, polydispersed,
 * particle-laden flows" (arXiv 2109.03972).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * source, header, table or helper with the HIP library; the two meet only
 * in the seeded input arrays.  It is written for a reader who checks it
 * against the paper: no blocking, no fusion, no reordering.
 *
 * Conventions (all arrays row-major, caller-owned, host memory):
 *   grid field     double [3][nz][ny][nx], x fastest; node (i,j,k) sits at
 *                  origin + (i + 1/2, j + 1/2, k + 1/2) h (cell centres of the
 *                  collocated finite-volume grid, Sec. 2.2.1).  A non-periodic
 *                  axis has walls at origin and origin + n h.
 *   particle data  double [3][np] (component-major).
 *   markers        CSR offsets moff[np+1]; body offsets o_l = X_l - x_p as
 *                  double [3][nm]; dV[p] is the marker volume of particle p.
 *
 * Return codes: 0 ok, -1 invalid argument, -2 an active marker's delta
 * support leaves the grid through a wall, -6 list capacity exceeded.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define R_OK 0
#define R_EINVAL (-1)
#define R_EDOMAIN (-2)
#define R_ECAPACITY (-6)

/* ------------------------------------------------------------------------ */
/* Regularized delta functions                                              */
/* ------------------------------------------------------------------------ */

/* Three-point function phi_3 of Roma et al. (Sec. 2.1, eq. 3pt-stencil). */
double ref_phi3(double r)
{
    double a = fabs(r);
    if (a <= 0.5)
        return (1.0 + sqrt(1.0 - 3.0 * a * a)) / 3.0;
    if (a <= 1.5)
        return (5.0 - 3.0 * a - sqrt(1.0 - 3.0 * (1.0 - a) * (1.0 - a))) / 6.0;
    return 0.0;
}

/* d phi_3 / d r, differentiated from the same formula. */
double ref_dphi3(double r)
{
    double a = fabs(r);
    double s = (r < 0.0) ? -1.0 : 1.0;
    if (a <= 0.5) {
        if (a == 0.0)
            return 0.0;
        return -r / sqrt(1.0 - 3.0 * r * r);
    }
    if (a <= 1.5) {
        double b = 1.0 - a;
        double q = sqrt(1.0 - 3.0 * b * b);
        if (q == 0.0)
            return 0.0;
        return s * (-0.5 - 0.5 * b / q);
    }
    return 0.0;
}

/* Four-point function phi_4 of Peskin (Sec. 2.2.3, eq. 4pt-stencil).  The
 * printed range of the first branch reads -2 <= r <= 1; the branch is the
 * mirror of the last one, i.e. -2 <= r <= -1. */
double ref_phi4(double r)
{
    if (r >= -2.0 && r <= -1.0)
        return (5.0 + 2.0 * r - sqrt(-7.0 - 12.0 * r - 4.0 * r * r)) / 8.0;
    if (r > -1.0 && r <= 0.0)
        return (3.0 + 2.0 * r + sqrt(1.0 - 4.0 * r - 4.0 * r * r)) / 8.0;
    if (r > 0.0 && r <= 1.0)
        return (3.0 - 2.0 * r + sqrt(1.0 + 4.0 * r - 4.0 * r * r)) / 8.0;
    if (r > 1.0 && r <= 2.0)
        return (5.0 - 2.0 * r - sqrt(-7.0 + 12.0 * r - 4.0 * r * r)) / 8.0;
    return 0.0;
}

double ref_dphi4(double r)
{
    if (r >= -2.0 && r <= -1.0) {
        double q = sqrt(-7.0 - 12.0 * r - 4.0 * r * r);
        return q == 0.0 ? 0.0 : (2.0 - (-12.0 - 8.0 * r) / (2.0 * q)) / 8.0;
    }
    if (r > -1.0 && r <= 0.0) {
        double q = sqrt(1.0 - 4.0 * r - 4.0 * r * r);
        return (2.0 + (-4.0 - 8.0 * r) / (2.0 * q)) / 8.0;
    }
    if (r > 0.0 && r <= 1.0) {
        double q = sqrt(1.0 + 4.0 * r - 4.0 * r * r);
        return (-2.0 + (4.0 - 8.0 * r) / (2.0 * q)) / 8.0;
    }
    if (r > 1.0 && r <= 2.0) {
        double q = sqrt(-7.0 + 12.0 * r - 4.0 * r * r);
        return q == 0.0 ? 0.0 : (-2.0 - (12.0 - 8.0 * r) / (2.0 * q)) / 8.0;
    }
    return 0.0;
}

static double phi_k(int kernel, double r) { return kernel == 4 ? ref_phi4(r) : ref_phi3(r); }
static double dphi_k(int kernel, double r) { return kernel == 4 ? ref_dphi4(r) : ref_dphi3(r); }

/* ------------------------------------------------------------------------ */
/* Delta support of one marker                                              */
/* ------------------------------------------------------------------------ */

typedef struct {
    int cnt[3];          /* nodes per axis with nonzero weight window      */
    long idx[3][4];      /* wrapped node index per axis                    */
    double w[3][4];      /* phi(r) per axis                                */
    double dw[3][4];     /* phi'(r) per axis                               */
} support_t;

/* Nodes whose 1-D delta weight can be nonzero: |x_i - X| / h < W/2, with
 * x_i = origin + (i + 1/2) h.  The product of the three 1-D weights is
 * delta_h,3D(x - X) h^3 (Sec. 2.1).  Periodic axes wrap the index; a node
 * beyond a wall makes the marker invalid. */
static int marker_support(const int *n, double h, const double *origin, const int *periodic,
                          int kernel, const double *X, support_t *sp)
{
    double half = (kernel == 4) ? 2.0 : 1.5;
    for (int a = 0; a < 3; ++a) {
        double s = (X[a] - origin[a]) / h;          /* position in units of h */
        long lo = (long)floor(s - 0.5 - half) + 1;   /* first i with i+1/2-s > -half */
        int c = 0;
        for (long i = lo; i < lo + 6; ++i) {
            double r = ((double)i + 0.5) - s;
            if (!(r < half))
                break;
            if (!(r > -half))
                continue;
            long ii = i;
            if (periodic[a]) {
                ii = i % n[a];
                if (ii < 0)
                    ii += n[a];
            } else if (i < 0 || i >= n[a]) {
                return R_EDOMAIN;
            }
            sp->idx[a][c] = ii;
            sp->w[a][c] = phi_k(kernel, r);
            sp->dw[a][c] = dphi_k(kernel, r);
            ++c;
        }
        sp->cnt[a] = c;
    }
    return R_OK;
}

static int check_markers(const int *n, double h, const double *origin, const int *periodic,
                         int kernel, int np, const int *moff, const double *body,
                         const double *xp, const unsigned char *mask)
{
    int nm = moff[np];
    for (int p = 0; p < np; ++p) {
        if (moff[p + 1] < moff[p])
            return R_EINVAL;
        for (int l = moff[p]; l < moff[p + 1]; ++l) {
            if (mask && !mask[l])
                continue;
            double X[3];
            support_t sp;
            for (int a = 0; a < 3; ++a)
                X[a] = xp[a * np + p] + body[a * nm + l];
            int st = marker_support(n, h, origin, periodic, kernel, X, &sp);
            if (st != R_OK)
                return st;
        }
    }
    return R_OK;
}

static void cross(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

/* U_l = sum_x w(x - X_l) g(x) for one marker (Sec. 2.2.2, step 1). */
static void interp3(const support_t *sp, long nx, long ny, long N, const double *g, double *U)
{
    U[0] = U[1] = U[2] = 0.0;
    for (int k = 0; k < sp->cnt[2]; ++k)
        for (int j = 0; j < sp->cnt[1]; ++j)
            for (int i = 0; i < sp->cnt[0]; ++i) {
                double w = sp->w[2][k] * sp->w[1][j] * sp->w[0][i];
                long node = sp->idx[0][i] + nx * (sp->idx[1][j] + ny * sp->idx[2][k]);
                for (int c = 0; c < 3; ++c)
                    U[c] += w * g[c * N + node];
            }
}

/* ------------------------------------------------------------------------ */
/* Outer forcing loop (Sec. 2.2.2)                                          */
/* ------------------------------------------------------------------------ */

/*
 * For m = 1..n_iter:
 *   U^{m-1}_l = sum_x u^{m-1}(x) delta_h(x - X_l) h^3             (step 1)
 *   F^{m-1}_l = (U^d_l - U^{m-1}_l) / c,  c = 2 alpha_k dt,
 *               U^d_l = u_p + omega_p x (X_l - x_p)              (step 2)
 *   f^{m-1}(x) = sum_l F^{m-1}_l delta_h(x - X_l) dV_l            (step 3)
 *   u^m = u^{m-1} + c f^{m-1}                                     (step 4)
 * Outputs: u <- u^{n_iter} (in place); f_tot += sum_m f^{m-1};
 * S_p = sum_m sum_l F_l dV_l and T_p = sum_m sum_l (X_l - x_p) x F_l dV_l
 * (the sums of Sec. 2.1, eq. basic-particle; the hydrodynamic force and
 * torque are -rho_f S_p and -rho_f T_p); resid[m-1] = sqrt(sum_l dV_l
 * |U^d_l - U^{m-1}_l|^2), the no-slip error of Sec. 2.2.2 weighted by the
 * marker volumes; resid[n_iter] (if final_resid) measures u^{n_iter}.
 * U_dbg (optional) receives U^{m-1}_l as [n_iter][3][nm] for active markers.
 * Markers with mask[l] == 0 take no part (Sec. 2.2.5, disabling markers).
 */
int ref_forcing(const int *n, double h, const double *origin, const int *periodic,
                int kernel, int n_iter, double c, int final_resid,
                int np, const int *moff, const double *body, const double *dV,
                const double *xp, const double *up, const double *wp,
                const unsigned char *mask,
                double *u, double *f_tot, double *S, double *T,
                double *resid, double *U_dbg)
{
    if (!n || n[0] <= 0 || n[1] <= 0 || n[2] <= 0 || !(h > 0.0) || n_iter < 1 ||
        !(c != 0.0) || np < 0 || (kernel != 3 && kernel != 4))
        return R_EINVAL;
    int st = check_markers(n, h, origin, periodic, kernel, np, moff, body, xp, mask);
    if (st != R_OK)
        return st;
    long nx = n[0], ny = n[1], N = (long)n[0] * n[1] * n[2];
    int nm = moff[np];
    double h3 = h * h * h;
    double *fm = (double *)malloc(sizeof(double) * 3 * (size_t)N);
    if (!fm)
        return R_EINVAL;
    for (int i = 0; i < 3 * np; ++i) {
        S[i] = 0.0;
        T[i] = 0.0;
    }
    for (int m = 1; m <= n_iter; ++m) {
        memset(fm, 0, sizeof(double) * 3 * (size_t)N);
        double rsq = 0.0;
        for (int p = 0; p < np; ++p) {
            double upp[3], wpp[3];
            for (int a = 0; a < 3; ++a) {
                upp[a] = up[a * np + p];
                wpp[a] = wp[a * np + p];
            }
            for (int l = moff[p]; l < moff[p + 1]; ++l) {
                if (mask && !mask[l])
                    continue;
                double o[3], X[3], U[3], Ud[3], wxo[3], F[3], oxF[3];
                support_t sp;
                for (int a = 0; a < 3; ++a) {
                    o[a] = body[a * nm + l];
                    X[a] = xp[a * np + p] + o[a];
                }
                marker_support(n, h, origin, periodic, kernel, X, &sp);
                interp3(&sp, nx, ny, N, u, U);                       /* step 1 */
                if (U_dbg)
                    for (int a = 0; a < 3; ++a)
                        U_dbg[((size_t)(m - 1) * 3 + a) * nm + l] = U[a];
                cross(wpp, o, wxo);
                for (int a = 0; a < 3; ++a) {
                    Ud[a] = upp[a] + wxo[a];
                    double r = Ud[a] - U[a];
                    rsq += dV[p] * r * r;
                    F[a] = r / c;                                    /* step 2 */
                    S[a * np + p] += F[a] * dV[p];
                }
                cross(o, F, oxF);
                for (int a = 0; a < 3; ++a)
                    T[a * np + p] += oxF[a] * dV[p];
                for (int k = 0; k < sp.cnt[2]; ++k)                   /* step 3 */
                    for (int j = 0; j < sp.cnt[1]; ++j)
                        for (int i = 0; i < sp.cnt[0]; ++i) {
                            double w = sp.w[2][k] * sp.w[1][j] * sp.w[0][i];
                            long node = sp.idx[0][i] + nx * (sp.idx[1][j] + ny * sp.idx[2][k]);
                            for (int a = 0; a < 3; ++a)
                                fm[a * N + node] += F[a] * (w / h3) * dV[p];
                        }
            }
        }
        if (resid)
            resid[m - 1] = sqrt(rsq);
        for (long x = 0; x < 3 * N; ++x) {                           /* step 4 */
            u[x] += c * fm[x];
            f_tot[x] += fm[x];
        }
    }
    if (final_resid && resid) {
        double rsq = 0.0;
        for (int p = 0; p < np; ++p)
            for (int l = moff[p]; l < moff[p + 1]; ++l) {
                if (mask && !mask[l])
                    continue;
                double o[3], X[3], U[3], wpp[3], wxo[3];
                support_t sp;
                for (int a = 0; a < 3; ++a) {
                    o[a] = body[a * nm + l];
                    X[a] = xp[a * np + p] + o[a];
                    wpp[a] = wp[a * np + p];
                }
                marker_support(n, h, origin, periodic, kernel, X, &sp);
                interp3(&sp, nx, ny, N, u, U);
                cross(wpp, o, wxo);
                for (int a = 0; a < 3; ++a) {
                    double r = up[a * np + p] + wxo[a] - U[a];
                    rsq += dV[p] * r * r;
                }
            }
        resid[n_iter] = sqrt(rsq);
    }
    free(fm);
    return R_OK;
}

/* ------------------------------------------------------------------------ */
/* Adjoint of the forcing loop                                              */
/* ------------------------------------------------------------------------ */

/*
 * Reverse-mode derivative of ref_forcing with the marker mask, the body
 * offsets, dV and c held fixed.  Given dL/du^{n} (g_u, may be NULL), dL/df_tot
 * (g_f, may be NULL), dL/dS (g_S) and dL/dT (g_T, may be NULL), writes dL/du^0
 * (gu0), dL/dx_p (gxp), dL/du_p (gup) and dL/domega_p (gwp).
 *
 * The forward loop is replayed first, storing every u^{m-1} and F^{m-1}.
 * Going backwards through each pass m, with ub = dL/du^m and
 * fb = c ub + g_f (the cotangent of f^{m-1}):
 *   Fb_l  = dV_l/h^3 (I fb)_l + dV_l (g_S,p + g_T,p x o_l)
 *   Ub_l  = -Fb_l / c           (cotangent of U^{m-1}_l)
 *   Udb_l = +Fb_l / c           (cotangent of U^d_l)
 *   ub   <- ub + I^T Ub         (cotangent of u^{m-1})
 *   Xb_l += sum_x grad_X w(x - X_l) [Ub_l . u^{m-1}(x) + dV_l/h^3 fb(x) . F_l]
 * and finally gup_p = sum_l Udb_l, gwp_p = sum_l o_l x Udb_l, gxp_p =
 * sum_l Xb_l (X_l = x_p + o_l), gu0 = ub.
 */
int ref_forcing_adjoint(const int *n, double h, const double *origin, const int *periodic,
                        int kernel, int n_iter, double c,
                        int np, const int *moff, const double *body, const double *dV,
                        const double *xp, const double *up, const double *wp,
                        const unsigned char *mask, const double *u0,
                        const double *g_f, const double *g_u, const double *g_S, const double *g_T,
                        double *gu0, double *gxp, double *gup, double *gwp)
{
    if (!n || n[0] <= 0 || n[1] <= 0 || n[2] <= 0 || !(h > 0.0) || n_iter < 1 ||
        !(c != 0.0) || np < 0 || (kernel != 3 && kernel != 4))
        return R_EINVAL;
    int st = check_markers(n, h, origin, periodic, kernel, np, moff, body, xp, mask);
    if (st != R_OK)
        return st;
    long nx = n[0], ny = n[1], N = (long)n[0] * n[1] * n[2];
    int nm = moff[np];
    double h3 = h * h * h;
    size_t G = 3 * (size_t)N;
    double *us = (double *)malloc(sizeof(double) * G * (size_t)(n_iter + 1));
    double *Fs = (double *)malloc(sizeof(double) * 3 * (size_t)nm * n_iter);
    double *fb = (double *)malloc(sizeof(double) * G);
    double *dub = (double *)malloc(sizeof(double) * G);
    double *ftmp = (double *)malloc(sizeof(double) * G);
    double *S = (double *)malloc(sizeof(double) * 3 * (size_t)(np ? np : 1));
    double *T = (double *)malloc(sizeof(double) * 3 * (size_t)(np ? np : 1));
    if (!us || !Fs || !fb || !dub || !ftmp || !S || !T) {
        free(us); free(Fs); free(fb); free(dub); free(ftmp); free(S); free(T);
        return R_EINVAL;
    }
    /* forward replay: one pass at a time, keeping u^{m-1} and F^{m-1} */
    memcpy(us, u0, sizeof(double) * G);
    for (int m = 1; m <= n_iter; ++m) {
        double *um1 = us + (size_t)(m - 1) * G;
        double *um = us + (size_t)m * G;
        memcpy(um, um1, sizeof(double) * G);
        memset(ftmp, 0, sizeof(double) * G);
        /* a single pass of the forward loop writes u^m and the markers' F */
        for (int p = 0; p < np; ++p)
            for (int l = moff[p]; l < moff[p + 1]; ++l) {
                if (mask && !mask[l])
                    continue;
                double o[3], X[3], U[3], wpp[3], wxo[3];
                support_t sp;
                for (int a = 0; a < 3; ++a) {
                    o[a] = body[a * nm + l];
                    X[a] = xp[a * np + p] + o[a];
                    wpp[a] = wp[a * np + p];
                }
                marker_support(n, h, origin, periodic, kernel, X, &sp);
                interp3(&sp, nx, ny, N, um1, U);
                cross(wpp, o, wxo);
                double F[3];
                for (int a = 0; a < 3; ++a) {
                    F[a] = (up[a * np + p] + wxo[a] - U[a]) / c;
                    Fs[((size_t)(m - 1) * 3 + a) * nm + l] = F[a];
                }
                for (int k = 0; k < sp.cnt[2]; ++k)
                    for (int j = 0; j < sp.cnt[1]; ++j)
                        for (int i = 0; i < sp.cnt[0]; ++i) {
                            double w = sp.w[2][k] * sp.w[1][j] * sp.w[0][i];
                            long node = sp.idx[0][i] + nx * (sp.idx[1][j] + ny * sp.idx[2][k]);
                            for (int a = 0; a < 3; ++a)
                                ftmp[a * N + node] += F[a] * (w / h3) * dV[p];
                        }
            }
        for (size_t x = 0; x < G; ++x)
            um[x] += c * ftmp[x];
    }
    /* reverse sweep */
    for (size_t x = 0; x < G; ++x)
        gu0[x] = g_u ? g_u[x] : 0.0;
    for (int i = 0; i < 3 * np; ++i) {
        gxp[i] = 0.0;
        gup[i] = 0.0;
        gwp[i] = 0.0;
    }
    for (int m = n_iter; m >= 1; --m) {
        const double *um1 = us + (size_t)(m - 1) * G;
        for (size_t x = 0; x < G; ++x)
            fb[x] = c * gu0[x] + (g_f ? g_f[x] : 0.0);
        memset(dub, 0, sizeof(double) * G);
        for (int p = 0; p < np; ++p) {
            double gS[3], gT[3];
            for (int a = 0; a < 3; ++a) {
                gS[a] = g_S ? g_S[a * np + p] : 0.0;
                gT[a] = g_T ? g_T[a * np + p] : 0.0;
            }
            for (int l = moff[p]; l < moff[p + 1]; ++l) {
                if (mask && !mask[l])
                    continue;
                double o[3], X[3], IF[3], F[3], gTxo[3], Fb[3], Ub[3], Udb[3], oxUdb[3];
                support_t sp;
                for (int a = 0; a < 3; ++a) {
                    o[a] = body[a * nm + l];
                    X[a] = xp[a * np + p] + o[a];
                    F[a] = Fs[((size_t)(m - 1) * 3 + a) * nm + l];
                }
                marker_support(n, h, origin, periodic, kernel, X, &sp);
                interp3(&sp, nx, ny, N, fb, IF);
                cross(gT, o, gTxo);
                for (int a = 0; a < 3; ++a) {
                    Fb[a] = dV[p] / h3 * IF[a] + dV[p] * (gS[a] + gTxo[a]);
                    Ub[a] = -Fb[a] / c;
                    Udb[a] = Fb[a] / c;
                    gup[a * np + p] += Udb[a];
                }
                cross(o, Udb, oxUdb);
                for (int a = 0; a < 3; ++a)
                    gwp[a * np + p] += oxUdb[a];
                double Xb[3] = {0.0, 0.0, 0.0};
                for (int k = 0; k < sp.cnt[2]; ++k)
                    for (int j = 0; j < sp.cnt[1]; ++j)
                        for (int i = 0; i < sp.cnt[0]; ++i) {
                            double wx = sp.w[0][i], wy = sp.w[1][j], wz = sp.w[2][k];
                            long node = sp.idx[0][i] + nx * (sp.idx[1][j] + ny * sp.idx[2][k]);
                            double w = wz * wy * wx;
                            /* r = (x - X)/h, so d w / d X_a = -(1/h) phi'(r_a) prod_others */
                            double gw[3] = {-sp.dw[0][i] * wy * wz / h,
                                            -wx * sp.dw[1][j] * wz / h,
                                            -wx * wy * sp.dw[2][k] / h};
                            double s1 = 0.0, s2 = 0.0;
                            for (int a = 0; a < 3; ++a) {
                                s1 += Ub[a] * um1[a * N + node];
                                s2 += fb[a * N + node] * F[a];
                            }
                            for (int a = 0; a < 3; ++a)
                                Xb[a] += gw[a] * (s1 + dV[p] / h3 * s2);
                            for (int a = 0; a < 3; ++a)
                                dub[a * N + node] += w * Ub[a];
                        }
                for (int a = 0; a < 3; ++a)
                    gxp[a * np + p] += Xb[a];
            }
        }
        for (size_t x = 0; x < G; ++x)
            gu0[x] += dub[x];
    }
    free(us); free(Fs); free(fb); free(dub); free(ftmp); free(S); free(T);
    return R_OK;
}

/* ------------------------------------------------------------------------ */
/* Pair pass: cell list, pair and wall lists, collision forces, marker mask */
/* ------------------------------------------------------------------------ */

/* Position wrapped into [origin, origin + L) on a periodic axis. */
static double wrap_pos(double x, double o, double L)
{
    double t = floor((x - o) / L);
    return x - t * L;
}

/* Minimum-image displacement on a periodic axis. */
static double min_image(double d, double L)
{
    while (d > 0.5 * L)
        d = d - L;
    while (d < -0.5 * L)
        d = d + L;
    return d;
}

static void wrapped_centre(const int *n, double h, const double *origin, const int *periodic,
                           int np, const double *xp, int p, double *x)
{
    for (int a = 0; a < 3; ++a) {
        double L = n[a] * h;
        x[a] = periodic[a] ? wrap_pos(xp[a * np + p], origin[a], L) : xp[a * np + p];
    }
}

/* Pair displacement x_q - x_p (minimum image) and squared distance, summed
 * in the order dx^2 + dy^2 + dz^2. */
static double pair_disp(const int *n, double h, const double *origin, const int *periodic,
                        int np, const double *xp, int p, int q, double *d)
{
    double a_[3], b_[3];
    wrapped_centre(n, h, origin, periodic, np, xp, p, a_);
    wrapped_centre(n, h, origin, periodic, np, xp, q, b_);
    for (int a = 0; a < 3; ++a) {
        d[a] = b_[a] - a_[a];
        if (periodic[a])
            d[a] = min_image(d[a], n[a] * h);
    }
    double d2 = d[0] * d[0];
    d2 = d2 + d[1] * d[1];
    d2 = d2 + d[2] * d[2];
    return d2;
}

/* Uniform cell grid for the neighbour search: per axis nc = max(1,
 * floor(L / (2 R_max + gap_cut))) cells of edge L / nc, so every pair
 * within reach lies in neighbouring cells.  cell = floor((x - origin) / edge)
 * of the wrapped centre, clamped to [0, nc - 1].  Particles are listed per
 * cell in increasing id (a stable counting sort). */
int ref_cell_list(const int *n, double h, const double *origin, const int *periodic,
                  int np, const double *xp, const double *radius, double gap_cut,
                  int *nc, int cap_cells, int *cell_of, int *cell_start, int *cell_particles)
{
    if (np < 0)
        return R_EINVAL;
    double rmax = 0.0;
    for (int p = 0; p < np; ++p)
        if (radius[p] > rmax)
            rmax = radius[p];
    double edge[3];
    for (int a = 0; a < 3; ++a) {
        double L = n[a] * h;
        int k = (int)floor(L / (2.0 * rmax + gap_cut));
        nc[a] = k < 1 ? 1 : k;
        edge[a] = L / nc[a];
    }
    long ncell = (long)nc[0] * nc[1] * nc[2];
    if (ncell > cap_cells)
        return R_ECAPACITY;
    for (long cidx = 0; cidx <= ncell; ++cidx)
        cell_start[cidx] = 0;
    for (int p = 0; p < np; ++p) {
        double x[3];
        int ci[3];
        wrapped_centre(n, h, origin, periodic, np, xp, p, x);
        for (int a = 0; a < 3; ++a) {
            double t = floor((x[a] - origin[a]) / edge[a]);
            int v = (int)t;
            if (t < 0.0)
                v = 0;
            if (t > (double)(nc[a] - 1))
                v = nc[a] - 1;
            ci[a] = v;
        }
        cell_of[p] = ci[0] + nc[0] * (ci[1] + nc[1] * ci[2]);
        cell_start[cell_of[p] + 1] += 1;
    }
    for (long cidx = 0; cidx < ncell; ++cidx)
        cell_start[cidx + 1] += cell_start[cidx];
    int *fill = (int *)calloc((size_t)ncell, sizeof(int));
    if (!fill)
        return R_EINVAL;
    for (int p = 0; p < np; ++p) {
        int cc = cell_of[p];
        cell_particles[cell_start[cc] + fill[cc]] = p;
        fill[cc] += 1;
    }
    free(fill);
    return R_OK;
}

/* All pairs i < j with centre distance below R_i + R_j + gap_cut (compared
 * squared), in lexicographic (i, j) order -- the brute-force definition of
 * the set the sum over q != p in eq. f_int runs over.  gap = d - R_i - R_j
 * is the separation zeta_n of Secs. 2.2.6-2.2.7. */
int ref_pairs_brute(const int *n, double h, const double *origin, const int *periodic,
                    int np, const double *xp, const double *radius, double gap_cut,
                    int cap, int *pairs, double *gap, int *npairs)
{
    int cnt = 0;
    for (int i = 0; i < np; ++i)
        for (int j = i + 1; j < np; ++j) {
            double d[3];
            double d2 = pair_disp(n, h, origin, periodic, np, xp, i, j, d);
            double cut = radius[i] + radius[j] + gap_cut;
            if (d2 < cut * cut) {
                if (cnt < cap) {
                    pairs[cnt] = i;
                    pairs[cap + cnt] = j;
                    gap[cnt] = sqrt(d2) - radius[i] - radius[j];
                }
                ++cnt;
            }
        }
    *npairs = cnt;
    return cnt > cap ? R_ECAPACITY : R_OK;
}

/* Wall entries (particle, side) with side = 2 axis + (0 lower, 1 upper) for
 * every non-periodic axis, listed when the surface gap to the wall is below
 * gap_cut, in (particle, side) order. */
int ref_walls(const int *n, double h, const double *origin, const int *periodic,
              int np, const double *xp, const double *radius, double gap_cut,
              int cap, int *walls, double *gap, int *nwall)
{
    int cnt = 0;
    for (int p = 0; p < np; ++p)
        for (int a = 0; a < 3; ++a) {
            if (periodic[a])
                continue;
            double L = n[a] * h;
            double x = xp[a * np + p];
            for (int side = 0; side < 2; ++side) {
                double dist = side == 0 ? (x - origin[a]) : (origin[a] + L - x);
                double g = dist - radius[p];
                if (g < gap_cut) {
                    if (cnt < cap) {
                        walls[cnt] = p;
                        walls[cap + cnt] = 2 * a + side;
                        gap[cnt] = g;
                    }
                    ++cnt;
                }
            }
        }
    *nwall = cnt;
    return cnt > cap ? R_ECAPACITY : R_OK;
}

/*
 * ACTM coefficients of the normal contact (Sec. 2.2.7, eq. ode).  In the
 * units z = zeta / (u_in T_c), t = time / T_c the normal overlap of a
 * contact obeys
 *     z'' + D z' + K z^p = 0,   z(0) = 0,  z'(0) = 1,
 * with k_n = K m_eff / (u_in^(p-1) T_c^(p+1)) and d_n = D m_eff / T_c, so the
 * two end conditions of the paper (the overlap closes at T_c, the rebound
 * speed is e_dry times the impact speed) fix K and D for given e_dry: the
 * contact must end at t = 1 with z'(1) = -e.  p = 3/2 is the Hertz law of
 * eq. hertz-contact; p = 1 gives the linear spring-dashpot, whose closed
 * form pins this solver.
 *
 * contact_run integrates the equation with classical RK4 at a fixed step
 * until z returns to zero (force zero once z <= 0), locates the crossing
 * on the cubic Hermite interpolant of the last step and takes one partial
 * RK4 step to it.  Returns 0 if the overlap does not close before t_max.
 */
static double actm_force(double K, double p, double z)
{
    if (z <= 0.0)
        return 0.0;
    if (p == 1.0)
        return K * z;
    if (p == 1.5)
        return K * z * sqrt(z);
    return K * pow(z, p);
}

static void actm_step(double K, double D, double p, double h, double z, double v, double *zn,
                      double *vn)
{
    double k1z = v, k1v = -D * v - actm_force(K, p, z);
    double z2 = z + 0.5 * h * k1z, v2 = v + 0.5 * h * k1v;
    double k2z = v2, k2v = -D * v2 - actm_force(K, p, z2);
    double z3 = z + 0.5 * h * k2z, v3 = v + 0.5 * h * k2v;
    double k3z = v3, k3v = -D * v3 - actm_force(K, p, z3);
    double z4 = z + h * k3z, v4 = v + h * k3v;
    double k4z = v4, k4v = -D * v4 - actm_force(K, p, z4);
    *zn = z + h / 6.0 * (k1z + 2.0 * k2z + 2.0 * k3z + k4z);
    *vn = v + h / 6.0 * (k1v + 2.0 * k2v + 2.0 * k3v + k4v);
}

static int contact_run(double K, double D, double p, double h, double t_max, double *T,
                       double *v_end)
{
    double t = 0.0, z = 0.0, v = 1.0;
    long nmax = (long)(t_max / h) + 1;
    for (long s = 0; s < nmax; ++s) {
        double zn, vn;
        actm_step(K, D, p, h, z, v, &zn, &vn);
        if (s > 0 && zn <= 0.0) {
            /* crossing inside [t, t + h]: bisection on the Hermite cubic */
            double a0 = 0.0, a1 = 1.0;
            double fa0 = -D * v - actm_force(K, p, z);   /* unused slopes kept for clarity */
            (void)fa0;
            for (int it = 0; it < 200; ++it) {
                double s_ = 0.5 * (a0 + a1);
                double h00 = (1 + 2 * s_) * (1 - s_) * (1 - s_), h10 = s_ * (1 - s_) * (1 - s_);
                double h01 = s_ * s_ * (3 - 2 * s_), h11 = s_ * s_ * (s_ - 1);
                double zs = h00 * z + h10 * h * v + h01 * zn + h11 * h * vn;
                if (zs > 0.0)
                    a0 = s_;
                else
                    a1 = s_;
            }
            double tau = 0.5 * (a0 + a1) * h, ze, ve;
            actm_step(K, D, p, tau, z, v, &ze, &ve);
            *T = t + tau;
            *v_end = ve;
            return 1;
        }
        z = zn;
        v = vn;
        t += h;
    }
    return 0;
}

/*
 * K and D for restitution e in (0, 1] and exponent p: nested bisection.
 * Inner: for a damping D the contact duration falls monotonically with K;
 * bisect log K until the duration is 1.  Outer: with the duration held at
 * 1 the rebound ratio falls monotonically with D; bisect D until it is e.
 */
static double actm_K_for_unit_duration(double D, double p, double h)
{
    double lo = log(1e-3), hi = log(1e5);
    for (int it = 0; it < 64; ++it) {
        double mid = 0.5 * (lo + hi), T, v;
        int ok = contact_run(exp(mid), D, p, h, 4.0, &T, &v);
        if (!ok || T > 1.0)
            lo = mid;     /* too soft: the contact lasts too long */
        else
            hi = mid;
    }
    return exp(0.5 * (lo + hi));
}

int ref_actm_coefficients(double e, double p, double *K_out, double *D_out)
{
    if (!(e > 0.0 && e <= 1.0) || !(p >= 1.0 && p <= 2.0))
        return R_EINVAL;
    const double h = 1.0 / 20000.0;
    if (e == 1.0) {
        *D_out = 0.0;
        *K_out = actm_K_for_unit_duration(0.0, p, h);
        return R_OK;
    }
    double lo = 0.0, hi = 8.0 * (-log(e)) + 1.0;
    for (int it = 0; it < 60; ++it) {
        double D = 0.5 * (lo + hi);
        double K = actm_K_for_unit_duration(D, p, h), T, v;
        contact_run(K, D, p, h, 4.0, &T, &v);
        if (-v > e)
            lo = D;       /* rebound too strong: more damping */
        else
            hi = D;
    }
    *D_out = 0.5 * (lo + hi);
    *K_out = actm_K_for_unit_duration(*D_out, p, h);
    return R_OK;
}

typedef struct {
    double rho_f, nu_f, eps_sep, lub_C, zeta_min_factor, e_dry, T_c, mu_s, mu_k, nu_poi, dt, h;
    int normal_model;      /* 0 linear spring-dashpot, 1 Hertz with ACTM */
    double St_crit, kn_grav_eps, g[3], K_hz, D_hz;
    int st_switch;
} coll_params;

#define HIST 4   /* history rows per contact: tangential spring (3), impact speed */

static coll_params coll_from(const double *cpar, double h)
{
    coll_params P;
    P.rho_f = cpar[0];
    P.nu_f = cpar[1];
    P.eps_sep = cpar[2];
    P.lub_C = cpar[3];
    P.zeta_min_factor = cpar[4];
    P.e_dry = cpar[5];
    P.T_c = cpar[6];
    P.mu_s = cpar[7];
    P.mu_k = cpar[8];
    P.nu_poi = cpar[9];
    P.dt = cpar[10];
    P.h = h;
    P.normal_model = (int)cpar[11];
    P.St_crit = cpar[12];
    P.kn_grav_eps = cpar[13];
    P.g[0] = cpar[14];
    P.g[1] = cpar[15];
    P.g[2] = cpar[16];
    P.K_hz = cpar[17];
    P.D_hz = cpar[18];
    P.st_switch = (int)cpar[19];
    return P;
}

/* rho_p d_p of a sphere of mass m and radius R: 3 m / (2 pi R^2). */
static double rho_d(double m, double R) { return 3.0 * m / (2.0 * M_PI * R * R); }

/* Gravity stiffness m g (eps d / 2)^(-3/2) of one particle (Sec. 2.2.7). */
static double kn_grav_one(const coll_params *P, double m, double R)
{
    double g = sqrt(P->g[0] * P->g[0] + P->g[1] * P->g[1] + P->g[2] * P->g[2]);
    double a = P->kn_grav_eps * R;
    return m * g / (a * sqrt(a));
}

/*
 * Collision force on particle p from a partner across the contact plane
 * with unit normal nvec (pointing from p to the partner).  Inputs: surface
 * gap zeta, relative contact-point velocity g (Sec. 2.2.8: g_cp), effective
 * radius and mass, rho d of the contact (for the Stokes number), the
 * gravity stiffness of the contact, the history of the last committed state
 * (tangential spring, impact speed; zero for a new contact) and the time
 * dt since that state.  Returns F (force on p), the tangential part Ft and
 * the updated history.
 *
 *   regime (Secs. 2.2.6-2.2.8, eq. f_int cases): contact if zeta < 0, lubrication if
 *   0 <= zeta < eps_sep, nothing otherwise.
 *   lubrication: F = -6 pi rho_f nu_f R_eff^2 psi / max(zeta_min, zeta) g_n,
 *     psi = erf(6 - C max(zeta_min, zeta)/h)/2 + 1/2 (Sec. 2.2.6, lubrication).
 *   impact speed u_in: the approach speed g . n at the first contact
 *     evaluation (kept while the contact lasts, clamped at zero).
 *   normal contact, linear: F_n = -k_n |zeta| n - d_n g_n, with k_n, d_n the
 *     damped-oscillator coefficients giving restitution e_dry over the
 *     contact time T_c (the linear form of eq. ode).
 *   normal contact, Hertz (eq. hertz-contact): F_n = -k_n |zeta|^(3/2) n -
 *     d_n g_n, k_n = K m_eff / (sqrt(u_in) T_c^(5/2)) and d_n = D m_eff / T_c
 *     (ACTM, eq. ode, K and D from ref_actm_coefficients) while u_in exceeds
 *     u_in,crit = 9 St_crit rho_f nu_f / (rho d) (eq. stokes_num); otherwise
 *     k_n = max(k_n,crit, k_n,grav), k_n,crit being the ACTM stiffness at
 *     u_in,crit.
 *   tangential contact (Sec. 2.2.8, tangential model): spring-dashpot
 *     F_dp = -k_t zeta_t - d_t g_t, capped by Coulomb friction; mu_s while
 *     sticking, mu_k when slipping, with the spring reset on slip.
 *     k_t = 2 (1 - nu)/(2 - nu) times the normal spring's stiffness (k_n,
 *     and for the Hertz law its secant k_n |zeta|^(1/2)).
 */
static void contact_law(const coll_params *P, double zeta, const double *nvec, const double *g,
                        double Reff, double meff, double zmin, double rhod, double kgrav,
                        const double *hist_old, double dt, double *F, double *Ft_out,
                        double *hist_new)
{
    double gn = g[0] * nvec[0] + g[1] * nvec[1] + g[2] * nvec[2];
    double gnv[3], gtv[3];
    for (int a = 0; a < 3; ++a) {
        gnv[a] = gn * nvec[a];
        gtv[a] = g[a] - gnv[a];
        F[a] = 0.0;
        Ft_out[a] = 0.0;
    }
    for (int a = 0; a < HIST; ++a)
        hist_new[a] = 0.0;
    if (zeta >= P->eps_sep)
        return;
    if (zeta >= 0.0) {
        double zz = zeta > zmin ? zeta : zmin;
        double psi = 0.5 * erf(6.0 - P->lub_C * zz / P->h) + 0.5;
        double coef = 6.0 * M_PI * P->rho_f * P->nu_f * Reff * Reff * psi / zz;
        for (int a = 0; a < 3; ++a)
            F[a] = -coef * gnv[a];
        return;
    }
    double u_in = hist_old[3] > 0.0 ? hist_old[3] : (gn > 0.0 ? gn : 0.0);
    double le = log(P->e_dry);
    double ze = fabs(zeta);
    double kn, dn, kspring, Fn[3];
    if (P->normal_model == 1) {
        double Tc52 = P->T_c * P->T_c * sqrt(P->T_c);
        double u_crit = 9.0 * P->St_crit * P->rho_f * P->nu_f / rhod;
        if (u_in > u_crit) {
            kn = P->K_hz * meff / (sqrt(u_in) * Tc52);
        } else {
            double kcrit = u_crit > 0.0 ? P->K_hz * meff / (sqrt(u_crit) * Tc52) : 0.0;
            kn = kcrit > kgrav ? kcrit : kgrav;
        }
        dn = P->D_hz * meff / P->T_c;
        kspring = kn * sqrt(ze);
        for (int a = 0; a < 3; ++a)
            Fn[a] = -kn * (ze * sqrt(ze)) * nvec[a] - dn * gnv[a];
    } else {
        kn = meff * (M_PI * M_PI + le * le) / (P->T_c * P->T_c);
        dn = -2.0 * meff * le / P->T_c;
        kspring = kn;
        for (int a = 0; a < 3; ++a)
            Fn[a] = -kn * ze * nvec[a] - dn * gnv[a];
    }
    double kt = 2.0 * (1.0 - P->nu_poi) / (2.0 - P->nu_poi) * kspring;
    double dt_ = 2.0 * sqrt(meff * kt) * (-le) / sqrt(M_PI * M_PI + le * le);
    /* spring: previous displacement projected on the current tangent plane,
     * plus g_t dt */
    double zon = hist_old[0] * nvec[0] + hist_old[1] * nvec[1] + hist_old[2] * nvec[2];
    double zt[3], Fdp[3];
    for (int a = 0; a < 3; ++a) {
        zt[a] = (hist_old[a] - zon * nvec[a]) + gtv[a] * dt;
        Fdp[a] = -kt * zt[a] - dt_ * gtv[a];
    }
    double nFdp = sqrt(Fdp[0] * Fdp[0] + Fdp[1] * Fdp[1] + Fdp[2] * Fdp[2]);
    double nFn = sqrt(Fn[0] * Fn[0] + Fn[1] * Fn[1] + Fn[2] * Fn[2]);
    double Ft[3];
    if (nFdp <= P->mu_s * nFn) {
        for (int a = 0; a < 3; ++a)
            Ft[a] = Fdp[a];
    } else {
        for (int a = 0; a < 3; ++a) {
            Ft[a] = P->mu_k * nFn * Fdp[a] / nFdp;
            zt[a] = -(Ft[a] + dt_ * gtv[a]) / kt;
        }
    }
    for (int a = 0; a < 3; ++a) {
        F[a] = Fn[a] + Ft[a];
        Ft_out[a] = Ft[a];
        hist_new[a] = zt[a];
    }
    hist_new[3] = u_in;
}

static int find_pair(int n_in, const int *pairs_in, int i, int j)
{
    for (int k = 0; k < n_in; ++k)
        if (pairs_in[k] == i && pairs_in[n_in + k] == j)
            return k;
    return -1;
}

/* Geometry and contact law of listed pair k = (p, q), p < q: force on p (F),
 * the torques on p and q, and the new history. */
static void pair_contact(const int *n, double h, const double *origin, const int *periodic,
                         const coll_params *P, int np, const double *xp, const double *radius,
                         const double *mass, const double *up, const double *wp, int p, int q,
                         const double *hold, double dt, double *F, double *Tp, double *Tq,
                         double *hnew)
{
    double dvec[3];
    double d = sqrt(pair_disp(n, h, origin, periodic, np, xp, p, q, dvec));
    double Rp = radius[p], Rq = radius[q];
    double zeta = d - Rp - Rq;
    double nvec[3] = {dvec[0] / d, dvec[1] / d, dvec[2] / d};
    double Rpc = 0.5 * (d + Rp - Rq), Rqc = 0.5 * (d + Rq - Rp);
    double wpn[3], wqn[3], g[3];
    double wpp[3] = {wp[p], wp[np + p], wp[2 * np + p]};
    double wqq[3] = {wp[q], wp[np + q], wp[2 * np + q]};
    cross(wpp, nvec, wpn);
    cross(wqq, nvec, wqn);
    for (int a = 0; a < 3; ++a)
        g[a] = (up[a * np + p] - up[a * np + q]) + Rpc * wpn[a] + Rqc * wqn[a];
    double Reff = Rp * Rq / (Rp + Rq);
    double meff = mass[p] * mass[q] / (mass[p] + mass[q]);
    double zmin = P->zeta_min_factor * (Rp < Rq ? Rp : Rq);
    double rhod = 0.5 * (rho_d(mass[p], Rp) + rho_d(mass[q], Rq));
    double kg_p = kn_grav_one(P, mass[p], Rp), kg_q = kn_grav_one(P, mass[q], Rq);
    double kgrav = kg_p > kg_q ? kg_p : kg_q;
    double Ft[3], nxFt[3];
    contact_law(P, zeta, nvec, g, Reff, meff, zmin, rhod, kgrav, hold, dt, F, Ft, hnew);
    cross(nvec, Ft, nxFt);
    for (int a = 0; a < 3; ++a) {
        Tp[a] = Rpc * nxFt[a];
        Tq[a] = Rqc * nxFt[a];
    }
}

/* Wall entry (p, side): a wall is the limit R_q, m_q -> infinity at rest:
 * R_eff = R_p, m_eff = m_p, lever arm |x_w - x_p| (Sec. 2.2.8). */
static void wall_contact(const int *n, double h, const double *origin, const coll_params *P,
                         int np, const double *xp, const double *radius, const double *mass,
                         const double *up, const double *wp, int p, int side,
                         const double *hold, double dt, double *F, double *T, double *hnew)
{
    int ax = side / 2, up_side = side % 2;
    double L = n[ax] * h;
    double x = xp[ax * np + p];
    double dist = up_side == 0 ? (x - origin[ax]) : (origin[ax] + L - x);
    double Rp = radius[p];
    double zeta = dist - Rp;
    double nvec[3] = {0.0, 0.0, 0.0};
    nvec[ax] = up_side == 0 ? -1.0 : 1.0;
    double wpp[3] = {wp[p], wp[np + p], wp[2 * np + p]};
    double wpn[3], g[3];
    cross(wpp, nvec, wpn);
    for (int a = 0; a < 3; ++a)
        g[a] = up[a * np + p] + dist * wpn[a];
    double Ft[3], nxFt[3];
    contact_law(P, zeta, nvec, g, Rp, mass[p], P->zeta_min_factor * Rp, rho_d(mass[p], Rp),
                kn_grav_one(P, mass[p], Rp), hold, dt, F, Ft, hnew);
    cross(nvec, Ft, nxFt);
    for (int a = 0; a < 3; ++a)
        T[a] = dist * nxFt[a];
}

/*
 * Collision force and torque on every particle (eq. f_int): the sum over
 * listed pairs and walls of F_n + F_t, and of R_cp n x F_t.  For a pair
 * (p, q), n = (x_q - x_p)/d, the contact-point lever arms are
 * R_p,cp = (d + R_p - R_q)/2 and R_q,cp = (d + R_q - R_p)/2 (Sec. 2.2.8), and
 * g = (u_p - u_q) + R_p,cp omega_p x n + R_q,cp omega_q x n.  p receives F,
 * q receives -F; both receive the torque R_cp n x F_t.  R_eff =
 * R_p R_q/(R_p + R_q), m_eff = m_p m_q/(m_p + m_q), zeta_min = factor *
 * min(R_p, R_q), rho d = the mean of the two particles' rho_p d_p, k_n,grav
 * = the larger of the two particles' values.
 * History ([4][n]: spring, impact speed) is looked up by the (i, j) key of
 * the previous call's list (and by (p, side) for walls); the spring
 * advances by the parameter dt.  Each particle's force and torque are
 * summed over its partners in increasing partner id, then its walls in
 * increasing side.
 */
typedef struct {
    int key;     /* partner id, or np + side for a wall */
    int k;       /* index in the pair or wall list */
    int role;    /* 0: p is the first of the pair, 1: the second, 2: wall */
} contact_ref;

static int cmp_contact(const void *a, const void *b)
{
    const contact_ref *x = a, *y = b;
    return (x->key > y->key) - (x->key < y->key);
}

static void sum_contacts(int np, int npairs, const int *pairs, int nwall, const int *walls,
                         const double *pF, const double *pTp, const double *pTq,
                         const double *wF, const double *wT, double *Fc, double *Tc)
{
    /* every contact of every particle, then sorted per particle by key */
    int *cnt = calloc((size_t)np + 1, sizeof(int));
    contact_ref *refs = malloc(sizeof(contact_ref) * (size_t)(2 * npairs + nwall + 1));
    int *fill = calloc((size_t)np + 1, sizeof(int));
    for (int k = 0; k < npairs; ++k) {
        cnt[pairs[k] + 1]++;
        cnt[pairs[npairs + k] + 1]++;
    }
    for (int k = 0; k < nwall; ++k)
        cnt[walls[k] + 1]++;
    for (int p = 0; p < np; ++p)
        cnt[p + 1] += cnt[p];
    for (int k = 0; k < npairs; ++k) {
        int i = pairs[k], j = pairs[npairs + k];
        contact_ref ri = {j, k, 0}, rj = {i, k, 1};
        refs[cnt[i] + fill[i]++] = ri;
        refs[cnt[j] + fill[j]++] = rj;
    }
    for (int k = 0; k < nwall; ++k) {
        int p = walls[k];
        contact_ref rw = {np + walls[nwall + k], k, 2};
        refs[cnt[p] + fill[p]++] = rw;
    }
    for (int p = 0; p < np; ++p) {
        qsort(refs + cnt[p], (size_t)(cnt[p + 1] - cnt[p]), sizeof(contact_ref), cmp_contact);
        double F[3] = {0.0, 0.0, 0.0}, T[3] = {0.0, 0.0, 0.0};
        for (int r = cnt[p]; r < cnt[p + 1]; ++r) {
            int k = refs[r].k;
            for (int a = 0; a < 3; ++a) {
                if (refs[r].role == 0) {
                    F[a] = F[a] + pF[a * npairs + k];
                    T[a] = T[a] + pTp[a * npairs + k];
                } else if (refs[r].role == 1) {
                    F[a] = F[a] - pF[a * npairs + k];
                    T[a] = T[a] + pTq[a * npairs + k];
                } else {
                    F[a] = F[a] + wF[a * nwall + k];
                    T[a] = T[a] + wT[a * nwall + k];
                }
            }
        }
        for (int a = 0; a < 3; ++a) {
            Fc[a * np + p] = F[a];
            Tc[a * np + p] = T[a];
        }
    }
    free(cnt);
    free(refs);
    free(fill);
}

/* One evaluation of every listed contact at the given particle state, with
 * history hold ([4][n] aligned with the lists) and spring time step dt. */
static int eval_contacts(const int *n, double h, const double *origin, const int *periodic,
                         const coll_params *P, int np, const double *xp, const double *radius,
                         const double *mass, const double *up, const double *wp, int npairs,
                         const int *pairs, int nwall, const int *walls, const double *hold,
                         const double *whold, double dt, double *hnew, double *whnew,
                         double *Fc, double *Tc)
{
    double *pF = calloc(3 * (size_t)(npairs + 1), sizeof(double));
    double *pTp = calloc(3 * (size_t)(npairs + 1), sizeof(double));
    double *pTq = calloc(3 * (size_t)(npairs + 1), sizeof(double));
    double *wF = calloc(3 * (size_t)(nwall + 1), sizeof(double));
    double *wT = calloc(3 * (size_t)(nwall + 1), sizeof(double));
    if (!pF || !pTp || !pTq || !wF || !wT) {
        free(pF); free(pTp); free(pTq); free(wF); free(wT);
        return R_EINVAL;
    }
    for (int k = 0; k < npairs; ++k) {
        double ho[HIST], hn[HIST], F[3], Tp[3], Tq[3];
        for (int a = 0; a < HIST; ++a)
            ho[a] = hold[a * npairs + k];
        pair_contact(n, h, origin, periodic, P, np, xp, radius, mass, up, wp, pairs[k],
                     pairs[npairs + k], ho, dt, F, Tp, Tq, hn);
        for (int a = 0; a < 3; ++a) {
            pF[a * npairs + k] = F[a];
            pTp[a * npairs + k] = Tp[a];
            pTq[a * npairs + k] = Tq[a];
        }
        if (hnew)
            for (int a = 0; a < HIST; ++a)
                hnew[a * npairs + k] = hn[a];
    }
    for (int k = 0; k < nwall; ++k) {
        double ho[HIST], hn[HIST], F[3], T[3];
        for (int a = 0; a < HIST; ++a)
            ho[a] = whold[a * nwall + k];
        wall_contact(n, h, origin, P, np, xp, radius, mass, up, wp, walls[k], walls[nwall + k],
                     ho, dt, F, T, hn);
        for (int a = 0; a < 3; ++a) {
            wF[a * nwall + k] = F[a];
            wT[a * nwall + k] = T[a];
        }
        if (whnew)
            for (int a = 0; a < HIST; ++a)
                whnew[a * nwall + k] = hn[a];
    }
    sum_contacts(np, npairs, pairs, nwall, walls, pF, pTp, pTq, wF, wT, Fc, Tc);
    free(pF); free(pTp); free(pTq); free(wF); free(wT);
    return R_OK;
}

int ref_pair_forces(const int *n, double h, const double *origin, const int *periodic,
                    int np, const double *xp, const double *radius, const double *mass,
                    const double *up, const double *wp, const double *cpar /* [20] */,
                    int npairs, const int *pairs, int nwall, const int *walls,
                    int npairs_in, const int *pairs_in, const double *hist_in,
                    int nwall_in, const int *walls_in, const double *whist_in,
                    double *Fc, double *Tc, double *hist_out, double *whist_out)
{
    coll_params P = coll_from(cpar, h);
    /* history of the previous call, aligned with the new lists */
    double *hold = calloc(HIST * (size_t)(npairs + 1), sizeof(double));
    double *whold = calloc(HIST * (size_t)(nwall + 1), sizeof(double));
    if (!hold || !whold) {
        free(hold); free(whold);
        return R_EINVAL;
    }
    for (int k = 0; k < npairs; ++k) {
        int kin = find_pair(npairs_in, pairs_in, pairs[k], pairs[npairs + k]);
        if (kin >= 0)
            for (int a = 0; a < HIST; ++a)
                hold[a * npairs + k] = hist_in[a * npairs_in + kin];
    }
    for (int k = 0; k < nwall; ++k)
        for (int kk = 0; kk < nwall_in; ++kk)
            if (walls_in[kk] == walls[k] && walls_in[nwall_in + kk] == walls[nwall + k])
                for (int a = 0; a < HIST; ++a)
                    whold[a * nwall + k] = whist_in[a * nwall_in + kk];
    int st = eval_contacts(n, h, origin, periodic, &P, np, xp, radius, mass, up, wp, npairs,
                           pairs, nwall, walls, hold, whold, P.dt, hist_out, whist_out, Fc, Tc);
    free(hold);
    free(whold);
    return st;
}

/*
 * Particle sub-stepping (Sec. 2.2.10): the particle state (x_p, u_p,
 * omega_p) advances by dt_total in n_sub sub-steps of dts = dt_total /
 * n_sub, each the three-stage Runge-Kutta predictor-corrector of the
 * improved particle update with the low-storage coefficients of Rai and
 * Moin: alpha = (4/15, 1/15, 1/6), gamma = (8/15, 5/12, 3/4), zeta = (0,
 * -17/60, -5/12).  For stage k, with F_c(s) the collision force at state s:
 *   u~ = u^{k-1} + dts/m (2 alpha_k F_h + gamma_k F_c(s^{k-1}) + zeta_k F_c(s^{k-2}))
 *        + 2 alpha_k dts g'
 *   w~ = w^{k-1} + dts/I (2 alpha_k T_h + gamma_k T_c(s^{k-1}) + zeta_k T_c(s^{k-2}))
 *   x~ = x^{k-1} + alpha_k dts (u~ + u^{k-1})
 *   u^k, w^k, x^k: the same with F_c(s~) in place of F_c(s^{k-1}) and
 *        F_c(s^{k-1}) in place of F_c(s^{k-2}).
 * g' = (1 - rho_f / rho_p) g, rho_p = m_p / (4/3 pi R_p^3), I_p = 2/5 m_p R_p^2.
 * F_h, T_h (the hydrodynamic force and torque) are held for the call; with
 * the St switch on, a particle whose committed contacts all have impact
 * Stokes numbers <= St_crit gets F_h = T_h = 0.
 * Contacts are evaluated on the given lists (built by the caller with a
 * gap cut-off that covers the motion of the call).  The history is
 * committed at each accepted state s^k (evaluated there with the spring
 * advanced by the time since the previous accepted state); the predictor
 * state s~ uses the committed history and the stage's time 2 alpha_k dts.
 * The call starts by evaluating the input state with the input history
 * (dt 0) and ends by evaluating the final state, whose history and forces
 * it returns.
 */
int ref_particle_substeps(const int *n, double h, const double *origin, const int *periodic,
                          int np, double *xp, double *up, double *wp, const double *radius,
                          const double *mass, const double *cpar, const double *Fh,
                          const double *Th, double dt_total, int n_sub, int npairs,
                          const int *pairs, int nwall, const int *walls, double *hist,
                          double *whist, double *Fc_out, double *Tc_out)
{
    static const double alpha[3] = {4.0 / 15.0, 1.0 / 15.0, 1.0 / 6.0};
    static const double gamma_[3] = {8.0 / 15.0, 5.0 / 12.0, 3.0 / 4.0};
    static const double zeta_[3] = {0.0, -17.0 / 60.0, -5.0 / 12.0};
    if (n_sub < 1 || np < 0)
        return R_EINVAL;
    coll_params P = coll_from(cpar, h);
    const double dts = dt_total / n_sub;
    size_t N3 = 3 * (size_t)(np > 0 ? np : 1);
    double *Fa = calloc(N3, sizeof(double)), *Ta = calloc(N3, sizeof(double));
    double *Fb = calloc(N3, sizeof(double)), *Tb = calloc(N3, sizeof(double));
    double *Fp = calloc(N3, sizeof(double)), *Tp = calloc(N3, sizeof(double));
    double *xt = calloc(N3, sizeof(double)), *ut = calloc(N3, sizeof(double));
    double *wt = calloc(N3, sizeof(double));
    double *sF = calloc((size_t)(np > 0 ? np : 1), sizeof(double));
    double *H = calloc(HIST * (size_t)(npairs + 1), sizeof(double));
    double *WH = calloc(HIST * (size_t)(nwall + 1), sizeof(double));
    double *Hn = calloc(HIST * (size_t)(npairs + 1), sizeof(double));
    double *WHn = calloc(HIST * (size_t)(nwall + 1), sizeof(double));
    int st = R_EINVAL;
    if (!Fa || !Ta || !Fb || !Tb || !Fp || !Tp || !xt || !ut || !wt || !sF || !H || !WH || !Hn ||
        !WHn)
        goto done;
    memcpy(H, hist, sizeof(double) * HIST * (size_t)npairs);
    memcpy(WH, whist, sizeof(double) * HIST * (size_t)nwall);
    /* St switch: per particle, from the impact speeds of the input history:
     * count each particle's committed contacts and those above St_crit */
    {
        int *contacts = calloc((size_t)np + 1, sizeof(int));
        int *fast = calloc((size_t)np + 1, sizeof(int));
        if (!contacts || !fast) {
            free(contacts);
            free(fast);
            goto done;
        }
        for (int k = 0; k < npairs; ++k) {
            int i = pairs[k], j = pairs[npairs + k];
            if (!(H[3 * npairs + k] > 0.0))
                continue;
            double rhod = 0.5 * (rho_d(mass[i], radius[i]) + rho_d(mass[j], radius[j]));
            double St = H[3 * npairs + k] * rhod / (9.0 * P.rho_f * P.nu_f);
            contacts[i]++;
            contacts[j]++;
            if (St > P.St_crit) {
                fast[i]++;
                fast[j]++;
            }
        }
        for (int k = 0; k < nwall; ++k) {
            int p = walls[k];
            if (!(WH[3 * nwall + k] > 0.0))
                continue;
            double St = WH[3 * nwall + k] * rho_d(mass[p], radius[p]) / (9.0 * P.rho_f * P.nu_f);
            contacts[p]++;
            if (St > P.St_crit)
                fast[p]++;
        }
        for (int p = 0; p < np; ++p)
            sF[p] = (P.st_switch && contacts[p] > 0 && fast[p] == 0) ? 0.0 : 1.0;
        free(contacts);
        free(fast);
    }
    double t_since = 0.0;
    for (int s = 0; s < n_sub; ++s) {
        for (int k = 0; k < 3; ++k) {
            const double a2 = 2.0 * alpha[k];
            /* F_c at the accepted state s^{k-1}, committing its history */
            st = eval_contacts(n, h, origin, periodic, &P, np, xp, radius, mass, up, wp, npairs,
                               pairs, nwall, walls, H, WH, t_since, Hn, WHn, Fa, Ta);
            if (st != R_OK)
                goto done;
            memcpy(H, Hn, sizeof(double) * HIST * (size_t)npairs);
            memcpy(WH, WHn, sizeof(double) * HIST * (size_t)nwall);
            /* predictor */
            for (int p = 0; p < np; ++p) {
                double m = mass[p], R = radius[p];
                double I = 0.4 * m * R * R;
                double rho_p = m / (4.0 / 3.0 * M_PI * R * R * R);
                for (int a = 0; a < 3; ++a) {
                    size_t i = (size_t)a * np + p;
                    double Fh_ = Fh ? sF[p] * Fh[i] : 0.0, Th_ = Th ? sF[p] * Th[i] : 0.0;
                    double gp = (1.0 - P.rho_f / rho_p) * P.g[a];
                    ut[i] = up[i] + dts / m * (a2 * Fh_ + gamma_[k] * Fa[i] + zeta_[k] * Fb[i]) +
                            a2 * dts * gp;
                    wt[i] = wp[i] + dts / I * (a2 * Th_ + gamma_[k] * Ta[i] + zeta_[k] * Tb[i]);
                    xt[i] = xp[i] + alpha[k] * dts * (ut[i] + up[i]);
                }
            }
            /* F_c at the predicted state (history not committed) */
            st = eval_contacts(n, h, origin, periodic, &P, np, xt, radius, mass, ut, wt, npairs,
                               pairs, nwall, walls, H, WH, a2 * dts, NULL, NULL, Fp, Tp);
            if (st != R_OK)
                goto done;
            /* corrector */
            for (int p = 0; p < np; ++p) {
                double m = mass[p], R = radius[p];
                double I = 0.4 * m * R * R;
                double rho_p = m / (4.0 / 3.0 * M_PI * R * R * R);
                for (int a = 0; a < 3; ++a) {
                    size_t i = (size_t)a * np + p;
                    double Fh_ = Fh ? sF[p] * Fh[i] : 0.0, Th_ = Th ? sF[p] * Th[i] : 0.0;
                    double gp = (1.0 - P.rho_f / rho_p) * P.g[a];
                    double un = up[i] + dts / m * (a2 * Fh_ + gamma_[k] * Fp[i] + zeta_[k] * Fa[i]) +
                                a2 * dts * gp;
                    double wn = wp[i] + dts / I * (a2 * Th_ + gamma_[k] * Tp[i] + zeta_[k] * Ta[i]);
                    xp[i] = xp[i] + alpha[k] * dts * (un + up[i]);
                    up[i] = un;
                    wp[i] = wn;
                }
            }
            memcpy(Fb, Fa, sizeof(double) * 3 * (size_t)np);
            memcpy(Tb, Ta, sizeof(double) * 3 * (size_t)np);
            t_since = a2 * dts;
        }
    }
    /* the final state: its forces and committed history */
    st = eval_contacts(n, h, origin, periodic, &P, np, xp, radius, mass, up, wp, npairs, pairs,
                       nwall, walls, H, WH, t_since, hist, whist, Fa, Ta);
    if (st == R_OK && Fc_out && Tc_out) {
        memcpy(Fc_out, Fa, sizeof(double) * 3 * (size_t)np);
        memcpy(Tc_out, Ta, sizeof(double) * 3 * (size_t)np);
    }
done:
    free(Fa); free(Ta); free(Fb); free(Tb); free(Fp); free(Tp); free(xt); free(ut); free(wt);
    free(sF); free(H); free(WH); free(Hn); free(WHn);
    return st;
}

/* SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014). */
uint64_t ref_splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/*
 * Marker disabling (Sec. 2.2.5): markers leave the forcing when a particle is
 * closer than eps_sep to a wall or closer than 2 eps_sep to another
 * particle; for a particle pair only one of the two, chosen at random, loses
 * markers.  The random choice for pair (p, q), p < q, is the low bit of
 * splitmix64(seed ^ (p << 32 | q)): 0 picks p, 1 picks q.
 *   mode 1 (local): the chosen particle loses the markers X_l with
 *     |X_l - x_partner| < R_partner + 2 eps_sep (compared squared); a
 *     particle near a wall loses the markers closer than eps_sep to it.
 *   mode 2 (whole): the chosen particle (or the particle near a wall) loses
 *     all its markers.
 *   mode 0: nothing is disabled.
 * mask[l] = 1 keeps marker l, 0 disables it.
 */
int ref_marker_mask(const int *n, double h, const double *origin, const int *periodic,
                    int np, const int *moff, const double *body, const double *xp,
                    const double *radius, double eps_sep, int mode, uint64_t seed,
                    int npairs, const int *pairs, const double *pgap,
                    int nwall, const int *walls, const double *wgap, unsigned char *mask)
{
    int nm = moff[np];
    for (int l = 0; l < nm; ++l)
        mask[l] = 1;
    if (mode == 0)
        return R_OK;
    for (int k = 0; k < npairs; ++k) {
        if (!(pgap[k] < 2.0 * eps_sep))
            continue;
        int p = pairs[k], q = pairs[npairs + k];
        uint64_t key = ((uint64_t)(uint32_t)p << 32) | (uint64_t)(uint32_t)q;
        int chosen = (ref_splitmix64(seed ^ key) & 1ULL) == 0 ? p : q;
        int partner = chosen == p ? q : p;
        double xc[3], xq[3];
        wrapped_centre(n, h, origin, periodic, np, xp, chosen, xc);
        wrapped_centre(n, h, origin, periodic, np, xp, partner, xq);
        double lim = radius[partner] + 2.0 * eps_sep;
        for (int l = moff[chosen]; l < moff[chosen + 1]; ++l) {
            if (mode == 2) {
                mask[l] = 0;
                continue;
            }
            double d[3];
            for (int a = 0; a < 3; ++a) {
                d[a] = (xc[a] + body[a * nm + l]) - xq[a];
                if (periodic[a])
                    d[a] = min_image(d[a], n[a] * h);
            }
            double d2 = d[0] * d[0];
            d2 = d2 + d[1] * d[1];
            d2 = d2 + d[2] * d[2];
            if (d2 < lim * lim)
                mask[l] = 0;
        }
    }
    for (int k = 0; k < nwall; ++k) {
        if (!(wgap[k] < eps_sep))
            continue;
        int p = walls[k], side = walls[nwall + k];
        int ax = side / 2, up_side = side % 2;
        double L = n[ax] * h;
        for (int l = moff[p]; l < moff[p + 1]; ++l) {
            if (mode == 2) {
                mask[l] = 0;
                continue;
            }
            double X = xp[ax * np + p] + body[ax * nm + l];
            double dist = up_side == 0 ? (X - origin[ax]) : (origin[ax] + L - X);
            if (dist < eps_sep)
                mask[l] = 0;
        }
    }
    return R_OK;
}

/* ------------------------------------------------------------------------ */
/* Level-set volume fraction and the fluid integrals over each particle      */
/* (Sec. 2.2.9, direct computation of the fluid inertia inside a particle)   */
/* ------------------------------------------------------------------------ */

/* Volume fraction of a cell in a sphere of radius R from the signed corner
 * distances phi_m = |x_m - x_p| - R (negative inside): alpha = sum over the
 * eight corners of -phi_m H(-phi_m), divided by sum |phi_m|.  A cell whose
 * corners all lie on the surface (zero denominator) counts as empty. */
static double level_set_alpha(const double *c0, double h, double R)
{
    double num = 0.0, den = 0.0;
    for (int m = 0; m < 8; ++m) {
        double d[3] = {c0[0] + (m & 1) * h, c0[1] + ((m >> 1) & 1) * h, c0[2] + ((m >> 2) & 1) * h};
        double phi = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) - R;
        if (phi <= 0.0)
            num += -phi;
        den += fabs(phi);
    }
    return den > 0.0 ? num / den : 0.0;
}

/* The same volume fraction for one cell with lowest corner c0 (relative to
 * the particle centre): exposed for the pins. */
double ref_cell_alpha(const double *c0, double h, double R) { return level_set_alpha(c0, h, R); }

/* For every particle p, over the cells whose box meets [x_p - R_p, x_p + R_p]
 * per axis (x_p wrapped into the domain on periodic axes; cells beyond a wall
 * are skipped):
 *   Iu_p = sum alpha h^3 u(cell),  Ir_p = sum alpha h^3 (r x u(cell)),
 * with r = cell centre - x_p (the cell index not wrapped, so r is the
 * displacement to the image of the cell next to the particle).  Iu and Ir
 * are double[3][np]; alpha_out (may be NULL) receives sum_p alpha per cell,
 * double[nz][ny][nx].  Particles are assumed smaller than half a periodic
 * axis (no cell is met twice by one particle). */
int ref_particle_integrals(const int *n, double h, const double *origin, const int *periodic,
                           int np, const double *xp, const double *radius, const double *u,
                           double *Iu, double *Ir, double *alpha_out)
{
    if (!n || !(h > 0.0) || np < 0 || (np > 0 && (!xp || !radius || !u || !Iu || !Ir)))
        return R_EINVAL;
    long nx = n[0], ny = n[1], N = (long)n[0] * n[1] * n[2];
    if (alpha_out)
        for (long i = 0; i < N; ++i)
            alpha_out[i] = 0.0;
    for (int p = 0; p < np; ++p) {
        double x[3];
        wrapped_centre(n, h, origin, periodic, np, xp, p, x);
        double R = radius[p];
        long lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
            lo[a] = (long)floor((x[a] - R - origin[a]) / h);
            hi[a] = (long)floor((x[a] + R - origin[a]) / h);
        }
        double su[3] = {0.0, 0.0, 0.0}, sr[3] = {0.0, 0.0, 0.0};
        for (long k = lo[2]; k <= hi[2]; ++k)
            for (long j = lo[1]; j <= hi[1]; ++j)
                for (long i = lo[0]; i <= hi[0]; ++i) {
                    long idx3[3] = {i, j, k};
                    int inside = 1;
                    for (int a = 0; a < 3; ++a) {
                        if (periodic[a]) {
                            idx3[a] = ((idx3[a] % n[a]) + n[a]) % n[a];
                        } else if (idx3[a] < 0 || idx3[a] >= n[a]) {
                            inside = 0;
                        }
                    }
                    if (!inside)
                        continue;
                    /* lowest corner and centre of the cell, relative to x_p */
                    double c0[3] = {origin[0] + i * h - x[0], origin[1] + j * h - x[1],
                                    origin[2] + k * h - x[2]};
                    double alpha = level_set_alpha(c0, h, R);
                    if (alpha == 0.0)
                        continue;
                    long g = (idx3[2] * ny + idx3[1]) * nx + idx3[0];
                    double uc[3] = {u[g], u[N + g], u[2 * N + g]};
                    double r[3] = {c0[0] + 0.5 * h, c0[1] + 0.5 * h, c0[2] + 0.5 * h};
                    double rxu[3];
                    cross(r, uc, rxu);
                    double w = alpha * h * h * h;
                    for (int a = 0; a < 3; ++a) {
                        su[a] += w * uc[a];
                        sr[a] += w * rxu[a];
                    }
                    if (alpha_out)
                        alpha_out[g] += alpha;
                }
        for (int a = 0; a < 3; ++a) {
            Iu[a * np + p] = su[a];
            Ir[a * np + p] = sr[a];
        }
    }
    return R_OK;
}

/* Volume average of a grid field per component (Sec. 2.2.4, the mean IBM
 * force of a triply periodic domain is minus this average of f_IBM). */
int ref_grid_mean(const int *n, const double *f, double *mean)
{
    long N = (long)n[0] * n[1] * n[2];
    for (int a = 0; a < 3; ++a) {
        double s = 0.0;
        for (long i = 0; i < N; ++i)
            s += f[a * N + i];
        mean[a] = s / (double)N;
    }
    return R_OK;
}
