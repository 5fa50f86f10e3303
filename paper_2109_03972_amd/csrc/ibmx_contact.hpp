// Contact geometry and collision law shared by the pair pass and the
// particle sub-stepping (Secs. 2.2.5-2.2.8, 2.2.10), FP64 throughout.
//
// Every listed contact is evaluated by each particle it touches, in the
// canonical orientation (first particle of the pair as p), so both sides
// obtain bit-identical values; each particle sums its contacts in
// increasing partner order (walls after the partners, by side) through a
// per-particle adjacency list, so forces and torques do not depend on
// thread scheduling.  The files including this header are compiled without
// FMA contraction.
#pragma once
#pragma clang fp contract(off)

#include <math.h>

#include "ibmx_internal.hpp"

namespace {

constexpr int kHist = IBMX_HIST;

struct PairC {
    double rho_f, nu_f, eps_sep, lub_C, zeta_min_factor, e_dry, T_c, mu_s, mu_k, nu_poi, dt;
    double gap_cut;
    double h;
    double L[3];
    double origin[3];
    double edge[3];
    int nc[3];
    int periodic[3];
    int ncell;
    // collision constants derived on the host
    int normal_model;     // 0 linear spring-dashpot, 1 Hertz with ACTM coefficients
    double le;            // ln e_dry
    double lin_k;         // pi^2 + ln^2 e_dry
    double sq_damp;       // sqrt(pi^2 + ln^2 e_dry)
    double kt_ratio;      // 2 (1 - nu) / (2 - nu)
    double K_hz, D_hz;    // ACTM coefficients of the Hertz law in contact-time units
    double Tc52;          // T_c^(5/2)
    double St_crit;
    double kn_grav_eps;
    double g_abs;         // |g|
    double g[3];
};

__device__ __forceinline__ double wrap_pos(double x, double o, double L)
{
    double t = floor((x - o) / L);
    return x - t * L;
}

__device__ __forceinline__ double min_image(double d, double L)
{
    while (d > 0.5 * L)
        d = d - L;
    while (d < -0.5 * L)
        d = d + L;
    return d;
}

__device__ __forceinline__ void centre(const PairC &P, int np, const double *xp, int p, double *x)
{
    for (int a = 0; a < 3; ++a) {
        double v = xp[(size_t)a * np + p];
        x[a] = P.periodic[a] ? wrap_pos(v, P.origin[a], P.L[a]) : v;
    }
}

__device__ __forceinline__ double disp2(const PairC &P, const double *a_, const double *b_, double *d)
{
    for (int a = 0; a < 3; ++a) {
        d[a] = b_[a] - a_[a];
        if (P.periodic[a])
            d[a] = min_image(d[a], P.L[a]);
    }
    double d2 = d[0] * d[0];
    d2 = d2 + d[1] * d[1];
    d2 = d2 + d[2] * d[2];
    return d2;
}

// rho_p d_p of a sphere: 3 m / (2 pi R^2)
__device__ __forceinline__ double rho_d(double m, double R) { return 3.0 * m / (2.0 * M_PI * R * R); }

// k_n,grav of one particle: m |g| (eps R)^(-3/2)
__device__ __forceinline__ double kn_grav(const PairC &P, double m, double R)
{
    double a = P.kn_grav_eps * R;
    return m * P.g_abs / (a * sqrt(a));
}

// ---------------------------------------------------------------------------
// collision law for one contact (force on p; n points from p to the partner)
//   lubrication   0 <= zeta < eps_sep: -6 pi rho_f nu_f R_eff^2 psi / zz g_n
//   contact       zeta < 0: normal spring-dashpot (linear, or Hertz with the
//                 ACTM stiffness for the impact speed u_in, bounded below by
//                 max(k_n,crit, k_n,grav) at or under the critical speed)
//                 plus the tangential spring-dashpot capped by friction
// History hold/hnew: tangential spring (3), impact speed; dt is the time
// since the state the history belongs to.
// ---------------------------------------------------------------------------
__device__ void contact_law(const PairC &P, double zeta, const double *n, const double *g,
                            double Reff, double meff, double zmin, double rhod, double kgrav,
                            const double *hold, double dt, double *F, double *Ft, double *hnew)
{
    double gn = g[0] * n[0] + g[1] * n[1] + g[2] * n[2];
    double gnv[3], gtv[3];
    for (int a = 0; a < 3; ++a) {
        gnv[a] = gn * n[a];
        gtv[a] = g[a] - gnv[a];
        F[a] = 0.0;
        Ft[a] = 0.0;
    }
    for (int a = 0; a < kHist; ++a)
        hnew[a] = 0.0;
    if (zeta >= P.eps_sep)
        return;
    if (zeta >= 0.0) {
        double zz = zeta > zmin ? zeta : zmin;
        double psi = 0.5 * erf(6.0 - P.lub_C * zz / P.h) + 0.5;
        double coef = 6.0 * M_PI * P.rho_f * P.nu_f * Reff * Reff * psi / zz;
        for (int a = 0; a < 3; ++a)
            F[a] = -coef * gnv[a];
        return;
    }
    const double u_in = hold[3] > 0.0 ? hold[3] : (gn > 0.0 ? gn : 0.0);
    const double ze = fabs(zeta);
    double kn, dn, ks, Fn[3];
    if (P.normal_model == 1) {
        const double u_crit = 9.0 * P.St_crit * P.rho_f * P.nu_f / rhod;
        if (u_in > u_crit) {
            kn = P.K_hz * meff / (sqrt(u_in) * P.Tc52);
        } else {
            double kcrit = u_crit > 0.0 ? P.K_hz * meff / (sqrt(u_crit) * P.Tc52) : 0.0;
            kn = kcrit > kgrav ? kcrit : kgrav;
        }
        dn = P.D_hz * meff / P.T_c;
        ks = kn * sqrt(ze);
        for (int a = 0; a < 3; ++a)
            Fn[a] = -kn * (ze * sqrt(ze)) * n[a] - dn * gnv[a];
    } else {
        kn = meff * P.lin_k / (P.T_c * P.T_c);
        dn = -2.0 * meff * P.le / P.T_c;
        ks = kn;
        for (int a = 0; a < 3; ++a)
            Fn[a] = -kn * ze * n[a] - dn * gnv[a];
    }
    double kt = P.kt_ratio * ks;
    double dtc = 2.0 * sqrt(meff * kt) * (-P.le) / P.sq_damp;
    double zon = hold[0] * n[0] + hold[1] * n[1] + hold[2] * n[2];
    double zt[3], Fdp[3];
    for (int a = 0; a < 3; ++a) {
        zt[a] = (hold[a] - zon * n[a]) + gtv[a] * dt;
        Fdp[a] = -kt * zt[a] - dtc * gtv[a];
    }
    double nFdp = sqrt(Fdp[0] * Fdp[0] + Fdp[1] * Fdp[1] + Fdp[2] * Fdp[2]);
    double nFn = sqrt(Fn[0] * Fn[0] + Fn[1] * Fn[1] + Fn[2] * Fn[2]);
    if (nFdp <= P.mu_s * nFn) {
        for (int a = 0; a < 3; ++a)
            Ft[a] = Fdp[a];
    } else {
        for (int a = 0; a < 3; ++a) {
            Ft[a] = P.mu_k * nFn * Fdp[a] / nFdp;
            zt[a] = -(Ft[a] + dtc * gtv[a]) / kt;
        }
    }
    for (int a = 0; a < 3; ++a) {
        F[a] = Fn[a] + Ft[a];
        hnew[a] = zt[a];
    }
    hnew[3] = u_in;
}

// Pair (p, q) of the list, p its first particle: force on p, torques on p
// and q, new history.  g = (u_p - u_q) + R_p,cp w_p x n + R_q,cp w_q x n with
// the lever arms R_p,cp = (d + R_p - R_q)/2, R_q,cp = (d + R_q - R_p)/2.
__device__ void pair_contact(const PairC &P, int np, const double *xp, const double *up,
                             const double *wp, const double *radius, const double *mass, int p,
                             int q, const double *hold, double dt, double *F, double *Tp,
                             double *Tq, double *hnew)
{
    double xa[3], xb[3], dvec[3];
    centre(P, np, xp, p, xa);
    centre(P, np, xp, q, xb);
    double d = sqrt(disp2(P, xa, xb, dvec));
    double Rp = radius[p], Rq = radius[q];
    double zeta = d - Rp - Rq;
    double n[3] = {dvec[0] / d, dvec[1] / d, dvec[2] / d};
    double Rpc = 0.5 * (d + Rp - Rq), Rqc = 0.5 * (d + Rq - Rp);
    double wpp[3], wqq[3];
    for (int a = 0; a < 3; ++a) {
        wpp[a] = wp[(size_t)a * np + p];
        wqq[a] = wp[(size_t)a * np + q];
    }
    double wpn[3] = {wpp[1] * n[2] - wpp[2] * n[1], wpp[2] * n[0] - wpp[0] * n[2],
                     wpp[0] * n[1] - wpp[1] * n[0]};
    double wqn[3] = {wqq[1] * n[2] - wqq[2] * n[1], wqq[2] * n[0] - wqq[0] * n[2],
                     wqq[0] * n[1] - wqq[1] * n[0]};
    double g[3];
    for (int a = 0; a < 3; ++a)
        g[a] = (up[(size_t)a * np + p] - up[(size_t)a * np + q]) + Rpc * wpn[a] + Rqc * wqn[a];
    double mp = mass[p], mq = mass[q];
    double Reff = Rp * Rq / (Rp + Rq);
    double meff = mp * mq / (mp + mq);
    double zmin = P.zeta_min_factor * (Rp < Rq ? Rp : Rq);
    double rhod = 0.5 * (rho_d(mp, Rp) + rho_d(mq, Rq));
    double kgp = kn_grav(P, mp, Rp), kgq = kn_grav(P, mq, Rq);
    double Ft[3];
    contact_law(P, zeta, n, g, Reff, meff, zmin, rhod, kgp > kgq ? kgp : kgq, hold, dt, F, Ft,
                hnew);
    double nxFt[3] = {n[1] * Ft[2] - n[2] * Ft[1], n[2] * Ft[0] - n[0] * Ft[2],
                      n[0] * Ft[1] - n[1] * Ft[0]};
    for (int a = 0; a < 3; ++a) {
        Tp[a] = Rpc * nxFt[a];
        Tq[a] = Rqc * nxFt[a];
    }
}

// Wall entry (p, side = 2 axis + upper): the wall as a partner of infinite
// radius and mass at rest, lever arm = the centre's distance to the wall.
__device__ void wall_contact(const PairC &P, int np, const double *xp, const double *up,
                             const double *wp, const double *radius, const double *mass, int p,
                             int side, const double *hold, double dt, double *F, double *T,
                             double *hnew)
{
    int ax = side / 2, upper = side % 2;
    double x = xp[(size_t)ax * np + p];
    double top = P.origin[ax] + P.L[ax];
    double dist = upper == 0 ? (x - P.origin[ax]) : (top - x);
    double Rp = radius[p], mp = mass[p];
    double zeta = dist - Rp;
    double n[3] = {0.0, 0.0, 0.0};
    n[ax] = upper == 0 ? -1.0 : 1.0;
    double wpp[3];
    for (int a = 0; a < 3; ++a)
        wpp[a] = wp[(size_t)a * np + p];
    double wpn[3] = {wpp[1] * n[2] - wpp[2] * n[1], wpp[2] * n[0] - wpp[0] * n[2],
                     wpp[0] * n[1] - wpp[1] * n[0]};
    double g[3];
    for (int a = 0; a < 3; ++a)
        g[a] = up[(size_t)a * np + p] + dist * wpn[a];
    double Ft[3];
    contact_law(P, zeta, n, g, Rp, mp, P.zeta_min_factor * Rp, rho_d(mp, Rp), kn_grav(P, mp, Rp),
                hold, dt, F, Ft, hnew);
    double nxFt[3] = {n[1] * Ft[2] - n[2] * Ft[1], n[2] * Ft[0] - n[0] * Ft[2],
                      n[0] * Ft[1] - n[1] * Ft[0]};
    for (int a = 0; a < 3; ++a)
        T[a] = dist * nxFt[a];
}

// ---------------------------------------------------------------------------
// per-particle adjacency of the contact lists, int2 {code, aux} per entry
//   code   pair k, p first:  2k;  pair k, p second: 2k + 1;  wall k: -(k + 1)
//   aux    the partner's id (pairs) or the wall's side (walls)
//   order  increasing partner id, then walls by side
// ---------------------------------------------------------------------------
struct ContactLists {
    int pair_cap, wall_cap;
    const int *pairs;     // [2][pair_cap]
    const int *walls;     // [2][wall_cap]
    const int *counts;    // device [2]: listed pairs, walls (clamped to the caps)
};

__device__ __forceinline__ int n_pairs(const ContactLists &C) { return min(C.counts[0], C.pair_cap); }
__device__ __forceinline__ int n_walls(const ContactLists &C) { return min(C.counts[1], C.wall_cap); }

// list entries the adjacency can hold: pairs i < j of particles in range,
// wall entries of a particle in range on a wall axis; others are skipped
// (and reported as EINVAL)
__device__ __forceinline__ bool pair_ok(const ContactLists &C, int np, int k)
{
    const int i = C.pairs[k], j = C.pairs[C.pair_cap + k];
    return i >= 0 && j < np && i < j;
}
__device__ __forceinline__ bool wall_ok(const ContactLists &C, int np, const int *periodic, int k)
{
    const int p = C.walls[k], side = C.walls[C.wall_cap + k];
    return p >= 0 && p < np && side >= 0 && side < 6 && !periodic[side / 2];
}

struct Periodic {
    int p[3];
};

__global__ void k_adj_count(ContactLists C, int np, Periodic per, int *deg, int *err)
{
    const int npairs = n_pairs(C), nwall = n_walls(C);
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < npairs + nwall;
         k += gridDim.x * blockDim.x) {
        if (k < npairs) {
            if (!pair_ok(C, np, k)) {
                atomicCAS(err, 0, (int)IBMX_EINVAL);
                continue;
            }
            atomicAdd(&deg[C.pairs[k]], 1);
            atomicAdd(&deg[C.pairs[C.pair_cap + k]], 1);
        } else {
            if (!wall_ok(C, np, per.p, k - npairs)) {
                atomicCAS(err, 0, (int)IBMX_EINVAL);
                continue;
            }
            atomicAdd(&deg[C.walls[k - npairs]], 1);
        }
    }
}

__global__ void k_adj_fill(ContactLists C, int np, Periodic per, const int *off, int *cursor,
                           int2 *adj)
{
    const int npairs = n_pairs(C), nwall = n_walls(C);
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < npairs + nwall;
         k += gridDim.x * blockDim.x) {
        if (k < npairs) {
            if (!pair_ok(C, np, k))
                continue;
            const int i = C.pairs[k], j = C.pairs[C.pair_cap + k];
            adj[off[i] + atomicAdd(&cursor[i], 1)] = make_int2(2 * k, j);
            adj[off[j] + atomicAdd(&cursor[j], 1)] = make_int2(2 * k + 1, i);
        } else {
            const int kw = k - npairs;
            if (!wall_ok(C, np, per.p, kw))
                continue;
            const int p = C.walls[kw];
            adj[off[p] + atomicAdd(&cursor[p], 1)] = make_int2(-(kw + 1), C.walls[C.wall_cap + kw]);
        }
    }
}

__device__ __forceinline__ int adj_key(int np, int2 e) { return e.x >= 0 ? e.y : np + e.y; }

// insertion sort of each particle's entries by key (a few dozen at most)
__global__ void k_adj_sort(int np, const int *off, int2 *adj)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np)
        return;
    int2 *a = adj + off[p];
    const int n = off[p + 1] - off[p];
    for (int i = 1; i < n; ++i) {
        const int2 v = a[i];
        const int kv = adj_key(np, v);
        int j = i - 1;
        while (j >= 0 && adj_key(np, a[j]) > kv) {
            a[j + 1] = a[j];
            --j;
        }
        a[j + 1] = v;
    }
}

// History of all contacts: pair k in rows [a * pair_cap + k], wall k in
// [a * wall_cap + k], a = 0 .. kHist - 1.
struct Hist {
    double *pair;
    double *wall;
};
struct HistC {
    const double *pair;
    const double *wall;
};

// ---------------------------------------------------------------------------
// one contact evaluation of every particle, optionally followed by a stage
// of the particle update
//
// kContactLanes lanes serve one particle: lane j evaluates the particle's
// adjacency entries j, j + kContactLanes, ... (the pair in its canonical
// orientation, so both particles of a pair obtain identical values), the
// particle's first lane sums the results in adjacency order (increasing
// partner id, walls after) and applies the update.  With hnew set, each
// pair's first particle and each wall's particle write the new history.
// ---------------------------------------------------------------------------
constexpr int kContactLanes = 8;
constexpr int kContactBlock = 256;

enum { kStageForces = 0, kStagePredict = 1, kStageCorrect = 2 };

struct Stage {
    double dts;       // sub-step length
    double a2;        // 2 alpha_k
    double alpha;     // alpha_k
    double gamma;     // gamma_k
    double zeta;      // zeta_k
};

struct Body {
    const double *radius, *mass;
    const double *Fh, *Th;   // or null
    const double *sF;        // per-particle factor of F_h, T_h
};

struct StageIO {
    const double *xs, *us, *ws;   // state the contacts are evaluated at
    double *xa, *ua, *wa;         // accepted state (own entries updated by the corrector)
    double *xt, *ut, *wt;         // predicted state (written by the predictor)
    double *Fcur;                 // [6][np] force and torque at the accepted state
    const double *Fprev;          // [6][np] the same one stage earlier
    double *Fc, *Tc;              // forces mode: outputs (or null)
};

// the contribution of adjacency entry ea to particle p: F (3), T (3)
__device__ __forceinline__ void entry_contact(const PairC &P, int np, const ContactLists &C,
                                              int p, int2 ea, const double *xs, const double *us,
                                              const double *ws, const double *radius,
                                              const double *mass, HistC hold, double dt,
                                              Hist hnew, double *f6)
{
    double ho[kHist], hn[kHist], f[3], t1[3], t2[3];
    const int e = ea.x;
    if (e >= 0) {
        const int k = e >> 1;
        for (int a = 0; a < kHist; ++a)
            ho[a] = hold.pair[(size_t)a * C.pair_cap + k];
        const int i = (e & 1) ? ea.y : p, j = (e & 1) ? p : ea.y;
        pair_contact(P, np, xs, us, ws, radius, mass, i, j, ho, dt, f, t1, t2, hn);
        if (e & 1) {
            for (int a = 0; a < 3; ++a) {
                f6[a] = -f[a];
                f6[3 + a] = t2[a];
            }
        } else {
            for (int a = 0; a < 3; ++a) {
                f6[a] = f[a];
                f6[3 + a] = t1[a];
            }
            if (hnew.pair)
                for (int a = 0; a < kHist; ++a)
                    hnew.pair[(size_t)a * C.pair_cap + k] = hn[a];
        }
    } else {
        const int k = -e - 1;
        for (int a = 0; a < kHist; ++a)
            ho[a] = hold.wall[(size_t)a * C.wall_cap + k];
        wall_contact(P, np, xs, us, ws, radius, mass, p, ea.y, ho, dt, f, t1, hn);
        for (int a = 0; a < 3; ++a) {
            f6[a] = f[a];
            f6[3 + a] = t1[a];
        }
        if (hnew.wall)
            for (int a = 0; a < kHist; ++a)
                hnew.wall[(size_t)a * C.wall_cap + k] = hn[a];
    }
}

// particle constants: I = 2/5 m R^2, g' = (1 - rho_f / rho_p) g
__device__ __forceinline__ void body_terms(const PairC &P, const Body &B, int p, double &m,
                                           double &I, double *gp)
{
    m = B.mass[p];
    const double R = B.radius[p];
    I = 0.4 * m * R * R;
    const double rho_p = m / (4.0 / 3.0 * M_PI * R * R * R);
    for (int a = 0; a < 3; ++a)
        gp[a] = (1.0 - P.rho_f / rho_p) * P.g[a];
}

template <int MODE>
__global__ __launch_bounds__(kContactBlock) void k_contact_stage(PairC P, int np, ContactLists C,
                                                                const int *off, const int2 *adj,
                                                                Body B, HistC hold, double dt,
                                                                Hist hnew, StageIO io, Stage S)
{
    __shared__ double part[kContactBlock][6];
    __shared__ int chunks;
    const int g = threadIdx.x / kContactLanes, j = threadIdx.x % kContactLanes;
    const int p = blockIdx.x * (kContactBlock / kContactLanes) + g;
    int lo = 0, deg = 0;
    if (p < np) {
        lo = off[p];
        deg = off[p + 1] - lo;
    }
    if (threadIdx.x == 0)
        chunks = 0;
    __syncthreads();
    if (j == 0 && deg > 0)
        atomicMax(&chunks, (deg + kContactLanes - 1) / kContactLanes);
    __syncthreads();
    const int nch = chunks;
    double F[3] = {0.0, 0.0, 0.0}, T[3] = {0.0, 0.0, 0.0};
    for (int c = 0; c < nch; ++c) {
        const int r = c * kContactLanes + j;
        if (r < deg) {
            double f6[6];
            entry_contact(P, np, C, p, adj[lo + r], io.xs, io.us, io.ws, B.radius, B.mass, hold,
                          dt, hnew, f6);
            for (int q = 0; q < 6; ++q)
                part[threadIdx.x][q] = f6[q];
        }
        __syncthreads();
        if (j == 0) {
            const int n = min(kContactLanes, deg - c * kContactLanes);
            for (int t = 0; t < n; ++t)
                for (int a = 0; a < 3; ++a) {
                    F[a] = F[a] + part[threadIdx.x + t][a];
                    T[a] = T[a] + part[threadIdx.x + t][3 + a];
                }
        }
        __syncthreads();
    }
    if (j != 0 || p >= np)
        return;
    if (MODE == kStageForces) {
        if (io.Fc)
            for (int a = 0; a < 3; ++a) {
                io.Fc[(size_t)a * np + p] = F[a];
                io.Tc[(size_t)a * np + p] = T[a];
            }
        return;
    }
    // the particle's own inputs are loaded only now: loading them before the
    // contacts raises the register count past three waves per SIMD
    double m, I, gp[3];
    body_terms(P, B, p, m, I, gp);
    const double sF = B.sF[p];
    for (int a = 0; a < 3; ++a) {
        const size_t i = (size_t)a * np + p;
        const double Fh = B.Fh ? sF * B.Fh[i] : 0.0, Th = B.Th ? sF * B.Th[i] : 0.0;
        const double u0 = io.ua[i], w0 = io.wa[i], x0 = io.xa[i];
        if (MODE == kStagePredict) {
            // F, T: the accepted state's force, kept for the corrector and
            // the next stage
            io.Fcur[i] = F[a];
            io.Fcur[(size_t)3 * np + i] = T[a];
            double fs = S.a2 * Fh + S.gamma * F[a];
            double ts = S.a2 * Th + S.gamma * T[a];
            if (S.zeta != 0.0) {
                fs = fs + S.zeta * io.Fprev[i];
                ts = ts + S.zeta * io.Fprev[(size_t)3 * np + i];
            }
            const double u1 = u0 + S.dts / m * fs + S.a2 * S.dts * gp[a];
            io.ut[i] = u1;
            io.wt[i] = w0 + S.dts / I * ts;
            io.xt[i] = x0 + S.alpha * S.dts * (u1 + u0);
        } else {
            // F, T: the predicted state's force
            const double fs = S.a2 * Fh + S.gamma * F[a] + S.zeta * io.Fcur[i];
            const double ts = S.a2 * Th + S.gamma * T[a] + S.zeta * io.Fcur[(size_t)3 * np + i];
            const double u1 = u0 + S.dts / m * fs + S.a2 * S.dts * gp[a];
            const double w1 = w0 + S.dts / I * ts;
            io.xa[i] = x0 + S.alpha * S.dts * (u1 + u0);
            io.ua[i] = u1;
            io.wa[i] = w1;
        }
    }
}

// Method parameters and the host-derived collision constants (everything
// but the cell grid).
inline void contact_constants(const ibmx_plan p, PairC *P)
{
    const ibmx_params &prm = p->prm;
    P->rho_f = prm.rho_f;
    P->nu_f = prm.nu_f;
    P->eps_sep = prm.eps_sep;
    P->lub_C = prm.lub_C;
    P->zeta_min_factor = prm.zeta_min_factor;
    P->e_dry = prm.e_dry;
    P->T_c = prm.T_c;
    P->mu_s = prm.mu_s;
    P->mu_k = prm.mu_k;
    P->nu_poi = prm.nu_poi;
    P->dt = prm.dt;
    P->gap_cut = prm.gap_cut;
    P->h = p->g.h;
    for (int a = 0; a < 3; ++a) {
        P->L[a] = p->g.n[a] * p->g.h;
        P->origin[a] = p->g.origin[a];
        P->periodic[a] = p->g.periodic[a];
        P->g[a] = prm.gravity[a];
    }
    P->normal_model = prm.normal_model;
    P->le = log(prm.e_dry);
    P->lin_k = M_PI * M_PI + P->le * P->le;
    P->sq_damp = sqrt(M_PI * M_PI + P->le * P->le);
    P->kt_ratio = 2.0 * (1.0 - prm.nu_poi) / (2.0 - prm.nu_poi);
    P->K_hz = p->actm_K;
    P->D_hz = p->actm_D;
    P->Tc52 = prm.T_c * prm.T_c * sqrt(prm.T_c);
    P->St_crit = prm.St_crit;
    P->kn_grav_eps = prm.kn_grav_eps;
    P->g_abs = sqrt(prm.gravity[0] * prm.gravity[0] + prm.gravity[1] * prm.gravity[1] +
                    prm.gravity[2] * prm.gravity[2]);
}

inline int contact_blocks(long long n, int b) { return n > 0 ? (int)((n + b - 1) / b) : 1; }

// One contact evaluation of every particle (and a stage update with MODE
// kStagePredict / kStageCorrect).
template <int MODE>
inline void contact_stage(const PairC &P, int np, const ContactLists &C, const int *off,
                          const int2 *adj, const Body &B, HistC hold, double dt, Hist hnew,
                          const StageIO &io, const Stage &S, hipStream_t s)
{
    if (np <= 0)
        return;
    const int per = kContactBlock / kContactLanes;
    hipLaunchKernelGGL(k_contact_stage<MODE>, dim3((np + per - 1) / per), dim3(kContactBlock), 0,
                       s, P, np, C, off, adj, B, hold, dt, hnew, io, S);
}

// Adjacency of the lists in C into the plan's contact workspace (c_off,
// c_adj), which holds np + 1 offsets and 2 pair_cap + wall_cap entries.
inline void contact_adjacency(ibmx_plan p, const ContactLists &C, hipStream_t s)
{
    const int np = p->np;
    const long long nmax = (long long)C.pair_cap + C.wall_cap;
    const int g = contact_blocks(nmax, 256) < 4096 ? contact_blocks(nmax, 256) : 4096;
    ZeroList z = {};
    z.add(p->c_deg, np + 1);
    z.add(p->c_cur, np);
    ibmx_zero_i32_multi(z, s);
    const Periodic per{{p->grid.periodic[0], p->grid.periodic[1], p->grid.periodic[2]}};
    hipLaunchKernelGGL(k_adj_count, dim3(g), dim3(256), 0, s, C, np, per, p->c_deg, p->d_err);
    ibmx_exclusive_scan(p->c_deg, p->c_off, np, p->scan_aux, s);
    hipLaunchKernelGGL(k_adj_fill, dim3(g), dim3(256), 0, s, C, np, per, (const int *)p->c_off,
                       p->c_cur, p->c_adj);
    hipLaunchKernelGGL(k_adj_sort, dim3(contact_blocks(np, 64)), dim3(64), 0, s, np,
                       (const int *)p->c_off, p->c_adj);
}

}  // namespace
