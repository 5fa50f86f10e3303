// Pair pass of the collision models (Secs. 2.2.5-2.2.8), FP64 throughout.
//
//   cell list   uniform cells of edge >= 2 R_max + gap_cut, particles listed
//               per cell by id (counting sort, then a per-cell sort);
//   pair list   27-cell search, count -> exclusive scan -> emit, each
//               particle's partners sorted by id, so the list is in (i, j)
//               order and independent of thread scheduling;
//   wall list   (p, side) for every wall closer than gap_cut;
//   forces      lubrication, linear spring-dashpot normal contact and capped
//               tangential spring-dashpot (eq. f_int), one thread per entry;
//   mask        the marker-disable rule, one workgroup per close pair/wall.
//
// Distances, gaps and cell indices are computed with the operation order
// documented in ibmx.h and without FMA contraction so that the integer
// outputs do not depend on the compiler's fusion choices.
#pragma clang fp contract(off)

#include <math.h>

#include "ibmx_internal.hpp"

namespace {

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

__device__ __forceinline__ void cell_coords(const PairC &P, const double *x, int *ci)
{
    for (int a = 0; a < 3; ++a) {
        double t = floor((x[a] - P.origin[a]) / P.edge[a]);
        int v = (int)t;
        if (t < 0.0)
            v = 0;
        if (t > (double)(P.nc[a] - 1))
            v = P.nc[a] - 1;
        ci[a] = v;
    }
}

// ---------------------------------------------------------------------------
// cell list
// ---------------------------------------------------------------------------
__global__ void k_cell_count(PairC P, int np, const double *xp, const double *radius,
                             double rmax, int *cell_of, int *count, int *err)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np)
        return;
    if (!(radius[p] <= rmax))
        atomicCAS(err, 0, (int)IBMX_EINVAL);
    double x[3];
    int ci[3];
    centre(P, np, xp, p, x);
    cell_coords(P, x, ci);
    int c = ci[0] + P.nc[0] * (ci[1] + P.nc[1] * ci[2]);
    cell_of[p] = c;
    atomicAdd(&count[c], 1);
}

__global__ void k_cell_scatter(int np, const int *cell_of, const int *start, int *cursor, int *cellp)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np)
        return;
    int c = cell_of[p];
    int pos = start[c] + atomicAdd(&cursor[c], 1);
    cellp[pos] = p;
}

// insertion sort of one segment (segments are short: particles per cell,
// partners per particle)
__device__ void sort_segment(int *a, int n)
{
    for (int i = 1; i < n; ++i) {
        int v = a[i];
        int j = i - 1;
        while (j >= 0 && a[j] > v) {
            a[j + 1] = a[j];
            --j;
        }
        a[j + 1] = v;
    }
}

__global__ void k_cell_sort(int ncell, const int *start, int *cellp)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell)
        return;
    sort_segment(cellp + start[c], start[c + 1] - start[c]);
}

// ---------------------------------------------------------------------------
// pair search over the neighbouring cells (deduplicated when nc < 3), one
// wave per particle i: the candidates of the (up to 27) cells are numbered
// 0 .. total-1 through a wave prefix sum of the cell sizes and dealt to the
// lanes; hits j > i are counted (EMIT = false) or written in candidate order
// to the scratch half of pairs_out, then sorted and completed by lane 0.
// ---------------------------------------------------------------------------
template <bool EMIT>
__global__ __launch_bounds__(256) void k_pairs(PairC P, int np, const double *xp,
                                               const double *radius, const int *cell_start,
                                               const int *cellp, int *count, const int *off,
                                               int cap, int *pairs_out, double *gap_out)
{
    const int lane = threadIdx.x & (IBMX_WAVE - 1);
    const int i = blockIdx.x * (blockDim.x / IBMX_WAVE) + threadIdx.x / IBMX_WAVE;
    if (i >= np)
        return;
    double xi[3];
    int ci[3];
    centre(P, np, xp, i, xi);
    cell_coords(P, xi, ci);
    int offs[3][3], noff[3];
    for (int a = 0; a < 3; ++a) {
        noff[a] = 0;
        for (int d = -1; d <= 1; ++d) {
            int v = ci[a] + d;
            if (P.periodic[a]) {
                v = (v + P.nc[a]) % P.nc[a];
            } else if (v < 0 || v >= P.nc[a]) {
                continue;
            }
            bool dup = false;
            for (int k = 0; k < noff[a]; ++k)
                dup |= offs[a][k] == v;
            if (!dup)
                offs[a][noff[a]++] = v;
        }
    }
    const int ncells = noff[0] * noff[1] * noff[2];
    // lane k < ncells holds cell k's range and the number of candidates before it
    int c_first = 0, c_len = 0;
    if (lane < ncells) {
        const int kx = lane % noff[0], ky = (lane / noff[0]) % noff[1], kz = lane / (noff[0] * noff[1]);
        const int c = offs[0][kx] + P.nc[0] * (offs[1][ky] + P.nc[1] * offs[2][kz]);
        c_first = cell_start[c];
        c_len = cell_start[c + 1] - c_first;
    }
    int c_pre = c_len;   // inclusive wave scan
    for (int d = 1; d < IBMX_WAVE; d <<= 1) {
        const int v = __shfl_up(c_pre, d, IBMX_WAVE);
        if (lane >= d)
            c_pre += v;
    }
    const int total = __shfl(c_pre, IBMX_WAVE - 1, IBMX_WAVE);
    c_pre -= c_len;   // exclusive
    const double Ri = radius[i];
    const int base = EMIT ? off[i] : 0;
    int cnt = 0;
    for (int t0 = 0; t0 < total; t0 += IBMX_WAVE) {
        const int t = t0 + lane;
        // the cell k holding candidate t: the last k with c_pre[k] <= t
        int first = 0, pre = 0;
        for (int k = 0; k < ncells; ++k) {
            const int pk = __shfl(c_pre, k, IBMX_WAVE);
            const int fk = __shfl(c_first, k, IBMX_WAVE);
            if (pk <= t) {
                pre = pk;
                first = fk;
            }
        }
        bool hit = false;
        int j = -1;
        if (t < total) {
            j = cellp[first + (t - pre)];
            if (j > i) {
                double xj[3], d[3];
                centre(P, np, xp, j, xj);
                const double d2 = disp2(P, xi, xj, d);
                double cut = Ri + radius[j];
                cut = cut + P.gap_cut;
                hit = d2 < cut * cut;
            }
        }
        const unsigned long long m = __ballot(hit);
        if (EMIT && hit) {
            const int pos = cnt + __popcll(m & ((1ULL << lane) - 1ULL));
            if (base + pos < cap)
                pairs_out[cap + base + pos] = j;   // partner ids, sorted below
        }
        cnt += __popcll(m);
    }
    if (!EMIT) {
        if (lane == 0)
            count[i] = cnt;
        return;
    }
    // sort the partners of i, then write i and the gaps in that order
    const int n = min(cnt, cap - base);
    if (n <= 0 || lane != 0)
        return;
    sort_segment(pairs_out + cap + base, n);
    for (int k = 0; k < n; ++k) {
        int j = pairs_out[cap + base + k];
        double xj[3], d[3];
        centre(P, np, xp, j, xj);
        double d2 = disp2(P, xi, xj, d);
        pairs_out[base + k] = i;
        double g = sqrt(d2) - Ri;
        gap_out[base + k] = g - radius[j];
    }
}

template <bool EMIT>
__global__ void k_walls(PairC P, int np, const double *xp, const double *radius, int *count,
                        const int *off, int cap, int *walls_out, double *gap_out)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np)
        return;
    int cnt = 0;
    const int base = EMIT ? off[p] : 0;
    for (int a = 0; a < 3; ++a) {
        if (P.periodic[a])
            continue;
        double x = xp[(size_t)a * np + p];
        for (int side = 0; side < 2; ++side) {
            double top = P.origin[a] + P.L[a];
            double dist = side == 0 ? (x - P.origin[a]) : (top - x);
            double g = dist - radius[p];
            if (g < P.gap_cut) {
                if (EMIT && base + cnt < cap) {
                    walls_out[base + cnt] = p;
                    walls_out[cap + base + cnt] = 2 * a + side;
                    gap_out[base + cnt] = g;
                }
                ++cnt;
            }
        }
    }
    if (!EMIT)
        count[p] = cnt;
}

__global__ void k_list_totals(const int *poff, const int *woff, int np, int pair_cap, int wall_cap,
                              int *counts_out, int *err)
{
    int np_ = poff[np], nw = woff[np];
    counts_out[0] = np_;
    counts_out[1] = nw;
    if (np_ > pair_cap || nw > wall_cap)
        atomicCAS(err, 0, (int)IBMX_ECAPACITY);
}

// ---------------------------------------------------------------------------
// collision law for one contact (force on p; n points from p to the partner)
// ---------------------------------------------------------------------------
__device__ void contact_law(const PairC &P, double zeta, const double *n, const double *g,
                            double Reff, double meff, double zmin, const double *zt_old,
                            double *F, double *Ft, double *zt_new)
{
    double gn = g[0] * n[0] + g[1] * n[1] + g[2] * n[2];
    double gnv[3], gtv[3];
    for (int a = 0; a < 3; ++a) {
        gnv[a] = gn * n[a];
        gtv[a] = g[a] - gnv[a];
        F[a] = 0.0;
        Ft[a] = 0.0;
        zt_new[a] = 0.0;
    }
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
    double le = log(P.e_dry);
    double kn = meff * (M_PI * M_PI + le * le) / (P.T_c * P.T_c);
    double dn = -2.0 * meff * le / P.T_c;
    double Fn[3];
    for (int a = 0; a < 3; ++a)
        Fn[a] = -kn * fabs(zeta) * n[a] - dn * gnv[a];
    double kt = 2.0 * (1.0 - P.nu_poi) / (2.0 - P.nu_poi) * kn;
    double dtc = 2.0 * sqrt(meff * kt) * (-le) / sqrt(M_PI * M_PI + le * le);
    double zon = zt_old[0] * n[0] + zt_old[1] * n[1] + zt_old[2] * n[2];
    double zt[3], Fdp[3];
    for (int a = 0; a < 3; ++a) {
        zt[a] = (zt_old[a] - zon * n[a]) + gtv[a] * P.dt;
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
        zt_new[a] = zt[a];
    }
}

// previous-call history of pair (i, j): binary search in the (i, j)-sorted list
__device__ int find_pair(int n_in, const int *pairs_in, int i, int j)
{
    long long key = ((long long)i << 32) | (unsigned)j;
    int lo = 0, hi = n_in - 1;
    while (lo <= hi) {
        int mid = (lo + hi) >> 1;
        long long k = ((long long)pairs_in[mid] << 32) | (unsigned)pairs_in[n_in + mid];
        if (k == key)
            return mid;
        if (k < key)
            lo = mid + 1;
        else
            hi = mid - 1;
    }
    return -1;
}

__global__ void k_pair_forces(PairC P, int np, const double *xp, const double *radius,
                              const double *mass, const double *up, const double *wp,
                              const int *counts, int cap, const int *pairs, int n_in,
                              const int *pairs_in, const double *hist_in, double *hist_out,
                              double *Fc, double *Tc)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    int npairs = min(counts[0], cap);
    if (k >= npairs)
        return;
    int p = pairs[k], q = pairs[cap + k];
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
    double Reff = Rp * Rq / (Rp + Rq);
    double meff = mass[p] * mass[q] / (mass[p] + mass[q]);
    double zmin = P.zeta_min_factor * (Rp < Rq ? Rp : Rq);
    double zold[3] = {0.0, 0.0, 0.0};
    int kin = n_in > 0 ? find_pair(n_in, pairs_in, p, q) : -1;
    if (kin >= 0)
        for (int a = 0; a < 3; ++a)
            zold[a] = hist_in[(size_t)a * n_in + kin];
    double F[3], Ft[3], zt[3];
    contact_law(P, zeta, n, g, Reff, meff, zmin, zold, F, Ft, zt);
    double nxFt[3] = {n[1] * Ft[2] - n[2] * Ft[1], n[2] * Ft[0] - n[0] * Ft[2],
                      n[0] * Ft[1] - n[1] * Ft[0]};
    for (int a = 0; a < 3; ++a) {
        atomicAdd(&Fc[(size_t)a * np + p], F[a]);
        atomicAdd(&Fc[(size_t)a * np + q], -F[a]);
        atomicAdd(&Tc[(size_t)a * np + p], Rpc * nxFt[a]);
        atomicAdd(&Tc[(size_t)a * np + q], Rqc * nxFt[a]);
        hist_out[(size_t)a * cap + k] = zt[a];
    }
}

__global__ void k_wall_forces(PairC P, int np, const double *xp, const double *radius,
                              const double *mass, const double *up, const double *wp,
                              const int *counts, int cap, const int *walls, int n_in,
                              const int *walls_in, const double *whist_in, double *whist_out,
                              double *Fc, double *Tc)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    int nwall = min(counts[1], cap);
    if (k >= nwall)
        return;
    int p = walls[k], side = walls[cap + k];
    int ax = side / 2, upper = side % 2;
    double x = xp[(size_t)ax * np + p];
    double top = P.origin[ax] + P.L[ax];
    double dist = upper == 0 ? (x - P.origin[ax]) : (top - x);
    double Rp = radius[p];
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
    double zold[3] = {0.0, 0.0, 0.0};
    for (int kk = 0; kk < n_in; ++kk)
        if (walls_in[kk] == p && walls_in[n_in + kk] == side)
            for (int a = 0; a < 3; ++a)
                zold[a] = whist_in[(size_t)a * n_in + kk];
    double F[3], Ft[3], zt[3];
    contact_law(P, zeta, n, g, Rp, mass[p], P.zeta_min_factor * Rp, zold, F, Ft, zt);
    double nxFt[3] = {n[1] * Ft[2] - n[2] * Ft[1], n[2] * Ft[0] - n[0] * Ft[2],
                      n[0] * Ft[1] - n[1] * Ft[0]};
    for (int a = 0; a < 3; ++a) {
        atomicAdd(&Fc[(size_t)a * np + p], F[a]);
        atomicAdd(&Tc[(size_t)a * np + p], dist * nxFt[a]);
        whist_out[(size_t)a * cap + k] = zt[a];
    }
}

// ---------------------------------------------------------------------------
// marker-disable mask
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x)
{
    unsigned long long z = x + 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

// one wave per pair (wall entry); lanes take the chosen particle's markers
__global__ __launch_bounds__(256) void k_mask_pairs(PairC P, int np, int nm, const int *moff,
                                                    const double *body, const double *xp,
                                                    const double *radius, int mode,
                                                    unsigned long long seed, const int *counts,
                                                    int cap, const int *pairs, const double *gap,
                                                    uint8_t *mask)
{
    const int npairs = min(counts[0], cap);
    const int lane = threadIdx.x & (IBMX_WAVE - 1);
    const int wpb = blockDim.x / IBMX_WAVE;
    for (int k = blockIdx.x * wpb + threadIdx.x / IBMX_WAVE; k < npairs; k += gridDim.x * wpb) {
        if (!(gap[k] < 2.0 * P.eps_sep))
            continue;
        int p = pairs[k], q = pairs[cap + k];
        unsigned long long key =
            ((unsigned long long)(unsigned)p << 32) | (unsigned long long)(unsigned)q;
        int chosen = (splitmix64(seed ^ key) & 1ULL) == 0 ? p : q;
        int partner = chosen == p ? q : p;
        double xc[3], xq[3];
        centre(P, np, xp, chosen, xc);
        centre(P, np, xp, partner, xq);
        double lim = radius[partner] + 2.0 * P.eps_sep;
        double lim2 = lim * lim;
        for (int l = moff[chosen] + lane; l < moff[chosen + 1]; l += IBMX_WAVE) {
            if (mode == 2) {
                mask[l] = 0;
                continue;
            }
            double d[3];
            for (int a = 0; a < 3; ++a) {
                d[a] = (xc[a] + body[(size_t)a * nm + l]) - xq[a];
                if (P.periodic[a])
                    d[a] = min_image(d[a], P.L[a]);
            }
            double d2 = d[0] * d[0];
            d2 = d2 + d[1] * d[1];
            d2 = d2 + d[2] * d[2];
            if (d2 < lim2)
                mask[l] = 0;
        }
    }
}

__global__ __launch_bounds__(256) void k_mask_walls(PairC P, int np, int nm, const int *moff,
                                                    const double *body, const double *xp, int mode,
                                                    const int *counts, int cap, const int *walls,
                                                    const double *wgap, uint8_t *mask)
{
    const int nwall = min(counts[1], cap);
    const int lane = threadIdx.x & (IBMX_WAVE - 1);
    const int wpb = blockDim.x / IBMX_WAVE;
    for (int k = blockIdx.x * wpb + threadIdx.x / IBMX_WAVE; k < nwall; k += gridDim.x * wpb) {
        if (!(wgap[k] < P.eps_sep))
            continue;
        int p = walls[k], side = walls[cap + k];
        int ax = side / 2, upper = side % 2;
        double top = P.origin[ax] + P.L[ax];
        for (int l = moff[p] + lane; l < moff[p + 1]; l += IBMX_WAVE) {
            if (mode == 2) {
                mask[l] = 0;
                continue;
            }
            double X = xp[(size_t)ax * np + p] + body[(size_t)ax * nm + l];
            double dist = upper == 0 ? (X - P.origin[ax]) : (top - X);
            if (dist < P.eps_sep)
                mask[l] = 0;
        }
    }
}

int blocks(long long n, int b = 256) { return (int)((n + b - 1) / b) > 0 ? (int)((n + b - 1) / b) : 1; }

}  // namespace

extern "C" ibmx_status ibmx_pairs(ibmx_plan p, const double *xp, const double *radius,
                                  double rmax, const double *mass, const double *up, const double *wp,
                                  int32_t npairs_in, const int32_t *pairs_in, const double *hist_in,
                                  int32_t nwall_in, const int32_t *walls_in, const double *whist_in,
                                  int32_t *cell_start, int32_t cell_cap, int32_t *cell_particles,
                                  int32_t *pairs_out, double *pair_gap, double *hist_out,
                                  int32_t pair_cap, int32_t *walls_out, double *wall_gap,
                                  double *whist_out, int32_t wall_cap, int32_t *counts_out,
                                  double *Fc, double *Tc, uint8_t *marker_active)
{
    if (!p)
        return IBMX_EINVAL;
    const int np = p->np, nm = p->nm;
    if (np > 0 && (!xp || !radius || !mass || !up || !wp || !cell_particles || !Fc || !Tc))
        return IBMX_EINVAL;
    if (!cell_start || !counts_out || pair_cap < 0 || wall_cap < 0 || npairs_in < 0 || nwall_in < 0)
        return IBMX_EINVAL;
    if ((pair_cap > 0 && (!pairs_out || !pair_gap || !hist_out)) ||
        (wall_cap > 0 && (!walls_out || !wall_gap || !whist_out)) ||
        (npairs_in > 0 && (!pairs_in || !hist_in)) || (nwall_in > 0 && (!walls_in || !whist_in)))
        return IBMX_EINVAL;
    if (marker_active && nm > 0 && !p->body)
        return IBMX_ESTATE;
    const ibmx_params &prm = p->prm;
    PairC P;
    P.rho_f = prm.rho_f;
    P.nu_f = prm.nu_f;
    P.eps_sep = prm.eps_sep;
    P.lub_C = prm.lub_C;
    P.zeta_min_factor = prm.zeta_min_factor;
    P.e_dry = prm.e_dry;
    P.T_c = prm.T_c;
    P.mu_s = prm.mu_s;
    P.mu_k = prm.mu_k;
    P.nu_poi = prm.nu_poi;
    P.dt = prm.dt;
    P.gap_cut = prm.gap_cut;
    P.h = p->g.h;
    if (np > 0 && !(rmax > 0.0 && isfinite(rmax)))
        return IBMX_EINVAL;
    long long ncell = 1;
    for (int a = 0; a < 3; ++a) {
        P.L[a] = p->g.n[a] * p->g.h;
        P.origin[a] = p->g.origin[a];
        P.periodic[a] = p->g.periodic[a];
        int k = (int)floor(P.L[a] / (2.0 * rmax + P.gap_cut));
        P.nc[a] = k < 1 ? 1 : k;
        P.edge[a] = P.L[a] / P.nc[a];
        ncell *= P.nc[a];
    }
    if (ncell + 1 > cell_cap)
        return IBMX_ECAPACITY;
    P.ncell = (int)ncell;
    if (!p->p_cursor || p->p_cell_cap < ncell) {
        if (p->p_cursor)
            (void)hipFree(p->p_cursor);
        p->p_cursor = nullptr;
        if (hipMalloc((void **)&p->p_cursor, sizeof(int) * (size_t)ncell) != hipSuccess)
            return IBMX_ENOMEM;
        p->p_cell_cap = (int)ncell;
    }
    if (ibmx_plan_scan_reserve(p, ncell) != IBMX_OK)
        return IBMX_ENOMEM;
    hipStream_t s = p->stream;
    ProfScope ps(p, IBMX_K_PAIRS);
    // cell list
    ibmx_fill_i32(cell_start, 0, ncell + 1, s);
    ibmx_fill_i32(p->p_cursor, 0, ncell, s);
    if (np > 0)
        hipLaunchKernelGGL(k_cell_count, dim3(blocks(np)), dim3(256), 0, s, P, np, xp, radius,
                           rmax, p->p_cell_of, cell_start, p->d_err);
    ibmx_exclusive_scan(cell_start, cell_start, (int)ncell, p->scan_aux, s);
    if (np > 0) {
        hipLaunchKernelGGL(k_cell_scatter, dim3(blocks(np)), dim3(256), 0, s, np, p->p_cell_of,
                           cell_start, p->p_cursor, cell_particles);
        hipLaunchKernelGGL(k_cell_sort, dim3(blocks(ncell)), dim3(256), 0, s, (int)ncell,
                           cell_start, cell_particles);
        // pair and wall lists
        hipLaunchKernelGGL(k_pairs<false>, dim3(blocks(np, 4)), dim3(256), 0, s, P, np, xp, radius,
                           cell_start, cell_particles, p->p_count, (const int *)nullptr, 0,
                           (int *)nullptr, (double *)nullptr);
        hipLaunchKernelGGL(k_walls<false>, dim3(blocks(np)), dim3(256), 0, s, P, np, xp, radius,
                           p->p_wcount, (const int *)nullptr, 0, (int *)nullptr, (double *)nullptr);
    }
    ibmx_exclusive_scan(p->p_count, p->p_off, np, p->scan_aux, s);
    ibmx_exclusive_scan(p->p_wcount, p->p_woff, np, p->scan_aux, s);
    if (np > 0) {
        hipLaunchKernelGGL(k_pairs<true>, dim3(blocks(np, 4)), dim3(256), 0, s, P, np, xp, radius,
                           cell_start, cell_particles, p->p_count, p->p_off, pair_cap, pairs_out,
                           pair_gap);
        hipLaunchKernelGGL(k_walls<true>, dim3(blocks(np)), dim3(256), 0, s, P, np, xp, radius,
                           p->p_wcount, p->p_woff, wall_cap, walls_out, wall_gap);
    }
    hipLaunchKernelGGL(k_list_totals, dim3(1), dim3(1), 0, s, p->p_off, p->p_woff, np, pair_cap,
                       wall_cap, counts_out, p->d_err);
    // forces
    ibmx_fill_f64(Fc, 0.0, 3LL * np, s);
    ibmx_fill_f64(Tc, 0.0, 3LL * np, s);
    if (pair_cap > 0)
        hipLaunchKernelGGL(k_pair_forces, dim3(blocks(pair_cap)), dim3(256), 0, s, P, np, xp,
                           radius, mass, up, wp, counts_out, pair_cap, pairs_out, npairs_in,
                           pairs_in, hist_in, hist_out, Fc, Tc);
    if (wall_cap > 0)
        hipLaunchKernelGGL(k_wall_forces, dim3(blocks(wall_cap)), dim3(256), 0, s, P, np, xp,
                           radius, mass, up, wp, counts_out, wall_cap, walls_out, nwall_in,
                           walls_in, whist_in, whist_out, Fc, Tc);
    // mask
    if (marker_active && nm > 0) {
        ibmx_fill_u8(marker_active, 1, nm, s);
        if (prm.disable_mode != 0) {
            if (pair_cap > 0)
                hipLaunchKernelGGL(k_mask_pairs, dim3(min(blocks(pair_cap, 4), 8192)), dim3(256), 0, s,
                                   P, np, nm,
                                   p->d_moff, p->body, xp, radius, prm.disable_mode,
                                   (unsigned long long)prm.disable_seed, counts_out, pair_cap,
                                   pairs_out, pair_gap, marker_active);
            if (wall_cap > 0)
                hipLaunchKernelGGL(k_mask_walls, dim3(min(blocks(wall_cap, 4), 8192)), dim3(256), 0, s,
                                   P, np, nm,
                                   p->d_moff, p->body, xp, prm.disable_mode, counts_out, wall_cap,
                                   walls_out, wall_gap, marker_active);
        }
    }
    return ibmx_launch_check();
}
