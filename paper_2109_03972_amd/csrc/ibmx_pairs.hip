// Pair pass of the collision models (Secs. 2.2.5-2.2.8), FP64 throughout.
//
//   cell list   uniform cells of edge >= 2 R_max + gap_cut, particles listed
//               per cell by id (counting sort, then a per-cell sort);
//   pair list   27-cell search, count -> exclusive scan -> emit, each
//               particle's partners sorted by id, so the list is in (i, j)
//               order and independent of thread scheduling;
//   wall list   (p, side) for every wall closer than gap_cut;
//   forces      lubrication, normal contact (linear or Hertz) and capped
//               tangential spring-dashpot (eq. f_int): a group of lanes per
//               particle evaluates its contacts, summed in partner order;
//   mask        the marker-disable rule, one workgroup per close pair/wall.
//
// Distances, gaps and cell indices are computed with the operation order
// documented in ibmx.h and without FMA contraction so that the integer
// outputs do not depend on the compiler's fusion choices.
#pragma clang fp contract(off)

#include <math.h>

#include "ibmx_contact.hpp"

namespace {

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

// previous-call history of wall entry (p, side): binary search in the
// (p, side)-sorted list
__device__ int find_wall(int n_in, const int *walls_in, int p, int side)
{
    long long key = (long long)p * 8 + side;
    int lo = 0, hi = n_in - 1;
    while (lo <= hi) {
        int mid = (lo + hi) >> 1;
        long long k = (long long)walls_in[mid] * 8 + walls_in[n_in + mid];
        if (k == key)
            return mid;
        if (k < key)
            lo = mid + 1;
        else
            hi = mid - 1;
    }
    return -1;
}

// history of the previous call, aligned with the new lists (zero for new
// contacts)
__global__ void k_hist_align(ContactLists C, int n_in, const int *pairs_in, const double *hist_in,
                             int nw_in, const int *walls_in, const double *whist_in, Hist hold)
{
    const int npairs = n_pairs(C), nwall = n_walls(C);
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < npairs + nwall;
         k += gridDim.x * blockDim.x) {
        if (k < npairs) {
            const int kin = n_in > 0 ? find_pair(n_in, pairs_in, C.pairs[k], C.pairs[C.pair_cap + k])
                                     : -1;
            for (int a = 0; a < kHist; ++a)
                hold.pair[(size_t)a * C.pair_cap + k] =
                    kin >= 0 ? hist_in[(size_t)a * n_in + kin] : 0.0;
        } else {
            const int kw = k - npairs;
            const int kin =
                nw_in > 0 ? find_wall(nw_in, walls_in, C.walls[kw], C.walls[C.wall_cap + kw]) : -1;
            for (int a = 0; a < kHist; ++a)
                hold.wall[(size_t)a * C.wall_cap + kw] =
                    kin >= 0 ? whist_in[(size_t)a * nw_in + kin] : 0.0;
        }
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
constexpr int MUNR = 8;   // marker rounds per batch of offset loads in the mask kernels

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
        const int l1 = moff[chosen + 1];
        if (mode == 2) {
            for (int l = moff[chosen] + lane; l < l1; l += IBMX_WAVE)
                mask[l] = 0;
            continue;
        }
        // MUNR rounds of offsets loaded before any test, so that a large
        // particle's markers cost few memory round trips
        for (int l0 = moff[chosen] + lane; l0 < l1; l0 += MUNR * IBMX_WAVE) {
            double o[MUNR][3];
#pragma unroll
            for (int r = 0; r < MUNR; ++r) {
                const int l = l0 + r * IBMX_WAVE;
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    o[r][a] = l < l1 ? body[(size_t)a * nm + l] : 0.0;
            }
#pragma unroll
            for (int r = 0; r < MUNR; ++r) {
                const int l = l0 + r * IBMX_WAVE;
                double d[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    d[a] = (xc[a] + o[r][a]) - xq[a];
                    if (P.periodic[a])
                        d[a] = min_image(d[a], P.L[a]);
                }
                double d2 = d[0] * d[0];
                d2 = d2 + d[1] * d[1];
                d2 = d2 + d[2] * d[2];
                if (l < l1 && d2 < lim2)
                    mask[l] = 0;
            }
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
        const int l1 = moff[p + 1];
        if (mode == 2) {
            for (int l = moff[p] + lane; l < l1; l += IBMX_WAVE)
                mask[l] = 0;
            continue;
        }
        const double xa = xp[(size_t)ax * np + p];
        for (int l0 = moff[p] + lane; l0 < l1; l0 += MUNR * IBMX_WAVE) {
            double o[MUNR];
#pragma unroll
            for (int r = 0; r < MUNR; ++r) {
                const int l = l0 + r * IBMX_WAVE;
                o[r] = l < l1 ? body[(size_t)ax * nm + l] : 0.0;
            }
#pragma unroll
            for (int r = 0; r < MUNR; ++r) {
                const int l = l0 + r * IBMX_WAVE;
                double X = xa + o[r];
                double dist = upper == 0 ? (X - P.origin[ax]) : (top - X);
                if (l < l1 && dist < P.eps_sep)
                    mask[l] = 0;
            }
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
    contact_constants(p, &P);
    if (np > 0 && !(rmax > 0.0 && isfinite(rmax)))
        return IBMX_EINVAL;
    long long ncell = 1;
    for (int a = 0; a < 3; ++a) {
        int k = (int)floor(P.L[a] / (2.0 * rmax + P.gap_cut));
        P.nc[a] = k < 1 ? 1 : k;
        P.edge[a] = P.L[a] / P.nc[a];
        ncell *= P.nc[a];
    }
    if (ncell + 1 > cell_cap)
        return IBMX_ECAPACITY;
    P.ncell = (int)ncell;
    // the workspace comes from ibmx_plan_reserve: this call allocates nothing
    if (!p->p_cursor || p->p_cell_cap < ncell || p->scan_cap < ncell || p->scan_cap < np ||
        !ibmx_contact_ready(p, pair_cap, wall_cap, 1))
        return IBMX_ESTATE;
    hipStream_t s = p->stream;
    ProfScope ps(p, IBMX_K_PAIRS);
    // cell list
    ZeroList z = {};
    z.add(cell_start, ncell + 1);
    z.add(p->p_cursor, ncell);
    ibmx_zero_i32_multi(z, s);
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
    // forces: previous history aligned with the new lists, per-particle
    // adjacency, then one thread per particle
    const ContactLists C{pair_cap, wall_cap, pairs_out, walls_out, counts_out};
    const Hist hold{p->c_hist, p->c_hist + (size_t)kHist * pair_cap};
    {
        const long long nmax = (long long)pair_cap + wall_cap;
        const int g = blocks(nmax) < 4096 ? blocks(nmax) : 4096;
        hipLaunchKernelGGL(k_hist_align, dim3(g), dim3(256), 0, s, C, npairs_in, pairs_in, hist_in,
                           nwall_in, walls_in, whist_in, hold);
    }
    contact_adjacency(p, C, s);
    StageIO io{};
    io.xs = xp;
    io.us = up;
    io.ws = wp;
    io.Fc = Fc;
    io.Tc = Tc;
    contact_stage<kStageForces>(P, np, C, p->c_off, (const int2 *)p->c_adj,
                                Body{radius, mass, nullptr, nullptr, nullptr},
                                HistC{hold.pair, hold.wall}, P.dt, Hist{hist_out, whist_out}, io,
                                Stage{}, s);
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
