// Plan life cycle: validation, workspace allocation, deferred status.
#include <math.h>
#include <stdlib.h>
#include <string.h>


#include "ibmx_internal.hpp"

namespace {

int bits_for(int n)
{
    int b = 0;
    while ((1 << b) < n)
        ++b;
    return b < 1 ? 1 : b;
}

void free_plan(ibmx_plan p)
{
    if (!p)
        return;
    void *ptrs[] = {p->d_moff,      p->d_pid,       p->d_err,        p->rpart,     p->d_count,
                    p->rec_tn,      p->rec_ud,      p->rec_src,      p->rec_Gp,    p->rec_G,
                    p->m_key,       p->m_inv,       p->tile_count, p->tile_start,
                    p->tile_cursor, p->halo_count,  p->halo_start,   p->halo_cursor,
                    p->halo_list,   p->tile_gmax,   p->scan_aux,     p->mean_part,    p->bw_u,
                    p->c_deg,       p->c_off,       p->c_cur,        p->c_adj,        p->c_hist,
                    p->s_buf,       p->fl_r,        p->fl_z,        p->fl_cp,        p->fl_tw[0],     p->fl_tw[1],
                    p->fl_tw[2],         p->p_cell_of, p->p_cursor,
                    p->p_count,     p->p_off,       p->p_wcount,     p->p_woff};
    for (void *q : ptrs)
        if (q)
            (void)hipFree(q);
    ibmx_plan_drop_graph(p);
    if (p->cap_stream)
        (void)hipStreamDestroy(p->cap_stream);
    if (p->ev) {
        for (int i = 0; i < 2 * p->ev_cap; ++i)
            (void)hipEventDestroy(p->ev[i]);
        free(p->ev);
        free(p->ev_kind);
    }
    free(p);
}

ibmx_status check_params(const ibmx_grid *g, const ibmx_params *prm)
{
    if (!g || !prm)
        return IBMX_EINVAL;
    long long nodes = 1;
    for (int a = 0; a < 3; ++a) {
        if (g->n[a] < 1 || (g->periodic[a] != 0 && g->periodic[a] != 1))
            return IBMX_EINVAL;
        nodes *= g->n[a];
    }
    if (nodes >= (1LL << 31))
        return IBMX_EINVAL;
    if (bits_for(g->n[0]) + bits_for(g->n[1]) + bits_for(g->n[2]) > 32)
        return IBMX_EUNSUPPORTED;
    if (!(g->h > 0.0) || !isfinite(g->h))
        return IBMX_EINVAL;
    if (prm->kernel != 3 && prm->kernel != 4)
        return IBMX_EUNSUPPORTED;
    if (prm->normal_model != 0 && prm->normal_model != 1)
        return IBMX_EUNSUPPORTED;
    if (!(prm->St_crit >= 0.0) || !isfinite(prm->St_crit) || !(prm->kn_grav_eps > 0.0) ||
        !isfinite(prm->kn_grav_eps) || (prm->st_switch != 0 && prm->st_switch != 1) ||
        prm->reserved != 0)
        return IBMX_EINVAL;
    for (int a = 0; a < 3; ++a)
        if (!isfinite(prm->gravity[a]))
            return IBMX_EINVAL;
    if (prm->n_iter < 1 || prm->n_iter > 64)
        return IBMX_EINVAL;
    if (!(prm->two_alpha_dt != 0.0) || !isfinite(prm->two_alpha_dt))
        return IBMX_EINVAL;
    if (prm->disable_mode < 0 || prm->disable_mode > 2)
        return IBMX_EINVAL;
    // the disable rule (Sec. 2.2.5) acts on every pair closer than 2 eps_sep:
    // the pair list must reach that far
    if (prm->disable_mode != 0 && !(prm->gap_cut >= 2.0 * prm->eps_sep))
        return IBMX_EINVAL;
    if (!(prm->eps_sep >= 0.0) || !(prm->gap_cut >= 0.0) || !(prm->T_c > 0.0) ||
        !(prm->e_dry > 0.0 && prm->e_dry <= 1.0) || !(prm->dt > 0.0))
        return IBMX_EINVAL;
    // periodic axes must hold at least the delta support twice over
    for (int a = 0; a < 3; ++a)
        if (g->periodic[a] && g->n[a] < 2 * prm->kernel)
            return IBMX_EINVAL;
    return IBMX_OK;
}

}  // namespace

 extern "C" ibmx_status ibmx_plan_create(ibmx_plan *out, const ibmx_grid *grid,
                                        const ibmx_params *params, int32_t np,
                                        const int32_t *moff_host, ibmx_precision precision,
                                        void *hip_stream)
{
    if (!out)
        return IBMX_EINVAL;
    *out = nullptr;
    ibmx_status st = check_params(grid, params);
    if (st != IBMX_OK)
        return st;
    if (np < 0 || (np > 0 && !moff_host) || (precision != IBMX_F64 && precision != IBMX_F32))
        return IBMX_EINVAL;
    long long nm = 0;
    if (np > 0) {
        if (moff_host[0] != 0)
            return IBMX_EINVAL;
        for (int i = 0; i < np; ++i)
            if (moff_host[i + 1] < moff_host[i])
                return IBMX_EINVAL;
        nm = moff_host[np];
    }
    if (nm >= (1LL << 31) - 64)
        return IBMX_EINVAL;

    ibmx_plan p = (ibmx_plan)calloc(1, sizeof(ibmx_plan_s));
    if (!p)
        return IBMX_ENOMEM;
    p->grid = *grid;
    p->prm = *params;
    p->np = np;
    p->nm = (int)nm;
    p->n_iter_cap = params->n_iter;
    p->prec = precision;
    p->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&p->device) != hipSuccess) {
        free(p);
        return IBMX_EDEVICE;
    }
    GridC &g = p->g;
    long long nodes = 1;
    for (int a = 0; a < 3; ++a) {
        g.n[a] = grid->n[a];
        g.periodic[a] = grid->periodic[a];
        g.origin[a] = grid->origin[a];
        nodes *= grid->n[a];
    }
    g.h = grid->h;
    g.inv_h3 = 1.0 / (grid->h * grid->h * grid->h);
    g.nodes = nodes;
    g.shift[0] = 0;
    g.shift[1] = bits_for(g.n[0]);
    g.shift[2] = g.shift[1] + bits_for(g.n[1]);

    const size_t Ts = precision == IBMX_F64 ? sizeof(double) : sizeof(float);
    const size_t nmz = nm > 0 ? (size_t)nm : 1;
    const size_t npz = np > 0 ? (size_t)np : 1;
    bool ok = true;
    auto A = [&](void **q, size_t bytes) {
        if (ok && hipMalloc(q, bytes) != hipSuccess)
            ok = false;
    };
    A((void **)&p->d_moff, sizeof(int) * (npz + 1));
    A((void **)&p->d_pid, sizeof(int) * nmz);
    A((void **)&p->d_err, sizeof(int) * 4);
    A((void **)&p->d_count, sizeof(long long) * 8 * IBMX_RSLOTS);
    A((void **)&p->mean_part, sizeof(double) * 3 * ibmx_mean_blocks());
    A(&p->rec_tn, Ts * 4 * nmz);
    A(&p->rec_ud, Ts * 4 * nmz);
    A(&p->rec_G, Ts * 4 * nmz);
    A(&p->rec_Gp, Ts * 4 * nmz * (size_t)p->n_iter_cap);
    A((void **)&p->rpart, sizeof(double) * (size_t)(p->n_iter_cap + 1) * npz);
    A((void **)&p->rec_src, sizeof(int) * nmz);
    A((void **)&p->m_key, sizeof(int) * nmz);
    A((void **)&p->m_inv, sizeof(int) * nmz);
    A((void **)&p->p_cell_of, sizeof(int) * npz);
    A((void **)&p->p_count, sizeof(int) * (npz + 1));
    A((void **)&p->p_off, sizeof(int) * (npz + 1));
    A((void **)&p->p_wcount, sizeof(int) * (npz + 1));
    A((void **)&p->p_woff, sizeof(int) * (npz + 1));
    A((void **)&p->c_deg, sizeof(int) * (npz + 1));
    A((void **)&p->c_off, sizeof(int) * (npz + 1));
    A((void **)&p->c_cur, sizeof(int) * npz);
    if (!ok) {
        free_plan(p);
        return IBMX_ENOMEM;
    }
    // marker -> particle map from the CSR offsets
    int *pid = (int *)malloc(sizeof(int) * nmz);
    int *moff = (int *)malloc(sizeof(int) * (npz + 1));
    if (!pid || !moff) {
        free(pid);
        free(moff);
        free_plan(p);
        return IBMX_ENOMEM;
    }
    moff[0] = 0;
    for (int i = 0; i < np; ++i) {
        moff[i + 1] = moff_host[i + 1];
        for (int l = moff_host[i]; l < moff_host[i + 1]; ++l)
            pid[l] = i;
    }
    if (np == 0)
        moff[1] = 0;
    hipError_t e1 = hipMemcpy(p->d_pid, pid, sizeof(int) * (size_t)nm, hipMemcpyHostToDevice);
    hipError_t e2 = hipMemcpy(p->d_moff, moff, sizeof(int) * (size_t)(np + 1), hipMemcpyHostToDevice);
    free(pid);
    free(moff);
    if (e1 != hipSuccess || e2 != hipSuccess ||
        hipMemset(p->d_err, 0, sizeof(int) * 4) != hipSuccess ||
        hipMemset(p->d_count, 0, sizeof(long long) * 8 * IBMX_RSLOTS) != hipSuccess) {
        free_plan(p);
        return IBMX_EDEVICE;
    }
    p->block = 256;
    p->stats.n_markers = nm;
    st = ibmx_plan_actm(p);
    if (st != IBMX_OK) {
        free_plan(p);
        return st;
    }
    // default tiles: 16 x 16 x 8 nodes
    st = ibmx_plan_scan_reserve(p, np);
    if (st == IBMX_OK)
        st = ibmx_plan_alloc_tiles(p, 16, 16, 8);
    if (st != IBMX_OK) {
        free_plan(p);
        return st;
    }
    *out = p;
    return IBMX_OK;
}

ibmx_status ibmx_plan_alloc_tiles(ibmx_plan p, int tx, int ty, int tz)
{
    int t[3] = {tx, ty, tz};
    int nt[3];
    long long ntiles = 1;
    const int W = 4;   // widest delta support
    // a staged row of B[0] + W - 1 nodes must fit one wave
    if (t[0] > 60)
        return IBMX_EINVAL;
    for (int a = 0; a < 3; ++a) {
        if (t[a] < W || t[a] > 64)
            return IBMX_EINVAL;
        const int n = p->g.n[a];
        // a short last tile must still hold a whole support: take the
        // nearest edge (smaller first) that leaves no remainder or one >= W
        auto fits = [&](int e) { return n % e == 0 || n % e >= W; };
        if (t[a] >= n) {
            t[a] = n;
        } else if (!fits(t[a])) {
            int e = -1;
            for (int d = 1; d < 64 && e < 0; ++d) {
                if (t[a] - d >= W && fits(t[a] - d))
                    e = t[a] - d;
                else if (t[a] + d <= 64 && t[a] + d < n && fits(t[a] + d))
                    e = t[a] + d;
            }
            if (e < 0) {
                if (n > 64)
                    return IBMX_EUNSUPPORTED;
                e = n;
            }
            t[a] = e;
        }
        nt[a] = (p->g.n[a] + t[a] - 1) / t[a];
        ntiles *= nt[a];
    }
    if (ntiles > (1LL << 28))
        return IBMX_EINVAL;
    if (t[0] > 60)
        return IBMX_EUNSUPPORTED;
    const size_t Ts = p->prec == IBMX_F64 ? sizeof(double) : sizeof(float);
    if ((size_t)3 * t[0] * t[1] * t[2] * Ts > 160 * 1024)
        return IBMX_EUNSUPPORTED;
    if (!p->tile_count || ntiles > p->tile_cap) {
        void *ptrs[] = {p->tile_count, p->tile_start, p->tile_cursor, p->halo_count,
                        p->halo_start, p->halo_cursor, p->tile_gmax};
        for (void *q : ptrs)
            if (q)
                (void)hipFree(q);
        p->tile_count = p->tile_start = p->tile_cursor = nullptr;
        p->halo_count = p->halo_start = p->halo_cursor = nullptr;
        p->tile_gmax = nullptr;
        p->tc.ntiles = 0;
        p->tile_cap = 0;
        size_t b = sizeof(int) * (size_t)(ntiles + 1);
        if (hipMalloc((void **)&p->tile_count, b) != hipSuccess ||
            hipMalloc((void **)&p->tile_start, b) != hipSuccess ||
            hipMalloc((void **)&p->tile_cursor, b) != hipSuccess ||
            hipMalloc((void **)&p->halo_count, b) != hipSuccess ||
            hipMalloc((void **)&p->halo_start, b) != hipSuccess ||
            hipMalloc((void **)&p->halo_cursor, b) != hipSuccess ||
            hipMalloc((void **)&p->tile_gmax, sizeof(float4) * 2 * (size_t)ntiles) != hipSuccess)
            return IBMX_ENOMEM;
        p->tile_cap = ntiles;
    }
    // every marker reaches at most 7 tiles besides its own
    long long cap = 7LL * (p->nm > 0 ? p->nm : 1);
    if (!p->halo_list || p->halo_cap < cap) {
        if (p->halo_list)
            (void)hipFree(p->halo_list);
        p->halo_list = nullptr;
        if (hipMalloc((void **)&p->halo_list, sizeof(int) * (size_t)cap) != hipSuccess)
            return IBMX_ENOMEM;
        p->halo_cap = cap;
    }
    for (int a = 0; a < 3; ++a) {
        p->tc.B[a] = t[a];
        p->tc.nt[a] = nt[a];
        p->tc.sh[a] = -1;
        for (int k = 0; k < 31; ++k)
            if ((1 << k) == t[a])
                p->tc.sh[a] = k;
        p->stats.tile[a] = t[a];
    }
    p->tc.ntiles = (int)ntiles;
    p->stats.tiles = ntiles;
    ibmx_plan_drop_graph(p);
    if (ibmx_plan_scan_reserve(p, ntiles) != IBMX_OK)
        return IBMX_ENOMEM;
    return ibmx_spread_allow_lds(p);
}

// Grow the scan workspace to serve scans of up to n elements.
ibmx_status ibmx_plan_scan_reserve(ibmx_plan p, long long n)
{
    if (p->scan_aux && p->scan_cap >= n)
        return IBMX_OK;
    if (p->scan_aux)
        (void)hipFree(p->scan_aux);
    p->scan_aux = nullptr;
    p->scan_cap = 0;
    if (hipMalloc((void **)&p->scan_aux, sizeof(int) * (size_t)ibmx_scan_aux_size(n)) != hipSuccess)
        return IBMX_ENOMEM;
    p->scan_cap = n;
    return IBMX_OK;
}

extern "C" ibmx_status ibmx_plan_destroy(ibmx_plan p)
{
    if (!p)
        return IBMX_EINVAL;
    (void)hipStreamSynchronize(p->stream);
    free_plan(p);
    return IBMX_OK;
}

extern "C" ibmx_status ibmx_plan_set_markers(ibmx_plan p, const double *body, const double *dV)
{
    if (!p || (p->nm > 0 && !body) || (p->np > 0 && !dV))
        return IBMX_EINVAL;
    p->body = body;
    p->dV = dV;
    ibmx_plan_drop_graph(p);
    return IBMX_OK;
}

extern "C" ibmx_status ibmx_plan_set_params(ibmx_plan p, const ibmx_params *prm)
{
    if (!p)
        return IBMX_EINVAL;
    ibmx_status st = check_params(&p->grid, prm);
    if (st != IBMX_OK)
        return st;
    if (prm->n_iter > p->n_iter_cap)
        return IBMX_EINVAL;
    const ibmx_params old = p->prm;
    p->prm = *prm;
    st = ibmx_plan_actm(p);
    if (st != IBMX_OK) {
        p->prm = old;
        return st;
    }
    ibmx_plan_drop_graph(p);
    return IBMX_OK;
}

extern "C" ibmx_status ibmx_plan_set_tiles(ibmx_plan p, int32_t tx, int32_t ty, int32_t tz)
{
    if (!p)
        return IBMX_EINVAL;
    if (hipStreamSynchronize(p->stream) != hipSuccess)
        return IBMX_EDEVICE;
    const int old[3] = {p->tc.B[0], p->tc.B[1], p->tc.B[2]};
    const ibmx_status st = ibmx_plan_alloc_tiles(p, tx, ty, tz);
    if (st != IBMX_OK)
        (void)ibmx_plan_alloc_tiles(p, old[0], old[1], old[2]);
    return st;
}

extern "C" ibmx_status ibmx_plan_set_launch(ibmx_plan p, int32_t block, int32_t persistent)
{
    if (!p || (block != 64 && block != 128 && block != 256) || (persistent != 0 && persistent != 1))
        return IBMX_EINVAL;
    p->block = block;
    p->persist = persistent;
    p->stats.block = block;
    p->stats.persistent = persistent;
    ibmx_plan_drop_graph(p);
    return IBMX_OK;
}

extern "C" ibmx_status ibmx_plan_set_stream(ibmx_plan p, void *stream)
{
    if (!p)
        return IBMX_EINVAL;
    p->stream = (hipStream_t)stream;
    return IBMX_OK;
}

extern "C" ibmx_status ibmx_plan_status(ibmx_plan p)
{
    if (!p)
        return IBMX_EINVAL;
    if (hipStreamSynchronize(p->stream) != hipSuccess)
        return IBMX_EDEVICE;
    int err = 0;
    if (hipMemcpy(&err, p->d_err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
        return IBMX_EDEVICE;
    if (err != 0 && hipMemset(p->d_err, 0, sizeof(int)) != hipSuccess)
        return IBMX_EDEVICE;
    return (ibmx_status)err;
}

extern "C" ibmx_status ibmx_plan_stats(ibmx_plan p, ibmx_stats *out)
{
    if (!p || !out)
        return IBMX_EINVAL;
    if (hipStreamSynchronize(p->stream) != hipSuccess)
        return IBMX_EDEVICE;
    long long *c = (long long *)malloc(sizeof(long long) * 8 * IBMX_RSLOTS);
    if (!c)
        return IBMX_ENOMEM;
    if (hipMemcpy(c, p->d_count, sizeof(long long) * 8 * IBMX_RSLOTS, hipMemcpyDeviceToHost) !=
        hipSuccess) {
        free(c);
        return IBMX_EDEVICE;
    }
    long long tot[3] = {0, 0, 0};
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < IBMX_RSLOTS; ++i)
            tot[k] += c[k * IBMX_RSLOTS + i];
    free(c);
    p->stats.n_active = tot[0];
    p->stats.shell_nodes = tot[1];
    p->stats.halo_entries = tot[2];
    p->stats.block = p->block;
    p->stats.persistent = p->persist;
    for (int i = 0; i < p->ev_used; ++i) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, p->ev[2 * i], p->ev[2 * i + 1]) != hipSuccess)
            return IBMX_EDEVICE;
        p->acc_ms[p->ev_kind[i]] += ms;
        p->acc_n[p->ev_kind[i]] += 1;
    }
    p->ev_used = 0;
    for (int k = 0; k < 8; ++k) {
        p->stats.kernel_ms[k] = p->acc_ms[k];
        p->stats.kernel_launches[k] = p->acc_n[k];
    }
    *out = p->stats;
    return IBMX_OK;
}

extern "C" ibmx_status ibmx_plan_profile(ibmx_plan p, int32_t enable)
{
    if (!p)
        return IBMX_EINVAL;
    if (hipStreamSynchronize(p->stream) != hipSuccess)
        return IBMX_EDEVICE;
    if (enable && !p->ev) {
        const int cap = 8192;
        p->ev = (hipEvent_t *)calloc(2 * cap, sizeof(hipEvent_t));
        p->ev_kind = (int *)calloc(cap, sizeof(int));
        if (!p->ev || !p->ev_kind)
            return IBMX_ENOMEM;
        for (int i = 0; i < 2 * cap; ++i)
            if (hipEventCreate(&p->ev[i]) != hipSuccess)
                return IBMX_EDEVICE;
        p->ev_cap = cap;
    }

    p->ev_used = 0;
    for (int k = 0; k < 8; ++k) {
        p->acc_ms[k] = 0.0;
        p->acc_n[k] = 0;
    }
    p->prof = enable ? 1 : 0;
    return IBMX_OK;
}

ibmx_status ibmx_plan_actm(ibmx_plan p)
{
    if (p->prm.normal_model != 1 || p->actm_e == p->prm.e_dry)
        return IBMX_OK;
    double K = 0.0, D = 0.0;
    const ibmx_status st = ibmx_actm_coefficients(p->prm.e_dry, &K, &D);
    if (st != IBMX_OK)
        return st;
    p->actm_K = K;
    p->actm_D = D;
    p->actm_e = p->prm.e_dry;
    return IBMX_OK;
}

long long ibmx_substep_doubles(int np) { return 22LL * (np > 0 ? np : 1); }

bool ibmx_contact_ready(ibmx_plan p, int pair_cap, int wall_cap, int hist_sets)
{
    const long long nadj = 2LL * pair_cap + wall_cap;
    const long long nh = (long long)hist_sets * IBMX_HIST * ((long long)pair_cap + wall_cap);
    return p->c_adj && p->c_adj_cap >= nadj && (nh == 0 || (p->c_hist && p->c_hist_cap >= nh));
}

extern "C" ibmx_status ibmx_plan_reserve(ibmx_plan p, int32_t pair_cap, int32_t wall_cap,
                                         int32_t cell_cap, int32_t flags)
{
    if (!p || pair_cap < 0 || wall_cap < 0 || cell_cap < 0 ||
        (flags & ~(IBMX_RESERVE_BACKWARD | IBMX_RESERVE_FLUID)) != 0)
        return IBMX_EINVAL;
    if ((flags & IBMX_RESERVE_FLUID) && !ibmx_fluid_grid_ok(p))
        return IBMX_EUNSUPPORTED;
    if (hipStreamSynchronize(p->stream) != hipSuccess)
        return IBMX_EDEVICE;
    // cell list of the pair pass: cell_cap - 1 cells
    const long long cells = cell_cap > 1 ? (long long)cell_cap - 1 : 1;
    if (!p->p_cursor || p->p_cell_cap < cells) {
        if (p->p_cursor)
            (void)hipFree(p->p_cursor);
        p->p_cursor = nullptr;
        p->p_cell_cap = 0;
        if (hipMalloc((void **)&p->p_cursor, sizeof(int) * (size_t)cells) != hipSuccess)
            return IBMX_ENOMEM;
        p->p_cell_cap = (int)cells;
    }
    if (ibmx_plan_scan_reserve(p, cells > p->np ? cells : p->np) != IBMX_OK)
        return IBMX_ENOMEM;
    // contact adjacency and two history sets (the sub-steps alternate them)
    if (ibmx_contact_reserve(p, pair_cap, wall_cap, 2) != IBMX_OK)
        return IBMX_ENOMEM;
    const long long need = ibmx_substep_doubles(p->np);
    if (!p->s_buf || p->s_cap < need) {
        if (p->s_buf)
            (void)hipFree(p->s_buf);
        p->s_buf = nullptr;
        p->s_cap = 0;
        if (hipMalloc((void **)&p->s_buf, sizeof(double) * (size_t)need) != hipSuccess)
            return IBMX_ENOMEM;
        p->s_cap = need;
    }
    if (flags & IBMX_RESERVE_BACKWARD) {
        const size_t nb = ibmx_backward_bytes(p);
        if (!p->bw_u || p->bw_bytes < nb) {
            if (p->bw_u)
                (void)hipFree(p->bw_u);
            p->bw_u = nullptr;
            p->bw_bytes = 0;
            if (hipMalloc(&p->bw_u, nb) != hipSuccess)
                return IBMX_ENOMEM;
            p->bw_bytes = nb;
        }
    }
    if (flags & IBMX_RESERVE_FLUID) {
        const ibmx_status st = ibmx_fluid_reserve(p);
        if (st != IBMX_OK)
            return st;
    }
    return IBMX_OK;
}

ibmx_status ibmx_contact_reserve(ibmx_plan p, int pair_cap, int wall_cap, int hist_sets)
{
    const long long nadj = 2LL * pair_cap + wall_cap;
    if (nadj > p->c_adj_cap || !p->c_adj) {
        if (p->c_adj)
            (void)hipFree(p->c_adj);
        p->c_adj = nullptr;
        p->c_adj_cap = 0;
        if (hipMalloc((void **)&p->c_adj, sizeof(int2) * (size_t)(nadj > 0 ? nadj : 1)) != hipSuccess)
            return IBMX_ENOMEM;
        p->c_adj_cap = nadj;
    }
    const long long nh = (long long)hist_sets * IBMX_HIST * ((long long)pair_cap + wall_cap);
    if (nh > p->c_hist_cap || (nh > 0 && !p->c_hist)) {
        if (p->c_hist)
            (void)hipFree(p->c_hist);
        p->c_hist = nullptr;
        p->c_hist_cap = 0;
        if (hipMalloc((void **)&p->c_hist, sizeof(double) * (size_t)nh) != hipSuccess)
            return IBMX_ENOMEM;
        p->c_hist_cap = nh;
    }
    return IBMX_OK;
}
