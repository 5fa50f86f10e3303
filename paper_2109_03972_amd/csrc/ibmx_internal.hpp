// Internal declarations of the ibmx HIP library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ibmx.h"

#include "ibmx_device.hpp"

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
struct ibmx_plan_s {
    ibmx_grid grid;
    ibmx_params prm;
    GridC g;
    int np;
    int nm;
    int n_iter_cap;
    ibmx_precision prec;
    hipStream_t stream;
    int device;

    // caller-owned marker data
    const double *body;
    const double *dV;

    // plan-owned device workspace
    int *d_moff;          // [np + 1]
    int *d_pid;           // [nm] marker -> particle
    int *d_err;           // [1] first deferred error (0 = none)
    long long *d_count;   // [8][IBMX_RSLOTS] counters (active markers, shell
                          // nodes, halo entries) as partial sums

    // marker records, sorted by spreading tile (T4 = float4 / double4)
    void *rec_tn;         // T4[nm] {t_x, t_y, t_z, packed base node (bits)}
    void *rec_ud;         // T4[nm] {U^d_x, U^d_y, U^d_z, dV}: rigid-body velocity
                          // u_p + omega_p x o at the marker and its volume
    void *rec_Gp;         // T4[n_iter_cap][nm] spreading amplitude G = F dV / h^3
                          // of each pass (the adjoint keeps Ub in its first nm)
    void *rec_G;          // T4[nm] G summed over the passes
    int *rec_src;         // [nm] original marker index
    int *m_key;           // [nm] per-marker tile slot (binning scratch)
    int *m_inv;           // [nm] sorted position of marker l (-1: inactive)

    // tiles
    TileC tc;
    long long tile_cap;   // tiles the tile arrays are sized for
    int *tile_count;      // [ntiles + 1]
    int *tile_start;      // [ntiles + 1]
    int *tile_cursor;     // [ntiles]
    int *halo_count;      // [ntiles + 1]
    int *halo_start;      // [ntiles + 1]
    int *halo_cursor;     // [ntiles]
    int *halo_list;       // [halo_cap]
    double *mean_part;    // [3][ibmx_mean_blocks()] partial sums of ibmx_grid_mean
    int *scan_aux;        // exclusive-scan workspace (ibmx_scan_aux_size ints)
    long long scan_cap;   // elements the workspace serves
    float4 *tile_gmax;    // [2][ntiles] largest |G| of the pass over each tile's
                          // own markers, and its sum over the passes so far
                          // (fixed-point spreading scales)
    double *rpart;        // [n_iter_cap + 1][np] residual partials per particle
    long long halo_cap;
    int block;            // threads per workgroup of the forcing passes
    int persist;          // 1: passes as a persistent grid looping over tiles

    // backward workspace (allocated by the first backward call): replay
    // grid T[3][nodes], per-pass amplitude and Jacobian T4[n_iter][3][nm],
    // per-marker cotangent sums double4[2][nm]
    void *bw_u;
    size_t bw_bytes;

    // captured forcing call (ibmx_forcing_graph)
    hipStream_t cap_stream;
    hipGraphExec_t gexec;
    const void *gkey[10];

    // pair-pass workspace
    int *p_cell_of;       // [np]
    int *p_cursor;        // [max cells]
    int *p_count;         // [np + 1]
    int *p_off;           // [np + 1]
    int p_cell_cap;
    int *p_wcount;        // [np + 1]
    int *p_woff;          // [np + 1]

    // contact workspace (pair pass and particle sub-stepping): per-particle
    // adjacency of the contact lists, history of the previous pair call
    // aligned with the new lists, stage states and forces of the sub-steps
    double actm_K, actm_D;  // ACTM coefficients for prm.e_dry (Hertz law)
    double actm_e;          // e_dry they were solved for (0: none)
    int *c_deg;           // [np + 1]
    int *c_off;           // [np + 1]
    int *c_cur;           // [np]
    int2 *c_adj;          // [c_adj_cap] {code, partner or side}
    long long c_adj_cap;
    double *c_hist;       // [c_hist_cap] history buffers
    long long c_hist_cap;
    double *s_buf;        // [s_cap] sub-step states, stage forces, F_h factors
    long long s_cap;

    // fluid-solve workspace (first ibmx_project / ibmx_fluid_helmholtz call)
    double *fl_r;         // real right-hand side / solution [nodes]
    double2 *fl_z;        // half spectrum [nz][ny][nx/2 + 1]
    double *fl_cp;        // elimination scratch [nz][ny][nx/2 + 1]
    double2 *fl_tw[3];

    // last-call statistics
    ibmx_stats stats;

    // per-kernel timing (ibmx_plan_profile)
    int prof;
    int ev_cap;
    int ev_used;
    hipEvent_t *ev;       // [2 * ev_cap]
    int *ev_kind;         // [ev_cap]
    double acc_ms[8];
    long long acc_n[8];
};

// Brackets the kernel launches of one scope with a pair of HIP events when
// profiling is on.
struct ProfScope {
    ibmx_plan p;
    int idx;
    ProfScope(ibmx_plan p_, int kind) : p(p_), idx(-1)
    {
        if (p->prof && p->ev_used < p->ev_cap) {
            idx = p->ev_used++;
            p->ev_kind[idx] = kind;
            (void)hipEventRecord(p->ev[2 * idx], p->stream);
        }
    }
    ~ProfScope()
    {
        if (idx >= 0)
            (void)hipEventRecord(p->ev[2 * idx + 1], p->stream);
    }
};

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------
#define IBMX_HIP_CHECK(expr)                                  \
    do {                                                      \
        hipError_t _e = (expr);                               \
        if (_e != hipSuccess)                                 \
            return IBMX_EDEVICE;                              \
    } while (0)

ibmx_status ibmx_launch_check();
ibmx_status ibmx_plan_alloc_tiles(ibmx_plan p, int tx, int ty, int tz);
ibmx_status ibmx_spread_allow_lds(ibmx_plan p);
void ibmx_plan_drop_graph(ibmx_plan p);
ibmx_status ibmx_plan_scan_reserve(ibmx_plan p, long long n);
int ibmx_mean_blocks();
// exclusive scan of n ints, out[n] = total; aux holds ibmx_scan_aux_size(n)
// ints of workspace
int ibmx_scan_aux_size(long long n);
// ACTM coefficients (K, D) of the Hertz law for restitution e (Sec. 2.2.7):
// in contact-time units z'' + D z' + K z^(3/2) = 0 closes at t = 1 with
// z'(1) = -e z'(0).  Host computation.
ibmx_status ibmx_actm_coefficients(double e, double *K, double *D);
// Solve the ACTM coefficients for the plan's e_dry when its normal model
// needs them (no-op otherwise or when already solved for that e_dry).
ibmx_status ibmx_plan_actm(ibmx_plan p);
// Grow the contact workspace to list capacities (pair_cap, wall_cap) with
// `hist_sets` history buffers of IBMX_HIST rows each.
ibmx_status ibmx_contact_reserve(ibmx_plan p, int pair_cap, int wall_cap, int hist_sets);
// whether the contact workspace serves these capacities
bool ibmx_contact_ready(ibmx_plan p, int pair_cap, int wall_cap, int hist_sets);
// doubles of sub-stepping state for np particles
long long ibmx_substep_doubles(int np);
// bytes of the adjoint's workspace
size_t ibmx_backward_bytes(ibmx_plan p);
// fluid-solve workspace: grid support, presence, allocation
bool ibmx_fluid_grid_ok(ibmx_plan p);
bool ibmx_fluid_ready(ibmx_plan p);
ibmx_status ibmx_fluid_reserve(ibmx_plan p);
void ibmx_exclusive_scan(const int *in, int *out, int n, int *aux, hipStream_t s);
void ibmx_fill_i32(int *p, int v, long long n, hipStream_t s);
// up to eight int arrays cleared by one launch
struct ZeroList {
    int *p[8];
    long long n[8];
    long long total;
    int k;
    void add(int *q, long long m)
    {
        if (m > 0 && k < 8) {
            p[k] = q;
            n[k] = m;
            total += m;
            ++k;
        }
    }
};
void ibmx_zero_i32_multi(const ZeroList &z, hipStream_t s);
void ibmx_fill_f64(double *p, double v, long long n, hipStream_t s);
void ibmx_fill_u8(uint8_t *p, uint8_t v, long long n, hipStream_t s);
