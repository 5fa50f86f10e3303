/*
 * ibmx.h -- C ABI of the MI355X (gfx950) library for the data-parallel hot
 * path of the collocated-grid direct-forcing immersed boundary method with
 * polydisperse collision models of Yao et al., arXiv 2109.03972:
 *
 *   - the outer forcing loop (Sec. 2.2.2): interpolate the collocated
 *     velocity to every particle's Lagrangian markers through the
 *     regularized delta (Sec. 2.1, eq. 3pt-stencil; Sec. 2.2.3 for the
 *     four-point variant), form the marker force from the rigid-body
 *     velocity u_p + omega_p x (X_l - x_p), spread it back to the grid,
 *     update the velocity, and sum each particle's force and torque
 *     (eq. basic-particle);
 *   - the pair pass (Secs. 2.2.5-2.2.8): cell list, pair and wall lists, the
 *     lubrication / normal / tangential collision forces and torques
 *     (eq. f_int), and the marker-disable mask.
 *
 * Conventions shared by every entry point
 *   * Grid fields are T[3][nz][ny][nx] (x fastest), T = double for
 *     IBMX_F64 and float for IBMX_F32.  Node (i,j,k) sits at
 *     origin + (i + 1/2, j + 1/2, k + 1/2) h (cell centres of the collocated
 *     finite-volume grid).  A non-periodic axis has walls at origin and
 *     origin + n h.
 *   * Particle arrays are double[3][np] (all x, then all y, then all z).
 *   * Markers are stored per particle in CSR order: marker_offset[np + 1]
 *     (host, int32); body offsets o_l = X_l - x_p are double[3][nm].
 *   * Every pointer passed to a compute call is a DEVICE pointer unless
 *     named *_host.  The caller owns every buffer; the library only reads
 *     or writes it inside the call, asynchronously on the plan's stream, so
 *     buffers must stay valid until the stream reaches the call.
 *   * Compute calls never synchronise the stream and never allocate, so
 *     every one of them can be captured into a HIP graph from its first
 *     call (ibmx_forcing_graph does that for ibmx_forcing).  The plan owns
 *     all workspace: the forcing loop's is sized by ibmx_plan_create and
 *     ibmx_plan_set_tiles; the pair pass, the particle sub-stepping, the
 *     adjoint and the fluid solves take theirs from ibmx_plan_reserve and
 *     return ESTATE when it is missing or too small.  Only ibmx_tune
 *     allocates (its scratch copies) and synchronises.  Errors that only the
 *     device can see (a delta support crossing a wall, a list capacity
 *     exceeded) are recorded in the plan and returned by ibmx_plan_status().
 *   * A plan is used by one host thread at a time; calls on one plan are
 *     ordered by its stream.
 *   * No exception, abort or exit crosses this interface.
 */
#ifndef IBMX_H
#define IBMX_H

#include <stdint.h>

#if defined(IBMX_BUILD)
#define IBMX_API __attribute__((visibility("default")))
#else
#define IBMX_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    IBMX_OK = 0,
    IBMX_EINVAL = -1,       /* bad argument, size or CSR                      */
    IBMX_EDOMAIN = -2,      /* an active marker's delta support leaves the
                               grid through a wall (deferred)                 */
    IBMX_ENOMEM = -3,       /* device allocation failed (plan creation only)  */
    IBMX_EDEVICE = -4,      /* a HIP runtime call failed                      */
    IBMX_ESTATE = -5,       /* plan not ready: markers not set, or workspace
                               not reserved for the call (ibmx_plan_reserve) */
    IBMX_ECAPACITY = -6,    /* pair or wall list longer than its capacity
                               (deferred; counts are still written)           */
    IBMX_EUNSUPPORTED = -7  /* option not built (e.g. a delta other than 3/4)  */
} ibmx_status;

typedef enum {
    IBMX_F64 = 0,           /* grid, delta weights and marker forces in FP64  */
    IBMX_F32 = 1            /* grid, delta weights and marker forces in FP32;
                               marker geometry, per-particle force and torque
                               sums, residuals and all pair-pass arithmetic
                               stay FP64                                      */
} ibmx_precision;

/* Uniform collocated grid.  n[a] >= 1, h > 0, n[0]*n[1]*n[2] < 2^31. */
typedef struct {
    int32_t n[3];
    int32_t periodic[3];    /* 1 periodic, 0 walls                            */
    double h;
    double origin[3];
} ibmx_grid;

/* Method parameters (units of the caller; the paper's values in brackets). */
typedef struct {
    int32_t kernel;          /* 3: three-point delta (Sec. 2.1), 4: four-point
                                (Sec. 2.2.3)                                   */
    int32_t n_iter;          /* interpolate-force-spread-update passes per
                                call (n_f + 1 in the paper's count), 1..64   */
    double two_alpha_dt;     /* c = 2 alpha_k dt of the current RK sub-step    */
    double rho_f;            /* fluid density                                  */
    double nu_f;             /* kinematic viscosity                            */
    double eps_sep;          /* lubrication / disable threshold [1.5h, 2h]     */
    double lub_C;            /* psi blending constant [5.5 three-point, 4]    */
    double zeta_min_factor;  /* zeta_min = factor * min(R_p, R_q) [3e-3]       */
    double e_dry;            /* dry restitution coefficient [0.97]            */
    double T_c;              /* contact duration [10 dt]                       */
    double mu_s;             /* static friction [0.11]                         */
    double mu_k;             /* kinetic friction [0.8]                         */
    double nu_poi;           /* Poisson ratio of the particles                 */
    double dt;               /* time step for the tangential spring            */
    double gap_cut;          /* pair/wall list cut-off on the surface gap; at
                                least 2 eps_sep when disable_mode != 0 (the
                                disable rule acts on gaps below 2 eps_sep),
                                else EINVAL                                    */
    int32_t disable_mode;    /* 0 none, 1 local markers, 2 whole particle      */
    int32_t normal_model;    /* 0 linear spring-dashpot, 1 Hertz law with ACTM
                                coefficients (Sec. 2.2.7)                      */
    uint64_t disable_seed;   /* seed of the per-pair random choice             */
    double St_crit;          /* critical Stokes number of a contact [5]        */
    double gravity[3];       /* gravitational acceleration g                   */
    double kn_grav_eps;      /* eps of the gravity stiffness k_n,grav [1e-3]   */
    int32_t st_switch;       /* 1: particle sub-stepping drops F_h, T_h of a
                                particle whose contacts all have St <= St_crit */
    int32_t reserved;        /* 0                                              */
} ibmx_params;

/* Rows of the per-contact history arrays: the tangential spring
 * displacement zeta_t (3 rows) and the impact speed u_in of the contact
 * (the approach speed g_cp . n at its first evaluation, clamped at zero;
 * zero for a contact that has not begun).  A history array for n contacts
 * is double[IBMX_HIST][n]. */
#define IBMX_HIST 4

typedef struct ibmx_plan_s *ibmx_plan;

/* Counters of the last forcing call (read by ibmx_plan_stats, which
 * synchronises the plan's stream). */
typedef struct {
    int64_t n_markers;        /* markers in the plan                           */
    int64_t n_active;         /* markers taking part in the last call          */
    int64_t shell_nodes;      /* distinct grid nodes with nonzero delta weight
                                 from some active marker (last call)           */
    int64_t tiles;            /* spatial tiles of the spreading pass          */
    int64_t halo_entries;     /* (marker, neighbour tile) spreading entries    */
    int32_t tile[3];          /* tile edge in nodes                            */
    int32_t block;            /* threads per workgroup of the forcing passes  */
    int32_t persistent;       /* 1: the passes run as a persistent grid        */
    int32_t reserved;
    /* Kernel timings accumulated while profiling is on (ibmx_plan_profile):
     * total milliseconds and launch counts per kernel class
     * IBMX_K_GEOMETRY .. IBMX_K_FTOT. */
    double kernel_ms[8];
    int64_t kernel_launches[8];
} ibmx_stats;

/* Kernel classes of ibmx_stats.kernel_ms. */
enum {
    IBMX_K_GEOMETRY = 0,      /* marker geometry, binning and sorting          */
    IBMX_K_INTERP = 1,        /* interpolation + marker force + particle sums  */
    IBMX_K_SPREAD = 2,        /* spreading + velocity update of one pass       */
    IBMX_K_BACKWARD = 3,      /* adjoint passes                                */
    IBMX_K_PAIRS = 4,         /* pair pass (lists, forces, mask)               */
    IBMX_K_OTHER = 5,         /* fills, residual finish                        */
    IBMX_K_FTOT = 6,          /* spreading of the pass-summed amplitudes into
                                 f_tot (calls with two or more passes)         */
    IBMX_K_GRAPH = 7          /* whole forcing call replayed as a HIP graph
                                 (ibmx_forcing_graph)                          */
};

/*
 * Create a plan for a grid, a parameter set and a fixed marker layout.
 *   out                 receives the handle.
 *   grid, params        copied.
 *   np                  number of particles (>= 0).
 *   marker_offset_host  host int32[np + 1], nondecreasing, [0] = 0.
 *   precision           IBMX_F64 or IBMX_F32.
 *   hip_stream          hipStream_t (NULL = default stream) used by every
 *                       call on this plan.
 * Allocates all device workspace.  Returns EINVAL (among others for a
 * periodic axis of fewer than 2 * kernel nodes, where a support would meet
 * itself across the seam), ENOMEM, EDEVICE or EUNSUPPORTED (kernel other
 * than 3/4, normal_model other than 0/1).
 * With normal_model 1 the plan solves the ACTM equation for e_dry on the
 * host (a few milliseconds), here and in ibmx_plan_set_params.
 */
IBMX_API ibmx_status ibmx_plan_create(ibmx_plan *out, const ibmx_grid *grid, const ibmx_params *params,
                             int32_t np, const int32_t *marker_offset_host,
                             ibmx_precision precision, void *hip_stream);

/* Release the plan and its workspace (synchronises its stream). */
IBMX_API ibmx_status ibmx_plan_destroy(ibmx_plan plan);

/* Attach the marker set: body offsets double[3][nm] and the marker volume
 * dV_l of each particle double[np] (Sec. 2.1: N_l dV_l is the shell volume).
 * Pointers are kept, not copied: they must stay valid while the plan is
 * used. */
IBMX_API ibmx_status ibmx_plan_set_markers(ibmx_plan plan, const double *body_offset, const double *dV);

/* Flags of ibmx_plan_reserve. */
#define IBMX_RESERVE_BACKWARD 1   /* replay workspace of ibmx_forcing_backward  */
#define IBMX_RESERVE_FLUID 2      /* FFT / elimination workspace of ibmx_project
                                     and ibmx_fluid_helmholtz                   */

/*
 * Size the workspace of the calls that need more than the forcing loop, so
 * that they allocate nothing:
 *   ibmx_pairs               a cell list of up to cell_cap - 1 cells and lists
 *                            of up to pair_cap pairs and wall_cap wall entries
 *                            (the capacities the call is given);
 *   ibmx_particle_substeps   lists of up to pair_cap / wall_cap entries, the
 *                            stage states of the plan's particles;
 *   IBMX_RESERVE_BACKWARD    ibmx_forcing_backward (the replay grid T[3][nodes]
 *                            and T4[n_iter][3][nm] of per-pass data);
 *   IBMX_RESERVE_FLUID       ibmx_project and ibmx_fluid_helmholtz (an FP64
 *                            real grid, the FP64 half spectrum, with walls in z
 *                            an FP64 elimination grid, twiddle tables);
 *                            EUNSUPPORTED on grids the solves do not take.
 * Workspace only grows; a call whose needs exceed the reservation returns
 * ESTATE.  Synchronises the plan's stream.  Growing it moves the workspace,
 * so graphs captured before must be captured again.  EINVAL for negative
 * sizes or unknown flags, ENOMEM.
 */
IBMX_API ibmx_status ibmx_plan_reserve(ibmx_plan plan, int32_t pair_cap, int32_t wall_cap,
                                       int32_t cell_cap, int32_t flags);

/* Change the parameters (n_iter may not exceed the value the plan was
 * created with). */
IBMX_API ibmx_status ibmx_plan_set_params(ibmx_plan plan, const ibmx_params *params);

/* Change the stream used by later calls. */
IBMX_API ibmx_status ibmx_plan_set_stream(ibmx_plan plan, void *hip_stream);

/* Set the tile shape (nodes per tile along x, y, z) of the forcing passes,
 * as ibmx_tune does for its choice.  Edges are 4..64 with x <= 60 (EINVAL
 * otherwise).  An edge whose last tile would be shorter than 4 nodes is
 * replaced by the nearest edge (smaller first) that divides the axis or
 * leaves at least 4; an edge of at least the axis length becomes the axis
 * length.  EUNSUPPORTED if the tile's LDS footprint is too large for the
 * precision.  Synchronises the stream; reallocates tile workspace. */
IBMX_API ibmx_status ibmx_plan_set_tiles(ibmx_plan plan, int32_t tx, int32_t ty, int32_t tz);

/* Set the launch form of the forcing passes, as ibmx_tune does for its
 * choice: block = threads per workgroup (64, 128 or 256; a thread takes one
 * marker at a time, so this is the number of markers a tile's workgroup
 * works on at once), persistent = 0 for one workgroup per tile, 1 for a
 * fixed grid (as many workgroups as the CUs hold at once) whose workgroups
 * loop over the tiles.  Results do not depend on either choice.  EINVAL for
 * other values. */
IBMX_API ibmx_status ibmx_plan_set_launch(ibmx_plan plan, int32_t block, int32_t persistent);

/* Synchronise the plan's stream and return (and clear) the first deferred
 * device error of the calls since the last ibmx_plan_status: EDOMAIN,
 * ECAPACITY, or EDEVICE. */
IBMX_API ibmx_status ibmx_plan_status(ibmx_plan plan);

/* Synchronise and report the counters of the last forcing call. */
IBMX_API ibmx_status ibmx_plan_stats(ibmx_plan plan, ibmx_stats *out);

/* Turn per-kernel timing on (enable = 1) or off (0).  While on, every kernel
 * launch of this plan is bracketed by a pair of HIP events recorded on the
 * plan's stream; ibmx_plan_stats sums their elapsed times per kernel class.
 * Turning it on clears the accumulated timings.  Do not capture a plan with
 * profiling on into a HIP graph. */
IBMX_API ibmx_status ibmx_plan_profile(ibmx_plan plan, int32_t enable);

/*
 * Outer forcing loop (Sec. 2.2.2), params.n_iter passes:
 *   U_l   = sum_x u(x) delta_h(x - X_l) h^3            X_l = x_p + o_l
 *   F_l   = (u_p + omega_p x o_l - U_l) / c
 *   f(x)  = sum_l F_l delta_h(x - X_l) dV_l
 *   u    <- u + c f
 * u            T[3][nz][ny][nx], in/out: u^0 in, u^{n_iter} out.
 * f_tot        T[3][nz][ny][nx], accumulate-into: f_tot += sum of the
 *              passes' f.  Only nodes in the delta support of active markers
 *              are read or written.
 * xp, up, wp   double[3][np]: centres, velocities, angular velocities.
 * marker_active uint8[nm] or NULL (all active): 0 drops marker l from every
 *              pass (the disable rule of Sec. 2.2.5, see ibmx_pairs).
 * S_out, T_out double[3][np], overwritten: sum over passes and active
 *              markers of F_l dV_l and of o_l x F_l dV_l.  The hydrodynamic
 *              force and torque of eq. basic-particle are -rho_f times these.
 * resid_out    double[n_iter + 1] or NULL: resid[m] = sqrt(sum_l dV_l
 *              |u_p + omega_p x o_l - U_l^m|^2) before pass m + 1; the last
 *              entry is measured on the final velocity.
 * U_debug      T[n_iter][3][nm] or NULL: the interpolated U_l of each pass
 *              (entries of inactive markers are not written).
 * Deferred error: EDOMAIN if an active marker's support crosses a wall (the
 * marker is then skipped).
 * The spreading accumulates in integer fixed point (per-tile power-of-two
 * scales), so the results do not depend on the order of the additions: a
 * call repeated on the same inputs gives the same bits.
 */
IBMX_API ibmx_status ibmx_forcing(ibmx_plan plan, void *u, void *f_tot,
                         const double *xp, const double *up, const double *wp,
                         const uint8_t *marker_active,
                         double *S_out, double *T_out, double *resid_out, void *U_debug);

/*
 * Reverse-mode derivative of ibmx_forcing with respect to u^0, x_p, u_p and
 * omega_p, holding the mask, body offsets, dV and c fixed (the adjoint of
 * each pass swaps interpolation and spreading; the delta gradient gives the
 * position terms).  Inputs are the forward inputs (u0 = the velocity BEFORE
 * the forward call) and the cotangents g_f = dL/df_tot (T grid or NULL),
 * g_u = dL/du^{n_iter} (T grid or NULL), g_S = dL/dS_out and g_T = dL/dT_out
 * (double[3][np] or NULL).  Outputs (overwritten): gu0 (T grid), gxp, gup,
 * gwp (double[3][np]).  The forward passes are recomputed, not stored by the
 * forward call; plan workspace holds the per-marker pass data
 * (ibmx_plan_reserve with IBMX_RESERVE_BACKWARD, else ESTATE).
 */
IBMX_API ibmx_status ibmx_forcing_backward(ibmx_plan plan, const void *u0,
                                  const double *xp, const double *up, const double *wp,
                                  const uint8_t *marker_active,
                                  const void *g_f, const void *g_u,
                                  const double *g_S, const double *g_T,
                                  void *gu0, double *gxp, double *gup, double *gwp);

/*
 * Pair pass (Secs. 2.2.5-2.2.8), all FP64:
 *  - cell list: nc[a] = max(1, floor(L_a / (2 R_max + gap_cut))) cells per
 *    axis; cell of p = floor((x_p - origin)/edge) of the periodically wrapped
 *    centre, clamped; cell_start int32[ncell + 1], cell_particles int32[np]
 *    listed by (cell, id);
 *  - pair list: every i < j with minimum-image centre distance below
 *    R_i + R_j + gap_cut, int32[2][pair_cap] in (i, j) order; pair_gap
 *    double[pair_cap] = d - R_i - R_j;
 *  - wall list: (p, side) with side = 2 axis + (0 lower, 1 upper) for walls
 *    closer than gap_cut, int32[2][wall_cap] in (p, side) order, wall_gap;
 *  - collision force and torque (eq. f_int): Fc, Tc double[3][np]
 *    (overwritten): lubrication for 0 <= gap < eps_sep, normal contact
 *    (params.normal_model) and capped tangential spring-dashpot for gap < 0;
 *    each particle's contacts are summed in increasing partner id, then its
 *    walls by side, so the sums do not depend on scheduling;
 *      linear: F_n = -k_n |gap| n - d_n g_n, k_n = m_eff (pi^2 + ln^2 e_dry)
 *        / T_c^2, d_n = -2 m_eff ln e_dry / T_c;
 *      Hertz (eq. hertz-contact): F_n = -k_n |gap|^(3/2) n - d_n g_n with the
 *        ACTM coefficients k_n = K m_eff / (sqrt(u_in) T_c^(5/2)), d_n =
 *        D m_eff / T_c (eq. ode: K, D make a contact last T_c and rebound
 *        with e_dry, solved once per e_dry by the plan) while u_in exceeds
 *        u_crit = 9 St_crit rho_f nu_f / (rho d); otherwise k_n =
 *        max(k_n,crit, k_n,grav), k_n,crit the ACTM value at u_crit,
 *        k_n,grav = max over the two particles of m |g| (kn_grav_eps R)^(-3/2);
 *        rho d = mean over the two particles of 3 m / (2 pi R^2);
 *      tangential stiffness 2 (1 - nu)/(2 - nu) times the normal spring's
 *        (k_n, for the Hertz law its secant k_n |gap|^(1/2));
 *  - contact history (IBMX_HIST rows): hist_in double[IBMX_HIST][npairs_in]
 *    keyed by pairs_in (the previous call's pair list in its (i, j) order,
 *    may be empty), whist_in likewise for walls (keyed by (p, side) in that
 *    order); hist_out double[IBMX_HIST][pair_cap], whist_out
 *    double[IBMX_HIST][wall_cap]; the spring advances by params.dt;
 *  - marker_active uint8[nm] (overwritten): the disable rule of
 *    params.disable_mode (1: the randomly chosen particle of each pair closer
 *    than 2 eps_sep loses the markers within 2 eps_sep of its partner's
 *    surface; markers closer than eps_sep to a wall are off; 2: whole
 *    particles).  The random choice for (p, q), p < q, is the low bit of
 *    SplitMix64(seed ^ (p << 32 | q)): 0 picks p.
 * radius_max (host) bounds every radius; it sizes the cell grid.  A radius
 * above it is reported as a deferred EINVAL.
 * counts_out int32[2] (device): number of pairs and of wall entries found.
 * cell_cap is the capacity of cell_start (ncell + 1 entries).
 * Deferred error: ECAPACITY if a list exceeds its capacity (entries beyond
 * it are dropped, forces of dropped entries are not applied).
 * The body offsets set with ibmx_plan_set_markers are needed for the mask.
 * ESTATE if ibmx_plan_reserve has not reserved the cell count (ncell above
 * its cell_cap - 1) or these list capacities.
 */
IBMX_API ibmx_status ibmx_pairs(ibmx_plan plan, const double *xp, const double *radius,
                       double radius_max, const double *mass, const double *up, const double *wp,
                       int32_t npairs_in, const int32_t *pairs_in, const double *hist_in,
                       int32_t nwall_in, const int32_t *walls_in, const double *whist_in,
                       int32_t *cell_start, int32_t cell_cap, int32_t *cell_particles,
                       int32_t *pairs_out, double *pair_gap, double *hist_out, int32_t pair_cap,
                       int32_t *walls_out, double *wall_gap, double *whist_out, int32_t wall_cap,
                       int32_t *counts_out, double *Fc, double *Tc, uint8_t *marker_active);

/*
 * ibmx_forcing through a HIP graph (the batching form of the loop: one graph
 * launch per call).  The first call, and any call whose pointer arguments
 * differ from the captured ones or that follows a change of the plan's
 * parameters, tiles or markers, captures ibmx_forcing's launches
 * into a graph kept by the plan (on a private capture stream, so the plan's
 * stream may be the default stream); every call then launches that graph on
 * the plan's stream.  Same arguments, results and deferred errors as
 * ibmx_forcing.  With profiling on, the whole call is timed as IBMX_K_GRAPH.
 */
IBMX_API ibmx_status ibmx_forcing_graph(ibmx_plan plan, void *u, void *f_tot,
                               const double *xp, const double *up, const double *wp,
                               const uint8_t *marker_active,
                               double *S_out, double *T_out, double *resid_out, void *U_debug);

/*
 * Autotune the launch of the forcing passes on the given inputs: runs
 * ibmx_forcing with each candidate tile shape that fits the LDS (edges
 * 4..32, x-edge <= 32) at 256 threads per workgroup, then, for the fastest
 * shape, with 128 and 64 threads and as a persistent grid (ibmx_plan_set_launch);
 * times each with HIP events on the plan's stream and keeps the fastest in
 * the plan (a candidate must beat the earlier ones by 2%).  Candidates that
 * raise a deferred error are skipped.
 * u and f_tot are restored after every trial, so the call leaves them
 * unchanged.  Allocates and frees its own scratch (copies of u and f_tot)
 * and synchronises the stream; not capturable.  The choice is reported by
 * ibmx_plan_stats (tile, block, persistent).
 */
IBMX_API ibmx_status ibmx_tune(ibmx_plan plan, void *u, void *f_tot,
                      const double *xp, const double *up, const double *wp,
                      const uint8_t *marker_active);

/*
 * Fluid integrals over every particle for the rate-of-change term of the
 * particle equations (Sec. 2.2.9), with the level-set volume fraction of
 * each cell: from the signed distances phi_m = |x_m - x_p| - R_p of the
 * cell's eight corners x_m (negative inside),
 *   alpha = sum_m -phi_m H(-phi_m) / sum_m |phi_m|   (0 if all phi_m = 0),
 *   Iu[a][p] = sum_cells alpha h^3 u_a(cell),
 *   Ir[a][p] = sum_cells alpha h^3 (r x u)_a(cell),  r = cell centre - x_p,
 * over the cells whose box meets [x_p - R_p, x_p + R_p] per axis (x_p
 * wrapped into the domain on periodic axes; cells beyond a wall are
 * skipped; r is the displacement to the image of the cell next to the
 * particle).  Cell (i, j, k) is the box [origin + (i, j, k) h,
 * origin + (i + 1, j + 1, k + 1) h] around node (i, j, k).
 * u            T[3][nz][ny][nx] (the plan's precision); geometry and sums
 *              are FP64, summed in a fixed order.
 * xp, radius   double[3][np], double[np].
 * Iu, Ir       double[3][np], overwritten.
 * alpha_out    T[nz][ny][nx] or NULL: sum over particles of alpha per cell,
 *              overwritten (added with atomics where particles overlap).
 * Particles must be smaller than half a periodic axis.
 */
IBMX_API ibmx_status ibmx_particle_integrals(ibmx_plan plan, const void *u, const double *xp,
                                    const double *radius, double *Iu, double *Ir,
                                    void *alpha_out);

/*
 * Volume average per component of a T[3][nz][ny][nx] grid field, in FP64:
 * mean[a] = sum_x f_a(x) / (nx ny nz), double[3] on the device.  For the
 * IBM force of a triply periodic domain, minus this average is the mean
 * forcing removed from the momentum equation (Sec. 2.2.4, eq. fe_IBM).
 * Partial sums over fixed chunks, added in a fixed order.
 */
IBMX_API ibmx_status ibmx_grid_mean(ibmx_plan plan, const void *f, double *mean);

/*
 * ibmx_grid_mean for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * It needs no plan and allocates nothing: its partial sums live in a static
 * device array of the library, [3][4096] doubles (96 KB on every device the
 * library runs on, held until the process ends).  Same kernels, result and
 * summation order as ibmx_grid_mean.
 *   f          device T[3][n_nodes] (T = double for IBMX_F64, float for
 *              IBMX_F32), the three components one after the other.
 *   n_nodes    nodes per component, 1 <= n_nodes < 2^31 (the library's grid
 *              limit), else EINVAL.
 *   mean       device double[3], overwritten: sum_x f_a(x) / n_nodes.
 *   hip_stream stream of the current device (NULL = default stream); the
 *              call is asynchronous on it.
 * Every call on one device shares that device's array: calls that overlap
 * on one device (different streams, or host threads) race and must be
 * ordered by the caller.  Returns EINVAL, EDEVICE (the array's address could
 * not be found) or EUNSUPPORTED (device index above 63).
 */
IBMX_API ibmx_status ibmx_grid_mean_noalloc(const void *f, int64_t n_nodes,
                                            ibmx_precision precision, double *mean,
                                            void *hip_stream);

/*
 * Particle sub-stepping (Sec. 2.2.10): advance every particle's centre,
 * velocity and angular velocity by dt_total in n_sub sub-steps of dts =
 * dt_total / n_sub, each the three-stage Runge-Kutta predictor-corrector of
 * the particle update with the low-storage coefficients of Rai and Moin,
 * alpha = (4/15, 1/15, 1/6), gamma = (8/15, 5/12, 3/4), zeta = (0, -17/60,
 * -5/12).  Stage k, with F_c(s) the collision force of the pair pass at
 * particle state s (and T_c its torque):
 *   u~ = u^{k-1} + dts/m (2 alpha_k F_h + gamma_k F_c(s^{k-1}) + zeta_k F_c(s^{k-2}))
 *        + 2 alpha_k dts g',
 *   w~ = w^{k-1} + dts/I (2 alpha_k T_h + gamma_k T_c(s^{k-1}) + zeta_k T_c(s^{k-2})),
 *   x~ = x^{k-1} + alpha_k dts (u~ + u^{k-1}),
 * then u^k, w^k, x^k the same with F_c(s~) for F_c(s^{k-1}) and F_c(s^{k-1})
 * for F_c(s^{k-2}).  g' = (1 - rho_f/rho_p) g, rho_p = m / (4/3 pi R^3),
 * I = 2/5 m R^2.  15 sub-steps of dt/15 are the paper's setting (45 stages).
 * The collision law is ibmx_pairs's (params.normal_model), evaluated on the
 * given lists (pair and wall lists of an ibmx_pairs call, with gap_cut
 * covering the motion of this call); contacts beyond the lists are not seen.
 * History: hist / whist double[IBMX_HIST][pair_cap / wall_cap], aligned
 * with the lists, in: the history of the input state; out: the history of
 * the final state.  It is committed at each accepted stage state (the
 * spring advancing by the time since the previous one); predicted states
 * use the committed history and the stage's time 2 alpha_k dts.
 *   xp, up, wp  double[3][np], in/out (centres are not wrapped).
 *   radius, mass double[np].
 *   Fh, Th      double[3][np] hydrodynamic force and torque held over the
 *               call (e.g. -rho_f S_p plus the rate of change of the fluid
 *               integrals), or NULL for zero.  With params.st_switch, a
 *               particle whose input history holds at least one contact and
 *               only contacts with St = u_in rho d / (9 rho_f nu_f) <=
 *               St_crit gets F_h = T_h = 0.
 *   counts      device int32[2]: listed pairs, walls (an ibmx_pairs
 *               counts_out; clamped to the capacities).  List entries that
 *               are not pairs i < j of particles 0 .. np-1, or wall entries
 *               of such a particle on a wall axis, are skipped and reported
 *               as a deferred EINVAL.
 *   Fc, Tc      double[3][np] or NULL: collision force and torque at the
 *               final state, overwritten.
 * Each particle's contacts are summed in increasing partner id, then its
 * walls by side: the results do not depend on scheduling.  ESTATE if
 * ibmx_plan_reserve has not reserved these list capacities.
 */
IBMX_API ibmx_status ibmx_particle_substeps(ibmx_plan plan, double dt_total, int32_t n_sub,
                                   double *xp, double *up, double *wp, const double *radius,
                                   const double *mass, const double *Fh, const double *Th,
                                   const int32_t *counts, int32_t pair_cap, const int32_t *pairs,
                                   int32_t wall_cap, const int32_t *walls, double *hist,
                                   double *whist, double *Fc, double *Tc);

/*
 * Pressure projection of one Runge-Kutta stage of the collocated fluid
 * solver (Sec. 2.2.1 and eq. fluid-solver, steps f-i), with c =
 * params.two_alpha_dt and nu = params.nu_f:
 *   u_f* = the mean of the two cells next to each face (walls: 0);
 *   L phi = div(u_f*) / c, L the compact Laplacian (phi_+ - 2 phi + phi_-)/h^2
 *     per axis with zero normal gradient at walls, phi of zero mean;
 *   u   = u* - c grad(phi), grad the mean of the cell's two face gradients;
 *   u_f = u_f* - c (phi_+ - phi)/h on every interior face;
 *   P   = (1 - theta) P_prev + phi - (c/2) nu L phi (theta 0: pressure
 *     projection, incremental; theta 1: pressure correction).
 * u      T[3][nz][ny][nx] (the plan's precision), in: u*, out: u at the end of
 *        the stage.
 * uf     T[3][nz][ny][nx], out: normal velocity on the +x, +y, +z face of
 *        each cell (0 on a wall face).
 * P      T[nz][ny][nx], in/out.  phi: T[nz][ny][nx] or NULL, out.
 * The solve is direct and FP64: FFTs along x and y (and z when periodic),
 * across walls in z a tridiagonal elimination per Fourier mode.  Needs
 * periodic x and y with power-of-two sizes up to 1024 (and the same for z
 * when periodic), else EUNSUPPORTED.  The solver workspace (an FP64 real
 * grid, the FP64 complex half spectrum of nx/2 + 1 modes per row, with walls
 * in z an FP64 grid of elimination coefficients of the same shape, and one
 * twiddle table per axis) comes from ibmx_plan_reserve with
 * IBMX_RESERVE_FLUID, else ESTATE.
 */
IBMX_API ibmx_status ibmx_project(ibmx_plan plan, void *u, void *uf, void *P, void *phi,
                                  double theta);

/*
 * Predictor of one Runge-Kutta stage of the collocated fluid solver (eq.
 * fluid-solver, step a), with alpha_k = params.two_alpha_dt / (2 dt):
 *   u~ = u + dt (2 alpha_k nu L u - 2 alpha_k grad P - gamma_k N - zeta_k N_prev),
 *   N  = (u . grad) u,
 * L the 7-point Laplacian, N by central differences, grad P the mean of the
 * cell's two face gradients; velocity vanishes on wall faces (ghost -u),
 * pressure has zero normal gradient there.
 * u       T[3][nz][ny][nx], the stage's input velocity (not modified).
 * u_out   T[3][nz][ny][nx], out: u~ (must not alias u).
 * N       T[3][nz][ny][nx], in: N of the previous stage (any finite values
 *         when zeta_k = 0), out: N of u.
 * lapnu   T[3][nz][ny][nx], out: nu L u (input of ibmx_fluid_helmholtz).
 * P       T[nz][ny][nx], the pressure of the previous stage.
 * Any grid.  Allocates nothing.
 */
IBMX_API ibmx_status ibmx_fluid_predictor(ibmx_plan plan, const void *u, void *u_out, void *N,
                                          void *lapnu, const void *P, double dt, double gamma,
                                          double zeta);

/*
 * Implicit viscous step of one stage (eq. fluid-solver, step e, Crank-
 * Nicolson): with c = params.two_alpha_dt and alpha_k = c / (2 dt), solves
 *   (I - alpha_k dt nu L) u* = u - c fbar + dt (-alpha_k lapnu + 2 alpha_k theta grad P)
 * per component, where u is the velocity after the forcing loop (u~ + c
 * f_IBM, as ibmx_forcing leaves it), lapnu = nu L of the stage's input
 * velocity (from ibmx_fluid_predictor), fbar the mean IBM force (device
 * double[3], e.g. from ibmx_grid_mean of f_tot, for triply periodic cases;
 * NULL for 0) and theta 0 (pressure projection) or 1 (pressure correction).
 * u is overwritten by u*.  The solve is FP64: FFTs along x and y (and z when
 * periodic), across walls in z a tridiagonal elimination per Fourier mode
 * with velocity 0 on the wall faces.  Same grid conditions and workspace as
 * ibmx_project (ESTATE without it).
 */
IBMX_API ibmx_status ibmx_fluid_helmholtz(ibmx_plan plan, void *u, const void *lapnu, const void *P,
                                          const double *fbar, double dt, double theta);

/* Static description of a status code. */
IBMX_API const char *ibmx_status_string(ibmx_status status);

/* Library version string. */
IBMX_API const char *ibmx_version(void);

#ifdef __cplusplus
}
#endif

#endif /* IBMX_H */
