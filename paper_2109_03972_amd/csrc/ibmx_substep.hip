// Particle sub-stepping (Sec. 2.2.10) and the ACTM coefficients of the
// Hertz normal contact (Sec. 2.2.7).
//
// One call advances the particles by n_sub sub-steps of three Runge-Kutta
// stages; each stage is two launches of a lane group per particle:
//   predictor  contacts at the accepted state s^{k-1} (committing the
//              contact history of that state), then s~ into a separate
//              state buffer;
//   corrector  contacts at s~ (history not committed), then s^k over the
//              particle's own s^{k-1}.
// Contacts read the partners' state from a buffer no launch in flight
// writes; the stage forces of s^{k-1} and s^{k-2} are kept per particle in
// two alternating buffers.

#include "ibmx_contact.hpp"

namespace {

// ---------------------------------------------------------------------------
// ACTM coefficients, host.  In contact-time units the overlap obeys
// z'' + D z' + K z^(3/2) = 0 from z = 0, z' = 1, and the contact must close
// at t = 1 with z' = -e.  The time change t -> t / b maps (K, D) to
// (K b^(5/2), D b), so it suffices to find the damping D1 of the K = 1
// problem whose rebound is e (the rebound falls with D1), read its
// duration T1, and scale: K = T1^(5/2), D = D1 T1.
// ---------------------------------------------------------------------------
struct UnitRun {
    bool closed;
    double T;       // contact duration
    double v_end;   // z' when the overlap closes
};

inline double hertz_force(double z) { return z > 0.0 ? z * sqrt(z) : 0.0; }

inline void unit_rk4(double D1, double h, double &z, double &v)
{
    const double a1 = v, b1 = -D1 * v - hertz_force(z);
    const double a2 = v + 0.5 * h * b1, b2 = -D1 * a2 - hertz_force(z + 0.5 * h * a1);
    const double a3 = v + 0.5 * h * b2, b3 = -D1 * a3 - hertz_force(z + 0.5 * h * a2);
    const double a4 = v + h * b3, b4 = -D1 * a4 - hertz_force(z + h * a3);
    z += h / 6.0 * (a1 + 2.0 * a2 + 2.0 * a3 + a4);
    v += h / 6.0 * (b1 + 2.0 * b2 + 2.0 * b3 + b4);
}

UnitRun unit_run(double D1)
{
    const double h = 5.0e-5;       // the undamped K = 1 contact lasts about 3.2
    const long steps = 800000;
    double z = 0.0, v = 1.0, t = 0.0;
    for (long s = 0; s < steps; ++s) {
        double zn = z, vn = v;
        unit_rk4(D1, h, zn, vn);
        if (s > 0 && zn <= 0.0) {
            // closing inside this step: bisect the length of a partial step
            double lo = 0.0, hi = h;
            for (int it = 0; it < 80; ++it) {
                const double mid = 0.5 * (lo + hi);
                double zm = z, vm = v;
                unit_rk4(D1, mid, zm, vm);
                (zm > 0.0 ? lo : hi) = mid;
            }
            double ze = z, ve = v;
            unit_rk4(D1, hi, ze, ve);
            return UnitRun{true, t + hi, ve};
        }
        z = zn;
        v = vn;
        t = (double)(s + 1) * h;   // not a running sum: no accumulated rounding
    }
    return UnitRun{false, t, v};
}

}  // namespace

ibmx_status ibmx_actm_coefficients(double e, double *K, double *D)
{
    if (!(e > 0.0 && e <= 1.0) || !K || !D)
        return IBMX_EINVAL;
    double D1 = 0.0;
    if (e < 1.0) {
        double lo = 0.0, hi = 0.25;
        for (int it = 0; it < 60; ++it) {
            const UnitRun r = unit_run(hi);
            if (r.closed && -r.v_end < e)
                break;
            lo = hi;
            hi *= 2.0;
        }
        for (int it = 0; it < 64; ++it) {
            const double mid = 0.5 * (lo + hi);
            const UnitRun r = unit_run(mid);
            if (r.closed && -r.v_end < e)
                hi = mid;
            else
                lo = mid;
        }
        D1 = 0.5 * (lo + hi);
    }
    const UnitRun r = unit_run(D1);
    if (!r.closed)
        return IBMX_EINVAL;
    *K = r.T * r.T * sqrt(r.T);
    *D = D1 * r.T;
    return IBMX_OK;
}

namespace {

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
// F_h, T_h factor of each particle: 0 when the switch is on and the input
// history holds at least one contact of the particle, all with St <= St_crit
__global__ __launch_bounds__(64) void k_st_factor(PairC P, int np, ContactLists C, const int *off,
                                                  const int2 *adj, const double *radius,
                                                  const double *mass, HistC h0, int on,
                                                  double *sF)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np)
        return;
    int contacts = 0, fast = 0;
    for (int r = off[p]; r < off[p + 1]; ++r) {
        const int e = adj[r].x;
        double u_in, rhod;
        if (e >= 0) {
            const int k = e >> 1;
            const int i = (e & 1) ? adj[r].y : p, j = (e & 1) ? p : adj[r].y;
            u_in = h0.pair[(size_t)3 * C.pair_cap + k];
            rhod = 0.5 * (rho_d(mass[i], radius[i]) + rho_d(mass[j], radius[j]));
        } else {
            const int k = -e - 1;
            u_in = h0.wall[(size_t)3 * C.wall_cap + k];
            rhod = rho_d(mass[p], radius[p]);
        }
        if (!(u_in > 0.0))
            continue;
        ++contacts;
        const double St = u_in * rhod / (9.0 * P.rho_f * P.nu_f);
        fast += St > P.St_crit;
    }
    sF[p] = (on && contacts > 0 && fast == 0) ? 0.0 : 1.0;
}

}  // namespace

extern "C" ibmx_status ibmx_particle_substeps(ibmx_plan p, double dt_total, int32_t n_sub,
                                              double *xp, double *up, double *wp,
                                              const double *radius, const double *mass,
                                              const double *Fh, const double *Th,
                                              const int32_t *counts, int32_t pair_cap,
                                              const int32_t *pairs, int32_t wall_cap,
                                              const int32_t *walls, double *hist, double *whist,
                                              double *Fc, double *Tc)
{
    if (!p || n_sub < 1 || !isfinite(dt_total) || pair_cap < 0 || wall_cap < 0)
        return IBMX_EINVAL;
    const int np = p->np;
    if (np > 0 && (!xp || !up || !wp || !radius || !mass))
        return IBMX_EINVAL;
    if ((pair_cap > 0 || wall_cap > 0) && !counts)
        return IBMX_EINVAL;
    if ((pair_cap > 0 && (!pairs || !hist)) || (wall_cap > 0 && (!walls || !whist)) ||
        (!Fc) != (!Tc))
        return IBMX_EINVAL;
    if (np == 0)
        return IBMX_OK;
    // the workspace comes from ibmx_plan_reserve: this call allocates nothing
    if (!ibmx_contact_ready(p, pair_cap, wall_cap, 2) || !p->s_buf ||
        p->s_cap < ibmx_substep_doubles(np))
        return IBMX_ESTATE;
    hipStream_t s = p->stream;
    ProfScope ps(p, IBMX_K_PAIRS);
    PairC P;
    contact_constants(p, &P);
    const ContactLists C{pair_cap, wall_cap, pairs, walls, counts};
    const size_t hset = (size_t)kHist * ((size_t)pair_cap + wall_cap);
    Hist H[2];
    for (int b = 0; b < 2; ++b)
        H[b] = Hist{p->c_hist + b * hset, p->c_hist + b * hset + (size_t)kHist * pair_cap};
    if (pair_cap > 0)
        IBMX_HIP_CHECK(hipMemcpyAsync(H[0].pair, hist, sizeof(double) * kHist * (size_t)pair_cap,
                                      hipMemcpyDeviceToDevice, s));
    if (wall_cap > 0)
        IBMX_HIP_CHECK(hipMemcpyAsync(H[0].wall, whist, sizeof(double) * kHist * (size_t)wall_cap,
                                      hipMemcpyDeviceToDevice, s));
    double *xt = p->s_buf, *ut = xt + 3 * (size_t)np, *wt = ut + 3 * (size_t)np;
    double *Fbuf[2] = {wt + 3 * (size_t)np, wt + 9 * (size_t)np};
    double *sF = wt + 15 * (size_t)np;
    const int nb = (np + 63) / 64;
    if (counts) {
        contact_adjacency(p, C, s);
    } else {
        ibmx_fill_i32(p->c_off, 0, np + 1, s);
    }
    hipLaunchKernelGGL(k_st_factor, dim3(nb), dim3(64), 0, s, P, np, C, (const int *)p->c_off,
                       (const int2 *)p->c_adj, radius, mass, HistC{H[0].pair, H[0].wall},
                       p->prm.st_switch, sF);
    static const double alpha[3] = {4.0 / 15.0, 1.0 / 15.0, 1.0 / 6.0};
    static const double gamma_[3] = {8.0 / 15.0, 5.0 / 12.0, 3.0 / 4.0};
    static const double zeta_[3] = {0.0, -17.0 / 60.0, -5.0 / 12.0};
    const double dts = dt_total / n_sub;
    const Body B{radius, mass, Fh, Th, sF};
    const int *off = p->c_off;
    const int2 *adj = p->c_adj;
    StageIO io{};
    io.xa = xp;
    io.ua = up;
    io.wa = wp;
    io.xt = xt;
    io.ut = ut;
    io.wt = wt;
    int cur = 0;
    double t_since = 0.0;
    long long gs = 0;
    for (int sub = 0; sub < n_sub; ++sub)
        for (int k = 0; k < 3; ++k, ++gs) {
            const Stage S{dts, 2.0 * alpha[k], alpha[k], gamma_[k], zeta_[k]};
            io.Fcur = Fbuf[gs & 1];
            io.Fprev = Fbuf[(gs + 1) & 1];
            // contacts at the accepted state (committing its history), then s~
            io.xs = xp;
            io.us = up;
            io.ws = wp;
            contact_stage<kStagePredict>(P, np, C, off, adj, B, HistC{H[cur].pair, H[cur].wall},
                                         t_since, H[1 - cur], io, S, s);
            // contacts at s~, then s^k
            io.xs = xt;
            io.us = ut;
            io.ws = wt;
            contact_stage<kStageCorrect>(P, np, C, off, adj, B,
                                         HistC{H[1 - cur].pair, H[1 - cur].wall}, S.a2 * dts,
                                         Hist{nullptr, nullptr}, io, S, s);
            cur = 1 - cur;
            t_since = S.a2 * dts;
        }
    // the final state: committed history and collision force
    io.xs = xp;
    io.us = up;
    io.ws = wp;
    io.Fc = Fc;
    io.Tc = Tc;
    contact_stage<kStageForces>(P, np, C, off, adj, B, HistC{H[cur].pair, H[cur].wall}, t_since,
                                Hist{pair_cap > 0 ? hist : nullptr, wall_cap > 0 ? whist : nullptr},
                                io, Stage{}, s);
    return ibmx_launch_check();
}
