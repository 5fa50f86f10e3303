// Outer forcing loop of the collocated direct-forcing IBM (Sec. 2.2.2).
//
// Per call:
//   geometry   X_l = x_p + o_l in FP64 -> base node and fractional offset per
//              axis, periodic wrap, wall check (deferred EDOMAIN);
//   per pass   interpolate u at the markers, form F_l = (U^d_l - U_l)/c,
//              accumulate the particle sums and the residual (FP64), then
//              spread c F_l dV_l delta into u and F_l dV_l delta into f_tot.
// The interpolation pass finishes before the spreading pass starts (kernel
// boundary), so u can be updated in place: u^m = u^{m-1} + c f^{m-1}.
#include <math.h>

#include "ibmx_internal.hpp"
#include "ibmx_delta.hpp"

namespace {

// ---------------------------------------------------------------------------
// packed base node
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned pack_node(const GridC &g, int bx, int by, int bz)
{
    return (unsigned)bx | ((unsigned)by << g.shift[1]) | ((unsigned)bz << g.shift[2]);
}

__device__ __forceinline__ void unpack_node(const GridC &g, unsigned v, int &bx, int &by, int &bz)
{
    bx = (int)(v & ((1u << g.shift[1]) - 1u));
    by = (int)((v >> g.shift[1]) & ((1u << (g.shift[2] - g.shift[1])) - 1u));
    bz = (int)(v >> g.shift[2]);
}

// node index along one axis for stencil offset k from base b
__device__ __forceinline__ int axis_node(const GridC &g, int a, int b, int k)
{
    int i = b + k;
    if (g.periodic[a])
        return i >= g.n[a] ? i - g.n[a] : i;
    // on a wall axis only a zero-weight last node can fall outside
    return i < g.n[a] ? i : g.n[a] - 1;
}

// ---------------------------------------------------------------------------
// geometry: one thread per marker (original order)
// ---------------------------------------------------------------------------
template <typename T, int W>
__global__ void k_geometry(GridC g, int np, int nm, const int *__restrict__ pid,
                           const double *__restrict__ body, const double *__restrict__ xp,
                           const uint8_t *__restrict__ mask, unsigned *__restrict__ rec_node,
                           T *__restrict__ rec_t, T *__restrict__ rec_o, int *__restrict__ rec_ok,
                           int *__restrict__ err, long long *__restrict__ count)
{
    int l = blockIdx.x * blockDim.x + threadIdx.x;
    int active = 0;
    if (l < nm) {
        active = mask ? (mask[l] != 0) : 1;
        if (active) {
            int p = pid[l];
            int b[3];
            for (int a = 0; a < 3; ++a) {
                double o = body[(size_t)a * nm + l];
                double X = xp[(size_t)a * np + p] + o;
                double s = (X - g.origin[a]) / g.h - Delta<W, T>::base_shift;
                double fl = floor(s);
                double t = s - fl;
                long long bb = (long long)fl - 1;
                if (g.periodic[a]) {
                    bb %= g.n[a];
                    if (bb < 0)
                        bb += g.n[a];
                } else {
                    long long last = (t == 0.0) ? bb + W - 2 : bb + W - 1;
                    if (bb < 0 || last > g.n[a] - 1) {
                        active = 0;
                        atomicCAS(err, 0, (int)IBMX_EDOMAIN);
                    }
                }
                b[a] = (int)bb;
                rec_t[(size_t)a * nm + l] = (T)t;
                rec_o[(size_t)a * nm + l] = (T)o;
            }
            if (active)
                rec_node[l] = pack_node(g, b[0], b[1], b[2]);
        }
        rec_ok[l] = active;
    }
    int c = wave_sum_i(active);
    if ((threadIdx.x & (IBMX_WAVE - 1)) == 0 && c)
        atomicAdd((unsigned long long *)count, (unsigned long long)c);
}

// ---------------------------------------------------------------------------
// interpolation + marker force + per-particle sums: one workgroup per particle
// ---------------------------------------------------------------------------
template <typename T, int W>
__device__ __forceinline__ void stencil_weights(const GridC &g, unsigned node, const T *tt,
                                                int ix[3][W], T w[3][W])
{
    int b[3];
    unpack_node(g, node, b[0], b[1], b[2]);
    for (int a = 0; a < 3; ++a) {
        Delta<W, T>::w(tt[a], w[a]);
#pragma unroll
        for (int k = 0; k < W; ++k)
            ix[a][k] = axis_node(g, a, b[a], k);
    }
}

constexpr int RED = 7;   // S (3), T (3), residual^2

template <typename T, int W>
__global__ __launch_bounds__(256) void k_interp_particle(
    GridC g, int np, int nm, int pass, int final_only, double c, const int *__restrict__ moff,
    const double *__restrict__ dV, const double *__restrict__ up, const double *__restrict__ wp,
    const unsigned *__restrict__ rec_node, const T *__restrict__ rec_t, const T *__restrict__ rec_o,
    const int *__restrict__ rec_ok, const T *__restrict__ u, T *__restrict__ rec_G,
    double *__restrict__ S_out, double *__restrict__ T_out, double *__restrict__ acc,
    T *__restrict__ U_dbg)
{
    const int p = blockIdx.x;
    const long long N = g.nodes;
    const double dVp = dV[p];
    const double upp[3] = {up[p], up[np + p], up[2 * np + p]};
    const double wpp[3] = {wp[p], wp[np + p], wp[2 * np + p]};
    double red[RED] = {0, 0, 0, 0, 0, 0, 0};
    for (int l = moff[p] + threadIdx.x; l < moff[p + 1]; l += blockDim.x) {
        if (!rec_ok[l])
            continue;
        T tt[3], oo[3];
        for (int a = 0; a < 3; ++a) {
            tt[a] = rec_t[(size_t)a * nm + l];
            oo[a] = rec_o[(size_t)a * nm + l];
        }
        int ix[3][W];
        T w[3][W];
        stencil_weights<T, W>(g, rec_node[l], tt, ix, w);
        T U[3] = {0, 0, 0};
#pragma unroll
        for (int k = 0; k < W; ++k)
#pragma unroll
            for (int j = 0; j < W; ++j) {
                const T wzy = w[2][k] * w[1][j];
                const long long row = ((long long)ix[2][k] * g.n[1] + ix[1][j]) * g.n[0];
#pragma unroll
                for (int i = 0; i < W; ++i) {
                    const T ww = wzy * w[0][i];
                    const long long nd = row + ix[0][i];
                    U[0] += ww * u[nd];
                    U[1] += ww * u[N + nd];
                    U[2] += ww * u[2 * N + nd];
                }
            }
        const double o[3] = {(double)oo[0], (double)oo[1], (double)oo[2]};
        const double Ud[3] = {upp[0] + (wpp[1] * o[2] - wpp[2] * o[1]),
                              upp[1] + (wpp[2] * o[0] - wpp[0] * o[2]),
                              upp[2] + (wpp[0] * o[1] - wpp[1] * o[0])};
        double r[3], F[3];
        for (int a = 0; a < 3; ++a) {
            r[a] = Ud[a] - (double)U[a];
            F[a] = r[a] / c;
            red[6] += dVp * r[a] * r[a];
        }
        if (final_only)
            continue;
        if (U_dbg)
            for (int a = 0; a < 3; ++a)
                U_dbg[((size_t)pass * 3 + a) * nm + l] = U[a];
        for (int a = 0; a < 3; ++a) {
            red[a] += F[a] * dVp;
            rec_G[(size_t)a * nm + l] = (T)(F[a] * dVp * g.inv_h3);
        }
        red[3] += (o[1] * F[2] - o[2] * F[1]) * dVp;
        red[4] += (o[2] * F[0] - o[0] * F[2]) * dVp;
        red[5] += (o[0] * F[1] - o[1] * F[0]) * dVp;
    }
    // workgroup reduction of the 7 sums
    __shared__ double part[RED][256 / IBMX_WAVE];
    const int lane = threadIdx.x & (IBMX_WAVE - 1), wv = threadIdx.x / IBMX_WAVE;
    for (int q = 0; q < RED; ++q) {
        double v = wave_sum(red[q]);
        if (lane == 0)
            part[q][wv] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot[RED];
        for (int q = 0; q < RED; ++q) {
            tot[q] = 0.0;
            for (int k = 0; k < (int)(blockDim.x / IBMX_WAVE); ++k)
                tot[q] += part[q][k];
        }
        if (!final_only)
            for (int a = 0; a < 3; ++a) {
                S_out[(size_t)a * np + p] += tot[a];
                T_out[(size_t)a * np + p] += tot[3 + a];
            }
        atomicAdd(&acc[pass], tot[6]);
    }
}

// ---------------------------------------------------------------------------
// spreading: one thread per marker, atomic adds into u and f_tot
// ---------------------------------------------------------------------------
template <typename T, int W>
__global__ void k_spread_atomic(GridC g, int nm, T c, const unsigned *__restrict__ rec_node,
                                const T *__restrict__ rec_t, const int *__restrict__ rec_ok,
                                const T *__restrict__ rec_G, T *__restrict__ u,
                                T *__restrict__ f_tot)
{
    int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nm || !rec_ok[l])
        return;
    const long long N = g.nodes;
    T tt[3], G[3];
    for (int a = 0; a < 3; ++a) {
        tt[a] = rec_t[(size_t)a * nm + l];
        G[a] = rec_G[(size_t)a * nm + l];
    }
    int ix[3][W];
    T w[3][W];
    stencil_weights<T, W>(g, rec_node[l], tt, ix, w);
    for (int k = 0; k < W; ++k)
        for (int j = 0; j < W; ++j) {
            const T wzy = w[2][k] * w[1][j];
            const long long row = ((long long)ix[2][k] * g.n[1] + ix[1][j]) * g.n[0];
            for (int i = 0; i < W; ++i) {
                const T ww = wzy * w[0][i];
                if (ww == T(0))
                    continue;
                const long long nd = row + ix[0][i];
                for (int a = 0; a < 3; ++a) {
                    const T f = ww * G[a];
                    unsafeAtomicAdd(&f_tot[a * N + nd], f);
                    unsafeAtomicAdd(&u[a * N + nd], c * f);
                }
            }
        }
}

// Distinct grid nodes with nonzero delta weight from some active marker
// (profiling only): a bitmap of touched nodes, counted on first touch.
template <typename T, int W>
__global__ void k_shell_count(GridC g, int nm, const unsigned *__restrict__ rec_node,
                              const T *__restrict__ rec_t, const int *__restrict__ rec_ok,
                              unsigned *__restrict__ bits, long long *__restrict__ count)
{
    int l = blockIdx.x * blockDim.x + threadIdx.x;
    int fresh = 0;
    if (l < nm && rec_ok[l]) {
        T tt[3];
        for (int a = 0; a < 3; ++a)
            tt[a] = rec_t[(size_t)a * nm + l];
        int ix[3][W];
        T w[3][W];
        stencil_weights<T, W>(g, rec_node[l], tt, ix, w);
        for (int k = 0; k < W; ++k)
            for (int j = 0; j < W; ++j)
                for (int i = 0; i < W; ++i) {
                    if (w[2][k] * w[1][j] * w[0][i] == T(0))
                        continue;
                    long long nd = ((long long)ix[2][k] * g.n[1] + ix[1][j]) * g.n[0] + ix[0][i];
                    unsigned bit = 1u << (nd & 31);
                    unsigned old = atomicOr(&bits[nd >> 5], bit);
                    fresh += (old & bit) ? 0 : 1;
                }
    }
    int c = wave_sum_i(fresh);
    if ((threadIdx.x & (IBMX_WAVE - 1)) == 0 && c)
        atomicAdd((unsigned long long *)&count[1], (unsigned long long)c);
}

__global__ void k_finish_resid(const double *acc, double *resid, int n)
{
    int i = threadIdx.x;
    if (i < n)
        resid[i] = sqrt(acc[i]);
}

template <typename T, int W>
ibmx_status run_forcing(ibmx_plan p, T *u, T *f_tot, const double *xp, const double *up,
                        const double *wp, const uint8_t *mask, double *S_out, double *T_out,
                        double *resid_out, T *U_dbg)
{
    hipStream_t s = p->stream;
    const int nm = p->nm, np = p->np, n_iter = p->prm.n_iter;
    const double c = p->prm.two_alpha_dt;
    ibmx_fill_f64(S_out, 0.0, 3LL * np, s);
    ibmx_fill_f64(T_out, 0.0, 3LL * np, s);
    ibmx_fill_f64(p->d_acc, 0.0, n_iter + 1, s);
    ibmx_fill_i32((int *)p->d_count, 0, 16, s);
    int *rec_ok = p->m_key;
    if (nm > 0) {
        ProfScope ps(p, IBMX_K_GEOMETRY);
        hipLaunchKernelGGL((k_geometry<T, W>), dim3((nm + 255) / 256), dim3(256), 0, s, p->g, np,
                           nm, p->d_pid, p->body, xp, mask, (unsigned *)p->rec_node,
                           (T *)p->rec_t, (T *)p->rec_o, rec_ok, p->d_err, p->d_count);
    }
    if (p->prof && p->shell_bits && nm > 0) {
        ibmx_fill_i32((int *)p->shell_bits, 0, (p->g.nodes + 31) / 32, s);
        hipLaunchKernelGGL((k_shell_count<T, W>), dim3((nm + 255) / 256), dim3(256), 0, s, p->g, nm,
                           (const unsigned *)p->rec_node, (const T *)p->rec_t, rec_ok,
                           p->shell_bits, p->d_count);
    }
    for (int m = 0; m < n_iter; ++m) {
        if (np > 0) {
            ProfScope ps(p, IBMX_K_INTERP);
            hipLaunchKernelGGL((k_interp_particle<T, W>), dim3(np), dim3(256), 0, s, p->g, np, nm,
                               m, 0, c, p->d_moff, p->dV, up, wp, (const unsigned *)p->rec_node,
                               (const T *)p->rec_t, (const T *)p->rec_o, rec_ok, u, (T *)p->rec_G,
                               S_out, T_out, p->d_acc, U_dbg);
        }
        if (nm > 0) {
            ProfScope ps(p, IBMX_K_SPREAD);
            hipLaunchKernelGGL((k_spread_atomic<T, W>), dim3((nm + 255) / 256), dim3(256), 0, s,
                               p->g, nm, (T)c, (const unsigned *)p->rec_node, (const T *)p->rec_t,
                               rec_ok, (const T *)p->rec_G, u, f_tot);
        }
    }
    if (resid_out) {
        if (np > 0)
            hipLaunchKernelGGL((k_interp_particle<T, W>), dim3(np), dim3(256), 0, s, p->g, np, nm,
                               n_iter, 1, c, p->d_moff, p->dV, up, wp,
                               (const unsigned *)p->rec_node, (const T *)p->rec_t,
                               (const T *)p->rec_o, rec_ok, u, (T *)p->rec_G, S_out, T_out,
                               p->d_acc, (T *)nullptr);
        hipLaunchKernelGGL(k_finish_resid, dim3(1), dim3(64), 0, s, p->d_acc, resid_out, n_iter + 1);
    }
    return ibmx_launch_check();
}

}  // namespace

extern "C" ibmx_status ibmx_forcing(ibmx_plan p, void *u, void *f_tot, const double *xp,
                                    const double *up, const double *wp,
                                    const uint8_t *marker_active, double *S_out, double *T_out,
                                    double *resid_out, void *U_debug)
{
    if (!p)
        return IBMX_EINVAL;
    if (p->nm > 0 && (!p->body || !p->dV))
        return IBMX_ESTATE;
    if (!u || !f_tot || (p->np > 0 && (!xp || !up || !wp || !S_out || !T_out)))
        return IBMX_EINVAL;
    if (p->n_iter_cap + 1 > 64)
        return IBMX_EINVAL;
    const int W = p->prm.kernel;
    if (p->prec == IBMX_F64) {
        if (W == 3)
            return run_forcing<double, 3>(p, (double *)u, (double *)f_tot, xp, up, wp,
                                          marker_active, S_out, T_out, resid_out, (double *)U_debug);
        return run_forcing<double, 4>(p, (double *)u, (double *)f_tot, xp, up, wp, marker_active,
                                      S_out, T_out, resid_out, (double *)U_debug);
    }
    if (W == 3)
        return run_forcing<float, 3>(p, (float *)u, (float *)f_tot, xp, up, wp, marker_active,
                                     S_out, T_out, resid_out, (float *)U_debug);
    return run_forcing<float, 4>(p, (float *)u, (float *)f_tot, xp, up, wp, marker_active, S_out,
                                 T_out, resid_out, (float *)U_debug);
}

extern "C" ibmx_status ibmx_forcing_backward(ibmx_plan, const void *, const double *,
                                             const double *, const double *, const uint8_t *,
                                             const void *, const void *, const double *,
                                             const double *, void *, double *, double *, double *)
{
    return IBMX_EUNSUPPORTED;
}

extern "C" ibmx_status ibmx_tune(ibmx_plan, void *, void *, const double *, const double *,
                                 const double *, const uint8_t *)
{
    return IBMX_EUNSUPPORTED;
}
