// Fluid integrals over each particle with the level-set volume fraction
// (Sec. 2.2.9), and the volume average of a grid field (Sec. 2.2.4).
#include <math.h>

#include <mutex>

#include "ibmx_internal.hpp"

namespace {

constexpr int PI_THREADS = 256;
constexpr int MEAN_BLOCKS = 4096;

// Volume fraction of the cell whose lowest corner is c0 (relative to the
// particle centre) in a sphere of radius R: the signed corner distances
// phi_m = |x_m - x_p| - R give alpha = sum -phi_m H(-phi_m) / sum |phi_m|.
__device__ __forceinline__ double cell_alpha(const double *c0, double h, double R)
{
    double num = 0.0, den = 0.0;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const double dx = c0[0] + (m & 1) * h, dy = c0[1] + ((m >> 1) & 1) * h,
                     dz = c0[2] + ((m >> 2) & 1) * h;
        const double phi = sqrt(dx * dx + dy * dy + dz * dz) - R;
        if (phi <= 0.0)
            num += -phi;
        den += fabs(phi);
    }
    return den > 0.0 ? num / den : 0.0;
}

// One workgroup per particle; its threads take the cells of the particle's
// bounding box.  Cells whose centre lies deeper than half a cell diagonal
// inside (outside) the surface have every corner inside (outside) and take
// alpha = 1 (0) without the corner distances, which is what the corner
// formula gives for them; the test compares squared distances.  FP64 sums:
// per thread in cell order, per wave by a fixed shuffle tree, over the waves
// in wave order.
template <typename T>
__global__ __launch_bounds__(PI_THREADS) void k_particle_integrals(GridC g, int np,
                                                                   const double *__restrict__ xp,
                                                                   const double *__restrict__ radius,
                                                                   const T *__restrict__ u,
                                                                   double *__restrict__ Iu,
                                                                   double *__restrict__ Ir,
                                                                   T *__restrict__ alpha_out)
{
    __shared__ double part[6][PI_THREADS / IBMX_WAVE];
    const int p = blockIdx.x;
    const int wv = threadIdx.x / IBMX_WAVE, lane = threadIdx.x & (IBMX_WAVE - 1);
    const double h = g.h, h3 = h * h * h, half_diag = 0.5 * sqrt(3.0) * h;
    const double R = radius[p];
    double x[3];
    int lo[3], ext[3];
    for (int a = 0; a < 3; ++a) {
        x[a] = xp[(size_t)a * np + p];
        if (g.periodic[a]) {
            const double L = g.n[a] * h;
            x[a] = x[a] - floor((x[a] - g.origin[a]) / L) * L;
        }
        lo[a] = (int)floor((x[a] - R - g.origin[a]) / h);
        ext[a] = (int)floor((x[a] + R - g.origin[a]) / h) - lo[a] + 1;
    }
    const int total = ext[0] * ext[1] * ext[2], exy = ext[0] * ext[1];
    const double r_in = R - half_diag, r_out = R + half_diag;
    const double r_in2 = r_in > 0.0 ? r_in * r_in : -1.0, r_out2 = r_out * r_out;
    const long long N = g.nodes;
    double s[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int q = threadIdx.x; q < total; q += blockDim.x) {
        const int qz = q / exy, qr = q - qz * exy, qy = qr / ext[0];
        const int c[3] = {lo[0] + qr - qy * ext[0], lo[1] + qy, lo[2] + qz};
        int gc[3];
        bool in = true;
        for (int a = 0; a < 3; ++a) {
            gc[a] = c[a];
            if (g.periodic[a])
                gc[a] = gc[a] < 0 ? gc[a] + g.n[a] : (gc[a] >= g.n[a] ? gc[a] - g.n[a] : gc[a]);
            else if (gc[a] < 0 || gc[a] >= g.n[a])
                in = false;
        }
        if (!in)
            continue;
        const double c0[3] = {g.origin[0] + c[0] * h - x[0], g.origin[1] + c[1] * h - x[1],
                              g.origin[2] + c[2] * h - x[2]};
        const double r[3] = {c0[0] + 0.5 * h, c0[1] + 0.5 * h, c0[2] + 0.5 * h};
        const double dc2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        double alpha;
        if (dc2 <= r_in2)
            alpha = 1.0;
        else if (dc2 >= r_out2)
            continue;
        else
            alpha = cell_alpha(c0, h, R);
        if (alpha == 0.0)
            continue;
        const long long gi = ((long long)gc[2] * g.n[1] + gc[1]) * g.n[0] + gc[0];
        const double uc[3] = {(double)u[gi], (double)u[N + gi], (double)u[2 * N + gi]};
        const double w = alpha * h3;
        s[0] += w * uc[0];
        s[1] += w * uc[1];
        s[2] += w * uc[2];
        s[3] += w * (r[1] * uc[2] - r[2] * uc[1]);
        s[4] += w * (r[2] * uc[0] - r[0] * uc[2]);
        s[5] += w * (r[0] * uc[1] - r[1] * uc[0]);
        if (alpha_out)
            atomicAdd(&alpha_out[gi], (T)alpha);
    }
#pragma unroll
    for (int k = 0; k < 6; ++k)
        s[k] = wave_sum(s[k]);
    if (lane == 0)
        for (int k = 0; k < 6; ++k)
            part[k][wv] = s[k];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 0; k < 6; ++k) {
            double v = part[k][0];
            for (int w = 1; w < (int)(blockDim.x / IBMX_WAVE); ++w)
                v += part[k][w];
            if (k < 3)
                Iu[(size_t)k * np + p] = v;
            else
                Ir[(size_t)(k - 3) * np + p] = v;
        }
}

// Partial FP64 sums of each component over contiguous chunks, one chunk per
// workgroup, then their sum in workgroup order: the mean does not depend on
// scheduling.
template <typename T>
__global__ __launch_bounds__(256) void k_mean_partial(const T *__restrict__ f, long long N,
                                                      double *__restrict__ part)
{
    __shared__ double wsum[256 / IBMX_WAVE];
    const long long chunk = (N + gridDim.x - 1) / gridDim.x;
    const long long lo = (long long)blockIdx.x * chunk;
    const long long hi = lo + chunk < N ? lo + chunk : N;
    const int wv = threadIdx.x / IBMX_WAVE, lane = threadIdx.x & (IBMX_WAVE - 1);
    constexpr int E = 16 / (int)sizeof(T);
    for (int a = 0; a < 3; ++a) {
        const T *fa = f + (size_t)a * N;
        double s = 0.0;
        if (((size_t)fa & 15) == 0 && lo % E == 0) {
            // 16-byte packets over the chunk, elements for its tail
            const long long nv = (hi - lo) / E;
            struct alignas(16) Packet {
                T e[E];
            };
            const Packet *pk = reinterpret_cast<const Packet *>(fa + lo);
            for (long long v = threadIdx.x; v < nv; v += blockDim.x) {
                const Packet q = pk[v];
#pragma unroll
                for (int k = 0; k < E; ++k)
                    s += (double)q.e[k];
            }
            for (long long i = lo + nv * E + threadIdx.x; i < hi; i += blockDim.x)
                s += (double)fa[i];
        } else {
            for (long long i = lo + threadIdx.x; i < hi; i += blockDim.x)
                s += (double)fa[i];
        }
        s = wave_sum(s);
        if (lane == 0)
            wsum[wv] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            double v = wsum[0];
            for (int w = 1; w < (int)(blockDim.x / IBMX_WAVE); ++w)
                v += wsum[w];
            part[(size_t)a * gridDim.x + blockIdx.x] = v;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_mean_finish(const double *__restrict__ part, int nb,
                                                     long long N, double *__restrict__ mean)
{
    __shared__ double wsum[256 / IBMX_WAVE];
    const int wv = threadIdx.x / IBMX_WAVE, lane = threadIdx.x & (IBMX_WAVE - 1);
    for (int a = 0; a < 3; ++a) {
        double s = 0.0;
        for (int i = threadIdx.x; i < nb; i += blockDim.x)
            s += part[(size_t)a * nb + i];
        s = wave_sum(s);
        if (lane == 0)
            wsum[wv] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            double v = wsum[0];
            for (int w = 1; w < (int)(blockDim.x / IBMX_WAVE); ++w)
                v += wsum[w];
            mean[a] = v / (double)N;
        }
        __syncthreads();
    }
}

template <typename T>
__global__ void k_fill_grid(T *__restrict__ p, long long n)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += stride)
        p[i] = T(0);
}

template <typename T>
ibmx_status run_integrals(ibmx_plan p, const T *u, const double *xp, const double *radius,
                          double *Iu, double *Ir, T *alpha_out)
{
    hipStream_t s = p->stream;
    ProfScope ps(p, IBMX_K_OTHER);
    if (alpha_out)
        hipLaunchKernelGGL((k_fill_grid<T>), dim3(4096), dim3(256), 0, s, alpha_out, p->g.nodes);
    if (p->np > 0)
        hipLaunchKernelGGL((k_particle_integrals<T>), dim3(p->np), dim3(PI_THREADS), 0, s, p->g,
                           p->np, xp, radius, u, Iu, Ir, alpha_out);
    return ibmx_launch_check();
}

template <typename T>
ibmx_status run_mean(ibmx_plan p, const T *f, double *mean)
{
    hipStream_t s = p->stream;
    ProfScope ps(p, IBMX_K_OTHER);
    hipLaunchKernelGGL((k_mean_partial<T>), dim3(MEAN_BLOCKS), dim3(256), 0, s, f, p->g.nodes,
                       p->mean_part);
    hipLaunchKernelGGL(k_mean_finish, dim3(1), dim3(256), 0, s, (const double *)p->mean_part,
                       MEAN_BLOCKS, p->g.nodes, mean);
    return ibmx_launch_check();
}

}  // namespace

int ibmx_mean_blocks() { return MEAN_BLOCKS; }

// Partial sums of ibmx_grid_mean_noalloc: [3][MEAN_BLOCKS] doubles (96 KB)
// in every device's copy of the library's code object, held until the
// process ends.  Host code never passes this name to a kernel: it stands for
// a host-side shadow, not the device address; the address comes from
// hipGetSymbolAddress per device.
static __device__ __align__(256) double scratch[3 * MEAN_BLOCKS];

namespace {

constexpr int SCRATCH_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[SCRATCH_DEVICES];   // address of scratch on each device

// Device address of scratch on the current device, looked up once per
// device with that device current.
ibmx_status scratch_on_current_device(double **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess)
        return IBMX_EDEVICE;
    if (dev < 0 || dev >= SCRATCH_DEVICES)
        return IBMX_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
            return IBMX_EDEVICE;
        g_scratch_ptr[dev] = (double *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return IBMX_OK;
}

}  // namespace

extern "C" ibmx_status ibmx_grid_mean_noalloc(const void *f, int64_t n_nodes,
                                              ibmx_precision precision, double *mean,
                                              void *hip_stream)
{
    if (!f || !mean || n_nodes < 1 || n_nodes >= (1LL << 31) ||
        (precision != IBMX_F64 && precision != IBMX_F32))
        return IBMX_EINVAL;
    double *part = nullptr;
    const ibmx_status st = scratch_on_current_device(&part);
    if (st != IBMX_OK)
        return st;
    hipStream_t s = (hipStream_t)hip_stream;
    // every partial slot is written by k_mean_partial before k_mean_finish
    // reads it: nothing to clear between calls
    if (precision == IBMX_F64)
        hipLaunchKernelGGL((k_mean_partial<double>), dim3(MEAN_BLOCKS), dim3(256), 0, s,
                           (const double *)f, (long long)n_nodes, part);
    else
        hipLaunchKernelGGL((k_mean_partial<float>), dim3(MEAN_BLOCKS), dim3(256), 0, s,
                           (const float *)f, (long long)n_nodes, part);
    hipLaunchKernelGGL(k_mean_finish, dim3(1), dim3(256), 0, s, (const double *)part, MEAN_BLOCKS,
                       (long long)n_nodes, mean);
    return ibmx_launch_check();
}

extern "C" ibmx_status ibmx_particle_integrals(ibmx_plan p, const void *u, const double *xp,
                                               const double *radius, double *Iu, double *Ir,
                                               void *alpha_out)
{
    if (!p || !u || (p->np > 0 && (!xp || !radius || !Iu || !Ir)))
        return IBMX_EINVAL;
    if (p->prec == IBMX_F64)
        return run_integrals<double>(p, (const double *)u, xp, radius, Iu, Ir, (double *)alpha_out);
    return run_integrals<float>(p, (const float *)u, xp, radius, Iu, Ir, (float *)alpha_out);
}

extern "C" ibmx_status ibmx_grid_mean(ibmx_plan p, const void *f, double *mean)
{
    if (!p || !f || !mean)
        return IBMX_EINVAL;
    if (p->prec == IBMX_F64)
        return run_mean<double>(p, (const double *)f, mean);
    return run_mean<float>(p, (const float *)f, mean);
}
