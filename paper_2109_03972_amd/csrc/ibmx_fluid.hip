// Pressure projection of the collocated fluid solver (Sec. 2.2.1 and eq.
// fluid-solver, steps f-i): face interpolation, compact Poisson equation,
// cell and face corrections, pressure update.
//
// The Poisson equation L phi = div(u_f*) / c, with L the compact Laplacian
// of the face gradients, is solved directly: complex FFTs along the periodic
// x and y axes (and z when periodic, then a division by the eigenvalues), or
// per (kx, ky) mode a tridiagonal elimination across the walls in z.  FFTs
// are radix-2 passes in place in LDS, several short lines per workgroup,
// loaded so that each wave reads contiguous memory; everything is FP64,
// whatever the grid precision.
#include <math.h>
#include <vector>

#include "ibmx_internal.hpp"

namespace {

constexpr int kFftThreads = 256;
constexpr int kFftElems = 512;      // elements per workgroup, contiguous lines
constexpr int kFftElemsStrided = 2048;   // strided lines: 32 KB of LDS, 4 lines of 512

struct FluidC {
    int n[3];
    int periodic[3];
    double h, c, nu, theta;
};

__device__ __forceinline__ long long cell_index(const FluidC &F, int i, int j, int k)
{
    return ((long long)k * F.n[1] + j) * F.n[0] + i;
}

// neighbour index along axis a (d = +1 / -1); -1 past a wall
__device__ __forceinline__ long long neighbour(const FluidC &F, int i, int j, int k, int a, int d)
{
    int q[3] = {i, j, k};
    q[a] += d;
    if (q[a] < 0 || q[a] >= F.n[a]) {
        if (!F.periodic[a])
            return -1;
        q[a] = q[a] < 0 ? q[a] + F.n[a] : q[a] - F.n[a];
    }
    return cell_index(F, q[0], q[1], q[2]);
}

// u_f* = mean of the two cells of each +a face (wall faces 0), and the
// right-hand side div(u_f*) / c as a complex field with zero imaginary part
template <typename T>
__global__ __launch_bounds__(256) void k_face_div(FluidC F, const T *__restrict__ u,
                                                  T *__restrict__ uf, double2 *__restrict__ Z)
{
    const long long N = (long long)F.n[0] * F.n[1] * F.n[2];
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < N;
         c += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(c % F.n[0]), j = (int)((c / F.n[0]) % F.n[1]),
                  k = (int)(c / ((long long)F.n[0] * F.n[1]));
        double div = 0.0;
        for (int a = 0; a < 3; ++a) {
            const T *ua = u + (size_t)a * N;
            const double uc = (double)ua[c];
            const long long up = neighbour(F, i, j, k, a, 1), dn = neighbour(F, i, j, k, a, -1);
            const double out = up >= 0 ? 0.5 * (uc + (double)ua[up]) : 0.0;
            const double in = dn >= 0 ? 0.5 * ((double)ua[dn] + uc) : 0.0;
            uf[(size_t)a * N + c] = (T)out;
            div = div + (out - in) / F.h;
        }
        Z[c] = make_double2(div / F.c, 0.0);
    }
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Batched complex FFT of lines of length n = 2^logn: iterative radix-2
// Cooley-Tukey in place in LDS (elements loaded in bit-reversed order).
// Line l of the batch starts at (l / A) * B + (l % A) * C and has element
// stride S; a workgroup takes `lpw` consecutive lines.  Contiguous lines
// (S = 1) are loaded line by line, strided ones element-major across the
// lines, so the loads of a wave are contiguous either way.  tw[m] =
// exp(-2 pi i m / n), m < n / 2, read through the cache; INV uses the
// conjugate (no 1/n scaling).
template <bool INV>
__global__ __launch_bounds__(kFftThreads) void k_fft(double2 *__restrict__ Z, int n, int logn,
                                                     int lpw, long long A, long long B, long long C,
                                                     long long S, const double2 *__restrict__ tw)
{
    extern __shared__ double2 buf[];
    const int total = lpw * n, half_n = n / 2;
    const long long line0 = (long long)blockIdx.x * lpw;
    auto addr = [&](int l, int s) -> long long {
        const long long line = line0 + l;
        return (line / A) * B + (line % A) * C + (long long)s * S;
    };
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
        const int l = S == 1 ? e / n : e % lpw, s = S == 1 ? e % n : e / lpw;
        const int r = logn > 0 ? (int)(__brev((unsigned)s) >> (32 - logn)) : 0;
        buf[l * n + r] = Z[addr(l, s)];
    }
    __syncthreads();
    for (int len = 2; len <= n; len <<= 1) {
        const int half = len >> 1, step = n / len;
        for (int b = threadIdx.x; b < lpw * half_n; b += blockDim.x) {
            const int l = b / half_n, jj = b % half_n, pos = jj % half;
            const int i0 = l * n + (jj / half) * len + pos, i1 = i0 + half;
            double2 wk = tw[pos * step];
            if (INV)
                wk.y = -wk.y;
            const double2 v0 = buf[i0], v1 = cmul(buf[i1], wk);
            buf[i0] = make_double2(v0.x + v1.x, v0.y + v1.y);
            buf[i1] = make_double2(v0.x - v1.x, v0.y - v1.y);
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
        const int l = S == 1 ? e / n : e % lpw, s = S == 1 ? e % n : e / lpw;
        Z[addr(l, s)] = buf[l * n + s];
    }
}

// eigenvalue of the periodic second difference for mode m of n points
__device__ __forceinline__ double lam(int m, int n, double h)
{
    return (2.0 * cospi(2.0 * m / (double)n) - 2.0) / (h * h);
}

// triply periodic: divide every mode by its eigenvalue (the mean mode is 0)
__global__ __launch_bounds__(256) void k_divide(FluidC F, double2 *__restrict__ Z)
{
    const long long N = (long long)F.n[0] * F.n[1] * F.n[2];
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < N;
         c += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(c % F.n[0]), j = (int)((c / F.n[0]) % F.n[1]),
                  k = (int)(c / ((long long)F.n[0] * F.n[1]));
        const double L = lam(i, F.n[0], F.h) + lam(j, F.n[1], F.h) + lam(k, F.n[2], F.h);
        const double2 z = Z[c];
        Z[c] = c == 0 ? make_double2(0.0, 0.0) : make_double2(z.x / L, z.y / L);
    }
}

// walls in z: per (kx, ky) mode the system (1/h^2)(phi_{k+1} - 2 phi_k +
// phi_{k-1}) + lambda_xy phi_k = rhs_k with zero-gradient ends, by
// elimination from the bottom; the (0, 0) mode is singular: its top value is
// pinned to 0, then its z-mean removed (the grid mean of phi).  cp holds the
// eliminated super-diagonal.
__global__ __launch_bounds__(256) void k_tridiag(FluidC F, double2 *__restrict__ Z,
                                                 double *__restrict__ cp)
{
    const int nxy = F.n[0] * F.n[1], nz = F.n[2];
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= nxy)
        return;
    const int i = col % F.n[0], j = col / F.n[0];
    const double ih2 = 1.0 / (F.h * F.h);
    const double lxy = lam(i, F.n[0], F.h) + lam(j, F.n[1], F.h);
    const bool singular = col == 0;
    double cprev = 0.0;
    double2 dprev = make_double2(0.0, 0.0);
    for (int k = 0; k < nz; ++k) {
        const size_t c = (size_t)k * nxy + col;
        double a = k > 0 ? ih2 : 0.0, sup = k < nz - 1 ? ih2 : 0.0;
        double b = lxy - (a + sup);
        double2 d = Z[c];
        if (singular && k == nz - 1) {
            a = 0.0;
            b = 1.0;
            d = make_double2(0.0, 0.0);
        }
        const double den = b - a * cprev;
        cprev = sup / den;
        dprev = make_double2((d.x - a * dprev.x) / den, (d.y - a * dprev.y) / den);
        cp[c] = cprev;
        Z[c] = dprev;
    }
    double2 x = dprev;
    double2 sum = x;
    for (int k = nz - 2; k >= 0; --k) {
        const size_t c = (size_t)k * nxy + col;
        const double2 d = Z[c];
        x = make_double2(d.x - cp[c] * x.x, d.y - cp[c] * x.y);
        Z[c] = x;
        sum.x += x.x;
        sum.y += x.y;
    }
    if (singular) {
        const double2 mean = make_double2(sum.x / nz, sum.y / nz);
        for (int k = 0; k < nz; ++k) {
            const size_t c = (size_t)k * nxy + col;
            Z[c] = make_double2(Z[c].x - mean.x, Z[c].y - mean.y);
        }
    }
}

// phi = Re(Z) / scale; u = u* - c grad(phi) (mean of the cell's two face
// gradients), u_f = u_f* - c (phi_+ - phi)/h, P = (1 - theta) P + phi -
// (c/2) nu L phi
template <typename T>
__global__ __launch_bounds__(256) void k_correct(FluidC F, const double2 *__restrict__ Z,
                                                 double scale, T *__restrict__ u,
                                                 T *__restrict__ uf, T *__restrict__ P,
                                                 T *__restrict__ phi_out)
{
    const long long N = (long long)F.n[0] * F.n[1] * F.n[2];
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < N;
         c += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(c % F.n[0]), j = (int)((c / F.n[0]) % F.n[1]),
                  k = (int)(c / ((long long)F.n[0] * F.n[1]));
        const double ph = Z[c].x * scale;
        double lap = 0.0;
        for (int a = 0; a < 3; ++a) {
            const long long up = neighbour(F, i, j, k, a, 1), dn = neighbour(F, i, j, k, a, -1);
            const double gp = up >= 0 ? (Z[up].x * scale - ph) / F.h : 0.0;
            const double gm = dn >= 0 ? (ph - Z[dn].x * scale) / F.h : 0.0;
            const size_t ia = (size_t)a * N + c;
            u[ia] = (T)((double)u[ia] - F.c * (0.5 * (gp + gm)));
            uf[ia] = (T)((double)uf[ia] - F.c * gp);
            lap = lap + (gp - gm) / F.h;
        }
        P[c] = (T)((1.0 - F.theta) * (double)P[c] + ph - 0.5 * F.c * F.nu * lap);
        if (phi_out)
            phi_out[c] = (T)ph;
    }
}

int grid_blocks(long long n) { return (int)(n / 256 + 1 < 16384 ? n / 256 + 1 : 16384); }

bool pow2(int n) { return n >= 2 && (n & (n - 1)) == 0; }

int log2i(int n)
{
    int l = 0;
    while ((1 << l) < n)
        ++l;
    return l;
}

// one FFT pass along axis a over the whole grid
template <bool INV>
void fft_axis(ibmx_plan p, const FluidC &F, int a, hipStream_t s)
{
    const int nx = F.n[0], ny = F.n[1], nz = F.n[2], n = F.n[a];
    long long A, B, C, S, lines;
    int lim;   // lines of one group must share the pattern below
    if (a == 0) {
        A = 1, B = nx, C = 0, S = 1, lines = (long long)ny * nz, lim = ny * nz;
    } else if (a == 1) {
        A = nx, B = (long long)nx * ny, C = 1, S = nx, lines = (long long)nx * nz, lim = nx;
    } else {
        A = (long long)nx * ny, B = 0, C = 1, S = (long long)nx * ny, lines = (long long)nx * ny,
        lim = nx * ny;
    }
    const int elems = a == 0 ? kFftElems : kFftElemsStrided;
    int lpw = n >= elems ? 1 : elems / n;
    while (lpw > 1 && (lpw > lim || lim % lpw != 0))
        lpw >>= 1;
    const size_t lds = sizeof(double2) * (size_t)lpw * n;
    hipLaunchKernelGGL((k_fft<INV>), dim3((unsigned)(lines / lpw)), dim3(kFftThreads), lds, s,
                       p->fl_z, n, log2i(n), lpw, A, B, C, S, (const double2 *)p->fl_tw[a]);
}

template <typename T>
ibmx_status run_project(ibmx_plan p, T *u, T *uf, T *P, T *phi, double theta)
{
    const ibmx_grid &g = p->grid;
    FluidC F;
    for (int a = 0; a < 3; ++a) {
        F.n[a] = g.n[a];
        F.periodic[a] = g.periodic[a];
    }
    F.h = g.h;
    F.c = p->prm.two_alpha_dt;
    F.nu = p->prm.nu_f;
    F.theta = theta;
    const long long N = p->g.nodes;
    hipStream_t s = p->stream;
    ProfScope ps(p, IBMX_K_OTHER);
    hipLaunchKernelGGL((k_face_div<T>), dim3(grid_blocks(N)), dim3(256), 0, s, F, (const T *)u, uf,
                       p->fl_z);
    fft_axis<false>(p, F, 0, s);
    fft_axis<false>(p, F, 1, s);
    double scale = 1.0 / ((double)F.n[0] * F.n[1]);
    if (F.periodic[2]) {
        fft_axis<false>(p, F, 2, s);
        hipLaunchKernelGGL(k_divide, dim3(grid_blocks(N)), dim3(256), 0, s, F, p->fl_z);
        fft_axis<true>(p, F, 2, s);
        scale /= F.n[2];
    } else {
        const int nxy = F.n[0] * F.n[1];
        hipLaunchKernelGGL(k_tridiag, dim3((nxy + 255) / 256), dim3(256), 0, s, F, p->fl_z,
                           p->fl_cp);
    }
    fft_axis<true>(p, F, 1, s);
    fft_axis<true>(p, F, 0, s);
    hipLaunchKernelGGL((k_correct<T>), dim3(grid_blocks(N)), dim3(256), 0, s, F,
                       (const double2 *)p->fl_z, scale, u, uf, P, phi);
    return ibmx_launch_check();
}

// workspace: the complex grid, the elimination scratch (walls in z) and
// one twiddle table per axis
ibmx_status fluid_reserve(ibmx_plan p)
{
    if (p->fl_z)
        return IBMX_OK;
    const size_t N = (size_t)p->g.nodes;
    if (hipMalloc((void **)&p->fl_z, sizeof(double2) * N) != hipSuccess)
        return IBMX_ENOMEM;
    if (!p->grid.periodic[2] && hipMalloc((void **)&p->fl_cp, sizeof(double) * N) != hipSuccess)
        return IBMX_ENOMEM;
    for (int a = 0; a < 3; ++a) {
        const int n = p->grid.n[a];
        std::vector<double2> tw((size_t)(n / 2 > 0 ? n / 2 : 1));
        for (int m = 0; m < n / 2; ++m) {
            const double ang = -2.0 * M_PI * (double)m / (double)n;
            tw[m] = make_double2(cos(ang), sin(ang));
        }
        if (hipMalloc((void **)&p->fl_tw[a], sizeof(double2) * tw.size()) != hipSuccess ||
            hipMemcpy(p->fl_tw[a], tw.data(), sizeof(double2) * tw.size(),
                      hipMemcpyHostToDevice) != hipSuccess)
            return IBMX_ENOMEM;
    }
    return IBMX_OK;
}

}  // namespace

extern "C" ibmx_status ibmx_project(ibmx_plan p, void *u, void *uf, void *P, void *phi,
                                    double theta)
{
    if (!p || !u || !uf || !P || !isfinite(theta))
        return IBMX_EINVAL;
    const ibmx_grid &g = p->grid;
    if (!g.periodic[0] || !g.periodic[1] || !pow2(g.n[0]) || !pow2(g.n[1]) || g.n[0] > 1024 ||
        g.n[1] > 1024 || (g.periodic[2] && (!pow2(g.n[2]) || g.n[2] > 1024)))
        return IBMX_EUNSUPPORTED;
    const ibmx_status st = fluid_reserve(p);
    if (st != IBMX_OK)
        return st;
    if (p->prec == IBMX_F64)
        return run_project<double>(p, (double *)u, (double *)uf, (double *)P, (double *)phi, theta);
    return run_project<float>(p, (float *)u, (float *)uf, (float *)P, (float *)phi, theta);
}
