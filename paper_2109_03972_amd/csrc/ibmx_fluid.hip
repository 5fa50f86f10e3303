// The collocated fluid solver's steps around the forcing loop (Sec. 2.2.1
// and eq. fluid-solver): the predictor (step a), the implicit viscous step
// (step e) and the pressure projection (steps f-i: face interpolation,
// compact Poisson equation, cell and face corrections, pressure update).
//
// Both implicit systems, (I - beta L) u* = r per velocity component and the
// compact Poisson equation L phi = div(u_f*) / c, are solved directly in
// FP64: complex FFTs along the periodic x and y axes (and z when periodic,
// then a division by the eigenvalues), or per (kx, ky) mode a tridiagonal
// elimination across the walls in z.  FFTs are radix-2 passes in place in
// LDS, several short lines per workgroup, loaded so that each wave reads
// contiguous memory.  Stencil kernels take one thread per cell with x along
// the block and y, z along the grid.
#include <math.h>
#include <vector>

#include "ibmx_internal.hpp"

namespace {

constexpr int kFftThreads = 256;
constexpr int kFftElems = 512;      // elements per workgroup, contiguous lines
constexpr int kFftElemsStrided = 2048;   // strided lines: 32 KB of LDS, 4 lines of 512
constexpr int kFftMaxLines = 1024;       // lines per workgroup (lines of 2 elements and up)

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
    {
        const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y, k = blockIdx.z;
        if (i >= F.n[0])
            return;
        const long long c = cell_index(F, i, j, k);
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
// Cooley-Tukey in place in LDS (elements loaded in bit-reversed order), two
// stages per pass.
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
    __shared__ long long lbase[kFftMaxLines];
    const int total = lpw * n, half_n = n / 2;
    const long long line0 = (long long)blockIdx.x * lpw;
    for (int l = threadIdx.x; l < lpw; l += blockDim.x) {
        const long long line = line0 + l;
        lbase[l] = (line / A) * B + (line % A) * C;
    }
    __syncthreads();
    auto addr = [&](int l, int s) -> long long { return lbase[l] + (long long)s * S; };
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
        const int l = S == 1 ? e / n : e % lpw, s = S == 1 ? e % n : e / lpw;
        const int r = logn > 0 ? (int)(__brev((unsigned)s) >> (32 - logn)) : 0;
        buf[l * n + r] = Z[addr(l, s)];
    }
    __syncthreads();
    // stages in pairs (len, 2 len): the four elements i, i + half, i + len,
    // i + len + half close under both stages, so a thread takes them through
    // both with one LDS read and write each; a last single stage when logn is
    // odd
    int len = 2;
    for (; 2 * len <= n; len <<= 2) {
        const int half = len >> 1, quarter_n = n / 4;
        for (int b = threadIdx.x; b < lpw * quarter_n; b += blockDim.x) {
            const int l = b / quarter_n, q = b % quarter_n, pos = q % half;
            const int i0 = l * n + (q / half) * (2 * len) + pos;
            double2 w1 = tw[pos * (n / len)], w2 = tw[pos * (n / (2 * len))],
                    w3 = tw[(pos + half) * (n / (2 * len))];
            if (INV) {
                w1.y = -w1.y;
                w2.y = -w2.y;
                w3.y = -w3.y;
            }
            const double2 a0 = buf[i0], a1 = cmul(buf[i0 + half], w1);
            const double2 a2 = buf[i0 + len], a3 = cmul(buf[i0 + len + half], w1);
            // stage len
            const double2 b0 = make_double2(a0.x + a1.x, a0.y + a1.y);
            const double2 b1 = make_double2(a0.x - a1.x, a0.y - a1.y);
            const double2 b2 = make_double2(a2.x + a3.x, a2.y + a3.y);
            const double2 b3 = make_double2(a2.x - a3.x, a2.y - a3.y);
            // stage 2 len: (i0, i0 + len) with w2, (i0 + half, i0 + len + half) with w3
            const double2 c2 = cmul(b2, w2), c3 = cmul(b3, w3);
            buf[i0] = make_double2(b0.x + c2.x, b0.y + c2.y);
            buf[i0 + len] = make_double2(b0.x - c2.x, b0.y - c2.y);
            buf[i0 + half] = make_double2(b1.x + c3.x, b1.y + c3.y);
            buf[i0 + len + half] = make_double2(b1.x - c3.x, b1.y - c3.y);
        }
        __syncthreads();
    }
    if (len <= n) {
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

// triply periodic: mode by mode x = d / (s0 + s1 lambda); with s0 = 0 the
// mean mode is 0
__global__ __launch_bounds__(256) void k_divide(FluidC F, double s0, double s1,
                                                double2 *__restrict__ Z)
{
    {
        const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y, k = blockIdx.z;
        if (i >= F.n[0])
            return;
        const long long c = cell_index(F, i, j, k);
        const double L = s0 + s1 * (lam(i, F.n[0], F.h) + lam(j, F.n[1], F.h) + lam(k, F.n[2], F.h));
        const double2 z = Z[c];
        Z[c] = (c == 0 && s0 == 0.0) ? make_double2(0.0, 0.0) : make_double2(z.x / L, z.y / L);
    }
}

// walls in z: per (kx, ky) mode the system s0 x + s1 (D_z + lambda_xy) x =
// rhs, D_z the second difference (1/h^2)(x_{k+1} - 2 x_k + x_{k-1}) closed
// at the walls by a zero gradient (Neumann, the pressure) or by the ghost
// -x (no slip, the velocity), solved by elimination from the bottom.  The
// Neumann system with s0 = 0 is singular in the (0, 0) mode: its top value
// is pinned to 0, then its z-mean removed (the grid mean of phi).  cp holds
// the eliminated super-diagonal.
__global__ __launch_bounds__(256) void k_tridiag(FluidC F, double s0, double s1, int dirichlet,
                                                 double2 *__restrict__ Z, double *__restrict__ cp)
{
    const int nxy = F.n[0] * F.n[1], nz = F.n[2];
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= nxy)
        return;
    const int i = col % F.n[0], j = col / F.n[0];
    const double ih2 = 1.0 / (F.h * F.h);
    const double lxy = lam(i, F.n[0], F.h) + lam(j, F.n[1], F.h);
    const bool singular = col == 0 && s0 == 0.0 && !dirichlet;
    double cprev = 0.0;
    double2 dprev = make_double2(0.0, 0.0);
    for (int k = 0; k < nz; ++k) {
        const size_t c = (size_t)k * nxy + col;
        const bool lo = k > 0, hi = k < nz - 1;
        const double dz = dirichlet ? -2.0 * ih2 - (lo ? 0.0 : ih2) - (hi ? 0.0 : ih2)
                                    : -((lo ? ih2 : 0.0) + (hi ? ih2 : 0.0));
        double a = lo ? s1 * ih2 : 0.0, sup = hi ? s1 * ih2 : 0.0;
        double b = s0 + s1 * (lxy + dz);
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
    {
        const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y, k = blockIdx.z;
        if (i >= F.n[0])
            return;
        const long long c = cell_index(F, i, j, k);
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

// value of field f at the neighbour (d = +1 / -1 along axis a) of cell c:
// behind a wall the no-slip ghost -f(c)
template <typename T>
__device__ __forceinline__ double nb_noslip(const FluidC &F, const T *f, long long c, int i, int j,
                                            int k, int a, int d)
{
    const long long q = neighbour(F, i, j, k, a, d);
    return q >= 0 ? (double)f[q] : -(double)f[c];
}

// mean of the two face gradients of P along axis a (zero on wall faces)
template <typename T>
__device__ __forceinline__ double cell_grad(const FluidC &F, const T *P, long long c, int i, int j,
                                            int k, int a)
{
    const double pc = (double)P[c];
    const long long up = neighbour(F, i, j, k, a, 1), dn = neighbour(F, i, j, k, a, -1);
    const double gp = up >= 0 ? ((double)P[up] - pc) / F.h : 0.0;
    const double gm = dn >= 0 ? (pc - (double)P[dn]) / F.h : 0.0;
    return 0.5 * (gp + gm);
}

// step a: u~ = u + dt (2 alpha nu L u - 2 alpha grad P - gamma N - zeta N_prev),
// N = (u . grad) u; N holds N_prev on entry and N on exit, lapnu = nu L u.
// A workgroup takes a PX x PY column of cells and marches it up in z: each
// plane of u and P is staged in LDS with a one-cell rim for the x and y
// neighbours, the planes below and above are kept in registers, so each
// value is read from memory about once.
constexpr int PX = 64, PY = 4;

template <typename T>
__global__ __launch_bounds__(PX * PY) void k_predict(FluidC F, const T *__restrict__ u,
                                                     T *__restrict__ ut, T *__restrict__ Nbuf,
                                                     T *__restrict__ lapnu,
                                                     const T *__restrict__ P, double dt,
                                                     double alpha, double gamma, double zeta)
{
    __shared__ double tile[4][PY + 2][PX + 2];
    const long long N = (long long)F.n[0] * F.n[1] * F.n[2];
    const int nx = F.n[0], ny = F.n[1], nz = F.n[2];
    const int tx = threadIdx.x % PX, ty = threadIdx.x / PX;
    const int i0 = blockIdx.x * PX, j0 = blockIdx.y * PY;
    const int i = i0 + tx, j = j0 + ty;
    const bool live = i < nx && j < ny;
    const T *fld[4] = {u, u + N, u + 2 * N, P};
    // value of field q at (i, j, kk) (kk already inside the grid)
    auto at = [&](int q, int ii, int jj, int kk) -> double {
        return (double)fld[q][((long long)kk * ny + jj) * nx + ii];
    };
    double zc[4] = {0, 0, 0, 0}, zn[4] = {0, 0, 0, 0}, zp[4] = {0, 0, 0, 0}, z0[4] = {0, 0, 0, 0};
    if (live)
        for (int q = 0; q < 4; ++q) {
            zc[q] = at(q, i, j, 0);
            z0[q] = zc[q];
            if (F.periodic[2])
                zp[q] = at(q, i, j, nz - 1);
        }
    // the rim-extended plane is loaded into registers one plane ahead
    // (each thread holds up to kPre of its slots), stored to LDS after the
    // previous plane's compute: the loads of plane k + 1 overlap the compute
    // of plane k
    constexpr int kSlots = (PY + 2) * (PX + 2), kPre = (kSlots + PX * PY - 1) / (PX * PY);
    double pre[kPre][4];
    auto load_plane = [&](int kk) {
        for (int r = 0; r < kPre; ++r) {
            const int e = threadIdx.x + r * PX * PY;
            if (e >= kSlots)
                break;
            const int ry = e / (PX + 2), rx = e % (PX + 2);
            int gi = i0 + rx - 1, gj = j0 + ry - 1;
            if (F.periodic[0])
                gi = gi < 0 ? gi + nx : (gi >= nx ? gi - nx : gi);
            if (F.periodic[1])
                gj = gj < 0 ? gj + ny : (gj >= ny ? gj - ny : gj);
            const bool in = gi >= 0 && gi < nx && gj >= 0 && gj < ny;
            for (int q = 0; q < 4; ++q)
                pre[r][q] = in ? at(q, gi, gj, kk) : 0.0;
        }
    };
    load_plane(0);
    for (int k = 0; k < nz; ++k) {
        __syncthreads();
        for (int r = 0; r < kPre; ++r) {
            const int e = threadIdx.x + r * PX * PY;
            if (e >= kSlots)
                break;
            const int ry = e / (PX + 2), rx = e % (PX + 2);
            for (int q = 0; q < 4; ++q)
                tile[q][ry][rx] = pre[r][q];
        }
        __syncthreads();
        const bool has_up = k + 1 < nz, has_dn = k > 0;
        // the plane above at this cell first (needed now), then the prefetch
        if (live)
            for (int q = 0; q < 4; ++q)
                zn[q] = has_up ? at(q, i, j, k + 1) : (F.periodic[2] ? z0[q] : 0.0);
        if (has_up)
            load_plane(k + 1);
        if (!live)
            continue;
        const bool in_xm = F.periodic[0] || i > 0, in_xp = F.periodic[0] || i + 1 < nx;
        const bool in_ym = F.periodic[1] || j > 0, in_yp = F.periodic[1] || j + 1 < ny;
        const bool in_zm = F.periodic[2] || has_dn, in_zp = F.periodic[2] || has_up;
        const long long c = ((long long)k * ny + j) * nx + i;
        double ua[3];
        for (int q = 0; q < 3; ++q)
            ua[q] = zc[q];
        for (int b = 0; b < 3; ++b) {
            // neighbours of component b along x, y, z (no-slip ghost -u behind a wall)
            const double ub = ua[b];
            const double nbr[3][2] = {
                {in_xp ? tile[b][ty + 1][tx + 2] : -ub, in_xm ? tile[b][ty + 1][tx] : -ub},
                {in_yp ? tile[b][ty + 2][tx + 1] : -ub, in_ym ? tile[b][ty][tx + 1] : -ub},
                {in_zp ? zn[b] : -ub, in_zm ? zp[b] : -ub}};
            double lap = 0.0, adv = 0.0;
            for (int a = 0; a < 3; ++a) {
                const double up = nbr[a][0], dn = nbr[a][1];
                lap = lap + (up - 2.0 * ub + dn) / (F.h * F.h);
                adv = adv + ua[a] * ((up - dn) / (2.0 * F.h));
            }
            // pressure gradient along b: mean of the two face gradients
            const double pc = zc[3];
            double pp, pm;
            bool hp, hm;
            if (b == 0) {
                pp = tile[3][ty + 1][tx + 2], pm = tile[3][ty + 1][tx], hp = in_xp, hm = in_xm;
            } else if (b == 1) {
                pp = tile[3][ty + 2][tx + 1], pm = tile[3][ty][tx + 1], hp = in_yp, hm = in_ym;
            } else {
                pp = zn[3], pm = zp[3], hp = in_zp, hm = in_zm;
            }
            const double gp = hp ? (pp - pc) / F.h : 0.0;
            const double gm = hm ? (pc - pm) / F.h : 0.0;
            const double gP = 0.5 * (gp + gm);
            const size_t ib = (size_t)b * N + c;
            const double ln = F.nu * lap;
            const double Np = (double)Nbuf[ib];
            ut[ib] = (T)(ub + dt * (2.0 * alpha * ln - 2.0 * alpha * gP - gamma * adv - zeta * Np));
            Nbuf[ib] = (T)adv;
            lapnu[ib] = (T)ln;
        }
        for (int q = 0; q < 4; ++q) {
            zp[q] = zc[q];
            zc[q] = zn[q];
        }
    }
}

// step e: the right-hand side u_f - c fbar + dt (-alpha lapnu + 2 alpha
// theta grad P) of component b0 into the real part of Z and of component b1
// (if >= 0) into the imaginary part: the operator is real, so one complex
// solve serves both
template <typename T>
__device__ __forceinline__ double helm_rhs(const FluidC &F, const T *u, const T *lapnu, const T *P,
                                           const double *fbar, int b, long long c, int i, int j,
                                           int k, double dt, double alpha)
{
    const long long N = (long long)F.n[0] * F.n[1] * F.n[2];
    const double fb = fbar ? fbar[b] : 0.0;
    const double gP = cell_grad(F, P, c, i, j, k, b);
    return (double)u[(size_t)b * N + c] - F.c * fb +
           dt * (-alpha * (double)lapnu[(size_t)b * N + c] + 2.0 * alpha * F.theta * gP);
}

template <typename T>
__global__ __launch_bounds__(256) void k_helm_rhs(FluidC F, const T *__restrict__ u,
                                                  const T *__restrict__ lapnu,
                                                  const T *__restrict__ P,
                                                  const double *__restrict__ fbar, int b0, int b1,
                                                  double dt, double alpha, double2 *__restrict__ Z)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y, k = blockIdx.z;
    if (i >= F.n[0])
        return;
    const long long c = cell_index(F, i, j, k);
    const double r0 = helm_rhs(F, u, lapnu, P, fbar, b0, c, i, j, k, dt, alpha);
    const double r1 = b1 >= 0 ? helm_rhs(F, u, lapnu, P, fbar, b1, c, i, j, k, dt, alpha) : 0.0;
    Z[c] = make_double2(r0, r1);
}

// the solution: real part into component b0, imaginary part into b1
template <typename T>
__global__ __launch_bounds__(256) void k_take(long long N, const double2 *__restrict__ Z,
                                              double scale, T *__restrict__ out0,
                                              T *__restrict__ out1)
{
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < N;
         c += (long long)gridDim.x * blockDim.x) {
        const double2 z = Z[c];
        out0[c] = (T)(z.x * scale);
        if (out1)
            out1[c] = (T)(z.y * scale);
    }
}

int grid_blocks(long long n) { return (int)(n / 256 + 1 < 16384 ? n / 256 + 1 : 16384); }

// one thread per cell: x along the block, y and z along the grid
struct CellLaunch {
    dim3 grid, block;
};
CellLaunch cells(const FluidC &F)
{
    const int bx = F.n[0] >= 256 ? 256 : ((F.n[0] + 63) / 64) * 64;
    return CellLaunch{dim3((F.n[0] + bx - 1) / bx, F.n[1], F.n[2]), dim3(bx)};
}

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

FluidC fluid_constants(const ibmx_plan p, double theta)
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
    return F;
}

// Z (a right-hand side in the cell layout) -> the solution of (s0 + s1 L) x
// = Z, times the returned scale (the inverse FFTs are unnormalised)
double solve_modes(ibmx_plan p, const FluidC &F, double s0, double s1, int dirichlet,
                   hipStream_t s)
{
    fft_axis<false>(p, F, 0, s);
    fft_axis<false>(p, F, 1, s);
    double scale = 1.0 / ((double)F.n[0] * F.n[1]);
    if (F.periodic[2]) {
        fft_axis<false>(p, F, 2, s);
        hipLaunchKernelGGL(k_divide, cells(F).grid, cells(F).block, 0, s, F, s0, s1, p->fl_z);
        fft_axis<true>(p, F, 2, s);
        scale /= F.n[2];
    } else {
        const int nxy = F.n[0] * F.n[1];
        hipLaunchKernelGGL(k_tridiag, dim3((nxy + 255) / 256), dim3(256), 0, s, F, s0, s1,
                           dirichlet, p->fl_z, p->fl_cp);
    }
    fft_axis<true>(p, F, 1, s);
    fft_axis<true>(p, F, 0, s);
    return scale;
}

template <typename T>
ibmx_status run_project(ibmx_plan p, T *u, T *uf, T *P, T *phi, double theta)
{
    const FluidC F = fluid_constants(p, theta);
    hipStream_t s = p->stream;
    ProfScope ps(p, IBMX_K_OTHER);
    hipLaunchKernelGGL((k_face_div<T>), cells(F).grid, cells(F).block, 0, s, F, (const T *)u, uf,
                       p->fl_z);
    const double scale = solve_modes(p, F, 0.0, 1.0, 0, s);
    hipLaunchKernelGGL((k_correct<T>), cells(F).grid, cells(F).block, 0, s, F,
                       (const double2 *)p->fl_z, scale, u, uf, P, phi);
    return ibmx_launch_check();
}

template <typename T>
ibmx_status run_predict(ibmx_plan p, const T *u, T *ut, T *Nbuf, T *lapnu, const T *P, double dt,
                        double gamma, double zeta)
{
    const FluidC F = fluid_constants(p, 0.0);
    const double alpha = F.c / (2.0 * dt);
    ProfScope ps(p, IBMX_K_OTHER);
    hipLaunchKernelGGL((k_predict<T>), dim3((F.n[0] + PX - 1) / PX, (F.n[1] + PY - 1) / PY),
                       dim3(PX * PY), 0, p->stream, F,
                       u, ut, Nbuf, lapnu, P, dt, alpha, gamma, zeta);
    return ibmx_launch_check();
}

template <typename T>
ibmx_status run_helmholtz(ibmx_plan p, T *u, const T *lapnu, const T *P, const double *fbar,
                          double dt, double theta)
{
    const FluidC F = fluid_constants(p, theta);
    const double alpha = F.c / (2.0 * dt);
    const long long N = p->g.nodes;
    hipStream_t s = p->stream;
    ProfScope ps(p, IBMX_K_OTHER);
    // x and y together, then z
    for (int b0 = 0; b0 < 3; b0 += 2) {
        const int b1 = b0 == 0 ? 1 : -1;
        hipLaunchKernelGGL((k_helm_rhs<T>), cells(F).grid, cells(F).block, 0, s, F, (const T *)u,
                           lapnu, P, fbar, b0, b1, dt, alpha, p->fl_z);
        const double scale = solve_modes(p, F, 1.0, -alpha * dt * F.nu, 1, s);
        hipLaunchKernelGGL((k_take<T>), dim3(grid_blocks(N)), dim3(256), 0, s, N,
                           (const double2 *)p->fl_z, scale, u + (size_t)b0 * N,
                           b1 >= 0 ? u + (size_t)b1 * N : (T *)nullptr);
    }
    return ibmx_launch_check();
}

bool solver_grid_ok(const ibmx_grid &g)
{
    return g.periodic[0] && g.periodic[1] && pow2(g.n[0]) && pow2(g.n[1]) && g.n[0] <= 1024 &&
           g.n[1] <= 1024 && (!g.periodic[2] || (pow2(g.n[2]) && g.n[2] <= 1024));
}

// workspace: the complex grid, the elimination scratch (walls in z) and
// one twiddle table per axis
ibmx_status fluid_reserve(ibmx_plan p)
{
    const size_t N = (size_t)p->g.nodes;
    if (!p->fl_z && hipMalloc((void **)&p->fl_z, sizeof(double2) * N) != hipSuccess) {
        p->fl_z = nullptr;
        return IBMX_ENOMEM;
    }
    if (!p->grid.periodic[2] && !p->fl_cp &&
        hipMalloc((void **)&p->fl_cp, sizeof(double) * N) != hipSuccess) {
        p->fl_cp = nullptr;
        return IBMX_ENOMEM;
    }
    for (int a = 0; a < 3; ++a) {
        if (p->fl_tw[a])
            continue;
        const int n = p->grid.n[a];
        std::vector<double2> tw((size_t)(n / 2 > 0 ? n / 2 : 1));
        for (int m = 0; m < n / 2; ++m) {
            const double ang = -2.0 * M_PI * (double)m / (double)n;
            tw[m] = make_double2(cos(ang), sin(ang));
        }
        double2 *d = nullptr;
        if (hipMalloc((void **)&d, sizeof(double2) * tw.size()) != hipSuccess)
            return IBMX_ENOMEM;
        if (hipMemcpy(d, tw.data(), sizeof(double2) * tw.size(), hipMemcpyHostToDevice) !=
            hipSuccess) {
            (void)hipFree(d);
            return IBMX_EDEVICE;
        }
        p->fl_tw[a] = d;
    }
    return IBMX_OK;
}

}  // namespace

extern "C" ibmx_status ibmx_project(ibmx_plan p, void *u, void *uf, void *P, void *phi,
                                    double theta)
{
    if (!p || !u || !uf || !P || !isfinite(theta))
        return IBMX_EINVAL;
    if (!solver_grid_ok(p->grid))
        return IBMX_EUNSUPPORTED;
    const ibmx_status st = fluid_reserve(p);
    if (st != IBMX_OK)
        return st;
    if (p->prec == IBMX_F64)
        return run_project<double>(p, (double *)u, (double *)uf, (double *)P, (double *)phi, theta);
    return run_project<float>(p, (float *)u, (float *)uf, (float *)P, (float *)phi, theta);
}

extern "C" ibmx_status ibmx_fluid_predictor(ibmx_plan p, const void *u, void *u_out, void *N,
                                            void *lapnu, const void *P, double dt, double gamma,
                                            double zeta)
{
    if (!p || !u || !u_out || !N || !lapnu || !P || u == u_out || !(dt > 0.0) ||
        !isfinite(gamma) || !isfinite(zeta))
        return IBMX_EINVAL;
    if (p->prec == IBMX_F64)
        return run_predict<double>(p, (const double *)u, (double *)u_out, (double *)N,
                                   (double *)lapnu, (const double *)P, dt, gamma, zeta);
    return run_predict<float>(p, (const float *)u, (float *)u_out, (float *)N, (float *)lapnu,
                              (const float *)P, dt, gamma, zeta);
}

extern "C" ibmx_status ibmx_fluid_helmholtz(ibmx_plan p, void *u, const void *lapnu, const void *P,
                                            const double *fbar, double dt, double theta)
{
    if (!p || !u || !lapnu || !P || !(dt > 0.0) || !isfinite(theta))
        return IBMX_EINVAL;
    if (!solver_grid_ok(p->grid))
        return IBMX_EUNSUPPORTED;
    const ibmx_status st = fluid_reserve(p);
    if (st != IBMX_OK)
        return st;
    if (p->prec == IBMX_F64)
        return run_helmholtz<double>(p, (double *)u, (const double *)lapnu, (const double *)P, fbar,
                                     dt, theta);
    return run_helmholtz<float>(p, (float *)u, (const float *)lapnu, (const float *)P, fbar, dt,
                                theta);
}
