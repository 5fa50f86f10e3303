// The collocated fluid solver's steps around the forcing loop (Sec. 2.2.1
// and eq. fluid-solver): the predictor (step a), the implicit viscous step
// (step e) and the pressure projection (steps f-i: face interpolation,
// compact Poisson equation, cell and face corrections, pressure update).
//
// Both implicit systems, (I - beta L) u* = r per velocity component and the
// compact Poisson equation L phi = div(u_f*) / c, are solved directly in
// FP64 for a real right-hand side: a real-to-complex FFT along x (the
// nx/2 + 1 modes of each row), complex FFTs along y (and z when periodic,
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
constexpr int kRowElems = 256;      // complex elements per workgroup in the x passes
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
// right-hand side div(u_f*) / c
template <typename T>
__global__ __launch_bounds__(256) void k_face_div(FluidC F, const T *__restrict__ u,
                                                  T *__restrict__ uf, double *__restrict__ R)
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
        R[c] = div / F.c;
    }
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ int log2i_dev(int n)
{
    int l = 0;
    while ((1 << l) < n)
        ++l;
    return l;
}

// In-place complex FFT of `lines` lines of length n = 2^logn held in LDS in
// bit-reversed order: iterative radix-2 Cooley-Tukey, two stages per pass
// (the four elements i, i + half, i + len, i + len + half close under both
// stages), a last single stage when logn is odd.  w(m) = tw[m * ts] =
// exp(-2 pi i m / n); INV uses the conjugate (no 1/n scaling).
template <bool INV>
__device__ void fft_lds(double2 *buf, int n, int lines, const double2 *__restrict__ tw, int ts)
{
    const int half_n = n / 2;
    auto w = [&](int m) {
        double2 v = tw[(size_t)m * ts];
        if (INV)
            v.y = -v.y;
        return v;
    };
    int len = 2;
    for (; 2 * len <= n; len <<= 2) {
        const int half = len >> 1, quarter_n = n / 4;
        for (int b = threadIdx.x; b < lines * quarter_n; b += blockDim.x) {
            const int l = b / quarter_n, q = b % quarter_n, pos = q % half;
            const int i0 = l * n + (q / half) * (2 * len) + pos;
            const double2 w1 = w(pos * (n / len)), w2 = w(pos * (n / (2 * len))),
                          w3 = w((pos + half) * (n / (2 * len)));
            const double2 a0 = buf[i0], a1 = cmul(buf[i0 + half], w1);
            const double2 a2 = buf[i0 + len], a3 = cmul(buf[i0 + len + half], w1);
            const double2 b0 = make_double2(a0.x + a1.x, a0.y + a1.y);
            const double2 b1 = make_double2(a0.x - a1.x, a0.y - a1.y);
            const double2 b2 = make_double2(a2.x + a3.x, a2.y + a3.y);
            const double2 b3 = make_double2(a2.x - a3.x, a2.y - a3.y);
            const double2 c2 = cmul(b2, w2), c3 = cmul(b3, w3);
            buf[i0] = make_double2(b0.x + c2.x, b0.y + c2.y);
            buf[i0 + len] = make_double2(b0.x - c2.x, b0.y - c2.y);
            buf[i0 + half] = make_double2(b1.x + c3.x, b1.y + c3.y);
            buf[i0 + len + half] = make_double2(b1.x - c3.x, b1.y - c3.y);
        }
        __syncthreads();
    }
    if (len <= n) {
        const int half = len >> 1;
        for (int b = threadIdx.x; b < lines * half_n; b += blockDim.x) {
            const int l = b / half_n, jj = b % half_n, pos = jj % half;
            const int i0 = l * n + (jj / half) * len + pos, i1 = i0 + half;
            const double2 wk = w(pos * (n / len));
            const double2 v0 = buf[i0], v1 = cmul(buf[i1], wk);
            buf[i0] = make_double2(v0.x + v1.x, v0.y + v1.y);
            buf[i1] = make_double2(v0.x - v1.x, v0.y - v1.y);
        }
        __syncthreads();
    }
}

__device__ __forceinline__ int bitrev(int s, int logn)
{
    return logn > 0 ? (int)(__brev((unsigned)s) >> (32 - logn)) : 0;
}

// Real-to-complex transform of rows along x (nx = 2 N2): each row's values
// r[2m] + i r[2m + 1] form N2 complex values whose FFT Z gives the row's
// modes X[k] = (Z[k] + Z*[N2 - k])/2 - i w^k (Z[k] - Z*[N2 - k])/2, k = 0..N2,
// w = exp(-2 pi i / nx); H holds N2 + 1 modes per row.  `rows` rows per
// workgroup.
__global__ __launch_bounds__(kFftThreads) void k_rfft_x(const double *__restrict__ R,
                                                        double2 *__restrict__ H, int nx, int rows,
                                                        long long nrows,
                                                        const double2 *__restrict__ tw)
{
    extern __shared__ double2 buf[];
    const int N2 = nx / 2, logn = log2i_dev(N2), mx = N2 + 1;
    const long long row0 = (long long)blockIdx.x * rows;
    const int nr = (int)(nrows - row0 < rows ? nrows - row0 : rows);
    const double2 *Rc = reinterpret_cast<const double2 *>(R);
    for (int e = threadIdx.x; e < nr * N2; e += blockDim.x) {
        const int l = e / N2, m = e % N2;
        buf[l * N2 + bitrev(m, logn)] = Rc[(row0 + l) * N2 + m];
    }
    __syncthreads();
    fft_lds<false>(buf, N2, nr, tw, 2);
    for (int e = threadIdx.x; e < nr * mx; e += blockDim.x) {
        const int l = e / mx, k = e % mx;
        const double2 zk = buf[l * N2 + (k == N2 ? 0 : k)];
        const double2 zc = buf[l * N2 + (k == 0 ? 0 : N2 - k)];
        const double2 sum = make_double2(0.5 * (zk.x + zc.x), 0.5 * (zk.y - zc.y));
        const double2 dif = make_double2(0.5 * (zk.x - zc.x), 0.5 * (zk.y + zc.y));
        // -i w^k dif, w^k = tw[k] of the nx-point table (k <= N2: its last entry
        // is -1 = w^(nx/2))
        const double2 wk = k < N2 ? tw[k] : make_double2(-1.0, 0.0);
        const double2 t = cmul(wk, dif);
        H[(row0 + l) * mx + k] = make_double2(sum.x + t.y, sum.y - t.x);
    }
}

// Complex-to-real inverse of k_rfft_x (unnormalised: the rows come back
// multiplied by N2): Z[k] = E + i O with E = (X[k] + X*[N2 - k])/2 and O =
// (X[k] - X*[N2 - k]) w^-k / 2, inverse FFT, r[2m] = Re z[m], r[2m + 1] =
// Im z[m].
__global__ __launch_bounds__(kFftThreads) void k_irfft_x(const double2 *__restrict__ H,
                                                         double *__restrict__ R, int nx, int rows,
                                                         long long nrows,
                                                         const double2 *__restrict__ tw)
{
    extern __shared__ double2 buf[];
    const int N2 = nx / 2, logn = log2i_dev(N2), mx = N2 + 1;
    const long long row0 = (long long)blockIdx.x * rows;
    const int nr = (int)(nrows - row0 < rows ? nrows - row0 : rows);
    for (int e = threadIdx.x; e < nr * N2; e += blockDim.x) {
        const int l = e / N2, k = e % N2;
        const double2 xk = H[(row0 + l) * mx + k];
        const double2 xc = H[(row0 + l) * mx + (N2 - k)];
        const double2 E = make_double2(0.5 * (xk.x + xc.x), 0.5 * (xk.y - xc.y));
        const double2 D = make_double2(0.5 * (xk.x - xc.x), 0.5 * (xk.y + xc.y));
        double2 wk = tw[k];
        wk.y = -wk.y;
        const double2 O = cmul(D, wk);
        buf[l * N2 + bitrev(k, logn)] = make_double2(E.x - O.y, E.y + O.x);
    }
    __syncthreads();
    fft_lds<true>(buf, N2, nr, tw, 2);
    double2 *Rc = reinterpret_cast<double2 *>(R);
    for (int e = threadIdx.x; e < nr * N2; e += blockDim.x) {
        const int l = e / N2, m = e % N2;
        Rc[(row0 + l) * N2 + m] = buf[l * N2 + m];
    }
}

// Complex FFT along a strided axis: each plane holds `A` lines, line a of
// plane q starting at q * B + a * C with element stride S; a workgroup takes
// up to `lpw` consecutive lines of one plane (fewer at the plane's end) and
// loads them element-major, so a wave reads lpw contiguous values per row.
template <bool INV>
__global__ __launch_bounds__(kFftThreads) void k_fft_strided(double2 *__restrict__ Z, int n,
                                                             int lpw, int A, long long B,
                                                             long long C, long long S,
                                                             const double2 *__restrict__ tw)
{
    extern __shared__ double2 buf[];
    const int logn = log2i_dev(n);
    const int groups = (A + lpw - 1) / lpw;
    const long long q = blockIdx.x / groups;
    const int a0 = (int)(blockIdx.x % groups) * lpw;
    const int nl = A - a0 < lpw ? A - a0 : lpw;
    const long long base = q * B + (long long)a0 * C;
    for (int e = threadIdx.x; e < nl * n; e += blockDim.x) {
        const int l = e % nl, sidx = e / nl;
        buf[l * n + bitrev(sidx, logn)] = Z[base + l * C + sidx * S];
    }
    __syncthreads();
    fft_lds<INV>(buf, n, nl, tw, 1);
    for (int e = threadIdx.x; e < nl * n; e += blockDim.x) {
        const int l = e % nl, sidx = e / nl;
        Z[base + l * C + sidx * S] = buf[l * n + sidx];
    }
}

// eigenvalue of the periodic second difference for mode m of n points
__device__ __forceinline__ double lam(int m, int n, double h)
{
    return (2.0 * cospi(2.0 * m / (double)n) - 2.0) / (h * h);
}

// triply periodic: mode by mode x = d / (s0 + s1 lambda) over the modes
// kx = 0 .. nx/2 held for real fields; with s0 = 0 the mean mode is 0
__global__ __launch_bounds__(256) void k_divide(FluidC F, double s0, double s1,
                                                double2 *__restrict__ Z)
{
    const int mx = F.n[0] / 2 + 1;
    {
        const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y, k = blockIdx.z;
        if (i >= mx)
            return;
        const long long c = ((long long)k * F.n[1] + j) * mx + i;
        const double L = s0 + s1 * (lam(i, F.n[0], F.h) + lam(j, F.n[1], F.h) + lam(k, F.n[2], F.h));
        const double2 z = Z[c];
        Z[c] = (c == 0 && s0 == 0.0) ? make_double2(0.0, 0.0) : make_double2(z.x / L, z.y / L);
    }
}

// walls in z: per (kx, ky) mode (kx = 0 .. nx/2) the system s0 x + s1 (D_z + lambda_xy) x =
// rhs, D_z the second difference (1/h^2)(x_{k+1} - 2 x_k + x_{k-1}) closed
// at the walls by a zero gradient (Neumann, the pressure) or by the ghost
// -x (no slip, the velocity), solved by elimination from the bottom.  The
// Neumann system with s0 = 0 is singular in the (0, 0) mode: its top value
// is pinned to 0, then its z-mean removed (the grid mean of phi).  cp holds
// the eliminated super-diagonal.
__global__ __launch_bounds__(256) void k_tridiag(FluidC F, double s0, double s1, int dirichlet,
                                                 double2 *__restrict__ Z, double *__restrict__ cp)
{
    const int mx = F.n[0] / 2 + 1, nxy = mx * F.n[1], nz = F.n[2];
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= nxy)
        return;
    const int i = col % mx, j = col / mx;
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

// phi = R * scale; u = u* - c grad(phi) (mean of the cell's two face
// gradients), u_f = u_f* - c (phi_+ - phi)/h, P = (1 - theta) P + phi -
// (c/2) nu L phi
template <typename T>
__global__ __launch_bounds__(256) void k_correct(FluidC F, const double *__restrict__ Z,
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
        const double ph = Z[c] * scale;
        double lap = 0.0;
        for (int a = 0; a < 3; ++a) {
            const long long up = neighbour(F, i, j, k, a, 1), dn = neighbour(F, i, j, k, a, -1);
            const double gp = up >= 0 ? (Z[up] * scale - ph) / F.h : 0.0;
            const double gm = dn >= 0 ? (ph - Z[dn] * scale) / F.h : 0.0;
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
// A workgroup takes a PX x PY column of cells over a run of kPlanes planes
// and marches it up in z.  Each plane of u and P, with a one-cell rim for the
// x and y neighbours, goes through a ring of kRing planes in LDS: while plane
// k is computed from planes k - 1, k and k + 1, plane k + 2 is loaded into
// registers (and N_prev of plane k + 1), so each value is read from memory
// about once (a run adds one plane at each end).  With four slots the store
// of plane k + 1 cannot meet a read of the slot it reuses (last read while
// computing plane k - 2), so one barrier per plane suffices.
constexpr int PX = 64, PY = 4, kPlanes = 32, kRing = 4;

template <typename T>
__global__ __launch_bounds__(PX * PY) void k_predict(FluidC F, const T *__restrict__ u,
                                                     T *__restrict__ ut, T *__restrict__ Nbuf,
                                                     T *__restrict__ lapnu,
                                                     const T *__restrict__ P, double dt,
                                                     double alpha, double gamma, double zeta)
{
    // values are held in T and widened to double where they are used
    __shared__ T tile[kRing][4][PY + 2][PX + 2];
    const long long N = (long long)F.n[0] * F.n[1] * F.n[2];
    const int nx = F.n[0], ny = F.n[1], nz = F.n[2];
    const int tx = threadIdx.x % PX, ty = threadIdx.x / PX;
    const int i0 = blockIdx.x * PX, j0 = blockIdx.y * PY;
    const int k0 = blockIdx.z * kPlanes, k1 = min(nz, k0 + kPlanes);
    const int i = i0 + tx, j = j0 + ty;
    const bool live = i < nx && j < ny;
    const T *fld[4] = {u, u + N, u + 2 * N, P};
    // plane above / below kk, -1 behind a wall
    auto z_up = [&](int kk) { return kk + 1 < nz ? kk + 1 : (F.periodic[2] ? 0 : -1); };
    auto z_dn = [&](int kk) { return kk > 0 ? kk - 1 : (F.periodic[2] ? nz - 1 : -1); };
    // ring slot of plane kk (kk >= k0 - 1)
    auto slot = [&](int kk) { return (kk - k0 + 1) & (kRing - 1); };
    constexpr int kSlots = (PY + 2) * (PX + 2), kPre = (kSlots + PX * PY - 1) / (PX * PY);
    T pre[kPre][4];
    // the rim-extended plane kk into registers (zeros behind a wall, kk < 0)
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
            const bool in = kk >= 0 && gi >= 0 && gi < nx && gj >= 0 && gj < ny;
            const long long o = ((long long)kk * ny + gj) * nx + gi;
            for (int q = 0; q < 4; ++q)
                pre[r][q] = in ? fld[q][o] : T(0);
        }
    };
    auto store_plane = [&](int sl) {
        for (int r = 0; r < kPre; ++r) {
            const int e = threadIdx.x + r * PX * PY;
            if (e >= kSlots)
                break;
            const int ry = e / (PX + 2), rx = e % (PX + 2);
            for (int q = 0; q < 4; ++q)
                tile[sl][q][ry][rx] = pre[r][q];
        }
    };
    // N_prev of the own cell on plane kk
    auto own_n = [&](T *v, int kk) {
        const long long c = ((long long)kk * ny + j) * nx + i;
        for (int b = 0; b < 3; ++b)
            v[b] = live ? Nbuf[(size_t)b * N + c] : T(0);
    };
    T Np[3], Nq[3] = {0, 0, 0};
    load_plane(z_dn(k0));
    store_plane(slot(k0 - 1));
    load_plane(k0);
    store_plane(slot(k0));
    load_plane(z_up(k0));
    own_n(Np, k0);
    const bool in_xm = F.periodic[0] || i > 0, in_xp = F.periodic[0] || i + 1 < nx;
    const bool in_ym = F.periodic[1] || j > 0, in_yp = F.periodic[1] || j + 1 < ny;
    for (int k = k0; k < k1; ++k) {
        store_plane(slot(k + 1));
        __syncthreads();
        if (k + 1 < k1) {
            load_plane(z_up(k + 1));
            own_n(Nq, k + 1);
        }
        if (live) {
            const bool in_zm = z_dn(k) >= 0, in_zp = z_up(k) >= 0;
            const int sd = slot(k - 1), sc = slot(k), su = slot(k + 1);
            const long long c = ((long long)k * ny + j) * nx + i;
            double ua[3];
            for (int q = 0; q < 3; ++q)
                ua[q] = (double)tile[sc][q][ty + 1][tx + 1];
            for (int b = 0; b < 3; ++b) {
                // neighbours of component b along x, y, z (no-slip ghost -u
                // behind a wall)
                const double ub = ua[b];
                const double nbr[3][2] = {
                    {in_xp ? (double)tile[sc][b][ty + 1][tx + 2] : -ub,
                     in_xm ? (double)tile[sc][b][ty + 1][tx] : -ub},
                    {in_yp ? (double)tile[sc][b][ty + 2][tx + 1] : -ub,
                     in_ym ? (double)tile[sc][b][ty][tx + 1] : -ub},
                    {in_zp ? (double)tile[su][b][ty + 1][tx + 1] : -ub,
                     in_zm ? (double)tile[sd][b][ty + 1][tx + 1] : -ub}};
                double lap = 0.0, adv = 0.0;
                for (int a = 0; a < 3; ++a) {
                    const double up = nbr[a][0], dn = nbr[a][1];
                    lap = lap + (up - 2.0 * ub + dn) / (F.h * F.h);
                    adv = adv + ua[a] * ((up - dn) / (2.0 * F.h));
                }
                // pressure gradient along b: mean of the two face gradients
                const double pc = (double)tile[sc][3][ty + 1][tx + 1];
                double pp, pm;
                bool hp, hm;
                if (b == 0) {
                    pp = tile[sc][3][ty + 1][tx + 2], pm = tile[sc][3][ty + 1][tx];
                    hp = in_xp, hm = in_xm;
                } else if (b == 1) {
                    pp = tile[sc][3][ty + 2][tx + 1], pm = tile[sc][3][ty][tx + 1];
                    hp = in_yp, hm = in_ym;
                } else {
                    pp = tile[su][3][ty + 1][tx + 1], pm = tile[sd][3][ty + 1][tx + 1];
                    hp = in_zp, hm = in_zm;
                }
                const double gp = hp ? (pp - pc) / F.h : 0.0;
                const double gm = hm ? (pc - pm) / F.h : 0.0;
                const double gP = 0.5 * (gp + gm);
                const size_t ib = (size_t)b * N + c;
                const double ln = F.nu * lap;
                ut[ib] = (T)(ub + dt * (2.0 * alpha * ln - 2.0 * alpha * gP - gamma * adv -
                                        zeta * (double)Np[b]));
                Nbuf[ib] = (T)adv;
                lapnu[ib] = (T)ln;
            }
        }
        for (int b = 0; b < 3; ++b)
            Np[b] = Nq[b];
    }
}

// step e, component b: the right-hand side u_f - c fbar + dt (-alpha lapnu
// + 2 alpha theta grad P) into R
template <typename T>
__global__ __launch_bounds__(256) void k_helm_rhs(FluidC F, const T *__restrict__ u,
                                                  const T *__restrict__ lapnu,
                                                  const T *__restrict__ P,
                                                  const double *__restrict__ fbar, int b,
                                                  double dt, double alpha, double *__restrict__ R)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y, k = blockIdx.z;
    if (i >= F.n[0])
        return;
    const long long N = (long long)F.n[0] * F.n[1] * F.n[2];
    const long long c = cell_index(F, i, j, k);
    const double fb = fbar ? fbar[b] : 0.0;
    const double gP = cell_grad(F, P, c, i, j, k, b);
    R[c] = (double)u[(size_t)b * N + c] - F.c * fb +
           dt * (-alpha * (double)lapnu[(size_t)b * N + c] + 2.0 * alpha * F.theta * gP);
}

// the solution R * scale into out
template <typename T>
__global__ __launch_bounds__(256) void k_take(long long N, const double *__restrict__ R,
                                              double scale, T *__restrict__ out)
{
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < N;
         c += (long long)gridDim.x * blockDim.x)
        out[c] = (T)(R[c] * scale);
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


// strided complex FFT along y (a = 1) or z (a = 2) over the half spectrum
// (nx/2 + 1 columns)
template <bool INV>
void fft_strided(ibmx_plan p, const FluidC &F, int a, hipStream_t s)
{
    const int mx = F.n[0] / 2 + 1, ny = F.n[1], nz = F.n[2], n = F.n[a];
    int A;
    long long B, S, planes;
    if (a == 1) {
        A = mx, B = (long long)mx * ny, S = mx, planes = nz;
    } else {
        A = mx * ny, B = 0, S = (long long)mx * ny, planes = 1;
    }
    int lpw = n >= kFftElemsStrided ? 1 : kFftElemsStrided / n;
    if (lpw > A)
        lpw = A;
    const long long blocks = planes * ((A + lpw - 1) / lpw);
    hipLaunchKernelGGL((k_fft_strided<INV>), dim3((unsigned)blocks), dim3(kFftThreads),
                       sizeof(double2) * (size_t)lpw * n, s, p->fl_z, n, lpw, A, B, 1LL, S,
                       (const double2 *)p->fl_tw[a]);
}

// rows along x: forward real-to-complex from fl_r into fl_z, or back
template <bool INV>
void fft_rows(ibmx_plan p, const FluidC &F, hipStream_t s)
{
    const int N2 = F.n[0] / 2;
    const long long nrows = (long long)F.n[1] * F.n[2];
    const int rows = N2 >= kRowElems ? 1 : kRowElems / N2;
    const unsigned blocks = (unsigned)((nrows + rows - 1) / rows);
    const size_t lds = sizeof(double2) * (size_t)rows * N2;
    if (INV)
        hipLaunchKernelGGL(k_irfft_x, dim3(blocks), dim3(kFftThreads), lds, s,
                           (const double2 *)p->fl_z, p->fl_r, F.n[0], rows, nrows,
                           (const double2 *)p->fl_tw[0]);
    else
        hipLaunchKernelGGL(k_rfft_x, dim3(blocks), dim3(kFftThreads), lds, s,
                           (const double *)p->fl_r, p->fl_z, F.n[0], rows, nrows,
                           (const double2 *)p->fl_tw[0]);
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

// fl_r (a real right-hand side in the cell layout) -> the solution of
// (s0 + s1 L) x = r in fl_r, times the returned scale (the inverse passes
// are unnormalised)
double solve_modes(ibmx_plan p, const FluidC &F, double s0, double s1, int dirichlet,
                   hipStream_t s)
{
    const int mx = F.n[0] / 2 + 1;
    fft_rows<false>(p, F, s);
    fft_strided<false>(p, F, 1, s);
    double scale = 1.0 / ((double)(F.n[0] / 2) * F.n[1]);
    if (F.periodic[2]) {
        fft_strided<false>(p, F, 2, s);
        hipLaunchKernelGGL(k_divide, dim3((mx + 255) / 256, F.n[1], F.n[2]), dim3(256), 0, s, F,
                           s0, s1, p->fl_z);
        fft_strided<true>(p, F, 2, s);
        scale /= F.n[2];
    } else {
        const int nxy = mx * F.n[1];
        hipLaunchKernelGGL(k_tridiag, dim3((nxy + 255) / 256), dim3(256), 0, s, F, s0, s1,
                           dirichlet, p->fl_z, p->fl_cp);
    }
    fft_strided<true>(p, F, 1, s);
    fft_rows<true>(p, F, s);
    return scale;
}

template <typename T>
ibmx_status run_project(ibmx_plan p, T *u, T *uf, T *P, T *phi, double theta)
{
    const FluidC F = fluid_constants(p, theta);
    hipStream_t s = p->stream;
    ProfScope ps(p, IBMX_K_OTHER);
    hipLaunchKernelGGL((k_face_div<T>), cells(F).grid, cells(F).block, 0, s, F, (const T *)u, uf,
                       p->fl_r);
    const double scale = solve_modes(p, F, 0.0, 1.0, 0, s);
    hipLaunchKernelGGL((k_correct<T>), cells(F).grid, cells(F).block, 0, s, F,
                       (const double *)p->fl_r, scale, u, uf, P, phi);
    return ibmx_launch_check();
}

template <typename T>
ibmx_status run_predict(ibmx_plan p, const T *u, T *ut, T *Nbuf, T *lapnu, const T *P, double dt,
                        double gamma, double zeta)
{
    const FluidC F = fluid_constants(p, 0.0);
    const double alpha = F.c / (2.0 * dt);
    ProfScope ps(p, IBMX_K_OTHER);
    hipLaunchKernelGGL((k_predict<T>),
                       dim3((F.n[0] + PX - 1) / PX, (F.n[1] + PY - 1) / PY,
                            (F.n[2] + kPlanes - 1) / kPlanes),
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
    for (int b = 0; b < 3; ++b) {
        hipLaunchKernelGGL((k_helm_rhs<T>), cells(F).grid, cells(F).block, 0, s, F, (const T *)u,
                           lapnu, P, fbar, b, dt, alpha, p->fl_r);
        const double scale = solve_modes(p, F, 1.0, -alpha * dt * F.nu, 1, s);
        hipLaunchKernelGGL((k_take<T>), dim3(grid_blocks(N)), dim3(256), 0, s, N,
                           (const double *)p->fl_r, scale, u + (size_t)b * N);
    }
    return ibmx_launch_check();
}

bool solver_grid_ok(const ibmx_grid &g)
{
    return g.periodic[0] && g.periodic[1] && pow2(g.n[0]) && pow2(g.n[1]) && g.n[0] <= 1024 &&
           g.n[1] <= 1024 && (!g.periodic[2] || (pow2(g.n[2]) && g.n[2] <= 1024));
}

// workspace: the real right-hand side / solution grid, the half spectrum
// (nx/2 + 1 modes along x), the elimination scratch (walls in z) and one
// twiddle table per axis
ibmx_status fluid_reserve(ibmx_plan p)
{
    const size_t N = (size_t)p->g.nodes;
    const size_t M = (size_t)(p->grid.n[0] / 2 + 1) * p->grid.n[1] * p->grid.n[2];
    if (!p->fl_r && hipMalloc((void **)&p->fl_r, sizeof(double) * N) != hipSuccess) {
        p->fl_r = nullptr;
        return IBMX_ENOMEM;
    }
    if (!p->fl_z && hipMalloc((void **)&p->fl_z, sizeof(double2) * M) != hipSuccess) {
        p->fl_z = nullptr;
        return IBMX_ENOMEM;
    }
    if (!p->grid.periodic[2] && !p->fl_cp &&
        hipMalloc((void **)&p->fl_cp, sizeof(double) * M) != hipSuccess) {
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
