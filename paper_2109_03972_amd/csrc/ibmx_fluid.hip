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
// elimination across the walls in z.  The half spectrum is stored with y
// fastest, mode (kx, y, z) at (z (nx/2 + 1) + kx) ny + y, so that the y
// passes read whole contiguous lines and the x passes, taking 8 or more
// consecutive rows per workgroup, read and write runs of consecutive y.  FFTs
// are radix-2 passes in place in LDS, several lines per workgroup.  The
// stencil kernels march columns of cells up in z through a ring of planes in
// LDS.
#include <math.h>
#include <vector>

#include "ibmx_internal.hpp"

namespace {

constexpr int kFftThreads = 256;
constexpr int kRowElems = 256;      // complex elements per workgroup in the x passes
constexpr int kMinRows = 8;         // and at least this many rows
constexpr int kFftElemsStrided = 1024;   // y and z lines: 16 KB of LDS, 2 lines of 512

struct FluidC {
    int n[3];
    int periodic[3];
    double h, c, nu, theta;
    double ih, ih2, i2h, ic;   // 1/h, 1/h^2, 1/(2h), 1/c: the stencils multiply
};

// index of cell (i, j, k) (a plan's grid has fewer than 2^31 cells)
__device__ __forceinline__ unsigned cell32(const FluidC &F, int i, int j, int k)
{
    return ((unsigned)k * (unsigned)F.n[1] + (unsigned)j) * (unsigned)F.n[0] + (unsigned)i;
}

// element i of a field: with O32 (every field spans less than 4 GB) a 32-bit
// byte offset from the field's uniform base, which the loads and stores take
// as is; otherwise a 64-bit index
template <bool O32, typename T>
__device__ __forceinline__ T &fat(T *base, unsigned i)
{
    if (O32)
        return *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + i * (unsigned)sizeof(T));
    return base[(size_t)i];
}
template <bool O32, typename T>
__device__ __forceinline__ const T &fat(const T *base, unsigned i)
{
    if (O32)
        return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) +
                                            i * (unsigned)sizeof(T));
    return base[(size_t)i];
}

// Stencil kernels that need neighbours in all three axes march a PX x PY
// column of cells up in z over a run of kPlanes planes.  The fields' planes,
// with a one-cell rim for the x and y neighbours, pass through a ring of
// kRing planes in LDS: plane k + 1 is stored, then, while plane k is
// computed from planes k - 1, k and k + 1, plane k + 2 is loaded into
// registers, so each value is read from memory about once (a run adds one
// plane at each end).  With four slots the store of plane k + 1 cannot meet
// a read of the slot it reuses (last read while computing plane k - 2), so
// one barrier per plane suffices.
constexpr int PX = 64, PY = 4, kPlanes = 32, kRing = 4;

// plane above / below kk, -1 behind a wall
__device__ __forceinline__ int z_up(const FluidC &F, int kk)
{
    return kk + 1 < F.n[2] ? kk + 1 : (F.periodic[2] ? 0 : -1);
}
__device__ __forceinline__ int z_dn(const FluidC &F, int kk)
{
    return kk > 0 ? kk - 1 : (F.periodic[2] ? F.n[2] - 1 : -1);
}

struct Column {
    int tx, ty, i0, j0, k0, k1, i, j;
    bool live;
    bool in_p[2], in_m[2];   // x and y neighbours inside the grid (or periodic)
    __device__ explicit Column(const FluidC &F)
    {
        tx = threadIdx.x % PX, ty = threadIdx.x / PX;
        i0 = blockIdx.x * PX, j0 = blockIdx.y * PY;
        k0 = blockIdx.z * kPlanes, k1 = min(F.n[2], k0 + kPlanes);
        i = i0 + tx, j = j0 + ty;
        live = i < F.n[0] && j < F.n[1];
        in_m[0] = F.periodic[0] || i > 0, in_p[0] = F.periodic[0] || i + 1 < F.n[0];
        in_m[1] = F.periodic[1] || j > 0, in_p[1] = F.periodic[1] || j + 1 < F.n[1];
    }
    // ring slot of plane kk (kk >= k0 - 1)
    __device__ int slot(int kk) const { return (kk - k0 + 1) & (kRing - 1); }
};

// NF fields of one rim-extended plane, in registers between the load from
// memory and the store into a ring slot; zeros outside the grid (kk < 0 is
// the plane behind a wall)
template <typename T, int NF, bool O32>
struct PlaneStage {
    static constexpr int kSlots = (PY + 2) * (PX + 2), kPre = (kSlots + PX * PY - 1) / (PX * PY);
    T pre[kPre][NF];
    __device__ void load(const FluidC &F, const T *const *fld, const Column &col, int kk)
    {
        const int nx = F.n[0], ny = F.n[1];
        for (int r = 0; r < kPre; ++r) {
            const int e = threadIdx.x + r * PX * PY;
            if (e >= kSlots)
                break;
            const int ry = e / (PX + 2), rx = e % (PX + 2);
            int gi = col.i0 + rx - 1, gj = col.j0 + ry - 1;
            if (F.periodic[0])
                gi = gi < 0 ? gi + nx : (gi >= nx ? gi - nx : gi);
            if (F.periodic[1])
                gj = gj < 0 ? gj + ny : (gj >= ny ? gj - ny : gj);
            const bool in = kk >= 0 && gi >= 0 && gi < nx && gj >= 0 && gj < ny;
            const unsigned o = ((unsigned)kk * (unsigned)ny + (unsigned)gj) * (unsigned)nx + (unsigned)gi;
            for (int q = 0; q < NF; ++q)
                pre[r][q] = in ? fat<O32>(fld[q], o) : T(0);
        }
    }
    __device__ void store(T (*ring)[NF][PY + 2][PX + 2], int sl) const
    {
        for (int r = 0; r < kPre; ++r) {
            const int e = threadIdx.x + r * PX * PY;
            if (e >= kSlots)
                break;
            const int ry = e / (PX + 2), rx = e % (PX + 2);
            for (int q = 0; q < NF; ++q)
                ring[sl][q][ry][rx] = pre[r][q];
        }
    }
    // fill slots of planes k0 - 1 and k0, leave plane k0 + 1 in registers
    __device__ void prologue(const FluidC &F, const T *const *fld, const Column &col,
                             T (*ring)[NF][PY + 2][PX + 2])
    {
        load(F, fld, col, z_dn(F, col.k0));
        store(ring, col.slot(col.k0 - 1));
        load(F, fld, col, col.k0);
        store(ring, col.slot(col.k0));
        load(F, fld, col, z_up(F, col.k0));
    }
};

// the value of field q at the own cell's neighbour along axis a (d = +1 /
// -1) from the ring (sd, sc, su: slots of planes k - 1, k, k + 1)
template <typename T, int NF>
__device__ __forceinline__ T ring_nb(const T (*ring)[NF][PY + 2][PX + 2], const Column &col,
                                     int sd, int sc, int su, int q, int a, int d)
{
    if (a == 0)
        return ring[sc][q][col.ty + 1][col.tx + 1 + d];
    if (a == 1)
        return ring[sc][q][col.ty + 1 + d][col.tx + 1];
    return ring[d > 0 ? su : sd][q][col.ty + 1][col.tx + 1];
}

dim3 column_grid(const FluidC &F)
{
    return dim3((F.n[0] + PX - 1) / PX, (F.n[1] + PY - 1) / PY, (F.n[2] + kPlanes - 1) / kPlanes);
}

// u_f* = mean of the two cells of each +a face (wall faces 0), and the
// right-hand side div(u_f*) / c
template <typename T, bool O32>
__global__ __launch_bounds__(PX * PY) void k_face_div(FluidC F, const T *__restrict__ u,
                                                      T *__restrict__ uf, double *__restrict__ R)
{
    __shared__ T ring[kRing][3][PY + 2][PX + 2];
    const long long N = (long long)F.n[0] * F.n[1] * F.n[2];
    const Column col(F);
    const T *fld[3] = {u, u + N, u + 2 * N};
    T *const ufb[3] = {uf, uf + N, uf + 2 * N};
    PlaneStage<T, 3, O32> st;
    st.prologue(F, fld, col, ring);
    for (int k = col.k0; k < col.k1; ++k) {
        st.store(ring, col.slot(k + 1));
        __syncthreads();
        if (k + 1 < col.k1)
            st.load(F, fld, col, z_up(F, k + 1));
        if (!col.live)
            continue;
        const int sd = col.slot(k - 1), sc = col.slot(k), su = col.slot(k + 1);
        const bool in_p[3] = {col.in_p[0], col.in_p[1], z_up(F, k) >= 0};
        const bool in_m[3] = {col.in_m[0], col.in_m[1], z_dn(F, k) >= 0};
        const unsigned c = cell32(F, col.i, col.j, k);
        double div = 0.0;
        for (int a = 0; a < 3; ++a) {
            const double uc = (double)ring[sc][a][col.ty + 1][col.tx + 1];
            const double out =
                in_p[a] ? 0.5 * (uc + (double)ring_nb<T, 3>(ring, col, sd, sc, su, a, a, 1))
                        : 0.0;
            const double in =
                in_m[a] ? 0.5 * ((double)ring_nb<T, 3>(ring, col, sd, sc, su, a, a, -1) + uc)
                        : 0.0;
            fat<O32>(ufb[a], c) = (T)out;
            div = div + (out - in) * F.ih;
        }
        fat<O32>(R, c) = div * F.ic;
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

// LDS lines are padded by one element every 16: element j of a line sits at
// pad16(j), so that the bit-reversed stores and the short-span butterflies,
// whose addresses are multiples of large powers of two apart, spread over the
// banks; a line of n elements takes plen(n).
__host__ __device__ __forceinline__ int pad16(int j) { return j + (j >> 4); }
__host__ __device__ __forceinline__ int plen(int n) { return n + (n >> 4); }

// In-place complex FFT of `lines` lines of length n = 2^logn held in LDS in
// bit-reversed order, line l at buf + l * ls: iterative radix-2 Cooley-Tukey,
// two stages per pass (the four elements i, i + half, i + len, i + len + half
// close under both stages), a last single stage when logn is odd.  w(m) =
// tw[m * ts] = exp(-2 pi i m / n); INV uses the conjugate (no 1/n scaling).
template <bool INV>
__device__ void fft_lds(double2 *buf, int n, int ls, int lines, const double2 *__restrict__ tw,
                        int ts)
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
            const int j0 = (q / half) * (2 * len) + pos;
            double2 *lb = buf + l * ls;
            const int p0 = pad16(j0), p1 = pad16(j0 + half), p2 = pad16(j0 + len),
                      p3 = pad16(j0 + len + half);
            const double2 w1 = w(pos * (n / len)), w2 = w(pos * (n / (2 * len))),
                          w3 = w((pos + half) * (n / (2 * len)));
            const double2 a0 = lb[p0], a1 = cmul(lb[p1], w1);
            const double2 a2 = lb[p2], a3 = cmul(lb[p3], w1);
            const double2 b0 = make_double2(a0.x + a1.x, a0.y + a1.y);
            const double2 b1 = make_double2(a0.x - a1.x, a0.y - a1.y);
            const double2 b2 = make_double2(a2.x + a3.x, a2.y + a3.y);
            const double2 b3 = make_double2(a2.x - a3.x, a2.y - a3.y);
            const double2 c2 = cmul(b2, w2), c3 = cmul(b3, w3);
            lb[p0] = make_double2(b0.x + c2.x, b0.y + c2.y);
            lb[p2] = make_double2(b0.x - c2.x, b0.y - c2.y);
            lb[p1] = make_double2(b1.x + c3.x, b1.y + c3.y);
            lb[p3] = make_double2(b1.x - c3.x, b1.y - c3.y);
        }
        __syncthreads();
    }
    if (len <= n) {
        const int half = len >> 1;
        for (int b = threadIdx.x; b < lines * half_n; b += blockDim.x) {
            const int l = b / half_n, jj = b % half_n, pos = jj % half;
            const int j0 = (jj / half) * len + pos;
            double2 *lb = buf + l * ls;
            const int p0 = pad16(j0), p1 = pad16(j0 + half);
            const double2 wk = w(pos * (n / len));
            const double2 v0 = lb[p0], v1 = cmul(lb[p1], wk);
            lb[p0] = make_double2(v0.x + v1.x, v0.y + v1.y);
            lb[p1] = make_double2(v0.x - v1.x, v0.y - v1.y);
        }
        __syncthreads();
    }
}

__device__ __forceinline__ int bitrev(int s, int logn)
{
    return logn > 0 ? (int)(__brev((unsigned)s) >> (32 - logn)) : 0;
}

// What the x passes read and write, as pairs of consecutive real values
// (complex index m = real index / 2): the FP64 real grid, or (forward) the
// implicit step's right-hand side of one component without a pressure term,
// computed from u and nu L u as it is read, or (inverse) the solution scaled
// and rounded into the caller's field (caller fields are accessed by
// element: they need only the alignment of T).

struct RealIn {
    const double *R;
    __device__ void prepare() {}
    __device__ double2 operator()(long long m) const { return reinterpret_cast<const double2 *>(R)[m]; }
};

template <typename T>
struct HelmRhsIn {
    const T *u, *lapnu;
    const double *fbar;   // device double[3] or NULL
    int b;
    double c, dt, alpha, fb;
    __device__ void prepare() { fb = fbar ? fbar[b] : 0.0; }
    __device__ double2 operator()(long long m) const
    {
        const long long r = 2 * m;
        return make_double2((double)u[r] - c * fb + dt * (-alpha * (double)lapnu[r]),
                            (double)u[r + 1] - c * fb + dt * (-alpha * (double)lapnu[r + 1]));
    }
};

struct RealOut {
    double *R;
    __device__ void operator()(long long m, double2 v) const { reinterpret_cast<double2 *>(R)[m] = v; }
};

template <typename T>
struct ScaledOut {
    T *out;
    double scale;
    __device__ void operator()(long long m, double2 v) const
    {
        out[2 * m] = (T)(v.x * scale);
        out[2 * m + 1] = (T)(v.y * scale);
    }
};

// Real-to-complex transform of rows along x (nx = 2 N2): each row's values
// r[2m] + i r[2m + 1] form N2 complex values whose FFT Z gives the row's
// modes X[k] = (Z[k] + Z*[N2 - k])/2 - i w^k (Z[k] - Z*[N2 - k])/2, k = 0..N2,
// w = exp(-2 pi i / nx).  `rows` consecutive rows per workgroup (row r = z ny
// + y), held in LDS with a stride of plen(N2) + 1; the modes go out
// y-fastest, mode k of row r at (z mx + k) ny + y, consecutive threads taking
// consecutive rows.
template <class Src>
__global__ __launch_bounds__(kFftThreads) void k_rfft_x(Src src, double2 *__restrict__ H, int nx,
                                                        int logny, int rows, long long nrows,
                                                        const double2 *__restrict__ tw)
{
    extern __shared__ double2 buf[];
    const int N2 = nx / 2, logn = log2i_dev(N2), mx = N2 + 1, ls = plen(N2) + 1;
    const long long row0 = (long long)blockIdx.x * rows;
    const int nr = (int)(nrows - row0 < rows ? nrows - row0 : rows);
    const long long ymask = (1LL << logny) - 1;
    // the first N2 entries of the nx-point table, after the rows
    double2 *twl = buf + (size_t)rows * ls;
    for (int e = threadIdx.x; e < N2; e += blockDim.x)
        twl[e] = tw[e];
    src.prepare();
    for (int e = threadIdx.x; e < nr * N2; e += blockDim.x) {
        const int l = e >> logn, m = e & (N2 - 1);
        buf[l * ls + pad16(bitrev(m, logn))] = src(row0 * N2 + e);
    }
    __syncthreads();
    fft_lds<false>(buf, N2, ls, nr, twl, 2);
    for (int e = threadIdx.x; e < nr * mx; e += blockDim.x) {
        const int k = e / nr, l = e - k * nr;
        const double2 zk = buf[l * ls + pad16(k == N2 ? 0 : k)];
        const double2 zc = buf[l * ls + pad16(k == 0 ? 0 : N2 - k)];
        const double2 sum = make_double2(0.5 * (zk.x + zc.x), 0.5 * (zk.y - zc.y));
        const double2 dif = make_double2(0.5 * (zk.x - zc.x), 0.5 * (zk.y + zc.y));
        // -i w^k dif, w^k = tw[k] of the nx-point table (k <= N2: its last entry
        // is -1 = w^(nx/2))
        const double2 wk = k < N2 ? twl[k] : make_double2(-1.0, 0.0);
        const double2 t = cmul(wk, dif);
        const long long r = row0 + l, z = r >> logny, y = r & ymask;
        H[((z * mx + k) << logny) + y] = make_double2(sum.x + t.y, sum.y - t.x);
    }
}

// Complex-to-real inverse of k_rfft_x (unnormalised: the rows come back
// multiplied by N2): Z[k] = E + i O with E = (X[k] + X*[N2 - k])/2 and O =
// (X[k] - X*[N2 - k]) w^-k / 2, inverse FFT, r[2m] = Re z[m], r[2m + 1] =
// Im z[m].  Modes are read y-fastest as k_rfft_x writes them.
template <class Dst>
__global__ __launch_bounds__(kFftThreads) void k_irfft_x(const double2 *__restrict__ H, Dst dst,
                                                         int nx, int logny, int rows,
                                                         long long nrows,
                                                         const double2 *__restrict__ tw)
{
    extern __shared__ double2 buf[];
    const int N2 = nx / 2, logn = log2i_dev(N2), mx = N2 + 1, ls = plen(N2) + 1;
    const long long row0 = (long long)blockIdx.x * rows;
    const int nr = (int)(nrows - row0 < rows ? nrows - row0 : rows);
    const long long ymask = (1LL << logny) - 1;
    double2 *twl = buf + (size_t)rows * ls;
    for (int e = threadIdx.x; e < N2; e += blockDim.x)
        twl[e] = tw[e];
    for (int e = threadIdx.x; e < nr * N2; e += blockDim.x) {
        const int k = e / nr, l = e - k * nr;
        const long long r = row0 + l, z = r >> logny, y = r & ymask;
        const long long base = ((z * mx) << logny) + y;
        const double2 xk = H[base + ((long long)k << logny)];
        const double2 xc = H[base + ((long long)(N2 - k) << logny)];
        const double2 E = make_double2(0.5 * (xk.x + xc.x), 0.5 * (xk.y - xc.y));
        const double2 D = make_double2(0.5 * (xk.x - xc.x), 0.5 * (xk.y + xc.y));
        double2 wk = tw[k];
        wk.y = -wk.y;
        const double2 O = cmul(D, wk);
        buf[l * ls + pad16(bitrev(k, logn))] = make_double2(E.x - O.y, E.y + O.x);
    }
    __syncthreads();
    fft_lds<true>(buf, N2, ls, nr, twl, 2);
    for (int e = threadIdx.x; e < nr * N2; e += blockDim.x) {
        const int l = e >> logn, m = e & (N2 - 1);
        dst(row0 * N2 + e, buf[l * ls + pad16(m)]);
    }
}

// Complex FFT of contiguous lines of n values (line L at Z + L n): a
// workgroup takes lpw consecutive lines (fewer at the end), read and written
// in memory order.
template <bool INV>
__global__ __launch_bounds__(kFftThreads) void k_fft_lines(double2 *__restrict__ Z, int n,
                                                           int lpw, long long nlines,
                                                           const double2 *__restrict__ tw)
{
    extern __shared__ double2 buf[];
    const int logn = log2i_dev(n);
    const long long L0 = (long long)blockIdx.x * lpw;
    const int nl = (int)(nlines - L0 < lpw ? nlines - L0 : lpw);
    double2 *Zb = Z + L0 * n;
    const int ls = plen(n);
    // the n/2 twiddles the transform uses, after the lines
    double2 *twl = buf + (size_t)lpw * ls;
    for (int e = threadIdx.x; e < n / 2; e += blockDim.x)
        twl[e] = tw[e];
    for (int e = threadIdx.x; e < nl * n; e += blockDim.x)
        buf[(e >> logn) * ls + pad16(bitrev(e & (n - 1), logn))] = Zb[e];
    __syncthreads();
    fft_lds<INV>(buf, n, ls, nl, twl, 1);
    for (int e = threadIdx.x; e < nl * n; e += blockDim.x)
        Zb[e] = buf[(e >> logn) * ls + pad16(e & (n - 1))];
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
    const int ls = plen(n);
    double2 *twl = buf + (size_t)lpw * ls;
    for (int e = threadIdx.x; e < n / 2; e += blockDim.x)
        twl[e] = tw[e];
    for (int e = threadIdx.x; e < nl * n; e += blockDim.x) {
        const int l = e % nl, sidx = e / nl;
        buf[l * ls + pad16(bitrev(sidx, logn))] = Z[base + l * C + sidx * S];
    }
    __syncthreads();
    fft_lds<INV>(buf, n, ls, nl, twl, 1);
    for (int e = threadIdx.x; e < nl * n; e += blockDim.x) {
        const int l = e % nl, sidx = e / nl;
        Z[base + l * C + sidx * S] = buf[l * ls + pad16(sidx)];
    }
}

// eigenvalue of the periodic second difference for mode m of n points
__device__ __forceinline__ double lam(int m, int n, double h)
{
    return (2.0 * cospi(2.0 * m / (double)n) - 2.0) / (h * h);
}

// triply periodic: mode by mode x = d / (s0 + s1 lambda) over the modes
// kx = 0 .. nx/2 held for real fields (y fastest); with s0 = 0 the mean mode
// is 0
__global__ __launch_bounds__(256) void k_divide(FluidC F, double s0, double s1,
                                                double2 *__restrict__ Z)
{
    const int mx = F.n[0] / 2 + 1;
    {
        const int j = blockIdx.x * blockDim.x + threadIdx.x, i = blockIdx.y, k = blockIdx.z;
        if (j >= F.n[1])
            return;
        const long long c = ((long long)k * mx + i) * F.n[1] + j;
        const double L = s0 + s1 * (lam(i, F.n[0], F.h) + lam(j, F.n[1], F.h) + lam(k, F.n[2], F.h));
        const double2 z = Z[c];
        Z[c] = (c == 0 && s0 == 0.0) ? make_double2(0.0, 0.0) : make_double2(z.x / L, z.y / L);
    }
}

// walls in z: per (kx, ky) mode (kx = 0 .. nx/2; modes y-fastest) the system
// s0 x + s1 (D_z + lambda_xy) x = rhs, D_z the second difference
// (1/h^2)(x_{k+1} - 2 x_k + x_{k-1}) closed
// at the walls by a zero gradient (Neumann, the pressure) or by the ghost
// -x (no slip, the velocity), solved by elimination from the bottom.  The
// Neumann system with s0 = 0 is singular in the (0, 0) mode: its top value
// is pinned to 0, then its z-mean removed (the grid mean of phi).  cp holds
// the eliminated super-diagonal.  The interior rows have the same
// coefficients, so once the eliminated super-diagonal repeats exactly on an
// interior row it keeps that value up to the last interior row: it is stored
// only up to there and the back substitution takes the constant beyond.
__global__ __launch_bounds__(256) void k_tridiag(FluidC F, double s0, double s1, int dirichlet,
                                                 double2 *__restrict__ Z, double *__restrict__ cp)
{
    const int mx = F.n[0] / 2 + 1, nxy = mx * F.n[1], nz = F.n[2];
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= nxy)
        return;
    const int i = col / F.n[1], j = col % F.n[1];
    const double ih2 = 1.0 / (F.h * F.h);
    const double lxy = lam(i, F.n[0], F.h) + lam(j, F.n[1], F.h);
    const bool singular = col == 0 && s0 == 0.0 && !dirichlet;
    double cprev = 0.0, cconv = 0.0;
    int kconv = nz;   // first row of the constant super-diagonal
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
        const double cnew = sup / den;
        dprev = make_double2((d.x - a * dprev.x) / den, (d.y - a * dprev.y) / den);
        if (k < kconv) {
            cp[c] = cnew;
            if (k >= 2 && k <= nz - 2 && cnew == cprev) {
                kconv = k;
                cconv = cnew;
            }
        }
        cprev = cnew;
        Z[c] = dprev;
    }
    double2 x = dprev;
    double2 sum = x;
    for (int k = nz - 2; k >= 0; --k) {
        const size_t c = (size_t)k * nxy + col;
        const double2 d = Z[c];
        const double ck = k > kconv ? cconv : cp[c];
        x = make_double2(d.x - ck * x.x, d.y - ck * x.y);
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
// (c/2) nu L phi.  phi passes through the plane ring; the own cell's u,
// u_f and P of the next plane are loaded while a plane is computed.
template <typename T, bool O32>
__global__ __launch_bounds__(PX * PY) void k_correct(FluidC F, const double *__restrict__ Z,
                                                     double scale, T *__restrict__ u,
                                                     T *__restrict__ uf, T *__restrict__ P,
                                                     T *__restrict__ phi_out)
{
    __shared__ double ring[kRing][1][PY + 2][PX + 2];
    const long long N = (long long)F.n[0] * F.n[1] * F.n[2];
    const Column col(F);
    const double *fld[1] = {Z};
    T *const ub[3] = {u, u + N, u + 2 * N}, *const ufb[3] = {uf, uf + N, uf + 2 * N};
    PlaneStage<double, 1, O32> st;
    st.prologue(F, fld, col, ring);
    // own u (3), u_f (3) and P of plane kk
    auto own = [&](T *v, int kk) {
        const unsigned c = cell32(F, col.i, col.j, kk);
        for (int a = 0; a < 3; ++a) {
            v[a] = col.live ? fat<O32>(ub[a], c) : T(0);
            v[3 + a] = col.live ? fat<O32>(ufb[a], c) : T(0);
        }
        v[6] = col.live ? fat<O32>(P, c) : T(0);
    };
    T ow[7], oq[7] = {0, 0, 0, 0, 0, 0, 0};
    own(ow, col.k0);
    for (int k = col.k0; k < col.k1; ++k) {
        st.store(ring, col.slot(k + 1));
        __syncthreads();
        if (k + 1 < col.k1) {
            st.load(F, fld, col, z_up(F, k + 1));
            own(oq, k + 1);
        }
        if (col.live) {
            const int sd = col.slot(k - 1), sc = col.slot(k), su = col.slot(k + 1);
            const bool in_p[3] = {col.in_p[0], col.in_p[1], z_up(F, k) >= 0};
            const bool in_m[3] = {col.in_m[0], col.in_m[1], z_dn(F, k) >= 0};
            const unsigned c = cell32(F, col.i, col.j, k);
            const double ph = ring[sc][0][col.ty + 1][col.tx + 1] * scale;
            double lap = 0.0;
            for (int a = 0; a < 3; ++a) {
                const double gp =
                    in_p[a] ? (ring_nb<double, 1>(ring, col, sd, sc, su, 0, a, 1) * scale - ph) * F.ih
                            : 0.0;
                const double gm =
                    in_m[a] ? (ph - ring_nb<double, 1>(ring, col, sd, sc, su, 0, a, -1) * scale) * F.ih
                            : 0.0;
                fat<O32>(ub[a], c) = (T)((double)ow[a] - F.c * (0.5 * (gp + gm)));
                fat<O32>(ufb[a], c) = (T)((double)ow[3 + a] - F.c * gp);
                lap = lap + (gp - gm) * F.ih;
            }
            fat<O32>(P, c) = (T)((1.0 - F.theta) * (double)ow[6] + ph - 0.5 * F.c * F.nu * lap);
            if (phi_out)
                fat<O32>(phi_out, c) = (T)ph;
        }
        for (int q = 0; q < 7; ++q)
            ow[q] = oq[q];
    }
}

// step a: u~ = u + dt (2 alpha nu L u - 2 alpha grad P - gamma N - zeta N_prev),
// N = (u . grad) u; N holds N_prev on entry and N on exit, lapnu = nu L u.
// u and P pass through the plane ring (values held in T, widened to double
// where they are used); N_prev of the next plane is loaded while a plane is
// computed.
template <typename T, bool O32>
__global__ __launch_bounds__(PX * PY) void k_predict(FluidC F, const T *__restrict__ u,
                                                     T *__restrict__ ut, T *__restrict__ Nbuf,
                                                     T *__restrict__ lapnu,
                                                     const T *__restrict__ P, double dt,
                                                     double alpha, double gamma, double zeta)
{
    __shared__ T ring[kRing][4][PY + 2][PX + 2];
    const long long N = (long long)F.n[0] * F.n[1] * F.n[2];
    const Column col(F);
    const T *fld[4] = {u, u + N, u + 2 * N, P};
    T *const nb[3] = {Nbuf, Nbuf + N, Nbuf + 2 * N};
    T *const utb[3] = {ut, ut + N, ut + 2 * N}, *const lb[3] = {lapnu, lapnu + N, lapnu + 2 * N};
    PlaneStage<T, 4, O32> st;
    st.prologue(F, fld, col, ring);
    // N_prev of the own cell on plane kk
    auto own_n = [&](T *v, int kk) {
        const unsigned c = cell32(F, col.i, col.j, kk);
        for (int b = 0; b < 3; ++b)
            v[b] = col.live ? fat<O32>(nb[b], c) : T(0);
    };
    T Np[3], Nq[3] = {0, 0, 0};
    own_n(Np, col.k0);
    for (int k = col.k0; k < col.k1; ++k) {
        st.store(ring, col.slot(k + 1));
        __syncthreads();
        if (k + 1 < col.k1) {
            st.load(F, fld, col, z_up(F, k + 1));
            own_n(Nq, k + 1);
        }
        if (col.live) {
            const int sd = col.slot(k - 1), sc = col.slot(k), su = col.slot(k + 1);
            const bool in_p[3] = {col.in_p[0], col.in_p[1], z_up(F, k) >= 0};
            const bool in_m[3] = {col.in_m[0], col.in_m[1], z_dn(F, k) >= 0};
            const unsigned c = cell32(F, col.i, col.j, k);
            double ua[3];
            for (int q = 0; q < 3; ++q)
                ua[q] = (double)ring[sc][q][col.ty + 1][col.tx + 1];
            const double pc = (double)ring[sc][3][col.ty + 1][col.tx + 1];
            for (int b = 0; b < 3; ++b) {
                // neighbours of component b (no-slip ghost -u behind a wall)
                const double ub = ua[b];
                double lap = 0.0, adv = 0.0;
                for (int a = 0; a < 3; ++a) {
                    const double up =
                        in_p[a] ? (double)ring_nb<T, 4>(ring, col, sd, sc, su, b, a, 1) : -ub;
                    const double dn =
                        in_m[a] ? (double)ring_nb<T, 4>(ring, col, sd, sc, su, b, a, -1) : -ub;
                    lap = lap + (up - 2.0 * ub + dn) * F.ih2;
                    adv = adv + ua[a] * ((up - dn) * F.i2h);
                }
                // pressure gradient along b: mean of the two face gradients
                const double gp =
                    in_p[b] ? ((double)ring_nb<T, 4>(ring, col, sd, sc, su, 3, b, 1) - pc) * F.ih
                            : 0.0;
                const double gm =
                    in_m[b] ? (pc - (double)ring_nb<T, 4>(ring, col, sd, sc, su, 3, b, -1)) * F.ih
                            : 0.0;
                const double gP = 0.5 * (gp + gm);
                const double ln = F.nu * lap;
                fat<O32>(utb[b], c) = (T)(ub + dt * (2.0 * alpha * ln - 2.0 * alpha * gP -
                                                     gamma * adv - zeta * (double)Np[b]));
                fat<O32>(nb[b], c) = (T)adv;
                fat<O32>(lb[b], c) = (T)ln;
            }
        }
        for (int b = 0; b < 3; ++b)
            Np[b] = Nq[b];
    }
}

// step e, component b: the right-hand side u_f - c fbar + dt (-alpha lapnu
// + 2 alpha theta grad P) into R, P through the plane ring, the own u_f and
// lapnu of the next plane loaded while a plane is computed.  (With theta = 0
// there is no pressure term and the x pass computes the right-hand side as
// it reads: HelmRhsIn.)
template <typename T, bool O32>
__global__ __launch_bounds__(PX * PY) void k_helm_rhs(FluidC F, const T *__restrict__ u,
                                                      const T *__restrict__ lapnu,
                                                      const T *__restrict__ P,
                                                      const double *__restrict__ fbar, int b,
                                                      double dt, double alpha,
                                                      double *__restrict__ R)
{
    __shared__ T ring[kRing][1][PY + 2][PX + 2];
    const long long N = (long long)F.n[0] * F.n[1] * F.n[2];
    const Column col(F);
    const T *fld[1] = {P};
    PlaneStage<T, 1, O32> st;
    st.prologue(F, fld, col, ring);
    const T *ub = u + (size_t)b * N, *lb = lapnu + (size_t)b * N;
    auto own = [&](T *v, int kk) {
        const unsigned c = cell32(F, col.i, col.j, kk);
        v[0] = col.live ? fat<O32>(ub, c) : T(0);
        v[1] = col.live ? fat<O32>(lb, c) : T(0);
    };
    const double fb = fbar ? fbar[b] : 0.0;
    T ow[2], oq[2] = {0, 0};
    own(ow, col.k0);
    for (int k = col.k0; k < col.k1; ++k) {
        st.store(ring, col.slot(k + 1));
        __syncthreads();
        if (k + 1 < col.k1) {
            st.load(F, fld, col, z_up(F, k + 1));
            own(oq, k + 1);
        }
        if (col.live) {
            const int sd = col.slot(k - 1), sc = col.slot(k), su = col.slot(k + 1);
            const bool hp = b < 2 ? col.in_p[b] : z_up(F, k) >= 0;
            const bool hm = b < 2 ? col.in_m[b] : z_dn(F, k) >= 0;
            const double pc = (double)ring[sc][0][col.ty + 1][col.tx + 1];
            // mean of the two face gradients along b (zero on wall faces)
            const double gp =
                hp ? ((double)ring_nb<T, 1>(ring, col, sd, sc, su, 0, b, 1) - pc) * F.ih : 0.0;
            const double gm =
                hm ? (pc - (double)ring_nb<T, 1>(ring, col, sd, sc, su, 0, b, -1)) * F.ih : 0.0;
            const double gP = 0.5 * (gp + gm);
            fat<O32>(R, cell32(F, col.i, col.j, k)) =
                (double)ow[0] - F.c * fb +
                dt * (-alpha * (double)ow[1] + 2.0 * alpha * F.theta * gP);
        }
        ow[0] = oq[0];
        ow[1] = oq[1];
    }
}


bool pow2(int n) { return n >= 2 && (n & (n - 1)) == 0; }


// complex FFT over the half spectrum along y (a = 1: contiguous lines) or
// along z (a = 2: lines of stride mx ny, consecutive lines adjacent)
template <bool INV>
void fft_axis(ibmx_plan p, const FluidC &F, int a, hipStream_t s)
{
    const int mx = F.n[0] / 2 + 1, ny = F.n[1], nz = F.n[2], n = F.n[a];
    int lpw = n >= kFftElemsStrided ? 1 : kFftElemsStrided / n;
    if (a == 1) {
        const long long nlines = (long long)mx * nz;
        if (lpw > nlines)
            lpw = (int)nlines;
        hipLaunchKernelGGL((k_fft_lines<INV>), dim3((unsigned)((nlines + lpw - 1) / lpw)),
                           dim3(kFftThreads), sizeof(double2) * ((size_t)lpw * plen(n) + n / 2), s, p->fl_z, n,
                           lpw, nlines, (const double2 *)p->fl_tw[1]);
        return;
    }
    const int A = mx * ny;
    if (lpw > A)
        lpw = A;
    hipLaunchKernelGGL((k_fft_strided<INV>), dim3((unsigned)((A + lpw - 1) / lpw)),
                       dim3(kFftThreads), sizeof(double2) * ((size_t)lpw * plen(n) + n / 2), s, p->fl_z, n, lpw,
                       A, 0LL, 1LL, (long long)A, (const double2 *)p->fl_tw[2]);
}

// rows along x: forward real-to-complex from src into fl_z, or back into dst
struct RowLaunch {
    int rows, logny;
    unsigned blocks;
    size_t lds;
    long long nrows;
};
RowLaunch row_launch(const FluidC &F)
{
    const int N2 = F.n[0] / 2;
    RowLaunch r;
    r.nrows = (long long)F.n[1] * F.n[2];
    // at least kMinRows rows (each mode's writes cover that many consecutive
    // y), within 64 KB of LDS with the N2 twiddles
    r.rows = N2 * kMinRows >= kRowElems ? kMinRows : kRowElems / N2;
    const int fit = (int)((65536 / sizeof(double2) - N2) / (plen(N2) + 1));
    if (r.rows > fit)
        r.rows = fit;
    r.blocks = (unsigned)((r.nrows + r.rows - 1) / r.rows);
    r.lds = sizeof(double2) * ((size_t)r.rows * (plen(N2) + 1) + N2);
    r.logny = 0;
    while ((1 << r.logny) < F.n[1])
        ++r.logny;
    return r;
}

template <class Src>
void rows_forward(ibmx_plan p, const FluidC &F, Src src, hipStream_t s)
{
    const RowLaunch r = row_launch(F);
    hipLaunchKernelGGL((k_rfft_x<Src>), dim3(r.blocks), dim3(kFftThreads), r.lds, s, src, p->fl_z,
                       F.n[0], r.logny, r.rows, r.nrows, (const double2 *)p->fl_tw[0]);
}

template <class Dst>
void rows_inverse(ibmx_plan p, const FluidC &F, Dst dst, hipStream_t s)
{
    const RowLaunch r = row_launch(F);
    hipLaunchKernelGGL((k_irfft_x<Dst>), dim3(r.blocks), dim3(kFftThreads), r.lds, s,
                       (const double2 *)p->fl_z, dst, F.n[0], r.logny, r.rows, r.nrows,
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
    F.ih = 1.0 / g.h;
    F.ih2 = 1.0 / (g.h * g.h);
    F.i2h = 1.0 / (2.0 * g.h);
    F.c = p->prm.two_alpha_dt;
    F.ic = 1.0 / F.c;
    F.nu = p->prm.nu_f;
    F.theta = theta;
    return F;
}

// the half spectrum in fl_z (after rows_forward) -> that of the solution of
// (s0 + s1 L) x = r (before rows_inverse); the passes are unnormalised, the
// result comes back multiplied by 1 / spectrum_scale
void solve_spectrum(ibmx_plan p, const FluidC &F, double s0, double s1, int dirichlet,
                    hipStream_t s)
{
    const int mx = F.n[0] / 2 + 1;
    fft_axis<false>(p, F, 1, s);
    if (F.periodic[2]) {
        fft_axis<false>(p, F, 2, s);
        hipLaunchKernelGGL(k_divide, dim3((F.n[1] + 255) / 256, mx, F.n[2]), dim3(256), 0, s, F,
                           s0, s1, p->fl_z);
        fft_axis<true>(p, F, 2, s);
    } else {
        const int nxy = mx * F.n[1];
        hipLaunchKernelGGL(k_tridiag, dim3((nxy + 255) / 256), dim3(256), 0, s, F, s0, s1,
                           dirichlet, p->fl_z, p->fl_cp);
    }
    fft_axis<true>(p, F, 1, s);
}

double spectrum_scale(const FluidC &F)
{
    double scale = 1.0 / ((double)(F.n[0] / 2) * F.n[1]);
    if (F.periodic[2])
        scale /= F.n[2];
    return scale;
}

// stencil kernels with 32-bit field offsets when every field (the FP64 real
// grid included) spans less than 4 GB
bool fields32(const FluidC &F)
{
    return (unsigned long long)F.n[0] * F.n[1] * F.n[2] * sizeof(double) < (1ULL << 32);
}

#define IBMX_STENCIL_LAUNCH(K, T, F, s, ...)                                                     \
    do {                                                                                        \
        if (fields32(F))                                                                         \
            hipLaunchKernelGGL((K<T, true>), column_grid(F), dim3(PX * PY), 0, s, F, __VA_ARGS__);  \
        else                                                                                     \
            hipLaunchKernelGGL((K<T, false>), column_grid(F), dim3(PX * PY), 0, s, F, __VA_ARGS__); \
    } while (0)

template <typename T>
ibmx_status run_project(ibmx_plan p, T *u, T *uf, T *P, T *phi, double theta)
{
    const FluidC F = fluid_constants(p, theta);
    hipStream_t s = p->stream;
    ProfScope ps(p, IBMX_K_OTHER);
    IBMX_STENCIL_LAUNCH(k_face_div, T, F, s, (const T *)u, uf, p->fl_r);
    rows_forward(p, F, RealIn{p->fl_r}, s);
    solve_spectrum(p, F, 0.0, 1.0, 0, s);
    rows_inverse(p, F, RealOut{p->fl_r}, s);
    IBMX_STENCIL_LAUNCH(k_correct, T, F, s, (const double *)p->fl_r, spectrum_scale(F), u, uf, P,
                        phi);
    return ibmx_launch_check();
}

template <typename T>
ibmx_status run_predict(ibmx_plan p, const T *u, T *ut, T *Nbuf, T *lapnu, const T *P, double dt,
                        double gamma, double zeta)
{
    const FluidC F = fluid_constants(p, 0.0);
    const double alpha = F.c / (2.0 * dt);
    ProfScope ps(p, IBMX_K_OTHER);
    IBMX_STENCIL_LAUNCH(k_predict, T, F, p->stream, u, ut, Nbuf, lapnu, P, dt, alpha, gamma, zeta);
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
        // the right-hand side: with a pressure term through the plane ring
        // into the real grid, without it computed by the x pass as it reads
        if (F.theta != 0.0) {
            IBMX_STENCIL_LAUNCH(k_helm_rhs, T, F, s, (const T *)u, lapnu, P, fbar, b, dt, alpha,
                                p->fl_r);
            rows_forward(p, F, RealIn{p->fl_r}, s);
        } else {
            HelmRhsIn<T> in;
            in.u = u + (size_t)b * N;
            in.lapnu = lapnu + (size_t)b * N;
            in.fbar = fbar;
            in.b = b;
            in.c = F.c;
            in.dt = dt;
            in.alpha = alpha;
            in.fb = 0.0;
            rows_forward(p, F, in, s);
        }
        solve_spectrum(p, F, 1.0, -alpha * dt * F.nu, 1, s);
        rows_inverse(p, F, ScaledOut<T>{u + (size_t)b * N, spectrum_scale(F)}, s);
    }
    return ibmx_launch_check();
}

bool solver_grid_ok(const ibmx_grid &g)
{
    return g.periodic[0] && g.periodic[1] && pow2(g.n[0]) && pow2(g.n[1]) && g.n[0] <= 1024 &&
           g.n[1] <= 1024 && (!g.periodic[2] || (pow2(g.n[2]) && g.n[2] <= 1024));
}

}  // namespace

// workspace: the real right-hand side / solution grid, the half spectrum
// (nx/2 + 1 modes along x), the elimination scratch (walls in z) and one
// twiddle table per axis
bool ibmx_fluid_ready(ibmx_plan p)
{
    return p->fl_r && p->fl_z && (p->grid.periodic[2] || p->fl_cp) && p->fl_tw[0] &&
           p->fl_tw[1] && p->fl_tw[2];
}

bool ibmx_fluid_grid_ok(ibmx_plan p) { return solver_grid_ok(p->grid); }

ibmx_status ibmx_fluid_reserve(ibmx_plan p)
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

extern "C" ibmx_status ibmx_project(ibmx_plan p, void *u, void *uf, void *P, void *phi,
                                    double theta)
{
    if (!p || !u || !uf || !P || !isfinite(theta))
        return IBMX_EINVAL;
    if (!solver_grid_ok(p->grid))
        return IBMX_EUNSUPPORTED;
    if (!ibmx_fluid_ready(p))
        return IBMX_ESTATE;   // workspace not reserved (ibmx_plan_reserve)
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
    if (!ibmx_fluid_ready(p))
        return IBMX_ESTATE;   // workspace not reserved (ibmx_plan_reserve)
    if (p->prec == IBMX_F64)
        return run_helmholtz<double>(p, (double *)u, (const double *)lapnu, (const double *)P, fbar,
                                     dt, theta);
    return run_helmholtz<float>(p, (float *)u, (const float *)lapnu, (const float *)P, fbar, dt,
                                theta);
}
