// Outer forcing loop of the collocated direct-forcing IBM (Sec. 2.2.2).
//
// Data flow of one ibmx_forcing call
//   binning (once)  marker geometry in FP64 (X_l = x_p + o_l -> base node,
//                   fractional offsets, periodic wrap, wall check), then a
//                   counting sort of the active markers by the spatial tile of
//                   their centre node, and per tile a halo list of the
//                   neighbouring tiles' markers whose delta support reaches
//                   into it.
//   passes          two launches per pass, one workgroup per tile.  The
//                   interpolation stages the tile's region of u^{m-1} in LDS,
//                   gives every own marker U, F = (U^d - U)/c in FP64 and the
//                   spreading amplitude G = F dV / h^3 (kept per pass), and
//                   its residual term.  The spreading adds w G of every marker
//                   whose support reaches the tile (own + halo) into an LDS
//                   copy of the tile in integer fixed point, and the
//                   workgroup, sole owner of its nodes, writes u^m = u^{m-1} +
//                   c f^m in place (the interpolation of the pass has ended).
//   sums (once)     per particle, in marker order, the FP64 sums over markers
//                   and passes of G and o x G (S_p, T_p), the residual terms,
//                   and every marker's pass-summed amplitude.
//   residual (once) an interpolation of the final velocity gives the residual
//                   terms of u^n, before the sums.
//   f_tot (once)    spreading is linear and the markers do not move during the
//                   call, so sum_m f^m is the spread of the summed amplitudes:
//                   one last tile pass adds it to f_tot.
// With a single pass that pass's spreading updates u and f_tot together.
#include <math.h>

#include "ibmx_internal.hpp"
#include "ibmx_delta.hpp"

namespace {

constexpr int NXCD = 8;              // MI355X: 8 XCDs, workgroups dealt round-robin

// Four-value records.  The w of a {fractions, packed node} record carries
// the node's bits: it is only ever stored, loaded, copied between registers
// and bit-cast back (from_bits / to_bits), never an operand of floating-point
// arithmetic, so no flush of denormal values can touch it.
template <typename T>
struct V4;
template <>
struct V4<float> {
    typedef float4 type;
    __device__ static float from_bits(unsigned v) { return __uint_as_float(v); }
    __device__ static unsigned to_bits(float v) { return __float_as_uint(v); }
};
template <>
struct V4<double> {
    typedef double4 type;
    __device__ static double from_bits(unsigned v) { return __longlong_as_double((long long)v); }
    __device__ static unsigned to_bits(double v) { return (unsigned)__double_as_longlong(v); }
};

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned pack_node(const GridC &g, int bx, int by, int bz)
{
    return (unsigned)bx | ((unsigned)by << g.shift[1]) | ((unsigned)bz << g.shift[2]);
}

__device__ __forceinline__ void unpack_node(const GridC &g, unsigned v, int *b)
{
    b[0] = (int)(v & ((1u << g.shift[1]) - 1u));
    b[1] = (int)((v >> g.shift[1]) & ((1u << (g.shift[2] - g.shift[1])) - 1u));
    b[2] = (int)(v >> g.shift[2]);
}

// node index along axis a for stencil offset k from base b (b already wrapped)
__device__ __forceinline__ int axis_node(const GridC &g, int a, int b, int k)
{
    int i = b + k;
    if (g.periodic[a])
        return i >= g.n[a] ? i - g.n[a] : i;
    // on a wall axis only a zero-weight last node can fall outside
    return i < g.n[a] ? i : g.n[a] - 1;
}

// Workgroups are dealt to the XCDs round-robin; give each XCD a contiguous
// range of tiles / marker chunks so that neighbouring tiles share its L2.
__device__ __forceinline__ int xcd_remap(int bid, int nblocks)
{
    const int q = nblocks / NXCD, r = nblocks % NXCD;
    const int x = bid % NXCD, k = bid / NXCD;
    return x * q + min(x, r) + k;
}

__device__ __forceinline__ unsigned long long lanemask_lt(int lane)
{
    return (1ull << lane) - 1ull;
}

// Marker geometry: base node b (wrapped) and fractional offset t per axis.
// Returns false if a nonzero-weight node falls beyond a wall.
template <int W>
__device__ __forceinline__ bool marker_geometry(const GridC &g, const double *X, int *b, double *t)
{
    bool ok = true;
    for (int a = 0; a < 3; ++a) {
        double s = (X[a] - g.origin[a]) / g.h - Delta<W, double>::base_shift;
        double fl = floor(s);
        t[a] = s - fl;
        long long bb = (long long)fl - 1;
        if (g.periodic[a]) {
            // the 64-bit remainder only for a base outside [0, n)
            if (bb < 0 || bb >= g.n[a]) {
                bb %= g.n[a];
                if (bb < 0)
                    bb += g.n[a];
            }
        } else {
            long long last = (t[a] == 0.0) ? bb + W - 2 : bb + W - 1;
            if (bb < 0 || last > g.n[a] - 1) {
                ok = false;
                bb = 0;
            }
        }
        b[a] = (int)bb;
    }
    return ok;
}

// tile of the marker's centre node (base + 1 on every axis)
__device__ __forceinline__ int home_tile(const GridC &g, const TileC &tc, const int *b)
{
    int ti[3];
    for (int a = 0; a < 3; ++a)
        ti[a] = tile_of(tc, a, axis_node(g, a, b[a], 1));
    return ti[0] + tc.nt[0] * (ti[1] + tc.nt[1] * ti[2]);
}


template <typename T, int W>
__device__ __forceinline__ void stencil(const GridC &g, unsigned node, const T *tt, int ix[3][W],
                                        T w[3][W])
{
    int b[3];
    unpack_node(g, node, b);
    for (int a = 0; a < 3; ++a) {
        Delta<W, T>::w(tt[a], w[a]);
#pragma unroll
        for (int k = 0; k < W; ++k)
            ix[a][k] = axis_node(g, a, b[a], k);
    }
}

// Marker force from the interpolated velocity: F = (U^d - U)/c in FP64 with
// U^d = u_p + omega_p x o and dV taken from the marker's record; rsq
// receives dV |U^d - U|^2 and G = F dV / h^3 is returned.
template <typename T>
__device__ __forceinline__ void marker_force(const GridC &g, double c,
                                             const typename V4<T>::type &ud, const T *U,
                                             double &rsq, T *G)
{
    const double dVp = (double)ud.w;
    const double Ud[3] = {(double)ud.x, (double)ud.y, (double)ud.z};
    rsq = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double r = Ud[a] - (double)U[a];
        rsq += dVp * r * r;
        G[a] = (T)(r / c * dVp * g.inv_h3);
    }
}

// Row walk over a tile's nodes for the write-out: each wave takes whole rows
// of B[0] nodes (64 / B[0] rows at a time), UNR row groups per step, so that
// every thread issues all its loads before any store.
struct TileWalk {
    int rpi, sub, lx, rows, nw;
    bool lane_ok;
    float inv_by;
    __device__ TileWalk(const TileC &tc, int e0)
    {
        const int lane = threadIdx.x & (IBMX_WAVE - 1);
        rpi = IBMX_WAVE / tc.B[0];
        sub = lane / tc.B[0];
        lx = lane - sub * tc.B[0];
        rows = tc.B[1] * tc.B[2];
        nw = blockDim.x / IBMX_WAVE;
        lane_ok = sub < rpi && lx < e0;
        inv_by = 1.0f / (float)tc.B[1];
    }
    // row index -> (ly, lz); exact for rows < 2^16
    __device__ void yz(int r, int by, int &ly, int &lz) const
    {
        lz = (int)(((float)r + 0.5f) * inv_by);
        ly = r - lz * by;
    }
};

constexpr int UNR = 2;    // row groups per write-out step
constexpr int SUNR = 16;  // row groups per staging step

// ---------------------------------------------------------------------------
// halo entries: a marker registers itself with every neighbouring tile its
// support reaches (at most 7: tiles are at least W nodes wide); a last
// support node of zero weight (t == 0) does not count.
// ---------------------------------------------------------------------------
template <typename T, int W>
__device__ __forceinline__ int halo_tiles(const GridC &g, const TileC &tc, const int *b,
                                          const T *tt, int *tgt)
{
    int tl[3][2], nt[3], home[3];
    for (int a = 0; a < 3; ++a) {
        const int last = tt[a] == T(0) ? W - 2 : W - 1;
        home[a] = tile_of(tc, a, axis_node(g, a, b[a], 1));
        const int t0 = tile_of(tc, a, axis_node(g, a, b[a], 0));
        const int t1 = tile_of(tc, a, axis_node(g, a, b[a], last));
        tl[a][0] = t0;
        tl[a][1] = t1;
        nt[a] = t1 == t0 ? 1 : 2;
    }
    int ntg = 0;
    for (int kz = 0; kz < nt[2]; ++kz)
        for (int ky = 0; ky < nt[1]; ++ky)
            for (int kx = 0; kx < nt[0]; ++kx) {
                const int tx = tl[0][kx], ty = tl[1][ky], tz = tl[2][kz];
                if (tx == home[0] && ty == home[1] && tz == home[2])
                    continue;
                tgt[ntg++] = tx + tc.nt[0] * (ty + tc.nt[1] * tz);
            }
    return ntg;
}

// Wave-aggregated halo counting: adds every lane's halo tiles to count[tile]
// (one atomic per distinct tile and round, results unused).
__device__ __forceinline__ void halo_count_wave(const int *tgt, int ntg, int *__restrict__ count)
{
    const int lane = threadIdx.x & (IBMX_WAVE - 1);
    for (int k = 0; k < 7; ++k) {
        const int key = k < ntg ? tgt[k] : -1;
        unsigned long long pending = __ballot(key >= 0);
        while (pending) {
            const int leader = __ffsll((long long)pending) - 1;
            const int kk = __shfl(key, leader, IBMX_WAVE);
            const unsigned long long m = __ballot(key == kk) & pending;
            if (lane == leader)
                atomicAdd(&count[kk], __popcll(m));
            pending &= ~m;
        }
    }
}

// Halo emission of a wave's records: the lanes' (round, tile) groups are
// collected in the wave's LDS lists first, then every group reserves its
// positions with one atomic on cursor[tile] -- all groups at once, so the
// atomics' round trips overlap -- and the lanes write their record index j.
constexpr int HGROUPS = 7 * IBMX_WAVE;
__device__ __forceinline__ void halo_emit_wave(const int *tgt, int ntg, int j,
                                               int *__restrict__ cursor,
                                               const int *__restrict__ halo_start,
                                               int *__restrict__ halo_list, long long cap,
                                               int *__restrict__ err, volatile int *g_key,
                                               volatile int *g_pos)
{
    const int lane = threadIdx.x & (IBMX_WAVE - 1);
    int grp[7], rank[7];
    int ng = 0;
    for (int k = 0; k < 7; ++k) {
        const int key = k < ntg ? tgt[k] : -1;
        grp[k] = -1;
        rank[k] = 0;
        unsigned long long pending = __ballot(key >= 0);
        while (pending) {
            const int leader = __ffsll((long long)pending) - 1;
            const int kk = __shfl(key, leader, IBMX_WAVE);
            const unsigned long long m = __ballot(key == kk) & pending;
            if (key == kk) {
                grp[k] = ng;
                rank[k] = __popcll(m & lanemask_lt(lane));
            }
            if (lane == leader) {
                g_key[ng] = kk;
                g_pos[ng] = __popcll(m);
            }
            ++ng;
            pending &= ~m;
        }
    }
    for (int q = lane; q < ng; q += IBMX_WAVE) {
        const int key = g_key[q];
        g_pos[q] = halo_start[key] + atomicAdd(&cursor[key], g_pos[q]);
    }
    for (int k = 0; k < 7; ++k) {
        if (grp[k] < 0)
            continue;
        const long long pos = (long long)g_pos[grp[k]] + rank[k];
        if (pos < cap)
            halo_list[pos] = j;
        else
            atomicCAS(err, 0, (int)IBMX_ECAPACITY);
    }
}

// Reservation of one slot per lane with key >= 0 in the segment of tile
// key: lanes with equal keys form a group, every group reserves its slots
// with one atomic on cursor[key] -- all groups of the wave at once, so the
// atomics' round trips overlap -- and the lane gets start[key] + base + its
// rank in the group (-1 for key < 0).
__device__ __forceinline__ int reserve_wave(int key, int *__restrict__ cursor,
                                            const int *__restrict__ start, volatile int *g_key,
                                            volatile int *g_pos)
{
    const int lane = threadIdx.x & (IBMX_WAVE - 1);
    int grp = -1, rank = 0, ng = 0;
    unsigned long long pending = __ballot(key >= 0);
    while (pending) {
        const int leader = __ffsll((long long)pending) - 1;
        const int kk = __shfl(key, leader, IBMX_WAVE);
        const unsigned long long m = __ballot(key == kk) & pending;
        if (key == kk) {
            grp = ng;
            rank = __popcll(m & lanemask_lt(lane));
        }
        if (lane == leader) {
            g_key[ng] = kk;
            g_pos[ng] = __popcll(m);
        }
        ++ng;
        pending &= ~m;
    }
    for (int q = lane; q < ng; q += IBMX_WAVE) {
        const int k = g_key[q];
        g_pos[q] = start[k] + atomicAdd(&cursor[k], g_pos[q]);
    }
    return grp >= 0 ? g_pos[grp] + rank : -1;
}

// ---------------------------------------------------------------------------
// binning step A: one thread per marker.  Home tile of every active marker
// (m_key, -1 when masked), and the per-tile marker and halo entry counts,
// aggregated over the lanes of a wave that share a tile.
// ---------------------------------------------------------------------------
template <typename T, int W>
__global__ __launch_bounds__(256) void k_bin_count(
    GridC g, TileC tc, int np, int nm, const int *__restrict__ pid_of,
    const double *__restrict__ body, const double *__restrict__ xp,
    const uint8_t *__restrict__ mask, int *__restrict__ m_key, int *__restrict__ tile_count,
    int *__restrict__ halo_count, int *__restrict__ err, long long *__restrict__ count)
{
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & (IBMX_WAVE - 1);
    int key = -1, ntg = 0;
    int tgt[7];
    if (l < nm && (!mask || mask[l])) {
        const int p = pid_of[l];
        double X[3], t[3];
        int b[3];
        for (int a = 0; a < 3; ++a)
            X[a] = xp[(size_t)a * np + p] + body[(size_t)a * nm + l];
        if (marker_geometry<W>(g, X, b, t)) {
            key = home_tile(g, tc, b);
            const T tt[3] = {(T)t[0], (T)t[1], (T)t[2]};
            ntg = halo_tiles<T, W>(g, tc, b, tt, tgt);
        } else {
            atomicCAS(err, 0, (int)IBMX_EDOMAIN);
        }
    }
    if (l < nm)
        m_key[l] = key;
    unsigned long long pending = __ballot(key >= 0);
    while (pending) {
        const int leader = __ffsll((long long)pending) - 1;
        const int kk = __shfl(key, leader, IBMX_WAVE);
        const unsigned long long m = __ballot(key == kk) & pending;
        if (lane == leader)
            atomicAdd(&tile_count[kk], __popcll(m));
        pending &= ~m;
    }
    halo_count_wave(tgt, ntg, halo_count);
    slot_add(count, block_sum<long long>(key >= 0 ? 1 : 0));
    slot_add(count + 2 * IBMX_RSLOTS, block_sum<long long>(ntg));
}

// ---------------------------------------------------------------------------
// binning step B: one thread per marker.  Reserve the marker's slot in its
// home tile's segment, write the sorted records and register the record in
// the halo lists of the neighbouring tiles its support reaches.  The order
// of the markers inside a tile's segment follows the reservations; no result
// depends on it (the spreading sums integers, the particle sums go by marker
// index).
// ---------------------------------------------------------------------------
template <typename T, int W>
__global__ __launch_bounds__(256) void k_bin_scatter(
    GridC g, TileC tc, int np, int nm, const int *__restrict__ pid_of,
    const double *__restrict__ body, const double *__restrict__ xp,
    const double *__restrict__ up, const double *__restrict__ wp, const double *__restrict__ dV,
    const int *__restrict__ m_key, const int *__restrict__ tile_start,
    int *__restrict__ tile_cursor, typename V4<T>::type *__restrict__ rec_tn,
    typename V4<T>::type *__restrict__ rec_ud, int *__restrict__ rec_src,
    int *__restrict__ m_inv, const int *__restrict__ halo_start, int *__restrict__ halo_cursor,
    int *__restrict__ halo_list, long long halo_cap, int *__restrict__ err)
{
    __shared__ int s_gkey[4][HGROUPS], s_gpos[4][HGROUPS];
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    const int wv = threadIdx.x / IBMX_WAVE;
    const int key = l < nm ? m_key[l] : -1;
    const int dst = reserve_wave(key, tile_cursor, tile_start, s_gkey[wv], s_gpos[wv]);
    int tgt[7];
    int ntg = 0;
    if (key >= 0) {
        m_inv[l] = dst;
        const int p = pid_of[l];
        double X[3], t[3], o[3];
        int b[3];
        for (int a = 0; a < 3; ++a) {
            o[a] = body[(size_t)a * nm + l];
            X[a] = xp[(size_t)a * np + p] + o[a];
        }
        marker_geometry<W>(g, X, b, t);
        const double upp[3] = {up[p], up[np + p], up[2 * np + p]};
        const double wpp[3] = {wp[p], wp[np + p], wp[2 * np + p]};
        typename V4<T>::type tn, ud;
        tn.x = (T)t[0];
        tn.y = (T)t[1];
        tn.z = (T)t[2];
        tn.w = V4<T>::from_bits(pack_node(g, b[0], b[1], b[2]));
        // rigid-body velocity at the marker, U^d = u_p + omega_p x o (FP64)
        ud.x = (T)(upp[0] + (wpp[1] * o[2] - wpp[2] * o[1]));
        ud.y = (T)(upp[1] + (wpp[2] * o[0] - wpp[0] * o[2]));
        ud.z = (T)(upp[2] + (wpp[0] * o[1] - wpp[1] * o[0]));
        ud.w = (T)dV[p];
        rec_tn[dst] = tn;
        rec_ud[dst] = ud;
        rec_src[dst] = l;
        const T tt[3] = {tn.x, tn.y, tn.z};
        ntg = halo_tiles<T, W>(g, tc, b, tt, tgt);
    } else if (l < nm) {
        m_inv[l] = -1;
    }
    halo_emit_wave(tgt, ntg, dst, halo_cursor, halo_start, halo_list, halo_cap, err, s_gkey[wv],
                   s_gpos[wv]);
}

// ---------------------------------------------------------------------------
// tile geometry shared by the tile kernels
// ---------------------------------------------------------------------------
struct TileBox {
    int o[3];   // first node of the tile
    int e[3];   // extent (last tile of an axis may be short)
    __device__ TileBox(const GridC &g, const TileC &tc, int tile)
    {
        const int t0 = tile % tc.nt[0], t1 = (tile / tc.nt[0]) % tc.nt[1];
        const int t2 = tile / (tc.nt[0] * tc.nt[1]);
        o[0] = t0 * tc.B[0];
        o[1] = t1 * tc.B[1];
        o[2] = t2 * tc.B[2];
        for (int a = 0; a < 3; ++a)
            e[a] = min(tc.B[a], g.n[a] - o[a]);
    }
};

template <typename V>
__device__ __forceinline__ V block_max(V v)
{
    __shared__ V part[16];
#pragma unroll
    for (int off = IBMX_WAVE / 2; off > 0; off >>= 1) {
        V w = __shfl_xor(v, off, IBMX_WAVE);
        v = w > v ? w : v;
    }
    __syncthreads();
    if ((threadIdx.x & (IBMX_WAVE - 1)) == 0)
        part[threadIdx.x / IBMX_WAVE] = v;
    __syncthreads();
    V r = part[0];
    for (int w = 1; w < (int)(blockDim.x / IBMX_WAVE); ++w)
        r = part[w] > r ? part[w] : r;
    return r;   // valid in every thread
}

// Element i of a grid component: with O32 (every component spans less than
// 4 GB) a 32-bit byte offset from the component's uniform base, which the
// loads and stores take as is; otherwise a 64-bit index.  Node indices fit 32
// bits (the grid has fewer than 2^31 nodes).
template <typename T, bool O32>
__device__ __forceinline__ T &grid_at(T *base, unsigned i)
{
    if (O32)
        return *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + i * (unsigned)sizeof(T));
    return base[(size_t)i];
}
template <typename V, typename T, bool O32>
__device__ __forceinline__ const V &grid_at_as(const T *base, unsigned i)
{
    if (O32)
        return *reinterpret_cast<const V *>(reinterpret_cast<const char *>(base) +
                                            i * (unsigned)sizeof(T));
    return *reinterpret_cast<const V *>(base + (size_t)i);
}

// LDS layout of a staged region of RV nodes: (x, y) pairs of every node,
// then the z components, so that a node is read with two LDS loads
template <typename T>
struct V2;
template <>
struct V2<float> {
    typedef float2 type;
};
template <>
struct V2<double> {
    typedef double2 type;
};

template <typename T>
__device__ __forceinline__ void reg_put(T *reg, int RV, int idx, T x, T y, T z)
{
    typename V2<T>::type xy;
    xy.x = x;
    xy.y = y;
    reinterpret_cast<typename V2<T>::type *>(reg)[idx] = xy;
    reg[2 * RV + idx] = z;
}

template <typename T>
__device__ __forceinline__ void reg_get(const T *reg, int RV, int idx, T &x, T &y, T &z)
{
    const typename V2<T>::type xy = reinterpret_cast<const typename V2<T>::type *>(reg)[idx];
    x = xy.x;
    y = xy.y;
    z = reg[2 * RV + idx];
}

// Stage v = scale * src (+ src2) over the tile's support region
// [o - 1, o + B + W - 2) per axis into LDS (nodes beyond a wall read 0),
// element by element: each wave loads 64 / R0 rows of R0 nodes per step, and
// every thread issues SUNR steps of loads before its LDS stores.
template <typename T, int W, bool O32>
__device__ __forceinline__ void stage_region_rows(const GridC &g, const TileC &tc,
                                                  const TileBox &box, const T *__restrict__ src,
                                                  T scale, const T *__restrict__ src2, T *reg)
{
    const int R0 = tc.B[0] + W - 1, R1 = tc.B[1] + W - 1, R2 = tc.B[2] + W - 1;
    const int RV = R0 * R1 * R2;
    const long long N = g.nodes;
    const T *const s1[3] = {src, src + N, src + 2 * N};
    const T *const s2[3] = {src2, src2 ? src2 + N : nullptr, src2 ? src2 + 2 * N : nullptr};
    const int lane = threadIdx.x & (IBMX_WAVE - 1), wave = threadIdx.x / IBMX_WAVE;
    const int nw = blockDim.x / IBMX_WAVE;
    const int rpi = IBMX_WAVE / R0;
    const int sub = lane / R0, rx = lane - sub * R0;
    const int step = nw * rpi, rows = R1 * R2;
    int gx = box.o[0] - 1 + rx;
    const bool lane_ok = sub < rpi;
    // a node beyond an x wall is stored as 0 like those beyond y and z walls
    bool inx = true;
    if (g.periodic[0])
        gx = gx < 0 ? gx + g.n[0] : (gx >= g.n[0] ? gx - g.n[0] : gx);
    else
        inx = gx >= 0 && gx < g.n[0];
    for (int r0 = wave * rpi + sub; r0 < rows; r0 += SUNR * step) {
        T v[SUNR][3];
        int li[SUNR];
#pragma unroll
        for (int q = 0; q < SUNR; ++q) {
            const int r = r0 + q * step;
            const int rz = r / R1, ry = r - rz * R1;
            int gy = box.o[1] - 1 + ry, gz = box.o[2] - 1 + rz;
            bool ok = lane_ok && r < rows;
            li[q] = ok ? (rz * R1 + ry) * R0 + rx : -1;
            ok = ok && inx;
            if (g.periodic[1])
                gy = gy < 0 ? gy + g.n[1] : (gy >= g.n[1] ? gy - g.n[1] : gy);
            else
                ok = ok && gy >= 0 && gy < g.n[1];
            if (g.periodic[2])
                gz = gz < 0 ? gz + g.n[2] : (gz >= g.n[2] ? gz - g.n[2] : gz);
            else
                ok = ok && gz >= 0 && gz < g.n[2];
            v[q][0] = v[q][1] = v[q][2] = T(0);
            if (ok) {
                const unsigned gi =
                    ((unsigned)gz * (unsigned)g.n[1] + (unsigned)gy) * (unsigned)g.n[0] + (unsigned)gx;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    v[q][c] = scale * grid_at_as<T, T, O32>(s1[c], gi);
                    if (src2)
                        v[q][c] += grid_at_as<T, T, O32>(s2[c], gi);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < SUNR; ++q) {
            if (li[q] < 0)
                continue;
            reg_put<T>(reg, RV, li[q], v[q][0], v[q][1], v[q][2]);
        }
    }
}

// 16-byte packet of grid values (4 floats or 2 doubles)
template <typename T>
struct alignas(16) Pack16 {
    T e[16 / sizeof(T)];
};

// The same staging with 16-byte loads: every row of the region is covered by
// the aligned packets of [floor_E(o - 1), ceil_E(o + B + W - 2)) (E values
// per packet); packets inside the grid are loaded whole, packets crossing an
// edge value by value (wrapped on a periodic axis, 0 beyond a wall).  Needs
// n_x and the field pointers to be multiples of E values / 16 bytes.
constexpr int VUNR = 5;   // row groups per vector staging step
template <typename T, int W, bool O32>
__device__ __forceinline__ void stage_region_vec(const GridC &g, const TileC &tc,
                                                 const TileBox &box, const T *__restrict__ src,
                                                 T scale, const T *__restrict__ src2, T *reg)
{
    constexpr int E = 16 / (int)sizeof(T);
    const int R0 = tc.B[0] + W - 1, R1 = tc.B[1] + W - 1, R2 = tc.B[2] + W - 1;
    const int RV = R0 * R1 * R2;
    const long long N = g.nodes;
    const T *const s1[3] = {src, src + N, src + 2 * N};
    const T *const s2[3] = {src2, src2 ? src2 + N : nullptr, src2 ? src2 + 2 * N : nullptr};
    const int xs = box.o[0] - 1, xe = box.o[0] + R0 - 1;   // needed x range
    const int X0 = xs >= 0 ? xs - xs % E : -E;               // xs >= -1
    const int nch = (xe + E - 1 - X0) / E;                 // packets per row (xe > 0)
    const int lane = threadIdx.x & (IBMX_WAVE - 1), wave = threadIdx.x / IBMX_WAVE;
    const int nw = blockDim.x / IBMX_WAVE;
    const int rpi = IBMX_WAVE / nch;
    const int sub = lane / nch, ch = lane - sub * nch;
    const int step = nw * rpi, rows = R1 * R2;
    const int x = X0 + ch * E;
    const bool lane_ok = sub < rpi;
    const bool whole = x >= 0 && x + E <= g.n[0];
    for (int r0 = wave * rpi + sub; r0 < rows; r0 += VUNR * step) {
        Pack16<T> v[VUNR][3];
        int rb[VUNR];
#pragma unroll
        for (int q = 0; q < VUNR; ++q) {
            const int r = r0 + q * step;
            const int rz = r / R1, ry = r - rz * R1;
            int gy = box.o[1] - 1 + ry, gz = box.o[2] - 1 + rz;
            bool ok = lane_ok && r < rows;
            if (g.periodic[1])
                gy = gy < 0 ? gy + g.n[1] : (gy >= g.n[1] ? gy - g.n[1] : gy);
            else
                ok = ok && gy >= 0 && gy < g.n[1];
            if (g.periodic[2])
                gz = gz < 0 ? gz + g.n[2] : (gz >= g.n[2] ? gz - g.n[2] : gz);
            else
                ok = ok && gz >= 0 && gz < g.n[2];
            rb[q] = lane_ok && r < rows ? (rz * R1 + ry) * R0 : -1;
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int k = 0; k < E; ++k)
                    v[q][c].e[k] = T(0);
            if (!ok)
                continue;
            const unsigned row = ((unsigned)gz * (unsigned)g.n[1] + (unsigned)gy) * (unsigned)g.n[0];
            if (whole) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    v[q][c] = grid_at_as<Pack16<T>, T, O32>(s1[c], row + (unsigned)x);
                    if (src2) {
                        const Pack16<T> w2 = grid_at_as<Pack16<T>, T, O32>(s2[c], row + (unsigned)x);
#pragma unroll
                        for (int k = 0; k < E; ++k)
                            v[q][c].e[k] = scale * v[q][c].e[k] + w2.e[k];
                    } else if (scale != T(1)) {
#pragma unroll
                        for (int k = 0; k < E; ++k)
                            v[q][c].e[k] = scale * v[q][c].e[k];
                    }
                }
            } else {
#pragma unroll
                for (int k = 0; k < E; ++k) {
                    int gx = x + k;
                    if (gx < xs || gx >= xe)
                        continue;
                    if (g.periodic[0])
                        gx = gx < 0 ? gx + g.n[0] : (gx >= g.n[0] ? gx - g.n[0] : gx);
                    else if (gx < 0 || gx >= g.n[0])
                        continue;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        T val = scale * grid_at_as<T, T, O32>(s1[c], row + (unsigned)gx);
                        if (src2)
                            val += grid_at_as<T, T, O32>(s2[c], row + (unsigned)gx);
                        v[q][c].e[k] = val;
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < VUNR; ++q) {
            if (rb[q] < 0)
                continue;
#pragma unroll
            for (int k = 0; k < E; ++k) {
                const int lx = x + k - xs;
                if (lx < 0 || lx >= R0)
                    continue;
                reg_put<T>(reg, RV, rb[q] + lx, v[q][0].e[k], v[q][1].e[k], v[q][2].e[k]);
            }
        }
    }
}

template <typename T, int W, bool O32 = false>
__device__ __forceinline__ void stage_region(const GridC &g, const TileC &tc, const TileBox &box,
                                             const T *__restrict__ src, T scale,
                                             const T *__restrict__ src2, T *reg)
{
    constexpr int E = 16 / (int)sizeof(T);
    const bool vec = g.n[0] % E == 0 && ((size_t)src & 15) == 0 &&
                     (!src2 || ((size_t)src2 & 15) == 0);
    if (vec)
        stage_region_vec<T, W, O32>(g, tc, box, src, scale, src2, reg);
    else
        stage_region_rows<T, W, O32>(g, tc, box, src, scale, src2, reg);
}

// Region index of a marker's base node per axis: the centre node b + 1 lies
// in the tile, so d is in [0, e); d >= e only when b wrapped below a periodic
// seam (b = n - 1 for a centre at node 0).
__device__ __forceinline__ void region_base(const GridC &g, const TileBox &box, const int *b, int *d)
{
    for (int a = 0; a < 3; ++a) {
        d[a] = b[a] - box.o[a] + 1;
        if (d[a] >= box.e[a])
            d[a] -= g.n[a];
    }
}

// ---------------------------------------------------------------------------
// LDS accumulation of the spread in fixed point.  On gfx950 an LDS float add
// costs about 195 cycles per wave instruction, an FP64 add 27, a 32-bit
// integer add 9 and a 64-bit integer add 15, so both precisions accumulate
// integers, and the integer sums do not depend on the order of the additions.
// Per component a power-of-two scale bounds every node's sum: with m the
// largest |G| that can reach the tile (m < 2^ex), n the number of markers
// whose supports reach the tile (no node lies in more supports) and w_max =
// 8/27 the largest weight product of the delta (phi(0)^3; 1/8 for the
// four-point delta), a node's sum is below n w_max m, so the scale
// 2^(30 - ex - cb) with 2^cb >= n w_max keeps it below 2^30 (FP32: 32-bit
// sums) and 2^(62 - ex - cb) below 2^62 (FP64: 64-bit sums).  No sum can
// wrap, however dense the markers; each term is rounded to the nearest
// integer, at most 2^(ex + cb - 31) (2^(ex + cb - 63)) of m.  FP32
// keeps (x, y) of a node in one 64-bit word, y 2^32 + x as a two's-complement
// sum (exact while both partial sums fit 32 bits, which the bound
// guarantees), and z in a 32-bit word: two atomics per node.
// ---------------------------------------------------------------------------
// floor(x + 1/2) by the hardware's single conversion instruction (|x| below
// 2^31)
__device__ __forceinline__ int round_half_up(float x)
{
    int r;
    asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

__device__ __forceinline__ int cover_bits(int n)
{
    // smallest cb >= 0 with 2^cb >= n * 8/27
    const float bound = (float)n * (8.0f / 27.0f);
    int cb = 0;
    if (bound > 1.0f) {
        frexpf(bound, &cb);     // bound < 2^cb
    }
    return cb;
}

template <typename T>
struct SpreadAcc;
typedef __attribute__((address_space(3))) unsigned char lds_u8;
typedef __attribute__((address_space(3))) int lds_i32;
typedef __attribute__((address_space(3))) unsigned long long lds_u64;
template <>
struct SpreadAcc<float> {
    static constexpr int BYTES = 12;   // per node
    __device__ static float scale_for(float m, int n)
    {
        int ex = 0;
        frexpf(m, &ex);                  // m < 2^ex
        return m > 0.0f ? ldexpf(1.0f, min(30 - ex - cover_bits(n), 126)) : 0.0f;
    }
    __device__ static float unscale_for(float s) { return s > 0.0f ? 1.0f / s : 0.0f; }
    __device__ static void zero(unsigned char *lds, int V)
    {
        int *a = reinterpret_cast<int *>(lds);
        for (int i = threadIdx.x; i < 3 * V; i += blockDim.x)
            a[i] = 0;
    }
    __device__ static void add(unsigned char *lds, int V, int li, float vx, float vy, float vz)
    {
        // nearest integer (halves up) in one conversion each; (x, y) as the
        // 64-bit two's-complement value y 2^32 + x: low word x, high word y
        // plus the sign extension of x
        const int x = round_half_up(vx), y = round_half_up(vy), z = round_half_up(vz);
        const unsigned long long xy =
            ((unsigned long long)(unsigned)(y + (x >> 31)) << 32) | (unsigned)x;
        lds_u64 *axy = (lds_u64 *)lds + li;
        lds_i32 *az = (lds_i32 *)((lds_u8 *)lds + 8 * V) + li;
        __hip_atomic_fetch_add(axy, xy, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_fetch_add(az, z, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    // values of node li; false when all three sums are zero
    __device__ static bool get(const unsigned char *lds, int V, int li, const float *unscale,
                               float *f)
    {
        const long long sxy = reinterpret_cast<const long long *>(lds)[li];
        const int x = (int)(unsigned)(unsigned long long)sxy;
        const int y = (int)((sxy - (long long)x) >> 32);
        const int z = reinterpret_cast<const int *>(lds)[2 * V + li];
        f[0] = (float)x * unscale[0];
        f[1] = (float)y * unscale[1];
        f[2] = (float)z * unscale[2];
        return (x | y | z) != 0;
    }
};
template <>
struct SpreadAcc<double> {
    static constexpr int BYTES = 24;
    __device__ static double scale_for(float m, int n)
    {
        int ex = 0;
        frexpf(m, &ex);
        return m > 0.0f ? ldexp(1.0, min(62 - ex - cover_bits(n), 1000)) : 0.0;
    }
    __device__ static double unscale_for(double s) { return s > 0.0 ? 1.0 / s : 0.0; }
    __device__ static void zero(unsigned char *lds, int V)
    {
        long long *a = reinterpret_cast<long long *>(lds);
        for (int i = threadIdx.x; i < 3 * V; i += blockDim.x)
            a[i] = 0;
    }
    __device__ static void add(unsigned char *lds, int V, int li, double vx, double vy, double vz)
    {
        unsigned long long *a = reinterpret_cast<unsigned long long *>(lds);
        atomicAdd(&a[li], (unsigned long long)__double2ll_rn(vx));
        atomicAdd(&a[V + li], (unsigned long long)__double2ll_rn(vy));
        atomicAdd(&a[2 * V + li], (unsigned long long)__double2ll_rn(vz));
    }
    __device__ static bool get(const unsigned char *lds, int V, int li, const double *unscale,
                               double *f)
    {
        const long long *a = reinterpret_cast<const long long *>(lds);
        const long long x = a[li], y = a[V + li], z = a[2 * V + li];
        f[0] = (double)x * unscale[0];
        f[1] = (double)y * unscale[1];
        f[2] = (double)z * unscale[2];
        return (x | y | z) != 0;
    }
};

// Tile index of neighbour ni = (dx + 1) + 3 (dy + 1) + 9 (dz + 1) of a tile
// (periodic wrap; -1 beyond a wall).
__device__ __forceinline__ int neighbour_tile(const GridC &g, const TileC &tc, int tile, int ni)
{
    const int d[3] = {ni % 3 - 1, (ni / 3) % 3 - 1, ni / 9 - 1};
    int t[3] = {tile % tc.nt[0], (tile / tc.nt[0]) % tc.nt[1], tile / (tc.nt[0] * tc.nt[1])};
    for (int a = 0; a < 3; ++a) {
        t[a] += d[a];
        if (t[a] < 0 || t[a] >= tc.nt[a]) {
            if (!g.periodic[a])
                return -1;
            t[a] = t[a] < 0 ? t[a] + tc.nt[a] : t[a] - tc.nt[a];
        }
    }
    return t[0] + tc.nt[0] * (t[1] + tc.nt[1] * t[2]);
}

// ---------------------------------------------------------------------------
// spreading, one workgroup per tile.  Every marker whose support reaches
// the tile (own + halo list) adds w G to the tile's nodes in LDS; then the
// workgroup, owner of its nodes, applies u += c f (add_u) and f_tot += f
// (add_f) with plain loads and stores.  tile_max (per tile, the largest |G|
// of its own markers) bounds the amplitudes from the tile and its 26
// neighbours (a support of at most W <= B nodes reaches one tile further at
// most); without it the workgroup takes the largest |G| of the markers it
// adds.  The fixed-point scale also takes the number n of markers the tile
// receives: no node lies in more than n supports.  count_shell adds the
// number of nodes that received a nonzero sum to a counter.
// ---------------------------------------------------------------------------
template <typename T, int W, bool O32, bool AU, bool AF>
__device__ __forceinline__ void spread_tile(int tile, const GridC &g, const TileC &tc, T c,
                                            int count_shell,
                                            const int *__restrict__ tile_start,
                                            const int *__restrict__ halo_start,
                                            const int *__restrict__ halo_list,
                                            const typename V4<T>::type *__restrict__ rec_tn,
                                            const typename V4<T>::type *__restrict__ rec_G,
                                            const float4 *__restrict__ tile_max,
                                            T *__restrict__ u, T *__restrict__ f_tot,
                                            long long *__restrict__ count)
{
    typedef typename V4<T>::type T4;
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned char *acc = smem;
    const int a0 = tile_start[tile], a1 = tile_start[tile + 1];
    const int h0 = halo_start[tile], h1 = halo_start[tile + 1];
    const int n_own = a1 - a0, n_tot = n_own + (h1 - h0);
    if (n_tot == 0)
        return;
    const TileBox box(g, tc, tile);
    // accumulator rows padded to B[0] + 1 nodes, so that nodes of one x
    // position in different rows fall in different LDS banks
    const int S0 = tc.B[0] + 1;
    const int V = S0 * tc.B[1] * tc.B[2];
    // first record of this thread, in flight during the set-up
    T4 ptn = {}, pgv = {};
    if ((int)threadIdx.x < n_tot) {
        const int e = threadIdx.x;
        const int j = e < n_own ? a0 + e : halo_list[h0 + e - n_own];
        ptn = rec_tn[j];
        pgv = rec_G[j];
    }
    __shared__ float s_gm[3];
    if (tile_max) {
        if (threadIdx.x < IBMX_WAVE) {
            float m[3] = {0.f, 0.f, 0.f};
            if (threadIdx.x < 27) {
                const int tt = neighbour_tile(g, tc, tile, threadIdx.x);
                if (tt >= 0) {
                    const float4 v = tile_max[tt];
                    m[0] = v.x;
                    m[1] = v.y;
                    m[2] = v.z;
                }
            }
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int off = IBMX_WAVE / 2; off > 0; off >>= 1)
                    m[a] = fmaxf(m[a], __shfl_xor(m[a], off, IBMX_WAVE));
            if (threadIdx.x == 0)
                for (int a = 0; a < 3; ++a)
                    s_gm[a] = m[a];
        }
    } else {
        float gm[3] = {0.f, 0.f, 0.f};
        for (int e = threadIdx.x; e < n_tot; e += blockDim.x) {
            const int j = e < n_own ? a0 + e : halo_list[h0 + e - n_own];
            const T4 gv = rec_G[j];
            gm[0] = fmaxf(gm[0], fabsf((float)gv.x));
            gm[1] = fmaxf(gm[1], fabsf((float)gv.y));
            gm[2] = fmaxf(gm[2], fabsf((float)gv.z));
        }
        for (int a = 0; a < 3; ++a) {
            gm[a] = block_max<float>(gm[a]);
            if (threadIdx.x == 0)
                s_gm[a] = gm[a];
        }
    }
    // The grid values of every thread's first PF write-out rows are loaded
    // now: they do not depend on the sums, and the accumulation hides their
    // latency.  Later rows load as they go.
    const long long N = g.nodes;
    const int wave = threadIdx.x / IBMX_WAVE;
    const TileWalk tw(tc, box.e[0]);
    const int rstep = tw.nw * tw.rpi, rbase = wave * tw.rpi + tw.sub;
    // component bases (node indices fit 32 bits: the grid has < 2^31 nodes)
    T *const ub[3] = {u, u ? u + N : nullptr, u ? u + 2 * N : nullptr};
    T *const fb[3] = {f_tot, f_tot ? f_tot + N : nullptr, f_tot ? f_tot + 2 * N : nullptr};
    constexpr int PF = 4;
    T pu[PF][3], pf[PF][3];
    // row r of the tile: its LDS index (-1 beyond the tile) and grid index
    auto row_at = [&](int r, int &li, unsigned &gi) {
        int ly, lz;
        tw.yz(r, tc.B[1], ly, lz);
        const bool ok = tw.lane_ok && r < tw.rows && ly < box.e[1] && lz < box.e[2];
        li = ok ? (lz * tc.B[1] + ly) * S0 + tw.lx : -1;
        gi = ((unsigned)(box.o[2] + lz) * (unsigned)g.n[1] + (unsigned)(box.o[1] + ly)) *
                 (unsigned)g.n[0] +
             (unsigned)(box.o[0] + tw.lx);
    };
#pragma unroll
    for (int q = 0; q < PF; ++q) {
        int li;
        unsigned gi;
        row_at(rbase + q * rstep, li, gi);
        if (li >= 0) {
            if (AF)
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    pf[q][a] = grid_at<T, O32>(fb[a], gi);
            if (AU)
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    pu[q][a] = grid_at<T, O32>(ub[a], gi);
        }
    }
    SpreadAcc<T>::zero(acc, V);
    __syncthreads();
    T scale[3], unscale[3];
    for (int a = 0; a < 3; ++a) {
        scale[a] = SpreadAcc<T>::scale_for(s_gm[a], n_tot);
        unscale[a] = SpreadAcc<T>::unscale_for(scale[a]);
    }
    for (int e = threadIdx.x; e < n_tot; e += blockDim.x) {
        const T4 tn = ptn, gv = pgv;
        if (e + (int)blockDim.x < n_tot) {
            const int en = e + blockDim.x;
            const int jn = en < n_own ? a0 + en : halo_list[h0 + en - n_own];
            ptn = rec_tn[jn];
            pgv = rec_G[jn];
        }
        const T tt[3] = {tn.x, tn.y, tn.z};
        const T Gs[3] = {gv.x * scale[0], gv.y * scale[1], gv.z * scale[2]};
        int ix[3][W];
        T w[3][W];
        stencil<T, W>(g, V4<T>::to_bits(tn.w), tt, ix, w);
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const int lz = ix[2][k] - box.o[2];
            if ((unsigned)lz >= (unsigned)box.e[2])
                continue;
#pragma unroll
            for (int jj = 0; jj < W; ++jj) {
                const int ly = ix[1][jj] - box.o[1];
                if ((unsigned)ly >= (unsigned)box.e[1])
                    continue;
                const T wzy = w[2][k] * w[1][jj];
                const int rowl = (lz * tc.B[1] + ly) * S0;
#pragma unroll
                for (int i = 0; i < W; ++i) {
                    const int lx = ix[0][i] - box.o[0];
                    if ((unsigned)lx >= (unsigned)box.e[0])
                        continue;
                    // a zero weight adds an integer 0: no test for it
                    const T ww = wzy * w[0][i];
                    const int li = rowl + lx;
                    SpreadAcc<T>::add(acc, V, li, ww * Gs[0], ww * Gs[1], ww * Gs[2]);
                }
            }
        }
    }
    __syncthreads();
    int touched = 0;
#pragma unroll
    for (int q = 0; q < PF; ++q) {
        int li;
        unsigned gi;
        row_at(rbase + q * rstep, li, gi);
        T fv[3];
        if (li < 0 || !SpreadAcc<T>::get(acc, V, li, unscale, fv))
            continue;
        ++touched;
        if (AF)
#pragma unroll
            for (int a = 0; a < 3; ++a)
                grid_at<T, O32>(fb[a], gi) = pf[q][a] + fv[a];
        if (AU)
#pragma unroll
            for (int a = 0; a < 3; ++a)
                grid_at<T, O32>(ub[a], gi) = pu[q][a] + c * fv[a];
    }
    for (int r0 = rbase + PF * rstep; r0 < tw.rows; r0 += UNR * rstep) {
        unsigned gi[UNR];
        bool act[UNR];
        T fv[UNR][3], fo[UNR][3], uo[UNR][3];
#pragma unroll
        for (int q = 0; q < UNR; ++q) {
            const int r = r0 + q * tw.nw * tw.rpi;
            int ly, lz;
            tw.yz(r, tc.B[1], ly, lz);
            const int li = (lz * tc.B[1] + ly) * S0 + tw.lx;
            act[q] = tw.lane_ok && r < tw.rows && ly < box.e[1] && lz < box.e[2];
            gi[q] = ((unsigned)(box.o[2] + lz) * (unsigned)g.n[1] + (unsigned)(box.o[1] + ly)) *
                        (unsigned)g.n[0] +
                    (unsigned)(box.o[0] + tw.lx);
            if (act[q])
                act[q] = SpreadAcc<T>::get(acc, V, li, unscale, fv[q]);
            if (act[q]) {
                if (AF)
#pragma unroll
                    for (int a = 0; a < 3; ++a)
                        fo[q][a] = grid_at<T, O32>(fb[a], gi[q]);
                if (AU)
#pragma unroll
                    for (int a = 0; a < 3; ++a)
                        uo[q][a] = grid_at<T, O32>(ub[a], gi[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < UNR; ++q) {
            if (!act[q])
                continue;
            ++touched;
            if (AF)
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    grid_at<T, O32>(fb[a], gi[q]) = fo[q][a] + fv[q][a];
            if (AU)
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    grid_at<T, O32>(ub[a], gi[q]) = uo[q][a] + c * fv[q][a];
        }
    }
    if (count_shell)
        slot_add(count + IBMX_RSLOTS, block_sum<long long>(touched));
}

// One workgroup per tile (PERSIST false), or a fixed grid of workgroups (a
// multiple of the 8 XCDs) each taking tiles blockIdx.x, blockIdx.x +
// gridDim.x, ... until the tiles run out (PERSIST true).
template <typename T, int W, bool O32, bool PERSIST, bool AU, bool AF>
__global__ __launch_bounds__(256) void k_spread(GridC g, TileC tc, T c, int count_shell,
                                                const int *__restrict__ tile_start,
                                                const int *__restrict__ halo_start,
                                                const int *__restrict__ halo_list,
                                                const typename V4<T>::type *__restrict__ rec_tn,
                                                const typename V4<T>::type *__restrict__ rec_G,
                                                const float4 *__restrict__ tile_max,
                                                T *__restrict__ u, T *__restrict__ f_tot,
                                                long long *__restrict__ count)
{
    if (PERSIST) {
        for (int v = blockIdx.x; v < tc.ntiles; v += gridDim.x) {
            spread_tile<T, W, O32, AU, AF>(xcd_remap(v, tc.ntiles), g, tc, c, count_shell,
                                           tile_start, halo_start, halo_list, rec_tn, rec_G,
                                           tile_max, u, f_tot, count);
            __syncthreads();
        }
    } else {
        spread_tile<T, W, O32, AU, AF>(xcd_remap(blockIdx.x, gridDim.x), g, tc, c, count_shell,
                                       tile_start, halo_start, halo_list, rec_tn, rec_G, tile_max,
                                       u, f_tot, count);
    }
}


// ---------------------------------------------------------------------------
// interpolation of one pass, one workgroup per tile.  The velocity of the
// tile and of the support halo around it (R[a] = B[a] + W - 1 nodes per
// axis, starting one node before the tile) is staged in LDS with coalesced
// row loads; each own marker then gathers its W^3 stencil from LDS, forms
// F = (U^d - U)/c in FP64 and G = F dV / h^3.  The first marker records of
// every thread are loaded before the staging so that their latency overlaps
// it.
// MODE 0 (a pass): writes {G, dV |U^d - U|^2} per marker into the pass's
// record, the pass's largest |G| per tile into tile_max[tile] and the sum of
// the passes' largest |G| (a bound of |sum_m G^m|) into tile_max[ntiles +
// tile].  MODE 2 (the residual on the final velocity): writes dV |U^d - U|^2
// into the w of the marker's record.  The residual terms are summed per
// particle in marker order afterwards, so the residual does not depend on
// the order of the markers within a tile.
// ---------------------------------------------------------------------------
template <typename T, int W, int MODE, bool O32>
__device__ __forceinline__ void interp_tile(int tile, const GridC &g, const TileC &tc, int nm,
                                            int pass, double c, const int *__restrict__ tile_start,
                                            const typename V4<T>::type *__restrict__ rec_tn,
                                            const typename V4<T>::type *__restrict__ rec_ud,
                                            const int *__restrict__ rec_src,
                                            const T *__restrict__ u,
                                            typename V4<T>::type *__restrict__ rec_G,
                                            T *__restrict__ U_dbg, float4 *__restrict__ tile_max)
{
    typedef typename V4<T>::type T4;
    extern __shared__ __align__(16) unsigned char smem[];
    T *reg = reinterpret_cast<T *>(smem);
    const int a0 = tile_start[tile], a1 = tile_start[tile + 1];
    const int n_own = a1 - a0;
    if (n_own == 0) {
        if (MODE == 0 && threadIdx.x == 0) {
            tile_max[tile] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (pass == 0)
                tile_max[tc.ntiles + tile] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
        return;
    }
    const TileBox box(g, tc, tile);
    const int R0 = tc.B[0] + W - 1, R1 = tc.B[1] + W - 1, R2 = tc.B[2] + W - 1;
    const int RV = R0 * R1 * R2;
    // first records of this thread, in flight during the staging
    T4 tn = {}, ud = {};
    if ((int)threadIdx.x < n_own) {
        tn = rec_tn[a0 + threadIdx.x];
        ud = rec_ud[a0 + threadIdx.x];
    }
    stage_region<T, W, O32>(g, tc, box, u, T(1), (const T *)nullptr, reg);
    __syncthreads();
    float gmax[3] = {0.f, 0.f, 0.f};
    for (int e = threadIdx.x; e < n_own; e += blockDim.x) {
        const int j = a0 + e;
        const T4 ctn = tn, cud = ud;
        if (e + (int)blockDim.x < n_own) {
            tn = rec_tn[j + blockDim.x];
            ud = rec_ud[j + blockDim.x];
        }
        const T tt[3] = {ctn.x, ctn.y, ctn.z};
        int b[3];
        unpack_node(g, V4<T>::to_bits(ctn.w), b);
        T w[3][W];
        int d[3];
        for (int a = 0; a < 3; ++a)
            Delta<W, T>::w(tt[a], w[a]);
        region_base(g, box, b, d);
        T U[3] = {T(0), T(0), T(0)};
#pragma unroll
        for (int k = 0; k < W; ++k)
#pragma unroll
            for (int jj = 0; jj < W; ++jj) {
                const T wzy = w[2][k] * w[1][jj];
                const int row = ((d[2] + k) * R1 + (d[1] + jj)) * R0 + d[0];
#pragma unroll
                for (int i = 0; i < W; ++i) {
                    const T ww = wzy * w[0][i];
                    T vx, vy, vz;
                    reg_get<T>(reg, RV, row + i, vx, vy, vz);
                    U[0] += ww * vx;
                    U[1] += ww * vy;
                    U[2] += ww * vz;
                }
            }
        T G[3];
        double r2;
        marker_force<T>(g, c, cud, U, r2, G);
        if (MODE == 0) {
            if (U_dbg) {
                const int src = rec_src[j];
                for (int a = 0; a < 3; ++a)
                    U_dbg[((size_t)pass * 3 + a) * nm + src] = U[a];
            }
            T4 gp;
            gp.x = G[0];
            gp.y = G[1];
            gp.z = G[2];
            gp.w = (T)r2;
            rec_G[j] = gp;
            gmax[0] = fmaxf(gmax[0], fabsf((float)G[0]));
            gmax[1] = fmaxf(gmax[1], fabsf((float)G[1]));
            gmax[2] = fmaxf(gmax[2], fabsf((float)G[2]));
        } else {
            reinterpret_cast<T *>(rec_G + j)[3] = (T)r2;
        }
    }
    if (MODE == 0) {
        for (int a = 0; a < 3; ++a)
            gmax[a] = block_max<float>(gmax[a]);
        if (threadIdx.x == 0) {
            tile_max[tile] = make_float4(gmax[0], gmax[1], gmax[2], 0.f);
            float4 sm = make_float4(gmax[0], gmax[1], gmax[2], 0.f);
            if (pass > 0) {
                const float4 o = tile_max[tc.ntiles + tile];
                sm.x += o.x;
                sm.y += o.y;
                sm.z += o.z;
            }
            tile_max[tc.ntiles + tile] = sm;
        }
    }
}

template <typename T, int W, int MODE, bool O32, bool PERSIST>
__global__ __launch_bounds__(256) void k_interp(
    GridC g, TileC tc, int nm, int pass, double c, const int *__restrict__ tile_start,
    const typename V4<T>::type *__restrict__ rec_tn, const typename V4<T>::type *__restrict__ rec_ud,
    const int *__restrict__ rec_src, const T *__restrict__ u,
    typename V4<T>::type *__restrict__ rec_G, T *__restrict__ U_dbg,
    float4 *__restrict__ tile_max)
{
    if (PERSIST) {
        for (int v = blockIdx.x; v < tc.ntiles; v += gridDim.x) {
            interp_tile<T, W, MODE, O32>(xcd_remap(v, tc.ntiles), g, tc, nm, pass, c, tile_start,
                                         rec_tn, rec_ud, rec_src, u, rec_G, U_dbg, tile_max);
            __syncthreads();
        }
    } else {
        interp_tile<T, W, MODE, O32>(xcd_remap(blockIdx.x, gridDim.x), g, tc, nm, pass, c,
                                     tile_start, rec_tn, rec_ud, rec_src, u, rec_G, U_dbg,
                                     tile_max);
    }
}

// Particle sums after the passes, one wave per particle, markers in index
// order (64 at a time) and passes in order, all in FP64:
//   S_p = h^3 sum_l sum_m G_l^m,  T_p = h^3 sum_l o_l x sum_m G_l^m,
//   rpart[m][p] = sum_l dV |U^d - U^m|^2 (m <= n_iter, the last from the
//   residual pass on the final velocity, when want_res),
// and the pass-summed amplitude of every marker (rounded to T) for the f_tot
// spreading.  Nothing depends on scheduling or on the markers' tile order.
template <typename T>
__global__ __launch_bounds__(256) void k_particle_sums(
    int np, int nm, int n_iter, int want_res, double h3, const int *__restrict__ moff,
    const double *__restrict__ body, const int *__restrict__ m_inv,
    const typename V4<T>::type *__restrict__ rec_Gm, typename V4<T>::type *__restrict__ rec_Gs,
    double *__restrict__ S_out, double *__restrict__ T_out, double *__restrict__ rpart)
{
    typedef typename V4<T>::type T4;
    __shared__ double racc[4][IBMX_MAX_PASSES + 1];
    const int wv = threadIdx.x / IBMX_WAVE, lane = threadIdx.x & (IBMX_WAVE - 1);
    const int p = blockIdx.x * 4 + wv;
    if (p >= np)
        return;
    if (want_res)
        for (int m = lane; m <= n_iter; m += IBMX_WAVE)
            racc[wv][m] = 0.0;
    double sm[6] = {0, 0, 0, 0, 0, 0};
    const int l0 = moff[p], l1 = moff[p + 1];
    for (int lb = l0; lb < l1; lb += IBMX_WAVE) {
        const int l = lb + lane;
        const int j = l < l1 ? m_inv[l] : -1;
        double G[3] = {0.0, 0.0, 0.0};
        for (int m = 0; m < n_iter; ++m) {
            double r2 = 0.0;
            if (j >= 0) {
                const T4 gv = rec_Gm[(size_t)m * nm + j];
                G[0] += (double)gv.x;
                G[1] += (double)gv.y;
                G[2] += (double)gv.z;
                r2 = (double)gv.w;
            }
            if (want_res) {
                r2 = wave_sum(r2);
                if (lane == 0)
                    racc[wv][m] += r2;
            }
        }
        if (want_res) {
            double r2 = j >= 0 ? (double)reinterpret_cast<const T *>(rec_Gs + j)[3] : 0.0;
            r2 = wave_sum(r2);
            if (lane == 0)
                racc[wv][n_iter] += r2;
        }
        if (j < 0)
            continue;
        T4 gs;
        gs.x = (T)G[0];
        gs.y = (T)G[1];
        gs.z = (T)G[2];
        gs.w = T(0);
        rec_Gs[j] = gs;
        const double o[3] = {body[l], body[(size_t)nm + l], body[2 * (size_t)nm + l]};
        sm[0] += G[0];
        sm[1] += G[1];
        sm[2] += G[2];
        sm[3] += o[1] * G[2] - o[2] * G[1];
        sm[4] += o[2] * G[0] - o[0] * G[2];
        sm[5] += o[0] * G[1] - o[1] * G[0];
    }
#pragma unroll
    for (int q = 0; q < 6; ++q)
        sm[q] = wave_sum(sm[q]);
    if (lane == 0)
        for (int a = 0; a < 3; ++a) {
            S_out[(size_t)a * np + p] = h3 * sm[a];
            T_out[(size_t)a * np + p] = h3 * sm[3 + a];
        }
    if (want_res && lane == 0)
        for (int m = 0; m <= n_iter; ++m)
            rpart[(size_t)m * np + p] = racc[wv][m];
}

// ---------------------------------------------------------------------------
// Adjoint of the forcing loop.
//
// Reverse mode with the mask, body offsets, dV and c fixed.  The forward
// passes are replayed on a scratch copy of u^0, keeping per marker and pass
// the amplitude G^m and the Jacobian J^m = d U^m / d X of the interpolated
// velocity (the grids are not stored).  Then, for m = n .. 1, with ub the
// cotangent of u^m and fb = c ub + dL/df_tot the cotangent of f^m:
//   Fb  = dV/h^3 (I fb) + dV (g_S + g_T x o)        cotangent of F^m
//   Ub  = -Fb / c, Udb = Fb / c                     of U^m and U^d
//   Xb += J^T Ub + sum_x dw/dX (fb(x) . G^m)         delta-gradient terms
//   ub <- ub + I^T Ub                               (tile spreading of Ub)
// and finally g_u0 = ub, g_up = sum Udb, g_wp = sum o x Udb, g_xp = sum Xb.
// ---------------------------------------------------------------------------

// Forward replay of one pass: U, G and J for own markers (LDS-staged u).
template <typename T, int W>
__global__ __launch_bounds__(256) void k_interp_jac(
    GridC g, TileC tc, int nm, double c, const int *__restrict__ tile_start,
    const typename V4<T>::type *__restrict__ rec_tn, const typename V4<T>::type *__restrict__ rec_ud,
    const T *__restrict__ u, typename V4<T>::type *__restrict__ GJ)
{
    typedef typename V4<T>::type T4;
    extern __shared__ __align__(16) unsigned char smem[];
    T *reg = reinterpret_cast<T *>(smem);
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    const int a0 = tile_start[tile], n_own = tile_start[tile + 1] - a0;
    if (n_own == 0)
        return;
    const TileBox box(g, tc, tile);
    const int R0 = tc.B[0] + W - 1, R1 = tc.B[1] + W - 1, RV = R0 * R1 * (tc.B[2] + W - 1);
    stage_region<T, W>(g, tc, box, u, T(1), (const T *)nullptr, reg);
    __syncthreads();
    const T inv_h = (T)(1.0 / g.h);
    for (int e = threadIdx.x; e < n_own; e += blockDim.x) {
        const int j = a0 + e;
        const T4 tn = rec_tn[j], ud = rec_ud[j];
        const T tt[3] = {tn.x, tn.y, tn.z};
        int b[3], d[3];
        unpack_node(g, V4<T>::to_bits(tn.w), b);
        region_base(g, box, b, d);
        T w[3][W], dw[3][W];
        for (int a = 0; a < 3; ++a)
            Delta<W, T>::wd(tt[a], w[a], dw[a]);
        T U[3] = {T(0), T(0), T(0)};
        T J[3][3] = {{T(0), T(0), T(0)}, {T(0), T(0), T(0)}, {T(0), T(0), T(0)}};
#pragma unroll
        for (int k = 0; k < W; ++k)
#pragma unroll
            for (int jj = 0; jj < W; ++jj) {
                const int row = ((d[2] + k) * R1 + (d[1] + jj)) * R0 + d[0];
#pragma unroll
                for (int i = 0; i < W; ++i) {
                    const T ww = w[2][k] * w[1][jj] * w[0][i];
                    const T dx = w[2][k] * w[1][jj] * dw[0][i];
                    const T dy = w[2][k] * dw[1][jj] * w[0][i];
                    const T dz = dw[2][k] * w[1][jj] * w[0][i];
                    T vv[3];
                    reg_get<T>(reg, RV, row + i, vv[0], vv[1], vv[2]);
#pragma unroll
                    for (int cc = 0; cc < 3; ++cc) {
                        const T v = vv[cc];
                        U[cc] += ww * v;
                        J[cc][0] += dx * v;
                        J[cc][1] += dy * v;
                        J[cc][2] += dz * v;
                    }
                }
            }
        double r2;
        T G[3];
        marker_force<T>(g, c, ud, U, r2, G);
        T4 q0, q1, q2;
        q0.x = G[0];
        q0.y = G[1];
        q0.z = G[2];
        q0.w = J[0][0] * inv_h;
        q1.x = J[0][1] * inv_h;
        q1.y = J[0][2] * inv_h;
        q1.z = J[1][0] * inv_h;
        q1.w = J[1][1] * inv_h;
        q2.x = J[1][2] * inv_h;
        q2.y = J[2][0] * inv_h;
        q2.z = J[2][1] * inv_h;
        q2.w = J[2][2] * inv_h;
        GJ[j] = q0;
        GJ[nm + j] = q1;
        GJ[2 * (size_t)nm + j] = q2;
    }
}

// Adjoint interpolation of one pass (own markers): Ub for the spreading,
// and the per-marker accumulation of Udb and Xb.
template <typename T, int W, int FIRST>
__global__ __launch_bounds__(256) void k_interp_adj(
    GridC g, TileC tc, int nm, int np, double c, const int *__restrict__ tile_start,
    const typename V4<T>::type *__restrict__ rec_tn, const int *__restrict__ rec_src,
    const double *__restrict__ body, const int *__restrict__ pid_of,
    const double *__restrict__ dV, const double *__restrict__ gS, const double *__restrict__ gT,
    const T *__restrict__ ub, const T *__restrict__ gf, const typename V4<T>::type *__restrict__ GJ,
    typename V4<T>::type *__restrict__ Ub_out, double4 *__restrict__ accA,
    double4 *__restrict__ accB)
{
    typedef typename V4<T>::type T4;
    extern __shared__ __align__(16) unsigned char smem[];
    T *reg = reinterpret_cast<T *>(smem);
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    const int a0 = tile_start[tile], n_own = tile_start[tile + 1] - a0;
    if (n_own == 0)
        return;
    const TileBox box(g, tc, tile);
    const int R0 = tc.B[0] + W - 1, R1 = tc.B[1] + W - 1, RV = R0 * R1 * (tc.B[2] + W - 1);
    stage_region<T, W>(g, tc, box, ub, (T)c, gf, reg);   // fb = c ub + g_f
    __syncthreads();
    const double inv_h = 1.0 / g.h;
    for (int e = threadIdx.x; e < n_own; e += blockDim.x) {
        const int j = a0 + e;
        const T4 tn = rec_tn[j];
        const int l = rec_src[j];
        const T tt[3] = {tn.x, tn.y, tn.z};
        const double o[3] = {body[l], body[(size_t)nm + l], body[2 * (size_t)nm + l]};
        const int pid = pid_of[l];
        const T4 q0 = GJ[j], q1 = GJ[nm + j], q2 = GJ[2 * (size_t)nm + j];
        const T G[3] = {q0.x, q0.y, q0.z};
        const double Jm[3][3] = {{(double)q0.w, (double)q1.x, (double)q1.y},
                                 {(double)q1.z, (double)q1.w, (double)q2.x},
                                 {(double)q2.y, (double)q2.z, (double)q2.w}};
        int b[3], d[3];
        unpack_node(g, V4<T>::to_bits(tn.w), b);
        region_base(g, box, b, d);
        T w[3][W], dw[3][W];
        for (int a = 0; a < 3; ++a)
            Delta<W, T>::wd(tt[a], w[a], dw[a]);
        T IF[3] = {T(0), T(0), T(0)}, P[3] = {T(0), T(0), T(0)};
#pragma unroll
        for (int k = 0; k < W; ++k)
#pragma unroll
            for (int jj = 0; jj < W; ++jj) {
                const int row = ((d[2] + k) * R1 + (d[1] + jj)) * R0 + d[0];
#pragma unroll
                for (int i = 0; i < W; ++i) {
                    const T ww = w[2][k] * w[1][jj] * w[0][i];
                    T f0, f1, f2;
                    reg_get<T>(reg, RV, row + i, f0, f1, f2);
                    IF[0] += ww * f0;
                    IF[1] += ww * f1;
                    IF[2] += ww * f2;
                    const T fg = f0 * G[0] + f1 * G[1] + f2 * G[2];
                    P[0] += w[2][k] * w[1][jj] * dw[0][i] * fg;
                    P[1] += w[2][k] * dw[1][jj] * w[0][i] * fg;
                    P[2] += dw[2][k] * w[1][jj] * w[0][i] * fg;
                }
            }
        const double dVp = dV[pid], v = dVp * g.inv_h3;
        double gs[3] = {0.0, 0.0, 0.0}, gt[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < 3; ++a) {
            if (gS)
                gs[a] = gS[(size_t)a * np + pid];
            if (gT)
                gt[a] = gT[(size_t)a * np + pid];
        }
        const double gtxo[3] = {gt[1] * o[2] - gt[2] * o[1], gt[2] * o[0] - gt[0] * o[2],
                                gt[0] * o[1] - gt[1] * o[0]};
        double Ubv[3], Udb[3];
        for (int a = 0; a < 3; ++a) {
            const double Fb = v * (double)IF[a] + dVp * (gs[a] + gtxo[a]);
            Ubv[a] = -Fb / c;
            Udb[a] = Fb / c;
        }
        double Xb[3];
        for (int a = 0; a < 3; ++a)
            Xb[a] = Jm[0][a] * Ubv[0] + Jm[1][a] * Ubv[1] + Jm[2][a] * Ubv[2] + (double)P[a] * inv_h;
        T4 ubo;
        ubo.x = (T)Ubv[0];
        ubo.y = (T)Ubv[1];
        ubo.z = (T)Ubv[2];
        ubo.w = T(0);
        Ub_out[j] = ubo;
        double4 A = make_double4(Udb[0], Udb[1], Udb[2], 0.0);
        double4 B = make_double4(Xb[0], Xb[1], Xb[2], 0.0);
        if (!FIRST) {
            const double4 A0 = accA[j], B0 = accB[j];
            A.x += A0.x;
            A.y += A0.y;
            A.z += A0.z;
            B.x += B0.x;
            B.y += B0.y;
            B.z += B0.z;
        }
        accA[j] = A;
        accB[j] = B;
    }
}

// Particle gradients from the per-marker accumulations (index order).
__global__ __launch_bounds__(256) void k_particle_grad(int np, int nm, const int *__restrict__ moff,
                                                       const double *__restrict__ body,
                                                       const int *__restrict__ m_inv,
                                                       const double4 *__restrict__ accA,
                                                       const double4 *__restrict__ accB,
                                                       double *__restrict__ gxp,
                                                       double *__restrict__ gup,
                                                       double *__restrict__ gwp)
{
    const int wv = threadIdx.x / IBMX_WAVE, lane = threadIdx.x & (IBMX_WAVE - 1);
    const int p = blockIdx.x * 4 + wv;
    if (p >= np)
        return;
    double sm[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int l = moff[p] + lane; l < moff[p + 1]; l += IBMX_WAVE) {
        const int j = m_inv[l];
        if (j < 0)
            continue;
        const double4 A = accA[j], B = accB[j];
        const double o[3] = {body[l], body[(size_t)nm + l], body[2 * (size_t)nm + l]};
        sm[0] += A.x;
        sm[1] += A.y;
        sm[2] += A.z;
        sm[3] += o[1] * A.z - o[2] * A.y;
        sm[4] += o[2] * A.x - o[0] * A.z;
        sm[5] += o[0] * A.y - o[1] * A.x;
        sm[6] += B.x;
        sm[7] += B.y;
        sm[8] += B.z;
    }
#pragma unroll
    for (int q = 0; q < 9; ++q)
        sm[q] = wave_sum(sm[q]);
    if (lane == 0)
        for (int a = 0; a < 3; ++a) {
            gup[(size_t)a * np + p] = sm[a];
            gwp[(size_t)a * np + p] = sm[3 + a];
            gxp[(size_t)a * np + p] = sm[6 + a];
        }
}

template <typename T>
__global__ void k_copy(T *__restrict__ dst, const T *__restrict__ src, long long n)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += stride)
        dst[i] = src[i];
}

template <typename T>
__global__ void k_zero(T *__restrict__ dst, long long n)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += stride)
        dst[i] = T(0);
}

// resid[pass] = sqrt of the sum of the pass's per-particle partials, added
// in a fixed order (one block per pass)
__global__ __launch_bounds__(1024) void k_finish_resid(const double *__restrict__ rpart, int np,
                                                       double *__restrict__ resid)
{
    double v = 0.0;
    for (int i = threadIdx.x; i < np; i += blockDim.x)
        v += rpart[(size_t)blockIdx.x * np + i];
    v = block_sum<double>(v);
    if (threadIdx.x == 0)
        resid[blockIdx.x] = sqrt(v);
}

int nblocks(long long n, int b) { return (int)((n + b - 1) / b) > 0 ? (int)((n + b - 1) / b) : 1; }

template <typename T, int W>
size_t interp_lds(const TileC &tc)
{
    return (size_t)3 * (tc.B[0] + W - 1) * (tc.B[1] + W - 1) * (tc.B[2] + W - 1) * sizeof(T);
}

template <typename T>
size_t spread_lds(const TileC &tc)
{
    return (size_t)SpreadAcc<T>::BYTES * (tc.B[0] + 1) * tc.B[1] * tc.B[2];
}

// Workgroups of a persistent pass launch: as many as the CUs hold at once
// (LDS-limited, at most 8 per CU), a multiple of the 8 XCDs, no more than
// the tiles.
int persist_grid(const ibmx_plan p, size_t lds)
{
    int per_cu = lds > 0 ? (int)((160 * 1024) / lds) : 8;
    per_cu = per_cu < 1 ? 1 : (per_cu > 8 ? 8 : per_cu);
    const long long g = 256LL * per_cu;
    const long long nt8 = ((long long)p->tc.ntiles + 7) / 8 * 8;
    return (int)(g < nt8 ? g : nt8);
}

// the tile kernels with 32-bit grid offsets when every component spans
// less than 4 GB
template <typename T>
bool offsets32(ibmx_plan p)
{
    return (unsigned long long)p->g.nodes * sizeof(T) < (1ULL << 32);
}

template <typename T, int W, int MODE, bool O32, typename... A>
void launch_interp_o(ibmx_plan p, size_t lds, hipStream_t s, A... args)
{
    if (p->persist)
        hipLaunchKernelGGL((k_interp<T, W, MODE, O32, true>), dim3(persist_grid(p, lds)),
                           dim3(p->block), lds, s, args...);
    else
        hipLaunchKernelGGL((k_interp<T, W, MODE, O32, false>), dim3(p->tc.ntiles),
                           dim3(p->block), lds, s, args...);
}

template <typename T, int W, int MODE, typename... A>
void launch_interp(ibmx_plan p, size_t lds, hipStream_t s, A... args)
{
    if (offsets32<T>(p))
        launch_interp_o<T, W, MODE, true>(p, lds, s, args...);
    else
        launch_interp_o<T, W, MODE, false>(p, lds, s, args...);
}

template <typename T, int W, bool O32, bool AU, bool AF, typename... A>
void launch_spread_k(ibmx_plan p, size_t lds, hipStream_t s, A... args)
{
    if (p->persist)
        hipLaunchKernelGGL((k_spread<T, W, O32, true, AU, AF>), dim3(persist_grid(p, lds)),
                           dim3(p->block), lds, s, args...);
    else
        hipLaunchKernelGGL((k_spread<T, W, O32, false, AU, AF>), dim3(p->tc.ntiles),
                           dim3(p->block), lds, s, args...);
}

// spreading launch: u += c f (add_u) and / or f_tot += f (add_f)
template <typename T, int W, bool O32, typename... A>
void launch_spread_o(ibmx_plan p, size_t lds, hipStream_t s, GridC g, TileC tc, T c, int add_u,
                     int add_f, A... args)
{
    if (add_u && add_f)
        launch_spread_k<T, W, O32, true, true>(p, lds, s, g, tc, c, args...);
    else if (add_u)
        launch_spread_k<T, W, O32, true, false>(p, lds, s, g, tc, c, args...);
    else
        launch_spread_k<T, W, O32, false, true>(p, lds, s, g, tc, c, args...);
}

template <typename T, int W, typename... A>
void launch_spread(ibmx_plan p, size_t lds, hipStream_t s, A... args)
{
    if (offsets32<T>(p))
        launch_spread_o<T, W, true>(p, lds, s, args...);
    else
        launch_spread_o<T, W, false>(p, lds, s, args...);
}

// Marker geometry and binning of one call: tile counts, sorted records,
// halo lists, and the zeroed per-call counters.
template <typename T, int W>
void bin_markers(ibmx_plan p, const double *xp, const double *up, const double *wp,
                 const uint8_t *mask)
{
    typedef typename V4<T>::type T4;
    hipStream_t s = p->stream;
    const int nm = p->nm, np = p->np;
    const TileC tc = p->tc;
    const int ntiles = tc.ntiles;
    T4 *rec_tn = (T4 *)p->rec_tn, *rec_ud = (T4 *)p->rec_ud;
    {
        ProfScope ps(p, IBMX_K_OTHER);
        ZeroList z = {};
        z.add((int *)p->d_count, 16LL * IBMX_RSLOTS);
        z.add(p->tile_count, ntiles + 1);
        z.add(p->tile_cursor, ntiles + 1);
        z.add(p->halo_count, ntiles + 1);
        z.add(p->halo_cursor, ntiles + 1);
        ibmx_zero_i32_multi(z, s);
    }
    ProfScope ps(p, IBMX_K_GEOMETRY);
    if (np > 0 && nm > 0) {
        const int gb = nblocks(nm, 256);
        hipLaunchKernelGGL((k_bin_count<T, W>), dim3(gb), dim3(256), 0, s, p->g, tc, np, nm,
                           p->d_pid, p->body, xp, mask, p->m_key, p->tile_count, p->halo_count,
                           p->d_err, p->d_count);
        ibmx_exclusive_scan(p->tile_count, p->tile_start, ntiles, p->scan_aux, s);
        ibmx_exclusive_scan(p->halo_count, p->halo_start, ntiles, p->scan_aux, s);
        hipLaunchKernelGGL((k_bin_scatter<T, W>), dim3(gb), dim3(256), 0, s, p->g, tc, np, nm,
                           p->d_pid, p->body, xp, up, wp, p->dV, p->m_key, p->tile_start,
                           p->tile_cursor, rec_tn, rec_ud, p->rec_src, p->m_inv, p->halo_start,
                           p->halo_cursor, p->halo_list, p->halo_cap, p->d_err);
    } else {
        ibmx_exclusive_scan(p->tile_count, p->tile_start, ntiles, p->scan_aux, s);
        ibmx_exclusive_scan(p->halo_count, p->halo_start, ntiles, p->scan_aux, s);
    }
}

template <typename T, int W>
ibmx_status run_forcing(ibmx_plan p, T *u, T *f_tot, const double *xp, const double *up,
                        const double *wp, const uint8_t *mask, double *S_out, double *T_out,
                        double *resid_out, T *U_dbg)
{
    typedef typename V4<T>::type T4;
    hipStream_t s = p->stream;
    const int nm = p->nm, np = p->np, n_iter = p->prm.n_iter;
    const double c = p->prm.two_alpha_dt;
    const TileC tc = p->tc;
    const int ntiles = tc.ntiles;
    T4 *rec_tn = (T4 *)p->rec_tn, *rec_ud = (T4 *)p->rec_ud;
    T4 *rec_Gm = (T4 *)p->rec_Gp, *rec_Gs = (T4 *)p->rec_G;
    // per-tile amplitude bounds: [0, ntiles) the pass, [ntiles, 2 ntiles)
    // the sum over the passes so far
    float4 *tmax = p->tile_gmax;
    if (nm == 0 || np == 0) {
        ProfScope ps(p, IBMX_K_OTHER);
        ibmx_fill_f64(S_out, 0.0, 3LL * np, s);
        ibmx_fill_f64(T_out, 0.0, 3LL * np, s);
        if (resid_out)
            ibmx_fill_f64(resid_out, 0.0, n_iter + 1, s);
        ibmx_fill_i32((int *)p->d_count, 0, 16LL * IBMX_RSLOTS, s);
        return ibmx_launch_check();
    }
    bin_markers<T, W>(p, xp, up, wp, mask);
    const size_t lds_i = interp_lds<T, W>(tc), lds_s = spread_lds<T>(tc);
    for (int m = 0; m < n_iter; ++m) {
        T4 *Gm = rec_Gm + (size_t)m * nm;
        {
            ProfScope ps(p, IBMX_K_INTERP);
            launch_interp<T, W, 0>(p, lds_i, s, p->g, tc, nm, m, c, (const int *)p->tile_start,
                                   (const T4 *)rec_tn, (const T4 *)rec_ud, (const int *)p->rec_src,
                                   (const T *)u, Gm, U_dbg, tmax);
        }
        // u += c f^m (and, with a single pass, f_tot += f^m)
        ProfScope ps(p, IBMX_K_SPREAD);
        launch_spread<T, W>(p, lds_s, s, p->g, tc, (T)c, 1, n_iter == 1 ? 1 : 0,
                            n_iter == 1 ? 1 : 0, (const int *)p->tile_start,
                            (const int *)p->halo_start, (const int *)p->halo_list,
                            (const T4 *)rec_tn, (const T4 *)Gm, (const float4 *)tmax, u, f_tot,
                            p->d_count);
    }
    if (resid_out) {
        // residual terms on the final velocity, into the w of the summed-
        // amplitude records (read by the particle sums before they write G)
        ProfScope ps(p, IBMX_K_OTHER);
        launch_interp<T, W, 2>(p, lds_i, s, p->g, tc, nm, n_iter, c, (const int *)p->tile_start,
                               (const T4 *)rec_tn, (const T4 *)rec_ud, (const int *)p->rec_src,
                               (const T *)u, rec_Gs, (T *)nullptr, (float4 *)nullptr);
    }
    {
        ProfScope ps(p, IBMX_K_OTHER);
        hipLaunchKernelGGL((k_particle_sums<T>), dim3(nblocks(np, 4)), dim3(256), 0, s, np, nm,
                           n_iter, resid_out ? 1 : 0, p->g.h * p->g.h * p->g.h,
                           (const int *)p->d_moff, p->body, (const int *)p->m_inv,
                           (const T4 *)rec_Gm, rec_Gs, S_out, T_out, p->rpart);
        if (resid_out)
            hipLaunchKernelGGL(k_finish_resid, dim3(n_iter + 1), dim3(1024), 0, s,
                               (const double *)p->rpart, np, resid_out);
    }
    if (n_iter >= 2) {
        // f_tot += spread of the amplitudes summed over the passes
        ProfScope ps(p, IBMX_K_FTOT);
        launch_spread<T, W>(p, lds_s, s, p->g, tc, (T)c, 0, 1, 1, (const int *)p->tile_start,
                            (const int *)p->halo_start, (const int *)p->halo_list,
                            (const T4 *)rec_tn, (const T4 *)rec_Gs,
                            (const float4 *)(tmax + ntiles), u, f_tot, p->d_count);
    }
    return ibmx_launch_check();
}

template <typename T, int W>
ibmx_status run_backward(ibmx_plan p, const T *u0, const double *xp, const double *up,
                         const double *wp, const uint8_t *mask, const T *g_f, const T *g_u,
                         const double *g_S, const double *g_T, T *gu0, double *gxp, double *gup,
                         double *gwp)
{
    typedef typename V4<T>::type T4;
    hipStream_t s = p->stream;
    const int nm = p->nm, np = p->np, n_iter = p->prm.n_iter;
    const double c = p->prm.two_alpha_dt;
    const TileC tc = p->tc;
    const int ntiles = tc.ntiles;
    const long long G3 = 3 * p->g.nodes;
    T4 *rec_tn = (T4 *)p->rec_tn, *rec_ud = (T4 *)p->rec_ud, *rec_Ub = (T4 *)p->rec_Gp;
    // workspace (from ibmx_plan_reserve): replay grid, per-pass G and
    // Jacobian, per-marker sums
    if (!p->bw_u || p->bw_bytes < ibmx_backward_bytes(p))
        return IBMX_ESTATE;
    T *us = (T *)p->bw_u;
    T4 *GJ = (T4 *)(us + G3);
    double4 *accA = (double4 *)(GJ + 3 * (size_t)nm * p->n_iter_cap);
    double4 *accB = accA + nm;
    bin_markers<T, W>(p, xp, up, wp, mask);
    const int cb = 4096;
    {
        ProfScope ps(p, IBMX_K_OTHER);
        hipLaunchKernelGGL((k_copy<T>), dim3(cb), dim3(256), 0, s, us, u0, G3);
        if (g_u)
            hipLaunchKernelGGL((k_copy<T>), dim3(cb), dim3(256), 0, s, gu0, g_u, G3);
        else
            hipLaunchKernelGGL((k_zero<T>), dim3(cb), dim3(256), 0, s, gu0, G3);
        ibmx_fill_f64(gxp, 0.0, 3LL * np, s);
        ibmx_fill_f64(gup, 0.0, 3LL * np, s);
        ibmx_fill_f64(gwp, 0.0, 3LL * np, s);
    }
    if (nm > 0) {
        const size_t lds_i = interp_lds<T, W>(tc), lds_s = spread_lds<T>(tc);
        ProfScope ps(p, IBMX_K_BACKWARD);
        for (int m = 0; m < n_iter; ++m) {
            T4 *GJm = GJ + 3 * (size_t)nm * m;
            hipLaunchKernelGGL((k_interp_jac<T, W>), dim3(ntiles), dim3(256), lds_i, s, p->g, tc, nm,
                               c, p->tile_start, (const T4 *)rec_tn, (const T4 *)rec_ud,
                               (const T *)us, GJm);
            if (m < n_iter - 1)
                launch_spread<T, W>(p, lds_s, s, p->g, tc, (T)c, 1, 0, 0,
                                    (const int *)p->tile_start, (const int *)p->halo_start,
                                    (const int *)p->halo_list, (const T4 *)rec_tn,
                                    (const T4 *)GJm, (const float4 *)nullptr, us, (T *)nullptr,
                                    p->d_count);
        }
        for (int m = n_iter - 1; m >= 0; --m) {
            const T4 *GJm = GJ + 3 * (size_t)nm * m;
            if (m == n_iter - 1)
                hipLaunchKernelGGL((k_interp_adj<T, W, 1>), dim3(ntiles), dim3(256), lds_i, s, p->g,
                                   tc, nm, np, c, p->tile_start, (const T4 *)rec_tn,
                                   p->rec_src, p->body, p->d_pid, p->dV, g_S, g_T,
                                   (const T *)gu0, g_f, GJm, rec_Ub, accA, accB);
            else
                hipLaunchKernelGGL((k_interp_adj<T, W, 0>), dim3(ntiles), dim3(256), lds_i, s, p->g,
                                   tc, nm, np, c, p->tile_start, (const T4 *)rec_tn,
                                   p->rec_src, p->body, p->d_pid, p->dV, g_S, g_T,
                                   (const T *)gu0, g_f, GJm, rec_Ub, accA, accB);
            launch_spread<T, W>(p, lds_s, s, p->g, tc, T(1), 1, 0, 0, (const int *)p->tile_start,
                                (const int *)p->halo_start, (const int *)p->halo_list,
                                (const T4 *)rec_tn, (const T4 *)rec_Ub, (const float4 *)nullptr,
                                gu0, (T *)nullptr, p->d_count);
        }
        if (np > 0)
            hipLaunchKernelGGL(k_particle_grad, dim3(nblocks(np, 4)), dim3(256), 0, s, np, nm,
                               p->d_moff, p->body, p->m_inv, (const double4 *)accA,
                               (const double4 *)accB, gxp, gup, gwp);
    }
    return ibmx_launch_check();
}

template <typename T, int W>
hipError_t allow_lds_w(int bytes_interp, int bytes_spread)
{
    hipError_t e;
    const void *spreads[] = {
        (const void *)k_spread<T, W, true, false, true, false>,
        (const void *)k_spread<T, W, false, false, true, false>,
        (const void *)k_spread<T, W, true, true, true, false>,
        (const void *)k_spread<T, W, false, true, true, false>,
        (const void *)k_spread<T, W, true, false, false, true>,
        (const void *)k_spread<T, W, false, false, false, true>,
        (const void *)k_spread<T, W, true, true, false, true>,
        (const void *)k_spread<T, W, false, true, false, true>,
        (const void *)k_spread<T, W, true, false, true, true>,
        (const void *)k_spread<T, W, false, false, true, true>,
        (const void *)k_spread<T, W, true, true, true, true>,
        (const void *)k_spread<T, W, false, true, true, true>};
    for (const void *f : spreads)
        if ((e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes_spread)) !=
            hipSuccess)
            return e;
    const void *interps[] = {(const void *)k_interp<T, W, 0, true, false>,
                             (const void *)k_interp<T, W, 2, true, false>,
                             (const void *)k_interp<T, W, 0, false, false>,
                             (const void *)k_interp<T, W, 2, false, false>,
                             (const void *)k_interp<T, W, 0, true, true>,
                             (const void *)k_interp<T, W, 2, true, true>,
                             (const void *)k_interp<T, W, 0, false, true>,
                             (const void *)k_interp<T, W, 2, false, true>,
                             (const void *)k_interp_jac<T, W>,
                             (const void *)k_interp_adj<T, W, 0>, (const void *)k_interp_adj<T, W, 1>};
    for (const void *f : interps)
        if ((e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes_interp)) !=
            hipSuccess)
            return e;
    return hipSuccess;
}

}  // namespace

// Adjoint workspace: the replay grid T[3][nodes], per-pass amplitude and
// Jacobian T4[n_iter][3][nm], two double4[nm] per-marker sums.
size_t ibmx_backward_bytes(ibmx_plan p)
{
    const size_t Ts = p->prec == IBMX_F64 ? sizeof(double) : sizeof(float);
    const size_t nm = (size_t)(p->nm > 0 ? p->nm : 1);
    return Ts * 3 * (size_t)p->g.nodes + 3 * 4 * Ts * nm * (size_t)p->n_iter_cap +
           2 * sizeof(double4) * nm;
}

// Allow the tile kernels the plan's LDS footprint (above 64 KB needs an
// explicit opt-in).
ibmx_status ibmx_spread_allow_lds(ibmx_plan p)
{
    const size_t ls = p->prec == IBMX_F64 ? spread_lds<double>(p->tc) : spread_lds<float>(p->tc);
    const size_t l3 = p->prec == IBMX_F64 ? interp_lds<double, 3>(p->tc) : interp_lds<float, 3>(p->tc);
    const size_t l4 = p->prec == IBMX_F64 ? interp_lds<double, 4>(p->tc) : interp_lds<float, 4>(p->tc);
    if (ls > 160 * 1024 || l4 > 160 * 1024)
        return IBMX_EUNSUPPORTED;
    hipError_t e;
    if (p->prec == IBMX_F64) {
        e = allow_lds_w<double, 3>((int)l3, (int)ls);
        if (e == hipSuccess)
            e = allow_lds_w<double, 4>((int)l4, (int)ls);
    } else {
        e = allow_lds_w<float, 3>((int)l3, (int)ls);
        if (e == hipSuccess)
            e = allow_lds_w<float, 4>((int)l4, (int)ls);
    }
    return e == hipSuccess ? IBMX_OK : IBMX_EUNSUPPORTED;
}

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
    // the particle sums keep n_iter + 1 residual slots per wave in LDS
    if (p->prm.n_iter < 1 || p->prm.n_iter > IBMX_MAX_PASSES)
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

extern "C" ibmx_status ibmx_forcing_backward(ibmx_plan p, const void *u0, const double *xp,
                                             const double *up, const double *wp,
                                             const uint8_t *marker_active, const void *g_f,
                                             const void *g_u, const double *g_S,
                                             const double *g_T, void *gu0, double *gxp,
                                             double *gup, double *gwp)
{
    if (!p)
        return IBMX_EINVAL;
    if (p->nm > 0 && (!p->body || !p->dV))
        return IBMX_ESTATE;
    if (!u0 || !gu0 || (p->np > 0 && (!xp || !up || !wp || !gxp || !gup || !gwp)))
        return IBMX_EINVAL;
    const int W = p->prm.kernel;
    if (p->prec == IBMX_F64) {
        if (W == 3)
            return run_backward<double, 3>(p, (const double *)u0, xp, up, wp, marker_active,
                                           (const double *)g_f, (const double *)g_u, g_S, g_T,
                                           (double *)gu0, gxp, gup, gwp);
        return run_backward<double, 4>(p, (const double *)u0, xp, up, wp, marker_active,
                                       (const double *)g_f, (const double *)g_u, g_S, g_T,
                                       (double *)gu0, gxp, gup, gwp);
    }
    if (W == 3)
        return run_backward<float, 3>(p, (const float *)u0, xp, up, wp, marker_active,
                                      (const float *)g_f, (const float *)g_u, g_S, g_T,
                                      (float *)gu0, gxp, gup, gwp);
    return run_backward<float, 4>(p, (const float *)u0, xp, up, wp, marker_active,
                                  (const float *)g_f, (const float *)g_u, g_S, g_T, (float *)gu0,
                                  gxp, gup, gwp);
}

