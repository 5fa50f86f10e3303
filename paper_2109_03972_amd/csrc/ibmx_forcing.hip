// Outer forcing loop of the collocated direct-forcing IBM (Sec. 2.2.2).
//
// Data flow of one ibmx_forcing call
//   binning    (once)  marker geometry in FP64 (X_l = x_p + o_l -> base node,
//                      fractional offsets, periodic wrap, wall check), then a
//                      counting sort of the active markers by the spatial tile
//                      of their centre node.  Markers of one particle stay
//                      contiguous and in index order inside a tile.
//   halo lists (once)  for every tile, the markers of neighbouring tiles whose
//                      delta support reaches into it.
//   per pass           interpolation (one thread per sorted marker, gathers
//                      through the caches): U_l, F_l = (U^d_l - U_l)/c, the
//                      spreading amplitude G_l = F_l dV_l / h^3, and the FP64
//                      particle sums and residual (wave-segmented reductions).
//                      Spreading (one workgroup per tile): every marker whose
//                      support reaches the tile adds w G_l into an LDS copy of
//                      the tile; the workgroup then owns the tile's nodes and
//                      updates u += c f and f_tot += f with plain stores -- no
//                      global atomics.
// The interpolation kernel of a pass finishes before its spreading kernel
// starts, so u is updated in place: u^m = u^{m-1} + c f^{m-1}.
#include <math.h>

#include "ibmx_internal.hpp"
#include "ibmx_delta.hpp"

namespace {

constexpr int TS = IBMX_BIN_SLOTS;   // per-particle tile table (open addressing)
constexpr int NXCD = 8;              // MI355X: 8 XCDs, workgroups dealt round-robin

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
            bb %= g.n[a];
            if (bb < 0)
                bb += g.n[a];
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
        ti[a] = axis_node(g, a, b[a], 1) / tc.B[a];
    return ti[0] + tc.nt[0] * (ti[1] + tc.nt[1] * ti[2]);
}

__device__ __forceinline__ unsigned long long lanemask_lt(int lane)
{
    return (1ull << lane) - 1ull;
}

// open-addressing lookup/insert of a tile id in a wave-private table
__device__ __forceinline__ int table_slot(volatile int *keys, int key)
{
    unsigned h = ((unsigned)key * 2654435761u) >> (32 - IBMX_BIN_SLOTS_LOG2);
    for (int probe = 0; probe < TS; ++probe) {
        int s = (int)((h + probe) & (TS - 1));
        int k = keys[s];
        if (k == key)
            return s;
        if (k < 0) {
            keys[s] = key;
            return s;
        }
    }
    return -1;
}

// ---------------------------------------------------------------------------
// binning step A: one wave per particle.  Tile key and rank of every active
// marker among the particle's markers of the same tile (in index order), and
// the per-tile counts.
// ---------------------------------------------------------------------------
template <int W>
__global__ __launch_bounds__(256) void k_bin_count(
    GridC g, TileC tc, int np, int nm, const int *__restrict__ moff,
    const double *__restrict__ body, const double *__restrict__ xp,
    const uint8_t *__restrict__ mask, int *__restrict__ m_key, int *__restrict__ m_rank,
    int *__restrict__ tab, int *__restrict__ tile_count, int *__restrict__ err,
    long long *__restrict__ count)
{
    __shared__ int s_keys[4][TS];
    __shared__ int s_cnt[4][TS];
    const int wv = threadIdx.x / IBMX_WAVE, lane = threadIdx.x & (IBMX_WAVE - 1);
    const int p = blockIdx.x * 4 + wv;
    if (p >= np)
        return;
    volatile int *keys = s_keys[wv];
    volatile int *cnt = s_cnt[wv];
    for (int s = lane; s < TS; s += IBMX_WAVE) {
        keys[s] = -1;
        cnt[s] = 0;
    }
    const double xc[3] = {xp[p], xp[np + p], xp[2 * np + p]};
    const int l0 = moff[p], l1 = moff[p + 1];
    int active = 0;
    for (int base = l0; base < l1; base += IBMX_WAVE) {
        const int l = base + lane;
        int key = -1;
        if (l < l1 && (!mask || mask[l])) {
            double X[3], t[3];
            int b[3];
            for (int a = 0; a < 3; ++a)
                X[a] = xc[a] + body[(size_t)a * nm + l];
            if (marker_geometry<W>(g, X, b, t))
                key = home_tile(g, tc, b);
            else
                atomicCAS(err, 0, (int)IBMX_EDOMAIN);
        }
        active += key >= 0;
        unsigned long long pending = __ballot(key >= 0);
        while (pending) {
            const int leader = __ffsll((long long)pending) - 1;
            const int k = __shfl(key, leader, IBMX_WAVE);
            const unsigned long long m = __ballot(key == k) & pending;
            int slot = 0;
            if (lane == leader)
                slot = table_slot(keys, k);
            slot = __shfl(slot, leader, IBMX_WAVE);
            if (slot < 0) {
                if (lane == leader)
                    atomicCAS(err, 0, (int)IBMX_EUNSUPPORTED);
                if (key == k)
                    m_key[l] = -1;
            } else {
                if (key == k) {
                    m_key[l] = slot;
                    m_rank[l] = cnt[slot] + __popcll(m & lanemask_lt(lane));
                }
                if (lane == leader)
                    cnt[slot] = cnt[slot] + __popcll(m);
            }
            pending &= ~m;
        }
        if (key < 0 && l < l1)
            m_key[l] = -1;
    }
    int *mytab = tab + (size_t)p * 2 * TS;
    for (int s = lane; s < TS; s += IBMX_WAVE) {
        int k = keys[s];
        mytab[s] = k;
        mytab[TS + s] = cnt[s];
        if (k >= 0)
            atomicAdd(&tile_count[k], cnt[s]);
    }
    active = wave_sum_i(active);
    if (lane == 0 && active)
        atomicAdd((unsigned long long *)&count[0], (unsigned long long)active);
}

// ---------------------------------------------------------------------------
// binning step B: one wave per particle.  Reserve the particle's segment in
// every tile it touches and write the sorted marker records.
// ---------------------------------------------------------------------------
template <typename T, int W>
__global__ __launch_bounds__(256) void k_bin_scatter(
    GridC g, int np, int nm, const int *__restrict__ moff, const double *__restrict__ body,
    const double *__restrict__ xp, const int *__restrict__ m_key, const int *__restrict__ m_rank,
    const int *__restrict__ tab, const int *__restrict__ tile_start, int *__restrict__ tile_cursor,
    unsigned *__restrict__ rec_node, T *__restrict__ rec_t, T *__restrict__ rec_o,
    int *__restrict__ rec_pid, int *__restrict__ rec_src)
{
    __shared__ int s_base[4][TS];
    const int wv = threadIdx.x / IBMX_WAVE, lane = threadIdx.x & (IBMX_WAVE - 1);
    const int p = blockIdx.x * 4 + wv;
    if (p >= np)
        return;
    volatile int *base_of = s_base[wv];
    const int *mytab = tab + (size_t)p * 2 * TS;
    for (int s = lane; s < TS; s += IBMX_WAVE) {
        int k = mytab[s];
        base_of[s] = k >= 0 ? tile_start[k] + atomicAdd(&tile_cursor[k], mytab[TS + s]) : 0;
    }
    const double xc[3] = {xp[p], xp[np + p], xp[2 * np + p]};
    const int l0 = moff[p], l1 = moff[p + 1];
    for (int l = l0 + lane; l < l1; l += IBMX_WAVE) {
        const int slot = m_key[l];
        if (slot < 0)
            continue;
        const int dst = base_of[slot] + m_rank[l];
        double X[3], t[3], o[3];
        int b[3];
        for (int a = 0; a < 3; ++a) {
            o[a] = body[(size_t)a * nm + l];
            X[a] = xc[a] + o[a];
        }
        marker_geometry<W>(g, X, b, t);
        rec_node[dst] = pack_node(g, b[0], b[1], b[2]);
        for (int a = 0; a < 3; ++a) {
            rec_t[(size_t)a * nm + dst] = (T)t[a];
            rec_o[(size_t)a * nm + dst] = (T)o[a];
        }
        rec_pid[dst] = p;
        rec_src[dst] = l;
    }
}

// ---------------------------------------------------------------------------
// halo lists: every sorted marker registers itself with each neighbouring
// tile its support reaches (at most 7: tiles are at least W nodes wide).
// ---------------------------------------------------------------------------
template <typename T, int W, bool EMIT>
__global__ __launch_bounds__(256) void k_halo(GridC g, TileC tc, int nm,
                                              const int *__restrict__ n_act_p,
                                              const unsigned *__restrict__ rec_node,
                                              const T *__restrict__ rec_t,
                                              int *__restrict__ halo_count,
                                              const int *__restrict__ halo_start,
                                              int *__restrict__ halo_cursor,
                                              int *__restrict__ halo_list, long long cap,
                                              long long *__restrict__ count, int *__restrict__ err)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int n_act = *n_act_p;
    int entries = 0;
    if (j < n_act) {
        int b[3];
        unpack_node(g, rec_node[j], b);
        int tl[3][2], nt[3], home[3];
        for (int a = 0; a < 3; ++a) {
            const int last = rec_t[(size_t)a * nm + j] == T(0) ? W - 2 : W - 1;
            home[a] = axis_node(g, a, b[a], 1) / tc.B[a];
            const int t0 = axis_node(g, a, b[a], 0) / tc.B[a];
            const int t1 = axis_node(g, a, b[a], last) / tc.B[a];
            tl[a][0] = t0;
            tl[a][1] = t1;
            nt[a] = t1 == t0 ? 1 : 2;
        }
        for (int kz = 0; kz < nt[2]; ++kz)
            for (int ky = 0; ky < nt[1]; ++ky)
                for (int kx = 0; kx < nt[0]; ++kx) {
                    const int tx = tl[0][kx], ty = tl[1][ky], tz = tl[2][kz];
                    if (tx == home[0] && ty == home[1] && tz == home[2])
                        continue;
                    const int tile = tx + tc.nt[0] * (ty + tc.nt[1] * tz);
                    if (EMIT) {
                        const long long pos =
                            (long long)halo_start[tile] + atomicAdd(&halo_cursor[tile], 1);
                        if (pos < cap)
                            halo_list[pos] = j;
                        else
                            atomicCAS(err, 0, (int)IBMX_ECAPACITY);
                    } else {
                        atomicAdd(&halo_count[tile], 1);
                    }
                    ++entries;
                }
    }
    if (!EMIT) {
        entries = wave_sum_i(entries);
        if ((threadIdx.x & (IBMX_WAVE - 1)) == 0 && entries)
            atomicAdd((unsigned long long *)&count[2], (unsigned long long)entries);
    }
}

// ---------------------------------------------------------------------------
// interpolation + marker force + particle sums: one thread per sorted marker
// ---------------------------------------------------------------------------
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

// Sum v over the run of equal keys each lane belongs to (runs are contiguous
// in the wave); the last lane of each run returns the run total.
__device__ __forceinline__ double segmented_sum(double v, int lane, int head_lane)
{
#pragma unroll
    for (int off = 1; off < IBMX_WAVE; off <<= 1) {
        double u = __shfl_up(v, off, IBMX_WAVE);
        if (lane - off >= head_lane)
            v += u;
    }
    return v;
}

template <typename T, int W>
__global__ __launch_bounds__(256) void k_interp(
    GridC g, int nm, int pass, int final_only, double c, int np, const int *__restrict__ n_act_p,
    const unsigned *__restrict__ rec_node, const T *__restrict__ rec_t, const T *__restrict__ rec_o,
    const int *__restrict__ rec_pid, const int *__restrict__ rec_src,
    const double *__restrict__ dV, const double *__restrict__ up, const double *__restrict__ wp,
    const T *__restrict__ u, T *__restrict__ rec_G, double *__restrict__ S_out,
    double *__restrict__ T_out, double *__restrict__ acc, T *__restrict__ U_dbg)
{
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int j = blk * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & (IBMX_WAVE - 1);
    const int n_act = *n_act_p;
    const long long N = g.nodes;
    int pid = -1;
    double red[7] = {0, 0, 0, 0, 0, 0, 0};
    if (j < n_act) {
        pid = rec_pid[j];
        T tt[3];
        double o[3];
        for (int a = 0; a < 3; ++a) {
            tt[a] = rec_t[(size_t)a * nm + j];
            o[a] = (double)rec_o[(size_t)a * nm + j];
        }
        int ix[3][W];
        T w[3][W];
        stencil<T, W>(g, rec_node[j], tt, ix, w);
        T U[3] = {0, 0, 0};
#pragma unroll
        for (int k = 0; k < W; ++k)
#pragma unroll
            for (int jj = 0; jj < W; ++jj) {
                const T wzy = w[2][k] * w[1][jj];
                const long long row = ((long long)ix[2][k] * g.n[1] + ix[1][jj]) * g.n[0];
#pragma unroll
                for (int i = 0; i < W; ++i) {
                    const T ww = wzy * w[0][i];
                    const long long nd = row + ix[0][i];
                    U[0] += ww * u[nd];
                    U[1] += ww * u[N + nd];
                    U[2] += ww * u[2 * N + nd];
                }
            }
        const double upp[3] = {up[pid], up[np + pid], up[2 * np + pid]};
        const double wpp[3] = {wp[pid], wp[np + pid], wp[2 * np + pid]};
        const double dVp = dV[pid];
        const double Ud[3] = {upp[0] + (wpp[1] * o[2] - wpp[2] * o[1]),
                              upp[1] + (wpp[2] * o[0] - wpp[0] * o[2]),
                              upp[2] + (wpp[0] * o[1] - wpp[1] * o[0])};
        double F[3];
        for (int a = 0; a < 3; ++a) {
            const double r = Ud[a] - (double)U[a];
            F[a] = r / c;
            red[6] += dVp * r * r;
        }
        if (!final_only) {
            if (U_dbg) {
                const int src = rec_src[j];
                for (int a = 0; a < 3; ++a)
                    U_dbg[((size_t)pass * 3 + a) * nm + src] = U[a];
            }
            for (int a = 0; a < 3; ++a) {
                red[a] = F[a] * dVp;
                rec_G[(size_t)a * nm + j] = (T)(F[a] * dVp * g.inv_h3);
            }
            red[3] = (o[1] * F[2] - o[2] * F[1]) * dVp;
            red[4] = (o[2] * F[0] - o[0] * F[2]) * dVp;
            red[5] = (o[0] * F[1] - o[1] * F[0]) * dVp;
        }
    }
    // residual: plain wave sum, one atomic per wave
    const double rs = wave_sum(red[6]);
    if (lane == 0 && rs != 0.0)
        atomicAdd(&acc[pass], rs);
    if (final_only)
        return;
    // particle sums: segmented over runs of equal particle id
    const int prev = __shfl_up(pid, 1, IBMX_WAVE);
    const bool head = lane == 0 || prev != pid;
    const unsigned long long heads = __ballot(head);
    const unsigned long long le = lane == 63 ? ~0ull : ((1ull << (lane + 1)) - 1ull);
    const int head_lane = 63 - __clzll((long long)(heads & le));
    const int next = __shfl_down(pid, 1, IBMX_WAVE);
    const bool tail = lane == IBMX_WAVE - 1 || next != pid;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const double s = segmented_sum(red[q], lane, head_lane);
        if (tail && pid >= 0) {
            double *dst = q < 3 ? &S_out[(size_t)q * np + pid] : &T_out[(size_t)(q - 3) * np + pid];
            atomicAdd(dst, s);
        }
    }
}

// ---------------------------------------------------------------------------
// spreading + velocity update: one workgroup per tile, LDS accumulation
// ---------------------------------------------------------------------------
template <typename T, int W>
__global__ __launch_bounds__(256) void k_spread(GridC g, TileC tc, int nm, T c, int count_shell,
                                                const int *__restrict__ tile_start,
                                                const int *__restrict__ halo_start,
                                                const int *__restrict__ halo_list,
                                                const unsigned *__restrict__ rec_node,
                                                const T *__restrict__ rec_t,
                                                const T *__restrict__ rec_G, T *__restrict__ u,
                                                T *__restrict__ f_tot,
                                                long long *__restrict__ count)
{
    extern __shared__ __align__(16) unsigned char smem[];
    T *acc = reinterpret_cast<T *>(smem);
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    const int a0 = tile_start[tile], a1 = tile_start[tile + 1];
    const int h0 = halo_start[tile], h1 = halo_start[tile + 1];
    const int n_own = a1 - a0, n_tot = n_own + (h1 - h0);
    if (n_tot == 0)
        return;
    const int tx = tile % tc.nt[0], ty = (tile / tc.nt[0]) % tc.nt[1];
    const int tz = tile / (tc.nt[0] * tc.nt[1]);
    const int o0 = tx * tc.B[0], o1 = ty * tc.B[1], o2 = tz * tc.B[2];
    const int e0 = min(tc.B[0], g.n[0] - o0), e1 = min(tc.B[1], g.n[1] - o1);
    const int e2 = min(tc.B[2], g.n[2] - o2);
    const int V = tc.B[0] * tc.B[1] * tc.B[2];
    for (int i = threadIdx.x; i < 3 * V; i += blockDim.x)
        acc[i] = T(0);
    __syncthreads();
    for (int e = threadIdx.x; e < n_tot; e += blockDim.x) {
        const int j = e < n_own ? a0 + e : halo_list[h0 + e - n_own];
        T tt[3], G[3];
        for (int a = 0; a < 3; ++a) {
            tt[a] = rec_t[(size_t)a * nm + j];
            G[a] = rec_G[(size_t)a * nm + j];
        }
        int ix[3][W];
        T w[3][W];
        stencil<T, W>(g, rec_node[j], tt, ix, w);
        int lx[W], ly[W], lz[W];
#pragma unroll
        for (int k = 0; k < W; ++k) {
            lx[k] = ix[0][k] - o0;
            ly[k] = ix[1][k] - o1;
            lz[k] = ix[2][k] - o2;
        }
#pragma unroll
        for (int k = 0; k < W; ++k) {
            if ((unsigned)lz[k] >= (unsigned)e2)
                continue;
#pragma unroll
            for (int jj = 0; jj < W; ++jj) {
                if ((unsigned)ly[jj] >= (unsigned)e1)
                    continue;
                const T wzy = w[2][k] * w[1][jj];
                const int rowl = (lz[k] * tc.B[1] + ly[jj]) * tc.B[0];
#pragma unroll
                for (int i = 0; i < W; ++i) {
                    if ((unsigned)lx[i] >= (unsigned)e0)
                        continue;
                    const T ww = wzy * w[0][i];
                    const int li = rowl + lx[i];
                    atomicAdd(&acc[li], ww * G[0]);
                    atomicAdd(&acc[V + li], ww * G[1]);
                    atomicAdd(&acc[2 * V + li], ww * G[2]);
                }
            }
        }
    }
    __syncthreads();
    const long long N = g.nodes;
    int touched = 0;
    for (int li = threadIdx.x; li < V; li += blockDim.x) {
        const int lx = li % tc.B[0], ly = (li / tc.B[0]) % tc.B[1], lz = li / (tc.B[0] * tc.B[1]);
        if (lx >= e0 || ly >= e1 || lz >= e2)
            continue;
        const T f0 = acc[li], f1 = acc[V + li], f2 = acc[2 * V + li];
        if (f0 == T(0) && f1 == T(0) && f2 == T(0))
            continue;
        ++touched;
        const long long gi = ((long long)(o2 + lz) * g.n[1] + (o1 + ly)) * g.n[0] + (o0 + lx);
        u[gi] += c * f0;
        u[N + gi] += c * f1;
        u[2 * N + gi] += c * f2;
        f_tot[gi] += f0;
        f_tot[N + gi] += f1;
        f_tot[2 * N + gi] += f2;
    }
    if (count_shell) {
        touched = wave_sum_i(touched);
        if ((threadIdx.x & (IBMX_WAVE - 1)) == 0 && touched)
            atomicAdd((unsigned long long *)&count[1], (unsigned long long)touched);
    }
}

__global__ void k_finish_resid(const double *acc, double *resid, int n)
{
    int i = threadIdx.x;
    if (i < n)
        resid[i] = sqrt(acc[i]);
}

int nblocks(long long n, int b) { return (int)((n + b - 1) / b) > 0 ? (int)((n + b - 1) / b) : 1; }

template <typename T, int W>
ibmx_status run_forcing(ibmx_plan p, T *u, T *f_tot, const double *xp, const double *up,
                        const double *wp, const uint8_t *mask, double *S_out, double *T_out,
                        double *resid_out, T *U_dbg)
{
    hipStream_t s = p->stream;
    const int nm = p->nm, np = p->np, n_iter = p->prm.n_iter;
    const double c = p->prm.two_alpha_dt;
    const TileC tc = p->tc;
    const int ntiles = tc.ntiles;
    const int *n_act = p->tile_start + ntiles;   // total after the scan
    {
        ProfScope ps(p, IBMX_K_OTHER);
        ibmx_fill_f64(S_out, 0.0, 3LL * np, s);
        ibmx_fill_f64(T_out, 0.0, 3LL * np, s);
        ibmx_fill_f64(p->d_acc, 0.0, n_iter + 1, s);
        ibmx_fill_i32((int *)p->d_count, 0, 16, s);
        ibmx_fill_i32(p->tile_count, 0, ntiles + 1, s);
        ibmx_fill_i32(p->tile_cursor, 0, ntiles + 1, s);
        ibmx_fill_i32(p->halo_count, 0, ntiles + 1, s);
        ibmx_fill_i32(p->halo_cursor, 0, ntiles + 1, s);
    }
    if (np > 0 && nm > 0) {
        ProfScope ps(p, IBMX_K_GEOMETRY);
        const int gb = nblocks(np, 4);
        hipLaunchKernelGGL((k_bin_count<W>), dim3(gb), dim3(256), 0, s, p->g, tc, np, nm, p->d_moff,
                           p->body, xp, mask, p->m_key, p->m_rank, p->bin_tab, p->tile_count,
                           p->d_err, p->d_count);
        ibmx_exclusive_scan(p->tile_count, p->tile_start, ntiles, s);
        hipLaunchKernelGGL((k_bin_scatter<T, W>), dim3(gb), dim3(256), 0, s, p->g, np, nm,
                           p->d_moff, p->body, xp, p->m_key, p->m_rank, p->bin_tab, p->tile_start,
                           p->tile_cursor, (unsigned *)p->rec_node, (T *)p->rec_t, (T *)p->rec_o,
                           p->rec_pid, p->rec_src);
        hipLaunchKernelGGL((k_halo<T, W, false>), dim3(nblocks(nm, 256)), dim3(256), 0, s, p->g,
                           tc, nm, n_act, (const unsigned *)p->rec_node, (const T *)p->rec_t,
                           p->halo_count, (const int *)nullptr, (int *)nullptr, (int *)nullptr,
                           p->halo_cap, p->d_count, p->d_err);
        ibmx_exclusive_scan(p->halo_count, p->halo_start, ntiles, s);
        hipLaunchKernelGGL((k_halo<T, W, true>), dim3(nblocks(nm, 256)), dim3(256), 0, s, p->g,
                           tc, nm, n_act, (const unsigned *)p->rec_node, (const T *)p->rec_t,
                           p->halo_count, p->halo_start, p->halo_cursor, p->halo_list, p->halo_cap,
                           p->d_count, p->d_err);
    } else {
        ibmx_exclusive_scan(p->tile_count, p->tile_start, ntiles, s);
        ibmx_exclusive_scan(p->halo_count, p->halo_start, ntiles, s);
    }
    const int gi = nblocks(nm, 256);
    const size_t lds = (size_t)3 * tc.B[0] * tc.B[1] * tc.B[2] * sizeof(T);
    for (int m = 0; m < n_iter && nm > 0; ++m) {
        {
            ProfScope ps(p, IBMX_K_INTERP);
            hipLaunchKernelGGL((k_interp<T, W>), dim3(gi), dim3(256), 0, s, p->g, nm, m, 0, c, np,
                               n_act, (const unsigned *)p->rec_node, (const T *)p->rec_t,
                               (const T *)p->rec_o, p->rec_pid, p->rec_src, p->dV, up, wp, u,
                               (T *)p->rec_G, S_out, T_out, p->d_acc, U_dbg);
        }
        {
            ProfScope ps(p, IBMX_K_SPREAD);
            hipLaunchKernelGGL((k_spread<T, W>), dim3(ntiles), dim3(256), lds, s, p->g, tc, nm,
                               (T)c, m == 0 ? 1 : 0, p->tile_start, p->halo_start, p->halo_list,
                               (const unsigned *)p->rec_node, (const T *)p->rec_t,
                               (const T *)p->rec_G, u, f_tot, p->d_count);
        }
    }
    if (resid_out) {
        if (nm > 0) {
            ProfScope ps(p, IBMX_K_INTERP);
            hipLaunchKernelGGL((k_interp<T, W>), dim3(gi), dim3(256), 0, s, p->g, nm, n_iter, 1, c,
                               np, n_act, (const unsigned *)p->rec_node, (const T *)p->rec_t,
                               (const T *)p->rec_o, p->rec_pid, p->rec_src, p->dV, up, wp, u,
                               (T *)p->rec_G, S_out, T_out, p->d_acc, (T *)nullptr);
        }
        hipLaunchKernelGGL(k_finish_resid, dim3(1), dim3(64), 0, s, p->d_acc, resid_out, n_iter + 1);
    }
    return ibmx_launch_check();
}

}  // namespace

// LDS bytes of the spreading kernel for the plan's tile and precision
size_t ibmx_spread_lds_bytes(ibmx_plan p)
{
    return (size_t)3 * p->tc.B[0] * p->tc.B[1] * p->tc.B[2] *
           (p->prec == IBMX_F64 ? sizeof(double) : sizeof(float));
}

// Allow the spreading kernels the plan's LDS footprint (above 64 KB needs
// an explicit opt-in).
ibmx_status ibmx_spread_allow_lds(ibmx_plan p)
{
    const int bytes = (int)ibmx_spread_lds_bytes(p);
    hipError_t e = hipSuccess;
    if (p->prec == IBMX_F64) {
        e = hipFuncSetAttribute((const void *)k_spread<double, 3>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void *)k_spread<double, 4>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    } else {
        e = hipFuncSetAttribute((const void *)k_spread<float, 3>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void *)k_spread<float, 4>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
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
    if (p->prm.n_iter + 1 > 64)
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
