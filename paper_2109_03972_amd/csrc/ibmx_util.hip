// Small device utilities: fills and an exclusive scan, plus status strings.
#include "ibmx_internal.hpp"

namespace {

__global__ void k_fill_i32(int *p, int v, long long n)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += stride)
        p[i] = v;
}

// several int arrays cleared to 0 by one launch (their index ranges laid end
// to end)
__global__ void k_zero_i32_multi(ZeroList z)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    int k = 0;
    long long base = 0;
    for (; i < z.total; i += stride) {
        while (i >= base + z.n[k]) {
            base += z.n[k];
            ++k;
        }
        z.p[k][i - base] = 0;
    }
}

__global__ void k_fill_f64(double *p, double v, long long n)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += stride)
        p[i] = v;
}

__global__ void k_fill_u8(uint8_t *p, uint8_t v, long long n)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += stride)
        p[i] = v;
}

// Exclusive scan of n ints in three launches: every workgroup of 256
// threads scans its SCAN_B = 2048 elements (8 consecutive per thread) and
// writes its total to aux; one workgroup scans the totals (out[n] receives
// the grand total); every workgroup then adds the scanned total of the
// workgroups before it.  With n <= SCAN_B the first launch does all.  in and
// out may alias (every element is read before it is written, by the same
// thread).
constexpr int SCAN_T = 256, SCAN_E = 8, SCAN_B = SCAN_T * SCAN_E;

__device__ __forceinline__ int wave_incl_scan(int v)
{
    const int lane = threadIdx.x & (IBMX_WAVE - 1);
#pragma unroll
    for (int d = 1; d < IBMX_WAVE; d <<= 1) {
        const int u = __shfl_up(v, d, IBMX_WAVE);
        if (lane >= d)
            v += u;
    }
    return v;
}

// exclusive scan of one value per thread over the workgroup; *total gets the sum
__device__ __forceinline__ int block_excl_scan(int v, int *total)
{
    __shared__ int wsum[SCAN_T / IBMX_WAVE];
    const int lane = threadIdx.x & (IBMX_WAVE - 1), wave = threadIdx.x / IBMX_WAVE;
    const int incl = wave_incl_scan(v);
    if (lane == IBMX_WAVE - 1)
        wsum[wave] = incl;
    __syncthreads();
    int before = 0, all = 0;
    for (int w = 0; w < SCAN_T / IBMX_WAVE; ++w) {
        before += w < wave ? wsum[w] : 0;
        all += wsum[w];
    }
    __syncthreads();
    *total = all;
    return before + incl - v;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_local(const int *in, int *out, int *aux, int n)
{
    const long long lo = (long long)blockIdx.x * SCAN_B + (long long)threadIdx.x * SCAN_E;
    int v[SCAN_E];
#pragma unroll
    for (int k = 0; k < SCAN_E; ++k)
        v[k] = lo + k < n ? in[lo + k] : 0;
    int sum = 0;
#pragma unroll
    for (int k = 0; k < SCAN_E; ++k)
        sum += v[k];
    int total;
    int run = block_excl_scan(sum, &total);
#pragma unroll
    for (int k = 0; k < SCAN_E; ++k) {
        if (lo + k < n)
            out[lo + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 0) {
        if (aux)
            aux[blockIdx.x] = total;
        else
            out[n] = total;
    }
}

__global__ __launch_bounds__(SCAN_T) void k_scan_aux(int *aux, int nb, int *out, int n)
{
    int carry = 0;
    for (int b0 = 0; b0 < nb; b0 += SCAN_T) {
        const int b = b0 + threadIdx.x;
        const int v = b < nb ? aux[b] : 0;
        int total;
        const int ex = block_excl_scan(v, &total);
        if (b < nb)
            aux[b] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0)
        out[n] = carry;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_add(int *out, const int *aux, int n)
{
    if (blockIdx.x == 0)
        return;
    const int add = aux[blockIdx.x];
    const long long lo = (long long)blockIdx.x * SCAN_B;
    for (int k = threadIdx.x; k < SCAN_B; k += SCAN_T)
        if (lo + k < n)
            out[lo + k] += add;
}

int fill_blocks(long long n)
{
    long long b = (n + 255) / 256;
    if (b > 4096)
        b = 4096;
    return b < 1 ? 1 : (int)b;
}

}  // namespace

void ibmx_fill_i32(int *p, int v, long long n, hipStream_t s)
{
    if (n > 0)
        hipLaunchKernelGGL(k_fill_i32, dim3(fill_blocks(n)), dim3(256), 0, s, p, v, n);
}

void ibmx_zero_i32_multi(const ZeroList &z, hipStream_t s)
{
    if (z.total > 0)
        hipLaunchKernelGGL(k_zero_i32_multi, dim3(fill_blocks(z.total)), dim3(256), 0, s, z);
}

void ibmx_fill_f64(double *p, double v, long long n, hipStream_t s)
{
    if (n > 0)
        hipLaunchKernelGGL(k_fill_f64, dim3(fill_blocks(n)), dim3(256), 0, s, p, v, n);
}

void ibmx_fill_u8(uint8_t *p, uint8_t v, long long n, hipStream_t s)
{
    if (n > 0)
        hipLaunchKernelGGL(k_fill_u8, dim3(fill_blocks(n)), dim3(256), 0, s, p, v, n);
}

int ibmx_scan_aux_size(long long n) { return (int)((n + SCAN_B - 1) / SCAN_B) + 1; }

void ibmx_exclusive_scan(const int *in, int *out, int n, int *aux, hipStream_t s)
{
    const int nb = (n + SCAN_B - 1) / SCAN_B;
    if (nb <= 1) {
        hipLaunchKernelGGL(k_scan_local, dim3(1), dim3(SCAN_T), 0, s, in, out, (int *)nullptr, n);
        return;
    }
    hipLaunchKernelGGL(k_scan_local, dim3(nb), dim3(SCAN_T), 0, s, in, out, aux, n);
    hipLaunchKernelGGL(k_scan_aux, dim3(1), dim3(SCAN_T), 0, s, aux, nb, out, n);
    hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(SCAN_T), 0, s, out, (const int *)aux, n);
}

ibmx_status ibmx_launch_check()
{
    return hipGetLastError() == hipSuccess ? IBMX_OK : IBMX_EDEVICE;
}

extern "C" const char *ibmx_status_string(ibmx_status st)
{
    switch (st) {
    case IBMX_OK: return "ok";
    case IBMX_EINVAL: return "invalid argument";
    case IBMX_EDOMAIN: return "delta support of an active marker crosses a wall";
    case IBMX_ENOMEM: return "device allocation failed";
    case IBMX_EDEVICE: return "HIP runtime error";
    case IBMX_ESTATE: return "plan not ready (markers not set)";
    case IBMX_ECAPACITY: return "list capacity exceeded";
    case IBMX_EUNSUPPORTED: return "unsupported option";
    }
    return "unknown status";
}

extern "C" const char *ibmx_version(void) { return "ibmx 0.1 (gfx950)"; }
