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

// Exclusive scan of n ints by one workgroup of 1024 threads: each thread
// sums a contiguous chunk, the chunk sums are scanned in LDS, then every
// thread writes its chunk.  out[n] receives the total.  in and out may alias.
constexpr int SCAN_T = 1024;

__global__ __launch_bounds__(SCAN_T) void k_scan(const int *in, int *out, int n)
{
    __shared__ int part[SCAN_T];
    const int tid = threadIdx.x;
    const int chunk = (n + SCAN_T - 1) / SCAN_T;
    const int lo = min(n, tid * chunk), hi = min(n, lo + chunk);
    int s = 0;
    for (int i = lo; i < hi; ++i)
        s += in[i];
    part[tid] = s;
    __syncthreads();
    for (int off = 1; off < SCAN_T; off <<= 1) {
        int v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int run = part[tid] - s;
    for (int i = lo; i < hi; ++i) {
        int v = in[i];
        out[i] = run;
        run += v;
    }
    if (tid == SCAN_T - 1)
        out[n] = part[SCAN_T - 1];
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

void ibmx_exclusive_scan(const int *in, int *out, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(SCAN_T), 0, s, in, out, n);
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
