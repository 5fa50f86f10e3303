// Device-side constants, kernel argument structs and helpers of the ibmx
// HIP library (gfx950, wave64), shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define IBMX_WAVE 64
#define IBMX_RSLOTS 1024          // spread-out accumulation slots per counter
#define IBMX_MAX_PASSES 64        // largest n_iter of a plan

// ---------------------------------------------------------------------------
// grid constants passed by value to kernels
// ---------------------------------------------------------------------------
struct GridC {
    int n[3];
    int periodic[3];
    double h;
    double inv_h3;
    double origin[3];
    long long nodes;   // nx * ny * nz
    int shift[3];      // bit offsets of the packed base-node coordinates
};

// spatial tiles of the spreading pass: B[a] nodes per tile (the last tile of
// an axis may be shorter but never narrower than the delta support)
struct TileC {
    int B[3];
    int nt[3];
    int ntiles;
    int sh[3];   // log2 B[a] when B[a] is a power of two, else -1
};

// tile coordinate of node x along axis a
__device__ __forceinline__ int tile_of(const TileC &tc, int a, int x)
{
    return tc.sh[a] >= 0 ? x >> tc.sh[a] : x / tc.B[a];
}

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T dev_sqrt(T x);
template <>
__device__ __forceinline__ float dev_sqrt<float>(float x) { return __builtin_sqrtf(x); }
template <>
__device__ __forceinline__ double dev_sqrt<double>(double x) { return __builtin_sqrt(x); }

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = IBMX_WAVE / 2; off > 0; off >>= 1)
        v += __shfl_xor(v, off, IBMX_WAVE);
    return v;
}

// Block-wide sum; every thread of the block must call it; the result is
// valid in thread 0.
template <typename V>
__device__ __forceinline__ V block_sum(V v)
{
    __shared__ V part[16];
#pragma unroll
    for (int off = IBMX_WAVE / 2; off > 0; off >>= 1)
        v += __shfl_xor(v, off, IBMX_WAVE);
    __syncthreads();
    if ((threadIdx.x & (IBMX_WAVE - 1)) == 0)
        part[threadIdx.x / IBMX_WAVE] = v;
    __syncthreads();
    V r = V(0);
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x / IBMX_WAVE); ++w)
            r += part[w];
    return r;
}

// Add a block's partial to one of IBMX_RSLOTS slots of an integer counter
// (thread 0), so that workgroups do not all hit one address; integer sums do
// not depend on the order of the adds.
__device__ __forceinline__ void slot_add(long long *slots, long long v)
{
    if (threadIdx.x == 0 && v != 0)
        atomicAdd((unsigned long long *)&slots[blockIdx.x & (IBMX_RSLOTS - 1)],
                  (unsigned long long)v);
}

__device__ __forceinline__ int wave_sum_i(int v)
{
#pragma unroll
    for (int off = IBMX_WAVE / 2; off > 0; off >>= 1)
        v += __shfl_xor(v, off, IBMX_WAVE);
    return v;
}
