// Hardware ceilings of the access patterns the sampled gradient is made of,
// measured on the device itself: each kernel below does one pattern as fast
// as the device allows it, with nothing else, so that the time of the real
// kernels can be set against what their memory and LDS traffic could cost at
// best.  Measurement tools only; no part of the method runs here.
//
//   random record reads    independent 16-byte loads at random positions of
//                          a large array (the nonzero-sample record read and
//                          the membership-table probe);
//   dependent row gathers  a random 16-byte record, then the three factor rows
//                          its key names, eight lanes of four floats per
//                          row (the sampling kernel's access chain);
//   LDS 64-bit CAS adds    compare-and-swap adds of float pairs into LDS at
//                          distinct words (the accumulation of the LDS-private
//                          and row-block scatters);
//   LDS row adds           float adds into a 256-row block of 32 floats, eight
//                          lanes of four columns per row drawn at random (the
//                          owner pass's pattern), by compare-and-swap pairs or
//                          by the native LDS float atomic;
//   global float atomics   one 128-byte row of float atomic adds per request
//                          at random rows of a small array (the atomic scatter);
//   stream copy            a device-to-device float4 copy (attainable HBM
//                          bandwidth).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "gcp_internal.hpp"

namespace gcp {
namespace {

__device__ __forceinline__ uint64_t cmix(uint64_t k)
{
    // murmur3 fmix64 finaliser: a cheap, well-spread index stream
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return k;
}

__device__ __forceinline__ uint64_t crange(uint64_t u, uint64_t n) { return __umul64hi(u, n); }

template <int U>
__global__ void __launch_bounds__(1024) k_ceil_reads(const uint4* __restrict__ rec, uint64_t nrec, int64_t nreads,
                                                   uint64_t seed, uint32_t* __restrict__ sink)
{
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    uint32_t acc = 0;
    for (int64_t i = tid * U; i < nreads; i += nth * U) {
        uint4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = rec[crange(cmix(seed + (uint64_t)(i + u)), nrec)];
#pragma unroll
        for (int u = 0; u < U; ++u) acc ^= v[u].x ^ v[u].z;
    }
    if (acc == 0x9e3779b9u) sink[tid & 1023] = acc;     // keeps the loads; practically never stores
}

// Eight lanes per sample, four floats each (rank 32); two samples in flight
// per lane group.  The record is random (SEQ = false: a dependent chain as
// in the sampling kernel) or the next one of a stream (SEQ = true: as the
// row-block owner pass reads its sorted entries).  A hash of the record's contents picks one row in each of
// three modes of dims0, dims1, dims2 rows (the one factor array holds
// dims0 + dims1 + dims2 rows of 32 floats).
template <bool SEQ>
__global__ void __launch_bounds__(1024) k_ceil_gathers(const uint4* __restrict__ rec, uint64_t nrec,
                                                     const float* __restrict__ A, uint32_t d0, uint32_t d1,
                                                     uint32_t d2, int64_t nsamples, uint64_t seed,
                                                     float* __restrict__ sink)
{
    constexpr int LANES = 8, S = 64 / LANES, U = 2;
    const int lane = threadIdx.x & 63, g = lane / LANES, cl = lane % LANES;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    float acc = 0.f;
    for (int64_t base = wave * S * U; base < nsamples; base += nwaves * S * U) {
        uint4 r[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t s = (uint64_t)(base + u * S + g);
            r[u] = rec[SEQ ? s % nrec : crange(cmix(seed + s), nrec)];
        }
        float4 a[U][3];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t h = cmix(((uint64_t)r[u].y << 32) | r[u].x);
            const uint32_t i0 = (uint32_t)(((h & 0xffffffffull) * d0) >> 32);
            const uint32_t i1 = d0 + (uint32_t)(((h >> 32) * d1) >> 32);
            const uint32_t i2 = d0 + d1 + (uint32_t)((((h >> 16) & 0xffffffffull) * d2) >> 32);
            a[u][0] = *reinterpret_cast<const float4*>(A + (uint64_t)i0 * 32 + cl * 4);
            a[u][1] = *reinterpret_cast<const float4*>(A + (uint64_t)i1 * 32 + cl * 4);
            a[u][2] = *reinterpret_cast<const float4*>(A + (uint64_t)i2 * 32 + cl * 4);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            acc += a[u][0].x * a[u][1].x * a[u][2].x + a[u][0].y * a[u][1].y * a[u][2].y +
                   a[u][0].z * a[u][1].z * a[u][2].z + a[u][0].w * a[u][1].w * a[u][2].w;
    }
    if (acc == 1234.5f) sink[threadIdx.x] = acc;
}

// Every lane adds float pairs into its own 8-byte LDS words (no two lanes of
// the workgroup share a word), so each compare-and-swap succeeds at once.
__global__ void __launch_bounds__(1024) k_ceil_lds_cas(int iters, float* __restrict__ sink)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    unsigned long long* w = reinterpret_cast<unsigned long long*>(smem);
    const int words = blockDim.x * 4;                  // 32 KB per 1024 threads
    for (int e = threadIdx.x; e < words; e += blockDim.x) w[e] = 0ull;
    __syncthreads();
    for (int it = 0; it < iters; ++it) {
        unsigned long long* p = w + threadIdx.x + (it & 3) * blockDim.x;
        unsigned long long old = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        for (;;) {
            const float lo = __uint_as_float((unsigned)old) + 1.0f;
            const float hi = __uint_as_float((unsigned)(old >> 32)) + 2.0f;
            const unsigned long long nv = (unsigned long long)__float_as_uint(lo) |
                                          ((unsigned long long)__float_as_uint(hi) << 32);
            if (__hip_atomic_compare_exchange_strong(p, &old, nv, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_WORKGROUP))
                break;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && w[0] == 7ull) sink[blockIdx.x] = 1.f;
}

// Eight lanes per row: every iteration each group of 8 lanes draws a row of
// the 256 x 32 block and each lane adds 4 values to its 4 columns.  FORM 0:
// float block (32 KB of LDS), two 64-bit compare-and-swap float-pair loops
// (the owner pass's form); FORM 1: float block, four native LDS float atomic
// adds; FORM 2: double block (64 KB), four native LDS double atomic adds.
__device__ __forceinline__ uint32_t hmix32(uint32_t x)
{
    // 32-bit integer finaliser (xorshift-multiply), cheap next to the adds
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

template <int FORM>
__global__ void __launch_bounds__(1024) k_ceil_lds_rows(int iters, float* __restrict__ sink)
{
    using V = typename std::conditional<FORM == 2, double, float>::type;
    __shared__ __attribute__((aligned(16))) V blk[256 * 32];
    for (int e = threadIdx.x; e < 256 * 32; e += blockDim.x) blk[e] = V(0);
    __syncthreads();
    const uint32_t grp = threadIdx.x >> 3;
    const int c4 = (threadIdx.x & 7) * 4;
    for (int it = 0; it < iters; ++it) {
        const uint32_t row = hmix32(blockIdx.x * 0x9e3779b9u + grp * 0x85ebca6bu + (uint32_t)it * 0xc2b2ae35u) & 255u;
        V* p = blk + row * 32 + c4;
        if constexpr (FORM == 0) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                unsigned long long* w = reinterpret_cast<unsigned long long*>(p + 2 * h);
                unsigned long long old = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                for (;;) {
                    const float lo = __uint_as_float((unsigned)old) + 1.0f;
                    const float hi = __uint_as_float((unsigned)(old >> 32)) + 2.0f;
                    const unsigned long long nv = (unsigned long long)__float_as_uint(lo) |
                                                  ((unsigned long long)__float_as_uint(hi) << 32);
                    if (__hip_atomic_compare_exchange_strong(w, &old, nv, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_WORKGROUP))
                        break;
                }
            }
        } else {
#pragma unroll
            for (int v = 0; v < 4; ++v)
                __hip_atomic_fetch_add(p + v, V(1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && blk[0] == V(-1)) sink[blockIdx.x] = 1.f;
}

// Groups of 32 lanes add one float each to a random row of 32 floats.
__global__ void __launch_bounds__(1024) k_ceil_atomics(float* __restrict__ G, uint64_t rows, int64_t nupdates,
                                                     uint64_t seed)
{
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t grp = tid >> 5, ngrp = ((int64_t)gridDim.x * blockDim.x) >> 5;
    const int col = threadIdx.x & 31;
    for (int64_t i = grp; i < nupdates; i += ngrp) {
        const uint64_t row = crange(cmix(seed + (uint64_t)i), rows);
        unsafeAtomicAdd(G + row * 32 + col, 1.0f);
    }
}

__global__ void __launch_bounds__(256) k_ceil_copy(const float4* __restrict__ src, float4* __restrict__ dst,
                                                 int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

unsigned grid_for(const void* fn, int block, size_t lds, int device)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block, lds) != hipSuccess || per_cu < 1) per_cu = 1;
    return (unsigned)(per_cu * device_cu_count(device) * 4);
}

}  // namespace
}  // namespace gcp

using namespace gcp;

extern "C" {

gcp_status gcp_ceiling_random_reads(const void* rec, int64_t nrec, int64_t nreads, int in_flight, int block,
                                    void* sink, hipStream_t stream)
{
    clear_error();
    if (!rec || !sink || nrec < 1 || nreads < 0 || block < 64 || block > 1024 || block % 64)
        return set_error(GCP_ERR_ARG, "gcp_ceiling_random_reads arguments");
    int dev = 0;
    GCP_HIP(hipGetDevice(&dev));
    if (in_flight == 4) {
        hipLaunchKernelGGL(k_ceil_reads<4>, dim3(grid_for((const void*)k_ceil_reads<4>, block, 0, dev)), dim3(block),
                           0, stream, (const uint4*)rec, (uint64_t)nrec, nreads, 12345ull, (uint32_t*)sink);
    } else if (in_flight == 1) {
        hipLaunchKernelGGL(k_ceil_reads<1>, dim3(grid_for((const void*)k_ceil_reads<1>, block, 0, dev)), dim3(block),
                           0, stream, (const uint4*)rec, (uint64_t)nrec, nreads, 12345ull, (uint32_t*)sink);
    } else {
        return set_error(GCP_ERR_ARG, "in_flight must be 1 or 4");
    }
    GCP_HIP(hipGetLastError());
    return GCP_OK;
}

gcp_status gcp_ceiling_dependent_gathers(const void* rec, int64_t nrec, const float* A, const int64_t* dims3,
                                         int64_t nsamples, int sequential, int block, void* sink, hipStream_t stream)
{
    clear_error();
    if (!rec || !A || !sink || !dims3 || nrec < 1 || nsamples < 0 || block < 64 || block > 1024 || block % 64)
        return set_error(GCP_ERR_ARG, "gcp_ceiling_dependent_gathers arguments");
    for (int k = 0; k < 3; ++k)
        if (dims3[k] < 1 || dims3[k] >= (int64_t(1) << 30)) return set_error(GCP_ERR_ARG, "dims3[%d]", k);
    int dev = 0;
    GCP_HIP(hipGetDevice(&dev));
    const void* fn = sequential ? (const void*)k_ceil_gathers<true> : (const void*)k_ceil_gathers<false>;
    hipLaunchKernelGGL(sequential ? k_ceil_gathers<true> : k_ceil_gathers<false>,
                       dim3(grid_for(fn, block, 0, dev)), dim3(block), 0, stream, (const uint4*)rec, (uint64_t)nrec,
                       A, (uint32_t)dims3[0], (uint32_t)dims3[1], (uint32_t)dims3[2], nsamples, 777ull,
                       (float*)sink);
    GCP_HIP(hipGetLastError());
    return GCP_OK;
}

gcp_status gcp_ceiling_lds_cas(int iters, int block, int grid, void* sink, hipStream_t stream)
{
    clear_error();
    if (!sink || iters < 1 || block < 64 || block > 1024 || block % 64 || grid < 1)
        return set_error(GCP_ERR_ARG, "gcp_ceiling_lds_cas arguments");
    const size_t lds = (size_t)block * 4 * 8;
    hipLaunchKernelGGL(k_ceil_lds_cas, dim3((unsigned)grid), dim3(block), lds, stream, iters, (float*)sink);
    GCP_HIP(hipGetLastError());
    return GCP_OK;
}

gcp_status gcp_ceiling_lds_row_adds(int form, int iters, int grid, void* sink, hipStream_t stream)
{
    clear_error();
    if (!sink || iters < 1 || grid < 1 || form < 0 || form > 2)
        return set_error(GCP_ERR_ARG, "gcp_ceiling_lds_row_adds arguments");
    if (form == 0)
        hipLaunchKernelGGL(k_ceil_lds_rows<0>, dim3((unsigned)grid), dim3(1024), 0, stream, iters, (float*)sink);
    else if (form == 1)
        hipLaunchKernelGGL(k_ceil_lds_rows<1>, dim3((unsigned)grid), dim3(1024), 0, stream, iters, (float*)sink);
    else
        hipLaunchKernelGGL(k_ceil_lds_rows<2>, dim3((unsigned)grid), dim3(1024), 0, stream, iters, (float*)sink);
    GCP_HIP(hipGetLastError());
    return GCP_OK;
}

gcp_status gcp_ceiling_global_atomics(float* G, int64_t rows, int64_t nupdates, int block, hipStream_t stream)
{
    clear_error();
    if (!G || rows < 1 || nupdates < 0 || block < 64 || block > 1024 || block % 64)
        return set_error(GCP_ERR_ARG, "gcp_ceiling_global_atomics arguments");
    int dev = 0;
    GCP_HIP(hipGetDevice(&dev));
    hipLaunchKernelGGL(k_ceil_atomics, dim3(grid_for((const void*)k_ceil_atomics, block, 0, dev)), dim3(block), 0,
                       stream, G, (uint64_t)rows, nupdates, 99ull);
    GCP_HIP(hipGetLastError());
    return GCP_OK;
}

gcp_status gcp_ceiling_copy(const void* src, void* dst, int64_t bytes, hipStream_t stream)
{
    clear_error();
    if (!src || !dst || bytes < 0 || bytes % 16) return set_error(GCP_ERR_ARG, "gcp_ceiling_copy arguments");
    int dev = 0;
    GCP_HIP(hipGetDevice(&dev));
    const int64_t n = bytes / 16;
    hipLaunchKernelGGL(k_ceil_copy, dim3((unsigned)(device_cu_count(dev) * 8)), dim3(256), 0, stream,
                       (const float4*)src, (float4*)dst, n);
    GCP_HIP(hipGetLastError());
    return GCP_OK;
}

}  // extern "C"
