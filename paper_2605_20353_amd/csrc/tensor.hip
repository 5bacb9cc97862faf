// Tensor handles: error reporting, COO packing, membership-table build,
// dense handles and the device status word.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <new>

#include "gcp_internal.hpp"

namespace gcp {

static thread_local char g_last_error[512] = "";

gcp_status set_error(gcp_status st, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
    return st;
}

gcp_status hip_error(hipError_t e, const char* what)
{
    if (e == hipErrorOutOfMemory)
        return set_error(GCP_ERR_OOM, "%s: %s", what, hipGetErrorString(e));
    return set_error(GCP_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

void clear_error() { g_last_error[0] = 0; }

int device_cu_count(int device)
{
    static int cached[64] = {};
    if (device < 0 || device >= 64) return 256;
    if (!cached[device]) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || n <= 0)
            n = 256;
        cached[device] = n;
    }
    return cached[device];
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

gcp_status prepare_lds(const void* fn, size_t bytes, int device)
{
    static int cached[64] = {};
    int maxb = 65536;
    if (device >= 0 && device < 64) {
        if (!cached[device]) {
            int v = 0;
            if (hipDeviceGetAttribute(&v, hipDeviceAttributeSharedMemPerBlockOptin, device) != hipSuccess || v <= 0)
                if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess || v <= 0)
                    v = 65536;
            cached[device] = v;
        }
        maxb = cached[device];
    }
    if (bytes > (size_t)maxb)
        return set_error(GCP_ERR_UNSUPPORTED, "kernel needs %zu bytes of LDS, the device allows %d", bytes, maxb);
    if (bytes > 65536)
        GCP_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    return GCP_OK;
}

static int bits_for(int64_t n)
{
    int b = 0;
    while (b < 63 && (int64_t(1) << b) < n) ++b;
    return b;
}

// Shared by sparse and dense handles: dims, row offsets, cell-key layout.
static gcp_status init_shape(gcp_tensor_s* t, int d, const int64_t* dims)
{
    if (d < 1 || d > kMaxModes) return set_error(GCP_ERR_ARG, "d = %d outside [1, %d]", d, kMaxModes);
    if (!dims) return set_error(GCP_ERR_ARG, "dims_host is NULL");
    t->d = d;
    t->layout.d = d;
    int total_bits = 0;
    uint64_t cells = 1;
    bool overflow = false;
    t->rowoff[0] = 0;
    for (int k = 0; k < d; ++k) {
        if (dims[k] < 1) return set_error(GCP_ERR_ARG, "dims[%d] = %lld < 1", k, (long long)dims[k]);
        if (dims[k] >= (int64_t(1) << 32))
            return set_error(GCP_ERR_UNSUPPORTED, "dims[%d] = %lld needs more than 32-bit indices", k,
                             (long long)dims[k]);
        t->dims[k] = dims[k];
        t->layout.dims[k] = dims[k];
        t->rowoff[k + 1] = t->rowoff[k] + dims[k];
        if (__builtin_mul_overflow(cells, (uint64_t)dims[k], &cells)) overflow = true;
    }
    if (t->rowoff[d] >= (int64_t(1) << 32))
        return set_error(GCP_ERR_UNSUPPORTED, "sum of the dimensions %lld needs more than 32-bit model rows",
                         (long long)t->rowoff[d]);
    if (overflow || cells == ~0ull)
        return set_error(GCP_ERR_UNSUPPORTED, "the cell count prod_k I_k is not below 2^64 - 1");
    for (int k = d - 1; k >= 0; --k) {
        int b = bits_for(dims[k]);
        t->layout.shift[k] = total_bits;
        t->layout.mask[k] = b == 0 ? 0 : ((1ull << b) - 1);
        total_bits += b;
    }
    // bit-packed keys when they fit 63 bits, else the mixed-radix linear index
    t->layout.radix = total_bits > 63 ? 1 : 0;
    uint64_t stride = 1;
    for (int k = d - 1; k >= 0; --k) {
        t->layout.stride[k] = stride;
        t->layout.inv[k] = 1.0 / (double)dims[k];
        stride *= (uint64_t)dims[k];
    }
    t->cells = cells;
    return GCP_OK;
}

// One thread per nonzero: validate and pack its coordinates, write its
// record, insert the key (CAS on the 64-bit slot, linear probing).
template <typename T>
__global__ void k_build(KeyLayout L, int64_t nnz, const int64_t* __restrict__ coords, const T* __restrict__ vals,
                        Record<T>* __restrict__ rec, unsigned long long* __restrict__ table, uint64_t mask, int log2n,
                        uint32_t* status)
{
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nnz) return;
    uint64_t key = 0;
    bool ok = true;
    for (int k = 0; k < L.d; ++k) {
        int64_t c = coords[j * L.d + k];
        if (c < 0 || c >= L.dims[k]) ok = false;
        else key += pack_coord(L, (uint64_t)c, k);
    }
    Record<T> r;
    r.key = ok ? key : 0;
    r.val = vals[j];
    rec[j] = r;
    if (!ok) {
        atomicOr(status, kStatusData);
        return;
    }
    uint64_t h = log2n > 0 ? (mix64(key) >> (64 - log2n)) : 0;
    for (;;) {
        unsigned long long old = atomicCAS(table + h, (unsigned long long)kEmptySlot, (unsigned long long)key);
        if (old == kEmptySlot) return;
        if (old == key) {
            atomicOr(status, kStatusData);   // repeated coordinate tuple
            return;
        }
        h = (h + 1) & mask;
    }
}

__global__ void k_fill_u64(unsigned long long* __restrict__ p, int64_t n, unsigned long long v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

}  // namespace gcp

using namespace gcp;

extern "C" {

const char* gcp_version(void) { return "gcp-mi355x 0.1 (gfx950)"; }

const char* gcp_last_error(void) { return g_last_error; }

static void free_tensor(gcp_tensor_s* t)
{
    if (!t) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(t->device);
    (void)hipDeviceSynchronize();
    if (t->rec) (void)hipFree(t->rec);
    if (t->table) (void)hipFree(t->table);
    if (t->status) (void)hipFree(t->status);
    if (t->ws) (void)hipFree(t->ws);
    (void)hipSetDevice(cur);
    delete t;
}

gcp_status gcp_tensor_create(gcp_tensor* out, int d, const int64_t* dims_host, int64_t nnz,
                             const int64_t* coords_dev, const void* vals_dev, gcp_dtype dt, hipStream_t stream)
{
    clear_error();
    if (!out) return set_error(GCP_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (dt != GCP_F32 && dt != GCP_F64) return set_error(GCP_ERR_ARG, "dtype %d", (int)dt);
    gcp_tensor_s* t = new (std::nothrow) gcp_tensor_s();
    if (!t) return set_error(GCP_ERR_OOM, "host allocation");
    gcp_status st = init_shape(t, d, dims_host);
    if (st != GCP_OK) { delete t; return st; }
    if (nnz < 1 || (uint64_t)nnz > t->cells) {
        delete t;
        return set_error(GCP_ERR_ARG, "nnz = %lld outside [1, prod dims]", (long long)nnz);
    }
    if (!coords_dev || !vals_dev) { delete t; return set_error(GCP_ERR_ARG, "coords_dev or vals_dev is NULL"); }
    t->nnz = nnz;
    t->dt = dt;
    (void)hipGetDevice(&t->device);
    // load factor <= 1/4: a wave waits for the longest probe chain of its 64
    // zero samples, and halving the load factor from 1/2 shortens that chain
    // by about one 16-byte probe round trip (3% of a sampled-gradient call at
    // 5e7 nonzeros) for 8 bytes per nonzero more of HBM
    int lg = 1;
    while ((int64_t(1) << lg) < 4 * nnz) ++lg;
    if (lg < 10) lg = 10;
    t->table_log2 = lg;
    t->table_mask = (uint64_t(1) << lg) - 1;
    size_t table_bytes = sizeof(uint64_t) << lg;
    size_t rec_bytes = 16 * (size_t)nnz;
    hipError_t e;
    if ((e = hipMalloc(&t->rec, rec_bytes)) != hipSuccess) { free_tensor(t); return hip_error(e, "hipMalloc(records)"); }
    if ((e = hipMalloc((void**)&t->table, table_bytes)) != hipSuccess) { free_tensor(t); return hip_error(e, "hipMalloc(table)"); }
    if ((e = hipMalloc((void**)&t->status, sizeof(uint32_t))) != hipSuccess) { free_tensor(t); return hip_error(e, "hipMalloc(status)"); }
    t->owned_bytes = (int64_t)(rec_bytes + table_bytes + sizeof(uint32_t));
    if ((e = hipMemsetAsync(t->status, 0, sizeof(uint32_t), stream)) != hipSuccess) { free_tensor(t); return hip_error(e, "memset"); }
    int64_t slots = int64_t(1) << lg;
    k_fill_u64<<<(unsigned)std::min<int64_t>(ceil_div(slots, 256), 65536), 256, 0, stream>>>(
        (unsigned long long*)t->table, slots, kEmptySlot);
    unsigned blocks = (unsigned)ceil_div(nnz, 256);
    if (dt == GCP_F32)
        k_build<float><<<blocks, 256, 0, stream>>>(t->layout, nnz, coords_dev, (const float*)vals_dev,
                                                  (Record<float>*)t->rec, (unsigned long long*)t->table,
                                                  t->table_mask, lg, t->status);
    else
        k_build<double><<<blocks, 256, 0, stream>>>(t->layout, nnz, coords_dev, (const double*)vals_dev,
                                                   (Record<double>*)t->rec, (unsigned long long*)t->table,
                                                   t->table_mask, lg, t->status);
    if ((e = hipGetLastError()) != hipSuccess) { free_tensor(t); return hip_error(e, "k_build launch"); }
    uint32_t hs = 0;
    if ((e = hipMemcpyAsync(&hs, t->status, sizeof(hs), hipMemcpyDeviceToHost, stream)) != hipSuccess ||
        (e = hipStreamSynchronize(stream)) != hipSuccess) {
        free_tensor(t);
        return hip_error(e, "tensor build");
    }
    if (hs & kStatusData) {
        free_tensor(t);
        return set_error(GCP_ERR_DATA, "coordinates out of range or repeated");
    }
    *out = t;
    return GCP_OK;
}

gcp_status gcp_tensor_create_dense(gcp_tensor* out, int d, const int64_t* dims_host, const void* vals_dev,
                                   gcp_dtype dt, hipStream_t stream)
{
    clear_error();
    if (!out) return set_error(GCP_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (dt != GCP_F32 && dt != GCP_F64) return set_error(GCP_ERR_ARG, "dtype %d", (int)dt);
    if (!vals_dev) return set_error(GCP_ERR_ARG, "vals_dev is NULL");
    gcp_tensor_s* t = new (std::nothrow) gcp_tensor_s();
    if (!t) return set_error(GCP_ERR_OOM, "host allocation");
    gcp_status st = init_shape(t, d, dims_host);
    if (st != GCP_OK) { delete t; return st; }
    if (t->cells >= (uint64_t(1) << 48)) {
        delete t;
        return set_error(GCP_ERR_ARG, "a dense tensor of %llu cells", (unsigned long long)t->cells);
    }
    t->dense = true;
    t->dt = dt;
    t->nnz = (int64_t)t->cells;
    t->dense_vals = vals_dev;
    (void)hipGetDevice(&t->device);
    hipError_t e;
    if ((e = hipMalloc((void**)&t->status, sizeof(uint32_t))) != hipSuccess) { free_tensor(t); return hip_error(e, "hipMalloc(status)"); }
    t->owned_bytes = sizeof(uint32_t);
    if ((e = hipMemsetAsync(t->status, 0, sizeof(uint32_t), stream)) != hipSuccess) { free_tensor(t); return hip_error(e, "memset"); }
    if ((e = hipStreamSynchronize(stream)) != hipSuccess) { free_tensor(t); return hip_error(e, "sync"); }
    *out = t;
    return GCP_OK;
}

gcp_status gcp_tensor_destroy(gcp_tensor t)
{
    clear_error();
    if (!t) return set_error(GCP_ERR_ARG, "tensor is NULL");
    free_tensor(t);
    return GCP_OK;
}

int64_t gcp_tensor_device_bytes(gcp_tensor t) { return t ? t->owned_bytes + t->ws_bytes : 0; }

gcp_status gcp_tensor_reserve(gcp_tensor t, int64_t max_samples, int R, hipStream_t stream)
{
    clear_error();
    if (!t) return set_error(GCP_ERR_ARG, "tensor is NULL");
    if (max_samples < 0 || max_samples > (int64_t(1) << 40)) return set_error(GCP_ERR_ARG, "max_samples");
    if (R < 1 || R > 256) return set_error(GCP_ERR_ARG, "R = %d outside [1, 256]", R);
    (void)stream;
    int cur = 0;
    GCP_HIP(hipGetDevice(&cur));
    GCP_HIP(hipSetDevice(t->device));
    GCP_HIP(hipDeviceSynchronize());
    if (t->ws) {
        GCP_HIP(hipFree(t->ws));
        t->ws = nullptr;
        t->ws_entries = t->ws_hist = t->ws_bytes = t->ws_max_samples = 0;
    }
    if (max_samples == 0) { GCP_HIP(hipSetDevice(cur)); return GCP_OK; }
    // smallest row block: 8 KiB of LDS; fewest samples per workgroup: 512
    const int64_t esize = t->dt == GCP_F32 ? 4 : 8;
    int br_shift = 0;
    while (((int64_t)2 << br_shift) * R * esize <= 8192 && br_shift < 30) ++br_shift;
    int64_t nb = 0;
    for (int k = 0; k < t->d; ++k) nb += ceil_div(t->dims[k], int64_t(1) << br_shift);
    nb = std::min<int64_t>(nb, 4096);
    const int64_t nblocks = ceil_div(max_samples, 512);
    const int64_t entries = (max_samples + 8192) * t->d;
    const int64_t hist = nb * nblocks;
    // the same region serves GCP_DETERMINISTIC calls
    const int64_t det = max_samples < (int64_t(1) << 32) ? det_workspace_bytes(t, max_samples) : 0;
    const int64_t bytes = std::max<int64_t>(entries * 16 + hist * 8, det);
    hipError_t e = hipMalloc(&t->ws, (size_t)bytes);
    if (e != hipSuccess) {
        t->ws = nullptr;
        (void)hipSetDevice(cur);
        return hip_error(e, "hipMalloc(workspace)");
    }
    t->ws_entries = entries;
    t->ws_hist = hist;
    t->ws_bytes = bytes;
    t->ws_max_samples = max_samples;
    GCP_HIP(hipSetDevice(cur));
    return GCP_OK;
}

gcp_status gcp_device_status(gcp_tensor t, hipStream_t stream)
{
    clear_error();
    if (!t) return set_error(GCP_ERR_ARG, "tensor is NULL");
    uint32_t hs = 0;
    GCP_HIP(hipMemcpyAsync(&hs, t->status, sizeof(hs), hipMemcpyDeviceToHost, stream));
    GCP_HIP(hipStreamSynchronize(stream));
    if (hs) {
        uint32_t zero = 0;
        GCP_HIP(hipMemcpyAsync(t->status, &zero, sizeof(zero), hipMemcpyHostToDevice, stream));
        GCP_HIP(hipStreamSynchronize(stream));
    }
    if (hs & kStatusData) return set_error(GCP_ERR_DATA, "a sample list held an out-of-range coordinate");
    if (hs & kStatusSampling)
        return set_error(GCP_ERR_SAMPLING, "a zero sample exhausted its rejection attempts");
    return GCP_OK;
}

}  // extern "C"
