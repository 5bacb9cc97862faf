// Drawing one sample of the sampled tensor (Sec. 3.1.1) on the device.
//
// Stratified: sample s < p is a nonzero j = floor(out0 N / 2^64) of the
// Philox block (s, step, 0, 0); sample s >= p is the zero sample z = s - p,
// whose attempt a draws a cell from the block(s) (z, step, 1 | a << 8, blk)
// and is kept as soon as the cell is not in the membership table.
// Semi-stratified: the first attempt is kept without a search.
// Uniform (dense tensors): cell from (s, step, 2, blk), value read from the
// dense array.
#pragma once

#include "gcp_internal.hpp"

namespace gcp {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <typename T>
__device__ __forceinline__ T record_value(u32x4 raw);
template <>
__device__ __forceinline__ float record_value<float>(u32x4 raw) { return __uint_as_float(raw.z); }
template <>
__device__ __forceinline__ double record_value<double>(u32x4 raw)
{
    return __hiloint2double((int)raw.w, (int)raw.z);
}

template <typename T>
struct SampleCtx {
    KeyLayout L;
    int d;
    int kind;                 // gcp_sampling
    int max_attempts;
    int64_t p, q, N;
    uint64_t seed, step, client;
    T w_nz, w_z;              // N/p and (M-N)/q (uniform: M/p in w_nz)
    const Record<T>* rec;     // sparse records
    const uint64_t* table;    // membership table
    uint64_t table_mask;
    int table_log2;
    const T* dense;           // dense values (uniform sampling)
    int64_t dense_stride[kMaxModes];
    uint32_t* status;
};

// Fills the cell key, value and weight of sample s in [0, p + q) of
// iteration `step` (the second Philox counter word).
template <typename T, int D>
__device__ __forceinline__ void draw_sample(const SampleCtx<T>& c, uint64_t step, int64_t s, uint64_t& key, T& x,
                                            T& w)
{
    if (c.kind == GCP_SAMPLE_UNIFORM) {
        key = draw_cell_key<D>(c.L, c.d, c.seed, c.client, (uint64_t)s, step, kStreamUniform, 0);
        int64_t lin = 0;
        const int dd = D > 0 ? D : c.d;
        constexpr int DM = D > 0 ? D : kMaxModes;
        uint32_t ci[DM];
        unpack_all<D == 0>(c.L, dd, key, ci);
#pragma unroll
        for (int k = 0; k < DM; ++k)
            if (k < dd) lin += (int64_t)ci[k] * c.dense_stride[k];
        x = c.dense[lin];
        w = c.w_nz;
        return;
    }
    if (s < c.p) {
        U64x4 o = philox4x64_10((uint64_t)s, step, kStreamNonzero, 0, c.seed, c.client);
        int64_t j = (int64_t)range_map(o.v[0], (uint64_t)c.N);
        // one 16-byte streaming load: records are touched once per draw
        u32x4 raw = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(c.rec + j));
        key = (uint64_t)raw.x | ((uint64_t)raw.y << 32);
        x = record_value<T>(raw);
        w = c.w_nz;
        return;
    }
    const uint64_t z = (uint64_t)(s - c.p);
    const bool search = c.kind == GCP_SAMPLE_STRATIFIED;
    for (int a = 0;; ++a) {
        key = draw_cell_key<D>(c.L, c.d, c.seed, c.client, z, step, kStreamZero, (uint64_t)a);
        if (!search || !table_contains(c.table, c.table_mask, c.table_log2, key)) break;
        if (a + 1 >= c.max_attempts) {
            atomicOr(c.status, kStatusSampling);
            break;
        }
    }
    x = T(0);
    w = c.w_z;
}

}  // namespace gcp

namespace gcp {

// Host side: validate (tensor, params) and fill the device sampling context.
// n_out receives the number of samples p + q.
template <typename T>
inline gcp_status make_sample_ctx(const gcp_tensor_s* t, const gcp_sample_params* sp, SampleCtx<T>& c,
                                  int64_t& n_out)
{
    if (!t) return set_error(GCP_ERR_ARG, "tensor is NULL");
    if (!sp) return set_error(GCP_ERR_ARG, "sample params are NULL");
    if (sp->p < 0 || sp->q < 0) return set_error(GCP_ERR_ARG, "negative sample count");
    if (sp->p > (int64_t(1) << 40) || sp->q > (int64_t(1) << 40))
        return set_error(GCP_ERR_ARG, "sample count above 2^40");
    c = SampleCtx<T>{};
    c.L = t->layout;
    c.d = t->d;
    c.kind = sp->kind;
    c.max_attempts = sp->max_attempts > 0 ? sp->max_attempts : 64;
    c.p = sp->p;
    c.q = sp->q;
    c.N = t->nnz;
    c.seed = sp->seed;
    c.step = sp->step;
    c.client = sp->client;
    c.status = t->status;
    switch (sp->kind) {
    case GCP_SAMPLE_STRATIFIED:
    case GCP_SAMPLE_SEMI_STRATIFIED:
        if (t->dense) return set_error(GCP_ERR_UNSUPPORTED, "stratified sampling needs a sparse tensor");
        if (sp->kind == GCP_SAMPLE_STRATIFIED && sp->q > 0 && (uint64_t)t->nnz >= t->cells)
            return set_error(GCP_ERR_ARG, "q > 0 but the tensor has no zero cells");
        c.w_nz = sp->p > 0 ? T((double)t->nnz / (double)sp->p) : T(0);
        c.w_z = sp->q > 0 ? T((double)(t->cells - t->nnz) / (double)sp->q) : T(0);
        c.rec = (const Record<T>*)t->rec;
        c.table = t->table;
        c.table_mask = t->table_mask;
        c.table_log2 = t->table_log2;
        break;
    case GCP_SAMPLE_UNIFORM:
        if (!t->dense) return set_error(GCP_ERR_UNSUPPORTED, "uniform sampling needs a dense tensor");
        if (sp->q != 0) return set_error(GCP_ERR_ARG, "uniform sampling takes q = 0");
        c.w_nz = sp->p > 0 ? T((double)t->cells / (double)sp->p) : T(0);
        c.w_z = T(0);
        c.dense = (const T*)t->dense_vals;
        {
            int64_t st = 1;
            for (int k = t->d - 1; k >= 0; --k) {
                c.dense_stride[k] = st;
                st *= t->dims[k];
            }
        }
        break;
    default:
        return set_error(GCP_ERR_ARG, "sampling kind %d", sp->kind);
    }
    n_out = sp->p + sp->q;
    return GCP_OK;
}

}  // namespace gcp
