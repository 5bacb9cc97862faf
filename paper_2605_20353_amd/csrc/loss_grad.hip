// gcp_loss_grad: the fused sampled objective and gradient (Sec. 3.1.1-3.1.2,
// "Fused Sampling-MTTKRP", here with stratified, uniform or semi-stratified
// samples).
//
// Work decomposition of k_loss_grad (one 64-lane wavefront takes 64 samples
// at a time):
//   phase 1, one lane per sample: draw the sample (Philox, nonzero record
//     read or zero-candidate hash probes) or read it from a materialised
//     list, and stage (cell key, x, w) in the wave's LDS slice;
//   phase 2, LANES lanes per sample with VEC consecutive columns each, 64 /
//     LANES samples per pass and U samples per lane group in flight: gather
//     the d factor rows, m = sum_r prod_k A_k[i_k, r] (eq. cp) by a butterfly
//     over the lane group, y = w f'(x, m), then scatter the leave-one-out
//     products y prod_{n != k} A_n[i_n, r] into G_k[i_k, :].
// Factor rows are read once per sample and the sampled tensor is never
// written to memory.  Three scatter strategies, chosen per mode (the paper's
// MTTKRP variants, Sec. 3.1.2):
//   * atomic: hardware float atomics straight into G (one 128-byte request
//     per row and sample);
//   * LDS-private: a small mode's whole gradient lives in each workgroup's
//     LDS and is flushed once ("thread privatization" per workgroup);
//   * bucketed (sort-by-row): each workgroup sorts its samples' (key, y) by
//     row block of the mode into a per-workgroup segment list in global
//     memory; k_bucket_accum then gives every row block to its own
//     workgroups, which re-gather the other modes' rows, accumulate the
//     block in LDS and flush it once.  This replaces d atomic requests per
//     sample by one 16-byte entry write and read per mode -- hardware float
//     atomics are executed beyond the L2 at a fixed request rate, which
//     bounds the atomic strategy at large sample counts.
#include <cmath>

#include "lg_kernels.hpp"

namespace gcp {

template <typename T, int D>
static BAKernel<T> pick_bucket_shape(int lanes, int vec)
{
#define GCP_CASE(LN, VC) \
    if (lanes == LN && vec == VC) return k_bucket_accum<T, D, LN, VC>;
    if constexpr (sizeof(T) == 4) {
        GCP_LG_SHAPES_F32(GCP_CASE)
    } else {
        GCP_LG_SHAPES_F64(GCP_CASE)
    }
#undef GCP_CASE
    return nullptr;
}

template <typename T>
static LGKernel<T> pick_kernel(int d, int src, int lanes, int vec)
{
    if (src >= 2) return pick_kernel_nonfused<T>(d, src, lanes, vec);
    if (src == 0) {
        if (d == 3) return pick_shape<T, 3, 0>(lanes, vec);
        if (d == 4) return pick_shape<T, 4, 0>(lanes, vec);
        return pick_shape<T, 0, 0>(lanes, vec);
    }
    if (d == 3) return pick_shape<T, 3, 1>(lanes, vec);
    if (d == 4) return pick_shape<T, 4, 1>(lanes, vec);
    return pick_shape<T, 0, 1>(lanes, vec);
}

template <typename T>
static BAKernel<T> pick_bucket_kernel(int d, int lanes, int vec)
{
    if (d == 3) return pick_bucket_shape<T, 3>(lanes, vec);
    if (d == 4) return pick_bucket_shape<T, 4>(lanes, vec);
    return pick_bucket_shape<T, 0>(lanes, vec);
}

// Default lane shape.  Global float atomics are executed past the L2 at a
// fixed rate per request, and one request covers at most one 128-byte line,
// so each gradient row is added by one instruction over consecutive lanes:
// one column per lane while R <= 64, else the fewest columns per lane.
template <typename T>
static void default_shape(int R, int& lanes, int& vec)
{
    const int vmax = 4;
    vec = 1;
    while (vec < vmax && R > 64 * vec && R % (2 * vec) == 0) vec *= 2;
    const int need = (R + vec - 1) / vec;
    lanes = 8;
    while (lanes < need && lanes < 64) lanes <<= 1;
}

// Widest vector that divides R (4 columns per lane in float32, 2 in
// float64), then the fewest power-of-two lanes covering R.
template <typename T>
static void wide_shape(int R, int& lanes, int& vec)
{
    const int vmax = sizeof(T) == 4 ? 4 : 2;
    vec = 1;
    while (vec < vmax && R % (2 * vec) == 0) vec *= 2;
    if (vec == 1) {                      // nothing to gain
        default_shape<T>(R, lanes, vec);
        return;
    }
    const int need = (R + vec - 1) / vec;
    lanes = vec == 4 ? 2 : 4;            // the narrowest shapes built
    while (lanes < need && lanes < 64) lanes <<= 1;
    if (lanes * vec < R) default_shape<T>(R, lanes, vec);
}

constexpr int kLdsPrivateBudget = 96 * 1024;    // bytes of private gradient per workgroup
constexpr int kBucketLdsBudget = 32 * 1024;     // default bytes of one row block in LDS
constexpr int kBucketMinSamples = 1 << 16;      // automatic bucketing only at or above this n
constexpr int kMaxBuckets = 4096;
constexpr int kBucketWgPerCu = 8;              // owner-pass workgroups per CU aimed at

template <typename T>
static gcp_status launch_loss_grad(const gcp_tensor_s* t, const gcp_sample_params* sp, const gcp_samples* smp,
                                   const void* A, int R, gcp_loss loss, unsigned flags, const void* scale_dev,
                                   void* G_out, double* loss_out, const gcp_tile* tile, const LGWorkspace& ws,
                                   hipStream_t stream, const LGOutputs* xo)
{
    LGParams<T> P{};
    int64_t n = 0;
    gcp_status st = make_sample_ctx<T>(t, sp, P.sc, n);
    if (st != GCP_OK) return st;
    const bool write_y = xo && xo->y_out;
    const bool loss_only = (flags & GCP_LOSS_ONLY) != 0 || write_y;
    const bool given_values = (int)loss == kLossGivenValues;
    const bool accumulate = (flags & GCP_ACCUMULATE) != 0;
    if (flags & ~(GCP_LOSS_ONLY | GCP_ACCUMULATE | GCP_SCALE_BY_DEV))
        return set_error(GCP_ERR_ARG, "unknown flags 0x%x", flags);
    if (!A) return set_error(GCP_ERR_ARG, "A is NULL");
    if (R < 1 || R > 256) return set_error(GCP_ERR_ARG, "R = %d outside [1, 256]", R);
    if ((loss < GCP_LOSS_GAUSSIAN || loss > GCP_LOSS_BERNOULLI_LOGIT) && !(given_values && smp))
        return set_error(GCP_ERR_ARG, "loss %d", (int)loss);
    if (!loss_only && !G_out) return set_error(GCP_ERR_ARG, "G_out is NULL");
    if ((flags & GCP_SCALE_BY_DEV) && !scale_dev) return set_error(GCP_ERR_ARG, "scale_dev is NULL");
    if (loss_only && !loss_out && !write_y) return set_error(GCP_ERR_ARG, "GCP_LOSS_ONLY without loss_out");
    if (write_y && (smp || !xo->coords_out)) return set_error(GCP_ERR_ARG, "sampled-tensor output needs coords_out");
    if (smp && (!smp->coords || !smp->x || (!smp->w && !given_values)) && n > 0)
        return set_error(GCP_ERR_ARG, "materialised sample list has a NULL array");
    if (given_values && loss_out) return set_error(GCP_ERR_ARG, "the MTTKRP of a given sampled tensor has no objective");

    const int d = t->d;
    const int cus = device_cu_count(t->device);

    // scatter strategy per mode: LDS-private, bucketed or atomic
    uint32_t lds_mask = 0, bucket_mask = 0;
    int64_t lds_elems = 0;
    const int req_lds = tile ? tile->lds_modes : -1;
    const int req_bucket = tile ? tile->bucket_modes : -1;
    if (!loss_only) {
        for (int k = 0; k < d; ++k) {
            const int64_t elems = t->dims[k] * (int64_t)R;
            const bool fits = (lds_elems + elems) * (int64_t)sizeof(T) <= kLdsPrivateBudget;
            bool want;
            // automatic: when the workgroups' final flushes are few next to
            // the per-sample global atomic requests they replace
            if (req_lds >= 0) want = (req_lds >> k) & 1;
            else want = fits && elems * 4 * (int64_t)cus <= n * R;
            if (want) {
                if (!fits) return set_error(GCP_ERR_ARG, "LDS-private modes exceed %d bytes", kLdsPrivateBudget);
                P.lds_off[k] = lds_elems;
                lds_elems += elems;
                lds_mask |= 1u << k;
            }
        }
        if (req_bucket > 0) bucket_mask = (uint32_t)req_bucket & ((1u << d) - 1) & ~lds_mask;
        else if (req_bucket < 0 && ws.base && n >= kBucketMinSamples && (ws.scratch_bytes > 0 || n <= ws.max_samples))
            bucket_mask = ((1u << d) - 1) & ~lds_mask;
    }
    // row-block geometry of the bucketed modes
    int br_shift = 0, nb = 0, nbm = 0, spb = 0;
    int64_t nblocks = 0;
    if (bucket_mask) {
        const int budget = (tile && tile->bucket_lds_bytes > 0) ? tile->bucket_lds_bytes : kBucketLdsBudget;
        if (budget < 8192) return set_error(GCP_ERR_ARG, "bucket_lds_bytes = %d < 8192", budget);
        while (((int64_t)2 << br_shift) * R * (int64_t)sizeof(T) <= budget && br_shift < 30) ++br_shift;
        int64_t nb_all = 0;
        for (int k = 0; k < d; ++k)
            if ((bucket_mask >> k) & 1u) nb_all += ceil_div(t->dims[k], int64_t(1) << br_shift);
        // automatic choice: modes with more row blocks than the owner pass
        // indexes (tall factor matrices, under one sample per row) keep the
        // atomic scatter
        if (req_bucket < 0 && nb_all > kMaxBuckets) bucket_mask = 0;
    }
    if (bucket_mask) {
        const int budget = (tile && tile->bucket_lds_bytes > 0) ? tile->bucket_lds_bytes : kBucketLdsBudget;
        for (int k = 0; k < d; ++k) {
            P.bucket_base[k] = nb;
            if ((bucket_mask >> k) & 1u) {
                if (nb + ceil_div(t->dims[k], int64_t(1) << br_shift) > kMaxBuckets)
                    return set_error(GCP_ERR_UNSUPPORTED, "more than %d row blocks of %d bytes", kMaxBuckets, budget);
                nb += (int)ceil_div(t->dims[k], int64_t(1) << br_shift);
                ++nbm;
            }
        }
        for (int k = d; k <= kMaxModes; ++k) P.bucket_base[k] = nb;
        if (tile && tile->bucket_block_samples > 0) {
            spb = tile->bucket_block_samples;
        } else {
            // 2048 samples per workgroup, fewer when that leaves under two
            // workgroups per CU
            spb = 2048;
            while (spb > 512 && ceil_div(n, spb) < 2 * (int64_t)cus) spb /= 2;
        }
        if (spb % 64 != 0 || spb < 512 || spb > 8192) return set_error(GCP_ERR_ARG, "bucket_block_samples = %d", spb);
        nblocks = ceil_div(n, spb);
        if (!ws.base) return set_error(GCP_ERR_ARG, "bucketed scatter needs gcp_tensor_reserve first");
        if (ws.scratch_bytes > 0) {
            // fixed scratch: entries first, then counts and starts
            const int64_t need = nblocks * spb * (int64_t)nbm * 16 + (int64_t)nb * nblocks * 8;
            if (need > ws.scratch_bytes) {
                if (req_bucket >= 0)
                    return set_error(GCP_ERR_ARG,
                                     "bucketed scatter of %lld samples needs %lld bytes of scratch, the maximum is %lld",
                                     (long long)n, (long long)need, (long long)ws.scratch_bytes);
                // automatic choice: hardware atomics need no scratch
                bucket_mask = 0;
                nb = nbm = spb = 0;
                nblocks = 0;
            }
        } else if (n > ws.max_samples || nblocks * spb * (int64_t)nbm > ws.entries || (int64_t)nb * nblocks > ws.hist) {
            return set_error(GCP_ERR_ARG, "workspace reserved by gcp_tensor_reserve is too small for this call");
        }
    }

    // lane shape: one column per lane while any mode scatters with global
    // atomics (one request per row); otherwise the widest vector, which
    // spreads each sample over the fewest lanes and so cuts the per-sample
    // instructions (the LDS and bucketed scatters issue no global atomics)
    const uint32_t all_modes = (1u << d) - 1;
    const bool no_global_atomics = loss_only || ((lds_mask | bucket_mask) == all_modes);
    int lanes = 0, vec = 0;
    default_shape<T>(R, lanes, vec);
    if (no_global_atomics) wide_shape<T>(R, lanes, vec);
    if (tile && tile->vec > 0) vec = tile->vec;
    if (tile && tile->lanes > 0) lanes = tile->lanes;
    else if (tile && tile->vec > 0) {
        const int need = (R + vec - 1) / vec;
        lanes = 2;
        while (lanes < need && lanes < 64) lanes <<= 1;
    }
    if (R % vec != 0) return set_error(GCP_ERR_ARG, "vec = %d does not divide R = %d", vec, R);
    if (lanes * vec < R) return set_error(GCP_ERR_ARG, "lanes*vec = %d < R = %d", lanes * vec, R);
    const int src = write_y ? 2 : smp ? (given_values ? 3 : 1) : 0;
    // the general-order float64 kernel with 64 lanes of one column needs 128
    // VGPRs and spills; even R takes 32 lanes of two columns instead
    if (sizeof(T) == 8 && kernel_order(t) == 0 && lanes == 64 && vec == 1 && R % 2 == 0 && !(tile && tile->lanes > 0)) {
        lanes = 32;
        vec = 2;
    }
    LGKernel<T> kern = pick_kernel<T>(kernel_order(t), src, lanes, vec);
    if (!kern) return set_error(GCP_ERR_UNSUPPORTED, "tile lanes = %d, vec = %d not built for this dtype", lanes, vec);
    const uintptr_t align = (uintptr_t)vec * sizeof(T);
    if (((uintptr_t)A % align) != 0) return set_error(GCP_ERR_ARG, "A is not %d-byte aligned", (int)align);

    int block = 256;
    if (lds_mask) block = 1024;
    else if (bucket_mask) block = 512;
    if (tile && tile->block > 0) {
        if (tile->block % 64 != 0 || tile->block > 1024) return set_error(GCP_ERR_ARG, "block = %d", tile->block);
        block = tile->block;
    }
    const int nwaves = block / 64;
    const int staging = nwaves * 64 * (8 + 2 * (int)sizeof(T));
    size_t lds_bytes = (size_t)staging + (size_t)lds_elems * sizeof(T);
    lds_bytes = (lds_bytes + 15) & ~(size_t)15;
    const int bucket_lds = (int)lds_bytes;
    if (bucket_mask) lds_bytes += (size_t)spb * (8 + sizeof(T)) + (size_t)nb * 8;
    const int64_t nchunks = ceil_div(n, 64);
    int64_t grid;
    st = prepare_lds(reinterpret_cast<const void*>(kern), lds_bytes, t->device);
    if (st != GCP_OK) return st;
    if (bucket_mask) {
        grid = nblocks;
    } else {
        int per_cu = 0;
        GCP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern), block,
                                                            lds_bytes));
        if (per_cu < 1) return set_error(GCP_ERR_UNSUPPORTED, "kernel does not fit on a CU (LDS %zu B)", lds_bytes);
        const int64_t resident = (int64_t)per_cu * cus;
        grid = std::max<int64_t>(1, std::min<int64_t>(resident, ceil_div(nchunks, nwaves)));
        if (tile && tile->grid > 0) grid = tile->grid;
    }

    P.n = n;
    P.nchunks = nchunks;
    if (smp) {
        P.m_coords = smp->coords;
        P.m_x = (const T*)smp->x;
        P.m_w = (const T*)smp->w;
    }
    P.A = (const T*)A;
    P.G = (T*)G_out;
    P.R = R;
    P.loss = loss;
    P.loss_only = loss_only;
    P.semi = sp->kind == GCP_SAMPLE_SEMI_STRATIFIED;
    P.scale = (flags & GCP_SCALE_BY_DEV) ? (const T*)scale_dev : nullptr;
    P.loss_out = loss_out;
    if (write_y) {
        P.y_out = (T*)xo->y_out;
        P.c_out = xo->coords_out;
    }
    if (xo && xo->loss_parts && loss_out) {
        if (bucket_mask) return set_error(GCP_ERR_ARG, "per-wave objective partials need an unbucketed launch");
        if (grid * nwaves > xo->loss_parts_cap)
            return set_error(GCP_ERR_ARG, "%lld objective partials exceed the %lld slots", (long long)(grid * nwaves),
                             (long long)xo->loss_parts_cap);
        P.loss_parts = xo->loss_parts;
        if (xo->parts_used) *xo->parts_used = grid * nwaves;
    }
    for (int k = 0; k < kMaxModes; ++k) P.rowoff[k] = k < d ? t->rowoff[k] : t->rowoff[d];
    P.lds_mask = lds_mask;
    P.lds_elems = lds_elems;
    P.staging_bytes = staging;
    P.bucket_mask = bucket_mask;
    P.n_bucket_modes = nbm;
    P.br_shift = br_shift;
    P.nb = nb;
    P.spb = spb;
    P.nblocks = nblocks;
    P.entry_cap = (int64_t)spb * nbm;
    P.bucket_lds = bucket_lds;
    if (bucket_mask) {
        const int64_t ent = ws.scratch_bytes > 0 ? nblocks * spb * (int64_t)nbm : ws.entries;
        const int64_t hist = ws.scratch_bytes > 0 ? (int64_t)nb * nblocks : ws.hist;
        P.entries = (uint4*)ws.base;
        P.hist = (int*)((char*)ws.base + ent * 16);
        P.start = P.hist + hist;
    }

    if (!accumulate) {
        const int64_t gn = loss_only ? 0 : t->rowoff[d] * R;
        if (gn > 0 || loss_out) {
            int64_t zb = std::max<int64_t>(1, std::min<int64_t>(ceil_div(gn, 256), 4096));
            k_zero<T><<<(unsigned)zb, 256, 0, stream>>>((T*)G_out, gn, loss_out);
            GCP_HIP(hipGetLastError());
        }
    }
    if (n == 0) return GCP_OK;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(block), lds_bytes, stream, P);
    GCP_HIP(hipGetLastError());
    if (bucket_mask) {
        BAKernel<T> bk = pick_bucket_kernel<T>(kernel_order(t), lanes, vec);
        if (!bk) return set_error(GCP_ERR_UNSUPPORTED, "no bucket kernel for lanes = %d, vec = %d", lanes, vec);
        const int bblock = (tile && tile->bucket_block > 0) ? tile->bucket_block : 1024;
        if (bblock % 64 != 0 || bblock > 1024) return set_error(GCP_ERR_ARG, "bucket_block = %d", bblock);
        const int bwaves = bblock / 64;
        // workgroups per row block: proportional to the entries a row block
        // of the mode expects (n * rows per block / I_k, samples uniform over
        // the rows), aiming at kBucketWgPerCu owner workgroups per CU.  Each
        // workgroup reads a whole number of segments per wave, since its waves
        // take its segments in turn and one wave with an extra segment would
        // hold up the workgroup
        const int64_t rows_blk = int64_t(1) << br_shift;
        double expect_total = 0.0;
        for (int k = 0; k < d; ++k)
            if ((bucket_mask >> k) & 1u) expect_total += (double)n;
        const double per_wg = std::max(1.0, expect_total / ((double)kBucketWgPerCu * cus));
        int64_t wg = 0, max_segs = 0;
        for (int k = 0; k < d; ++k) {
            P.bwg_base[k] = wg;
            P.bsplits[k] = 1;
            P.bsegs[k] = (int)nblocks;
            if (!((bucket_mask >> k) & 1u)) continue;
            int64_t segs;
            if (tile && tile->bucket_splits > 0) {
                segs = ceil_div(nblocks, (int64_t)tile->bucket_splits);
            } else {
                const double per_block = (double)n * (double)std::min<int64_t>(rows_blk, t->dims[k]) / (double)t->dims[k];
                const double target = std::max(1.0, std::ceil(per_block / per_wg));
                const int64_t per_wave = std::max<int64_t>(1, std::llround((double)nblocks / (target * bwaves)));
                segs = per_wave * bwaves;
            }
            segs = std::max<int64_t>(1, std::min<int64_t>(segs, nblocks));
            P.bsegs[k] = (int)segs;
            P.bsplits[k] = (int)ceil_div(nblocks, segs);
            max_segs = std::max<int64_t>(max_segs, segs);
            wg += (int64_t)(P.bucket_base[k + 1] - P.bucket_base[k]) * P.bsplits[k];
        }
        for (int k = d; k <= kMaxModes; ++k) P.bwg_base[k] = wg;
        const size_t part_bytes = ((((size_t)1 << br_shift) * R * sizeof(T) + 15) & ~(size_t)15) + 8 * (size_t)max_segs;
        st = prepare_lds(reinterpret_cast<const void*>(bk), part_bytes, t->device);
        if (st != GCP_OK) return st;
        hipLaunchKernelGGL(bk, dim3((unsigned)wg), dim3(bblock), part_bytes, stream, P);
        GCP_HIP(hipGetLastError());
    }
    return GCP_OK;
}

gcp_status loss_grad_with_workspace(gcp_tensor_s* t, const gcp_sample_params* sp, const gcp_samples* smp,
                                    const void* A, int R, gcp_loss loss, unsigned flags, const void* scale_dev,
                                    void* G_out, double* loss_out, const gcp_tile* tile, const LGWorkspace& ws,
                                    hipStream_t stream, const LGOutputs* xo)
{
    if (t->dt == GCP_F32)
        return launch_loss_grad<float>(t, sp, smp, A, R, loss, flags, scale_dev, G_out, loss_out, tile, ws, stream,
                                       xo);
    return launch_loss_grad<double>(t, sp, smp, A, R, loss, flags, scale_dev, G_out, loss_out, tile, ws, stream,
                                    xo);
}

static LGWorkspace reserved_workspace(const gcp_tensor_s* t)
{
    LGWorkspace ws;
    ws.base = t->ws;
    ws.entries = t->ws_entries;
    ws.hist = t->ws_hist;
    ws.max_samples = t->ws_max_samples;
    return ws;
}

}  // namespace gcp

extern "C" gcp_status gcp_loss_grad(gcp_tensor t, const gcp_sample_params* sp, const gcp_samples* smp,
                                    const void* A, int R, gcp_loss loss, unsigned flags, const void* scale_dev,
                                    void* G_out, double* loss_out, const gcp_tile* tile, hipStream_t stream)
{
    gcp::clear_error();
    if (!t) return gcp::set_error(GCP_ERR_ARG, "tensor is NULL");
    if (flags & GCP_DETERMINISTIC)
        return gcp::loss_grad_deterministic(t, sp, smp, A, R, loss, flags, scale_dev, G_out, loss_out, tile, stream);
    return gcp::loss_grad_with_workspace(t, sp, smp, A, R, loss, flags, scale_dev, G_out, loss_out, tile,
                                         gcp::reserved_workspace(t), stream);
}

extern "C" gcp_status gcp_sample_y(gcp_tensor t, const gcp_sample_params* sp, const void* A, int R, gcp_loss loss,
                                   int64_t* coords_out, void* y_out, double* loss_out, const gcp_tile* tile,
                                   hipStream_t stream)
{
    gcp::clear_error();
    if (!t) return gcp::set_error(GCP_ERR_ARG, "tensor is NULL");
    if (!y_out || !coords_out) return gcp::set_error(GCP_ERR_ARG, "coords_out or y_out is NULL");
    gcp::LGOutputs xo;
    xo.y_out = y_out;
    xo.coords_out = coords_out;
    gcp_tile tl = tile ? *tile : gcp_tile{};
    tl.lds_modes = 0;               // this kernel scatters nothing
    tl.bucket_modes = 0;
    return gcp::loss_grad_with_workspace(t, sp, nullptr, A, R, loss, 0u, nullptr, nullptr, loss_out, &tl,
                                         gcp::LGWorkspace{}, stream, &xo);
}

extern "C" gcp_status gcp_mttkrp(gcp_tensor t, int64_t n, const int64_t* coords, const void* y, const void* A,
                                 int R, unsigned flags, const void* scale_dev, void* G_out, const gcp_tile* tile,
                                 hipStream_t stream)
{
    gcp::clear_error();
    if (!t) return gcp::set_error(GCP_ERR_ARG, "tensor is NULL");
    if (n < 0) return gcp::set_error(GCP_ERR_ARG, "n < 0");
    if (flags & GCP_LOSS_ONLY) return gcp::set_error(GCP_ERR_ARG, "GCP_LOSS_ONLY makes no sense for the MTTKRP");
    gcp_sample_params sp{};
    sp.kind = t->dense ? GCP_SAMPLE_UNIFORM : GCP_SAMPLE_STRATIFIED;
    sp.p = n;
    sp.q = 0;
    gcp_samples smp{coords, y, nullptr};
    return gcp::loss_grad_with_workspace(t, &sp, &smp, A, R, (gcp_loss)gcp::kLossGivenValues, flags, scale_dev, G_out,
                                         nullptr, tile, gcp::reserved_workspace(t), stream);
}
