// Deterministic sampled gradient (gcp_loss_grad with GCP_DETERMINISTIC): the
// same gradient and objective, bit for bit, on every run with the same
// samples, model, tile and device.  The default scatters add floats in an
// order that depends on timing (atomics, LDS compare-and-swap, per-workgroup
// flushes); here every sum has a fixed order:
//   1. the sampling kernel (k_loss_grad, SRC = 2) writes the sampled tensor
//      -- coordinates and y = w f'(x, m) of every sample -- and each
//      wavefront's partial objective into its own slot;
//   2. k_det_pairs lists (model row, sample) for every sample and mode;
//   3. a stable radix sort by row (rocPRIM) groups each row's samples in
//      sample order;
//   4. k_det_starts finds where each row's run begins, and rocPRIM's unique
//      lists the rows whose run is not empty (in row order);
//   5. k_det_reduce gives each listed gradient row to one lane group, which adds
//      y prod_{j != k} A_j[i_j, :] over the row's run in an order fixed by
//      the sorted run (the sampled MTTKRP of eq. gcp-gradient, Sec. 3.1.2)
//      and writes the row;
//   6. k_det_loss adds the objective partials in slot order.
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_select.hpp>

#include "lg_kernels.hpp"

namespace gcp {
namespace {

struct DetModes {
    int d;
    uint32_t rowoff[kMaxModes + 1];
};

// (row, sample) of mode k for sample s at k * n + s.
__global__ void __launch_bounds__(256) k_det_pairs(const int64_t* __restrict__ coords, int64_t n, DetModes M,
                                                   uint32_t* __restrict__ keys, uint32_t* __restrict__ vals)
{
    const int64_t total = n * M.d;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = i / n, s = i - k * n;
        keys[i] = M.rowoff[k] + (uint32_t)coords[s * M.d + k];
        vals[i] = (uint32_t)s;
    }
}

// start[r] = first position of row r in the sorted keys (rows + 1 entries,
// start[rows] = total); every row gets a value, empty rows an empty run.
__global__ void __launch_bounds__(256) k_det_starts(const uint32_t* __restrict__ skeys, int64_t total, uint32_t rows,
                                                    uint32_t* __restrict__ start)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t lo = i == 0 ? 0 : (int64_t)skeys[i - 1] + 1;      // rows after the previous key
        const int64_t hi = i == total ? (int64_t)rows : (int64_t)skeys[i];
        for (int64_t r = lo; r <= hi; ++r) start[r] = (uint32_t)i;
    }
}

// Lanes per gradient row in k_det_reduce: R rounded up to a power of two,
// at most 64.
__host__ __device__ inline int det_group_lanes(int R)
{
    int rp = 1;
    while (rp < R && rp < 64) rp <<= 1;
    return rp;
}

// Value of `v` in lane `src` of the wavefront; doubles move as two 32-bit
// halves.
__device__ __forceinline__ float lane_get(float v, int src) { return __shfl(v, src, 64); }
__device__ __forceinline__ double lane_get(double v, int src)
{
    const long long b = __double_as_longlong(v);
    const int lo = __shfl((int)(b & 0xffffffffll), src, 64);
    const int hi = __shfl((int)(b >> 32), src, 64);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// One lane group per gradient row: RP lanes (RP = R rounded up to a power of
// two, at most 64; wider ranks take the columns 64 at a time), so a
// wavefront holds H = 64 / RP rows at once.  A group reads its row's run of
// sorted (row, sample) pairs RP at a time, one pair per lane: the lane loads
// the sample's y and the model rows of the other modes.  Lane shuffles inside
// the group then hand the pairs out in run order; the group gathers the other
// modes' rows and adds y prod_{j != k} A_j[i_j, :] in that order.  Every sum
// thus has an order fixed by the sorted run alone.  Only the listed rows
// (those with pairs) are visited; when the call does not accumulate, G is zeroed
// before this kernel, so rows without pairs hold 0.
template <typename T, int D>
__global__ void __launch_bounds__(256) k_det_reduce(const uint32_t* __restrict__ start,
                                                    const uint32_t* __restrict__ runs,
                                                    const uint32_t* __restrict__ nruns,
                                                    const uint32_t* __restrict__ svals,
                                                    const int64_t* __restrict__ coords, const T* __restrict__ y,
                                                    const T* __restrict__ A, DetModes M, int R,
                                                    const T* __restrict__ scale, int accumulate, T* __restrict__ G)
{
    constexpr int DM = D > 0 ? D : kMaxModes;
    constexpr int DO = DM - 1;
    constexpr int U = 4;
    const int dd = D > 0 ? D : M.d;
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const T sc = scale ? *scale : T(1);
    const int RP = det_group_lanes(R);
    const int H = 64 / RP;
    const int h = lane / RP, cg = lane % RP, gl0 = h * RP;
    const int64_t nr = *nruns;
    for (int64_t j0 = wave * H; j0 < nr; j0 += nw * H) {
        const int64_t j = j0 + h;
        if (j >= nr) break;               // no row for this group; shuffles stay inside a group
        const uint32_t r = runs[j];
        int k = 0;
        for (int kk = 1; kk < dd; ++kk)
            if (M.rowoff[kk] <= r) k = kk;
        const uint32_t b = start[r], e = start[r + 1];
        for (int c0 = 0; c0 < R; c0 += RP) {
            const int c = c0 + cg;
            const bool col = c < R;
            const uint64_t colL = col ? (uint32_t)c : 0u;
            T acc = T(0);
            for (uint32_t i0 = b; i0 < e; i0 += (uint32_t)RP) {
                const uint32_t nv = min(e - i0, (uint32_t)RP);
                // lane cg of the group: pair i0 + cg (past the run's end: its last pair)
                const uint32_t sl = svals[i0 + min((uint32_t)cg, nv - 1)];
                const T yl = y[sl] * sc;
                uint32_t orow[DO];
#pragma unroll
                for (int o = 0; o < DO; ++o) {
                    const int m = o + (o >= k ? 1 : 0);
                    orow[o] = (D > 0 || m < dd) ? M.rowoff[m] + (uint32_t)coords[(uint64_t)sl * dd + m] : 0u;
                }
                for (uint32_t q0 = 0; q0 < nv; q0 += U) {
                    T yq[U], prod[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int q = gl0 + (int)min(q0 + (uint32_t)u, nv - 1);
                        yq[u] = lane_get(yl, q);
                        prod[u] = T(1);
#pragma unroll
                        for (int o = 0; o < DO; ++o) {
                            if (D == 0 && o >= dd - 1) break;
                            const uint32_t row = (uint32_t)__shfl((int)orow[o], q, 64);
                            prod[u] *= A[(uint64_t)row * (uint32_t)R + colL];
                        }
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u)
                        if (q0 + (uint32_t)u < nv) acc += yq[u] * prod[u];
                }
            }
            if (col) {
                T* g = G + (uint64_t)r * (uint32_t)R + c;
                *g = accumulate ? *g + acc : acc;
            }
        }
    }
}

__global__ void k_det_loss(const double* __restrict__ parts, int64_t n, int accumulate, double* __restrict__ out)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += parts[i];
    *out = accumulate ? *out + s : s;
}

constexpr int64_t kDetLossSlots = 1 << 16;

int sort_bits(uint32_t rows)
{
    int b = 1;
    while (b < 32 && ((uint64_t)1 << b) < rows) ++b;
    return b;
}

struct DetLayout {
    int64_t coords, y, keys_in, vals_in, keys_out, vals_out, start, runs, nruns, parts, scratch_loss, sort_tmp, total;
    size_t sort_bytes;
};

int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

gcp_status det_layout(const gcp_tensor_s* t, int64_t n, DetLayout& L)
{
    const int64_t esize = t->dt == GCP_F32 ? 4 : 8;
    const int64_t pairs = n * t->d;
    const uint32_t rows = (uint32_t)t->rowoff[t->d];
    L.sort_bytes = 0;
    hipError_t e = rocprim::radix_sort_pairs(nullptr, L.sort_bytes, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                             (const uint32_t*)nullptr, (uint32_t*)nullptr, (size_t)pairs, 0,
                                             (unsigned)sort_bits(rows + 1), (hipStream_t)0);
    if (e != hipSuccess) return hip_error(e, "rocprim::radix_sort_pairs (size query)");
    size_t unique_bytes = 0;
    e = rocprim::unique(nullptr, unique_bytes, (const uint32_t*)nullptr, (uint32_t*)nullptr, (uint32_t*)nullptr,
                        (size_t)pairs, rocprim::equal_to<uint32_t>(), (hipStream_t)0);
    if (e != hipSuccess) return hip_error(e, "rocprim::unique (size query)");
    L.sort_bytes = std::max(L.sort_bytes, unique_bytes);          // the two use the region one after the other
    int64_t off = 0;
    L.coords = off; off = align256(off + pairs * 8);
    L.y = off; off = align256(off + n * esize);
    L.keys_in = off; off = align256(off + pairs * 4);
    L.vals_in = off; off = align256(off + pairs * 4);
    L.keys_out = off; off = align256(off + pairs * 4);
    L.vals_out = off; off = align256(off + pairs * 4);
    L.start = off; off = align256(off + ((int64_t)rows + 1) * 4);
    L.runs = off; off = align256(off + std::min<int64_t>(rows, pairs) * 4);
    L.nruns = off; off = align256(off + 4);
    L.parts = off; off = align256(off + kDetLossSlots * 8);
    L.scratch_loss = off; off = align256(off + 8);
    L.sort_tmp = off; off = align256(off + (int64_t)L.sort_bytes);
    L.total = off;
    return GCP_OK;
}

template <typename T>
gcp_status launch_det(gcp_tensor_s* t, const gcp_sample_params* sp, const void* A, int R, gcp_loss loss,
                      unsigned flags, const void* scale_dev, void* G_out, double* loss_out, const gcp_tile* tile,
                      hipStream_t stream)
{
    if (!t->ws || !sp) return set_error(GCP_ERR_ARG, "GCP_DETERMINISTIC needs gcp_tensor_reserve first");
    if (flags & GCP_LOSS_ONLY) return set_error(GCP_ERR_ARG, "GCP_DETERMINISTIC with GCP_LOSS_ONLY");
    if (!G_out) return set_error(GCP_ERR_ARG, "G_out is NULL");
    if ((flags & GCP_SCALE_BY_DEV) && !scale_dev) return set_error(GCP_ERR_ARG, "scale_dev is NULL");
    const int64_t n = sp->p + sp->q;
    if (n < 0 || n > t->ws_max_samples)
        return set_error(GCP_ERR_ARG, "GCP_DETERMINISTIC: %lld samples exceed the reserved %lld",
                         (long long)n, (long long)t->ws_max_samples);
    // (row, sample) pairs are indexed with 32 bits (run starts, sorted values)
    if (n * t->d >= (int64_t(1) << 32))
        return set_error(GCP_ERR_ARG, "GCP_DETERMINISTIC: %lld samples x %d modes reach 2^32 (row, sample) pairs",
                         (long long)n, t->d);
    DetLayout L{};
    gcp_status st = det_layout(t, n, L);
    if (st != GCP_OK) return st;
    if (L.total > t->ws_bytes) return set_error(GCP_ERR_ARG, "the reserved workspace is too small for this call");
    char* ws = (char*)t->ws;
    const bool accumulate = (flags & GCP_ACCUMULATE) != 0;
    const uint32_t rows = (uint32_t)t->rowoff[t->d];
    // 1. the sampled tensor and the per-wavefront objective partials; the
    //    launch's own objective target is a scratch word, so that loss_out
    //    keeps its accumulate semantics
    LGOutputs xo;
    xo.y_out = ws + L.y;
    xo.coords_out = (int64_t*)(ws + L.coords);
    xo.loss_parts = loss_out ? (double*)(ws + L.parts) : nullptr;
    xo.loss_parts_cap = kDetLossSlots;
    int64_t parts = 0;
    xo.parts_used = &parts;
    gcp_tile tl = tile ? *tile : gcp_tile{};
    tl.lds_modes = 0;
    tl.bucket_modes = 0;
    st = loss_grad_with_workspace(t, sp, nullptr, A, R, loss, 0u, nullptr, nullptr,
                                  loss_out ? (double*)(ws + L.scratch_loss) : nullptr, &tl, LGWorkspace{}, stream,
                                  &xo);
    if (st != GCP_OK) return st;
    if (n == 0) {
        if (!accumulate) {
            const int64_t gn = (int64_t)rows * R;
            const unsigned zb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(gn, 256), 4096));
            k_zero<T><<<zb, 256, 0, stream>>>((T*)G_out, gn, loss_out);
            GCP_HIP(hipGetLastError());
        }
        return GCP_OK;
    }
    DetModes M{};
    M.d = t->d;
    for (int k = 0; k <= t->d; ++k) M.rowoff[k] = (uint32_t)t->rowoff[k];
    const int cus = device_cu_count(t->device);
    const int64_t pairs = n * t->d;
    // 2. (row, sample) pairs
    const unsigned pg = (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(pairs, 256), (int64_t)cus * 16));
    hipLaunchKernelGGL(k_det_pairs, dim3(pg), dim3(256), 0, stream, (const int64_t*)(ws + L.coords), n, M,
                       (uint32_t*)(ws + L.keys_in), (uint32_t*)(ws + L.vals_in));
    GCP_HIP(hipGetLastError());
    // 3. stable sort by row
    size_t sort_bytes = L.sort_bytes;
    GCP_HIP(rocprim::radix_sort_pairs(ws + L.sort_tmp, sort_bytes, (const uint32_t*)(ws + L.keys_in),
                                      (uint32_t*)(ws + L.keys_out), (const uint32_t*)(ws + L.vals_in),
                                      (uint32_t*)(ws + L.vals_out), (size_t)pairs, 0,
                                      (unsigned)sort_bits(rows + 1), stream));
    // 4. run starts and the list of rows with pairs
    const unsigned sg = (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(pairs + 1, 256), (int64_t)cus * 16));
    hipLaunchKernelGGL(k_det_starts, dim3(sg), dim3(256), 0, stream, (const uint32_t*)(ws + L.keys_out), pairs, rows,
                       (uint32_t*)(ws + L.start));
    GCP_HIP(hipGetLastError());
    size_t unique_bytes = L.sort_bytes;
    GCP_HIP(rocprim::unique(ws + L.sort_tmp, unique_bytes, (const uint32_t*)(ws + L.keys_out),
                            (uint32_t*)(ws + L.runs), (uint32_t*)(ws + L.nruns), (size_t)pairs,
                            rocprim::equal_to<uint32_t>(), stream));
    // 5. one lane group per listed gradient row (all others stay as they
    //    are, or 0 when the call does not accumulate)
    if (!accumulate) {
        const int64_t gn = (int64_t)rows * R;
        const unsigned zb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(gn, 256), (int64_t)cus * 16));
        k_zero<T><<<zb, 256, 0, stream>>>((T*)G_out, gn, nullptr);
        GCP_HIP(hipGetLastError());
    }
    const int64_t max_runs = std::min<int64_t>(rows, pairs);
    const int64_t rows_per_wg = 4 * (64 / det_group_lanes(R));          // 4 wavefronts of 64 / RP rows
    const unsigned rg =
        (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(max_runs, rows_per_wg), (int64_t)cus * 32));
    auto reduce = t->d == 3 ? k_det_reduce<T, 3> : t->d == 4 ? k_det_reduce<T, 4> : k_det_reduce<T, 0>;
    hipLaunchKernelGGL(reduce, dim3(rg), dim3(256), 0, stream, (const uint32_t*)(ws + L.start),
                       (const uint32_t*)(ws + L.runs), (const uint32_t*)(ws + L.nruns),
                       (const uint32_t*)(ws + L.vals_out), (const int64_t*)(ws + L.coords), (const T*)(ws + L.y),
                       (const T*)A, M, R, (flags & GCP_SCALE_BY_DEV) ? (const T*)scale_dev : nullptr,
                       accumulate ? 1 : 0, (T*)G_out);
    GCP_HIP(hipGetLastError());
    // 6. the objective, partials in slot order
    if (loss_out) {
        hipLaunchKernelGGL(k_det_loss, dim3(1), dim3(64), 0, stream, (const double*)(ws + L.parts), parts,
                           accumulate ? 1 : 0, loss_out);
        GCP_HIP(hipGetLastError());
    }
    return GCP_OK;
}

}  // namespace

int64_t det_workspace_bytes(const gcp_tensor_s* t, int64_t max_samples)
{
    DetLayout L{};
    if (det_layout(t, max_samples, L) != GCP_OK) return -1;
    return L.total;
}

gcp_status loss_grad_deterministic(gcp_tensor_s* t, const gcp_sample_params* sp, const gcp_samples* smp,
                                   const void* A, int R, gcp_loss loss, unsigned flags, const void* scale_dev,
                                   void* G_out, double* loss_out, const gcp_tile* tile, hipStream_t stream)
{
    if (smp) return set_error(GCP_ERR_UNSUPPORTED, "GCP_DETERMINISTIC takes drawn samples only (smp must be NULL)");
    if (!A) return set_error(GCP_ERR_ARG, "A is NULL");
    if (R < 1 || R > 256) return set_error(GCP_ERR_ARG, "R = %d outside [1, 256]", R);
    const unsigned f = flags & ~(unsigned)GCP_DETERMINISTIC;
    if (t->dt == GCP_F32) return launch_det<float>(t, sp, A, R, loss, f, scale_dev, G_out, loss_out, tile, stream);
    return launch_det<double>(t, sp, A, R, loss, f, scale_dev, G_out, loss_out, tile, stream);
}

}  // namespace gcp
