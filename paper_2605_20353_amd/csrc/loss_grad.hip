// gcp_loss_grad: the fused sampled objective and gradient (Sec. 3.1.1-3.1.2,
// "Fused Sampling-MTTKRP", here with stratified, uniform or semi-stratified
// samples).
//
// Work decomposition (one 64-lane wavefront takes 64 samples at a time):
//   phase 1, one lane per sample: draw the sample (Philox, nonzero record
//     read or zero-candidate hash probes) or read it from a materialised
//     list, and stage (packed key, x, w) in the wave's LDS slice;
//   phase 2, LANES lanes per sample with VEC consecutive columns each, 64 /
//     LANES samples per pass: gather the d factor rows (coalesced LANES*VEC
//     columns), m = sum_r prod_k A_k[i_k, r] (eq. cp) by a butterfly over
//     the lane group, y = w f'(x, m), then the leave-one-out products
//     y prod_{n != k} A_n[i_n, r] are added into G_k[i_k, :] with hardware
//     float atomics -- into global memory, or into an LDS-private copy of a
//     small mode's gradient that the workgroup flushes once at the end (the
//     paper's "thread privatization", per workgroup).
// Factor rows are read once per sample and the sampled tensor is never
// written to memory.
#include <algorithm>

#include "sampling.hpp"

namespace gcp {

template <typename T>
struct LGParams {
    SampleCtx<T> sc;
    int64_t n;            // samples p + q
    int64_t nchunks;      // ceil(n / 64)
    const int64_t* m_coords;  // materialised list (SRC = 1)
    const T* m_x;
    const T* m_w;
    const T* A;
    T* G;
    int R;
    int loss;
    int loss_only;
    int semi;             // semi-stratified: samples s < p get f'(x,m) - f'(0,m)
    const T* scale;       // nullable device scalar
    double* loss_out;     // nullable
    int64_t rowoff[kMaxModes];
    uint32_t lds_mask;    // modes accumulated in LDS
    int64_t lds_off[kMaxModes];
    int64_t lds_elems;
    int staging_bytes;
};

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T, int V>
__device__ __forceinline__ void load_cols(const T* __restrict__ p, T (&out)[V])
{
    if constexpr (V == 4 && sizeof(T) == 4) {
        float4 f = *reinterpret_cast<const float4*>(p);
        out[0] = f.x; out[1] = f.y; out[2] = f.z; out[3] = f.w;
    } else if constexpr (V == 2 && sizeof(T) == 4) {
        float2 f = *reinterpret_cast<const float2*>(p);
        out[0] = f.x; out[1] = f.y;
    } else if constexpr (V == 2 && sizeof(T) == 8) {
        double2 f = *reinterpret_cast<const double2*>(p);
        out[0] = f.x; out[1] = f.y;
    } else {
#pragma unroll
        for (int v = 0; v < V; ++v) out[v] = p[v];
    }
}

template <typename T>
__device__ __forceinline__ void global_add(T* p, T v)
{
    unsafeAtomicAdd(p, v);
}

template <typename T, int D, int LANES, int VEC, int SRC>
__global__ void __launch_bounds__(1024) k_loss_grad(const LGParams<T> P)
{
    constexpr int S = 64 / LANES;                  // samples per pass
    constexpr int DM = D > 0 ? D : kMaxModes;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int nwaves = blockDim.x >> 6;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint64_t* skey = reinterpret_cast<uint64_t*>(smem) + wave * 64;
    T* sx = reinterpret_cast<T*>(smem + (size_t)nwaves * 64 * 8) + wave * 64;
    T* sw = reinterpret_cast<T*>(smem + (size_t)nwaves * 64 * (8 + sizeof(T))) + wave * 64;
    T* priv = reinterpret_cast<T*>(smem + P.staging_bytes);

    if (P.lds_mask) {
        for (int64_t e = threadIdx.x; e < P.lds_elems; e += blockDim.x) priv[e] = T(0);
        __syncthreads();
    }
    const int dd = D > 0 ? D : P.sc.d;
    const int R = P.R;
    const int g = lane / LANES, cl = lane % LANES;
    const int col0 = cl * VEC;
    const bool col_ok = col0 < R;          // VEC divides R
    const T scale = P.scale ? *P.scale : T(1);
    double lacc = 0.0;

    for (int64_t chunk = (int64_t)blockIdx.x * nwaves + wave; chunk < P.nchunks;
         chunk += (int64_t)gridDim.x * nwaves) {
        const int64_t s0 = chunk * 64;
        {   // phase 1: one lane per sample
            const int64_t s = s0 + lane;
            uint64_t key = 0;
            T x = T(0), w = T(0);
            if (s < P.n) {
                if constexpr (SRC == 0) {
                    draw_sample<T, D>(P.sc, s, key, x, w);
                } else {
                    bool ok = true;
#pragma unroll
                    for (int k = 0; k < DM; ++k) {
                        if (k < dd) {
                            int64_t c = P.m_coords[s * dd + k];
                            if (c < 0 || c >= P.sc.L.dims[k]) ok = false;
                            else key |= (uint64_t)c << P.sc.L.shift[k];
                        }
                    }
                    x = P.m_x[s];
                    w = P.m_w[s];
                    if (!ok) {
                        atomicOr(P.sc.status, kStatusData);
                        key = 0;
                        w = T(0);
                    }
                }
            }
            skey[lane] = key;
            sx[lane] = x;
            sw[lane] = w;
        }
        wave_sync();
        // phase 2: LANES lanes per sample
        for (int it = 0; it < LANES; ++it) {
            const int slot = it * S + g;
            const int64_t s = s0 + slot;
            if (s >= P.n) break;
            const uint64_t key = skey[slot];
            const T x = sx[slot], w = sw[slot];
            int64_t row[DM];
            T a[DM][VEC];
#pragma unroll
            for (int k = 0; k < DM; ++k) {
                if (k < dd) {
                    row[k] = P.rowoff[k] + (int64_t)unpack(P.sc.L, key, k);
                    if (col_ok) {
                        load_cols<T, VEC>(P.A + row[k] * R + col0, a[k]);
                    } else {
#pragma unroll
                        for (int v = 0; v < VEC; ++v) a[k][v] = T(0);
                    }
                }
            }
            T part = T(0);
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                T prod = a[0][v];
#pragma unroll
                for (int k = 1; k < DM; ++k)
                    if (k < dd) prod *= a[k][v];
                part += prod;
            }
#pragma unroll
            for (int off = LANES / 2; off >= 1; off >>= 1) part += __shfl_xor(part, off, 64);
            const T m = part;
            const bool semi_nz = P.semi && s < P.sc.p;
            T y = w * loss_df<T>(P.loss, x, m);
            if (semi_nz) y -= w * loss_df<T>(P.loss, T(0), m);
            if (P.loss_out && cl == 0) {
                T l = w * loss_f<T>(P.loss, x, m);
                if (semi_nz) l -= w * loss_f<T>(P.loss, T(0), m);
                lacc += (double)l;
            }
            if (P.loss_only || !col_ok) continue;
            y *= scale;
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                // leave-one-out products by prefix and suffix running products
                T pre[DM];
                pre[0] = y;
#pragma unroll
                for (int k = 1; k < DM; ++k)
                    if (k < dd) pre[k] = pre[k - 1] * a[k - 1][v];
                T suf = T(1);
#pragma unroll
                for (int k = DM - 1; k >= 0; --k) {
                    if (k < dd) {
                        const T c = pre[k] * suf;
                        suf *= a[k][v];
                        if ((P.lds_mask >> k) & 1u) {
                            atomicAdd(priv + P.lds_off[k] + (row[k] - P.rowoff[k]) * R + col0 + v, c);
                        } else {
                            global_add(P.G + row[k] * R + col0 + v, c);
                        }
                    }
                }
            }
        }
        wave_sync();
    }

    if (P.loss_out) {
        for (int off = 32; off >= 1; off >>= 1) lacc += __shfl_xor(lacc, off, 64);
        if (lane == 0 && lacc != 0.0) atomicAdd(P.loss_out, lacc);
    }
    if (P.lds_mask) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < DM; ++k) {
            if (k < dd && ((P.lds_mask >> k) & 1u)) {
                const int64_t rows = P.sc.L.dims[k];
                T* dst = P.G + P.rowoff[k] * R;
                const T* src = priv + P.lds_off[k];
                for (int64_t e = threadIdx.x; e < rows * R; e += blockDim.x) {
                    const T v = src[e];
                    if (v != T(0)) global_add(dst + e, v);
                }
            }
        }
    }
}

template <typename T>
__global__ void k_zero(T* __restrict__ p, int64_t n, double* __restrict__ loss_out)
{
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i0 == 0 && loss_out) *loss_out = 0.0;
    for (int64_t i = i0; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = T(0);
}

template <typename T>
using LGKernel = void (*)(const LGParams<T>);

// (lanes, vec) shapes built for each dtype
#define GCP_LG_SHAPES_F32(X) X(8, 1) X(16, 1) X(32, 1) X(64, 1) X(2, 4) X(4, 4) X(8, 4) X(16, 4) X(32, 4) X(64, 4) X(4, 2) X(8, 2) X(16, 2)
#define GCP_LG_SHAPES_F64(X) X(8, 1) X(16, 1) X(32, 1) X(64, 1) X(4, 2) X(8, 2) X(16, 2) X(32, 2)

template <typename T, int D, int SRC>
static LGKernel<T> pick_shape(int lanes, int vec)
{
#define GCP_CASE(LN, VC) \
    if (lanes == LN && vec == VC) return k_loss_grad<T, D, LN, VC, SRC>;
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
    if (src == 0) {
        if (d == 3) return pick_shape<T, 3, 0>(lanes, vec);
        if (d == 4) return pick_shape<T, 4, 0>(lanes, vec);
        return pick_shape<T, 0, 0>(lanes, vec);
    }
    if (d == 3) return pick_shape<T, 3, 1>(lanes, vec);
    if (d == 4) return pick_shape<T, 4, 1>(lanes, vec);
    return pick_shape<T, 0, 1>(lanes, vec);
}

// Default lane shape: the widest vector that divides R, then the fewest
// lanes (power of two) that cover R.
template <typename T>
static void default_shape(int R, int& lanes, int& vec)
{
    const int vmax = sizeof(T) == 4 ? 4 : 2;
    vec = 1;
    for (int v = vmax; v >= 2; v >>= 1)
        if (R % v == 0 && R / v >= 2) { vec = v; break; }
    const int need = (R + vec - 1) / vec;
    lanes = 8;
    while (lanes < need && lanes < 64) lanes <<= 1;
    if (sizeof(T) == 4 && vec == 4 && need <= 4) lanes = need <= 2 ? 2 : 4;
    if (vec == 2 && need <= 4) lanes = 4;
}

constexpr int kLdsPrivateBudget = 96 * 1024;   // bytes of private gradient per workgroup

template <typename T>
static gcp_status launch_loss_grad(const gcp_tensor_s* t, const gcp_sample_params* sp, const gcp_samples* smp,
                                   const void* A, int R, gcp_loss loss, unsigned flags, const void* scale_dev,
                                   void* G_out, double* loss_out, const gcp_tile* tile, hipStream_t stream)
{
    LGParams<T> P{};
    int64_t n = 0;
    gcp_status st = make_sample_ctx<T>(t, sp, P.sc, n);
    if (st != GCP_OK) return st;
    const bool loss_only = (flags & GCP_LOSS_ONLY) != 0;
    const bool accumulate = (flags & GCP_ACCUMULATE) != 0;
    if (flags & ~(GCP_LOSS_ONLY | GCP_ACCUMULATE | GCP_SCALE_BY_DEV))
        return set_error(GCP_ERR_ARG, "unknown flags 0x%x", flags);
    if (!A) return set_error(GCP_ERR_ARG, "A is NULL");
    if (R < 1 || R > 256) return set_error(GCP_ERR_ARG, "R = %d outside [1, 256]", R);
    if (loss < GCP_LOSS_GAUSSIAN || loss > GCP_LOSS_BERNOULLI_LOGIT) return set_error(GCP_ERR_ARG, "loss %d", (int)loss);
    if (!loss_only && !G_out) return set_error(GCP_ERR_ARG, "G_out is NULL");
    if ((flags & GCP_SCALE_BY_DEV) && !scale_dev) return set_error(GCP_ERR_ARG, "scale_dev is NULL");
    if (loss_only && !loss_out) return set_error(GCP_ERR_ARG, "GCP_LOSS_ONLY without loss_out");
    if (smp && (!smp->coords || !smp->x || !smp->w) && n > 0)
        return set_error(GCP_ERR_ARG, "materialised sample list has a NULL array");

    int lanes = 0, vec = 0;
    default_shape<T>(R, lanes, vec);
    if (tile && tile->vec > 0) vec = tile->vec;
    if (tile && tile->lanes > 0) lanes = tile->lanes;
    else if (tile && tile->vec > 0) {
        const int need = (R + vec - 1) / vec;
        lanes = 2;
        while (lanes < need && lanes < 64) lanes <<= 1;
    }
    if (R % vec != 0) return set_error(GCP_ERR_ARG, "vec = %d does not divide R = %d", vec, R);
    if (lanes * vec < R) return set_error(GCP_ERR_ARG, "lanes*vec = %d < R = %d", lanes * vec, R);
    const int src = smp ? 1 : 0;
    LGKernel<T> kern = pick_kernel<T>(t->d, src, lanes, vec);
    if (!kern) return set_error(GCP_ERR_UNSUPPORTED, "tile lanes = %d, vec = %d not built for this dtype", lanes, vec);
    const uintptr_t align = (uintptr_t)vec * sizeof(T);
    if (((uintptr_t)A % align) != 0) return set_error(GCP_ERR_ARG, "A is not %d-byte aligned", (int)align);

    // LDS privatisation of small modes
    int block = 256;
    int64_t nchunks = ceil_div(n, 64);
    uint32_t mask = 0;
    int64_t lds_elems = 0;
    const int req_mask = tile ? tile->lds_modes : -1;
    if (!loss_only) {
        for (int k = 0; k < t->d; ++k) {
            const int64_t elems = t->dims[k] * (int64_t)R;
            const bool fits = (lds_elems + elems) * (int64_t)sizeof(T) <= kLdsPrivateBudget;
            bool want;
            if (req_mask >= 0) want = (req_mask >> k) & 1;
            else want = fits && elems * 4 * (int64_t)device_cu_count(t->device) <= n * R;  // flush << scatter
            if (want) {
                if (!fits) return set_error(GCP_ERR_ARG, "LDS-private modes exceed %d bytes", kLdsPrivateBudget);
                P.lds_off[k] = lds_elems;
                lds_elems += elems;
                mask |= 1u << k;
            }
        }
    }
    if (mask) block = 1024;
    if (tile && tile->block > 0) {
        if (tile->block % 64 != 0 || tile->block > 1024) return set_error(GCP_ERR_ARG, "block = %d", tile->block);
        block = tile->block;
    }
    const int nwaves = block / 64;
    const int staging = nwaves * 64 * (8 + 2 * (int)sizeof(T));
    const size_t lds_bytes = (size_t)staging + (size_t)lds_elems * sizeof(T);
    int64_t grid;
    {
        int per_cu = 0;
        GCP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern), block,
                                                            lds_bytes));
        if (per_cu < 1) return set_error(GCP_ERR_UNSUPPORTED, "kernel does not fit on a CU (LDS %zu B)", lds_bytes);
        const int64_t resident = (int64_t)per_cu * device_cu_count(t->device);
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
    for (int k = 0; k < kMaxModes; ++k) P.rowoff[k] = k < t->d ? t->rowoff[k] : t->rowoff[t->d];
    P.lds_mask = mask;
    P.lds_elems = lds_elems;
    P.staging_bytes = staging;

    if (!accumulate) {
        const int64_t gn = loss_only ? 0 : t->rowoff[t->d] * R;
        if (gn > 0 || loss_out) {
            int64_t zb = std::max<int64_t>(1, std::min<int64_t>(ceil_div(gn, 256), 4096));
            k_zero<T><<<(unsigned)zb, 256, 0, stream>>>((T*)G_out, gn, loss_out);
            GCP_HIP(hipGetLastError());
        }
    }
    if (n == 0) return GCP_OK;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(block), lds_bytes, stream, P);
    GCP_HIP(hipGetLastError());
    return GCP_OK;
}

}  // namespace gcp

extern "C" gcp_status gcp_loss_grad(gcp_tensor t, const gcp_sample_params* sp, const gcp_samples* smp,
                                    const void* A, int R, gcp_loss loss, unsigned flags, const void* scale_dev,
                                    void* G_out, double* loss_out, const gcp_tile* tile, hipStream_t stream)
{
    gcp::clear_error();
    if (!t) return gcp::set_error(GCP_ERR_ARG, "tensor is NULL");
    if (t->dt == GCP_F32)
        return gcp::launch_loss_grad<float>(t, sp, smp, A, R, loss, flags, scale_dev, G_out, loss_out, tile, stream);
    return gcp::launch_loss_grad<double>(t, sp, smp, A, R, loss, flags, scale_dev, G_out, loss_out, tile, stream);
}
