// Kernel templates of the sampled loss/gradient (k_loss_grad, the row-block
// owner pass k_bucket_accum, k_zero) and the table of lane shapes they are
// built for.  Included by the translation units that instantiate them: the
// fused and materialised forms (loss_grad.hip) and the non-fused forms
// (nonfused.hip).
#pragma once

#include <cmath>

#include "lg_core.hpp"

namespace gcp {

template <typename T, int D, int LANES, int VEC, int SRC>
__global__ void __launch_bounds__(1024) k_loss_grad(const LGParams<T> P)
{
    constexpr int DM = D > 0 ? D : kMaxModes;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int nwaves = blockDim.x >> 6;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint64_t* skey = reinterpret_cast<uint64_t*>(smem) + wave * 64;
    T* sx = reinterpret_cast<T*>(smem + (size_t)nwaves * 64 * 8) + wave * 64;
    T* sw = reinterpret_cast<T*>(smem + (size_t)nwaves * 64 * (8 + sizeof(T))) + wave * 64;
    T* priv = reinterpret_cast<T*>(smem + P.staging_bytes);
    // bucketed scatter staging: the workgroup's samples in order
    uint64_t* bkey = reinterpret_cast<uint64_t*>(smem + P.bucket_lds);
    T* by = reinterpret_cast<T*>(smem + P.bucket_lds + (size_t)P.spb * 8);
    int* bcnt = reinterpret_cast<int*>(smem + P.bucket_lds + (size_t)P.spb * (8 + sizeof(T)));
    int* boff = bcnt + P.nb;

    if (P.lds_mask) {
        for (int64_t e = threadIdx.x; e < P.lds_elems; e += blockDim.x) priv[e] = T(0);
        __syncthreads();
    }
    const int dd = D > 0 ? D : P.sc.d;
    const int R = P.R;
    const T scale = P.scale ? *P.scale : T(1);
    const bool tiled = P.bucket_mask != 0;
    const int64_t block_s0 = tiled ? (int64_t)blockIdx.x * P.spb : 0;
    double lacc = 0.0;

    // tiled launches give workgroup j the chunks of samples [j*spb, (j+1)*spb)
    int64_t chunk, chunk_end, chunk_step;
    if (tiled) {
        chunk = block_s0 / 64 + wave;
        chunk_end = std::min<int64_t>(P.nchunks, (block_s0 + P.spb) / 64);
        chunk_step = nwaves;
    } else {
        chunk = (int64_t)blockIdx.x * nwaves + wave;
        chunk_end = P.nchunks;
        chunk_step = (int64_t)gridDim.x * nwaves;
    }

    for (; chunk < chunk_end; chunk += chunk_step) {
        lg_chunk<T, D, LANES, VEC, SRC>(P, chunk, lane, skey, sx, sw, priv, bkey, by, block_s0, tiled, scale,
                                        lacc, P.sc.step);
    }

    if (P.loss_out) {
        for (int off = 32; off >= 1; off >>= 1) lacc += xor_shfl(lacc, off);
        if (P.loss_parts) {
            if (lane == 0) P.loss_parts[(int64_t)blockIdx.x * nwaves + wave] = lacc;
        } else if (lane == 0 && lacc != 0.0) {
            atomicAdd(P.loss_out, lacc);
        }
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
    if (tiled && !P.loss_only)
        bucket_write_out<T, D>(P, blockIdx.x, (int)std::min<int64_t>(P.spb, P.n - block_s0), bkey, by, bcnt, boff);
}

// Row-block owner pass of the bucketed scatter.  Workgroup (b, split) owns
// rows [r0, r0 + 2^br_shift) of bucket b's mode k and reads the segments of
// workgroups [j0, j1) of the sampling launch: per entry it gathers the other
// modes' rows, forms y prod_{n != k} A_n[i_n, :] and adds it to the LDS copy
// of its rows; the block is flushed to G once.
template <typename T, int D, int LANES, int VEC>
__global__ void __launch_bounds__(1024) k_bucket_accum(const LGParams<T> P)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    T* part = reinterpret_cast<T*>(smem);
    const int R = P.R;
    const int dd = D > 0 ? D : P.sc.d;

    // the mode whose workgroup range holds this workgroup (ranges of modes
    // that are not bucketed are empty), then its row block and split
    int k = 0;
    for (int kk = 0; kk < dd; ++kk)
        if (P.bwg_base[kk] <= (int64_t)blockIdx.x && (int64_t)blockIdx.x < P.bwg_base[kk + 1]) k = kk;
    const int splits = P.bsplits[k];
    const int64_t local = (int64_t)blockIdx.x - P.bwg_base[k];
    const int b = P.bucket_base[k] + (int)(local / splits);
    const int split = (int)(local % splits);
    const int64_t r0 = (int64_t)(b - P.bucket_base[k]) << P.br_shift;
    const int64_t rows = std::min<int64_t>((int64_t)1 << P.br_shift, P.sc.L.dims[k] - r0);
    // whole segments per workgroup (the host makes it a multiple of the
    // waves per workgroup); the last split takes the remainder
    const int64_t j0 = (int64_t)split * P.bsegs[k];
    const int64_t j1 = std::min<int64_t>(P.nblocks, j0 + P.bsegs[k]);
    int* seg_cnt = reinterpret_cast<int*>(smem + (((size_t)rows * R * sizeof(T) + 15) & ~(size_t)15));
    bucket_accumulate<T, D, LANES, VEC>(P, k, b, r0, rows, j0, j1, part, seg_cnt);
    __syncthreads();
    T* dst = P.G + (P.rowoff[k] + r0) * R;
    for (int64_t e = threadIdx.x; e < rows * R; e += blockDim.x) {
        const T v = part[e];
        if (v != T(0)) global_add(dst + e, v);
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
template <typename T>
using BAKernel = void (*)(const LGParams<T>);

// (lanes, vec) shapes built for each dtype
#define GCP_LG_SHAPES_F32(X) \
    X(8, 1) X(16, 1) X(32, 1) X(64, 1) X(4, 2) X(8, 2) X(16, 2) X(32, 2) X(64, 2) X(2, 4) X(4, 4) X(8, 4) X(16, 4) X(32, 4) X(64, 4)
#define GCP_LG_SHAPES_F64(X) X(8, 1) X(16, 1) X(32, 1) X(64, 1) X(4, 2) X(8, 2) X(16, 2) X(32, 2) X(64, 2) X(64, 4)

template <typename T, int D, int SRC>
inline LGKernel<T> pick_shape(int lanes, int vec)
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

// Non-fused forms (Sec. 3.1.2), instantiated in nonfused.hip: SRC = 2 draws
// the samples and writes the sampled tensor, SRC = 3 reads a sampled tensor
// whose values are the derivative values.
template <typename T>
LGKernel<T> pick_kernel_nonfused(int d, int src, int lanes, int vec);

}  // namespace gcp
