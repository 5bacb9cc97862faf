// Device core of the fused sampled loss/gradient: kernel parameters, small
// helpers and the per-chunk body shared by the HIP kernels.
#pragma once

#include <algorithm>

#include "sampling.hpp"

namespace gcp {

template <typename T>
struct LGParams {
    SampleCtx<T> sc;
    int64_t n;            // samples p + q
    int64_t nchunks;      // ceil(n / 64)
    const int64_t* m_coords;  // materialised list (SRC = 1, 3)
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
    // bucketed scatter
    uint32_t bucket_mask;      // modes scattered through row-block buckets
    int n_bucket_modes;
    int br_shift;              // rows per bucket = 1 << br_shift
    int nb;                    // buckets over all bucketed modes
    int bucket_base[kMaxModes + 1];
    int spb;                   // samples per workgroup (tiled launch)
    int64_t nblocks;           // workgroups of the tiled launch (J)
    int64_t entry_cap;         // entries per workgroup segment list = spb * n_bucket_modes
    int bucket_lds;            // byte offset of the bucket staging in LDS
    uint4* entries;            // [J][entry_cap] 16-byte {key, y}
    int* hist;                 // [nb][J] entries per (bucket, workgroup)
    int* start;                // [nb][J] first entry of the bucket in the workgroup's list
    // owner pass: mode k's row blocks use workgroups [bwg_base[k], bwg_base[k+1]),
    // bsplits[k] per row block, each reading bsegs[k] consecutive segments
    int64_t bwg_base[kMaxModes + 1];
    int bsplits[kMaxModes];
    int bsegs[kMaxModes];
    // non-fused sampling step (SRC = 2): each sample's y, the sampled
    // tensor's values, and its coordinates [n x d], written instead of
    // scattering (last, so that the fields above keep their kernel-argument
    // offsets)
    T* y_out;
    int64_t* c_out;
    // deterministic objective: each wave's partial sum goes to its own slot
    // (workgroup * waves + wave) instead of an atomic add into loss_out
    double* loss_parts;
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

// Float add into LDS as a compare-and-swap loop on the bit pattern.  The
// native LDS float atomic (ds_add_f32) retires about one lane per three
// clocks on gfx950, while this loop costs a few LDS integer operations per
// wave instruction when the lanes hit distinct words (one gradient row per
// lane group).  Lanes that collide are serialised by the hardware, so every
// pass of the loop completes at least one of them.
__device__ __forceinline__ void lds_add(float* p, float v)
{
    unsigned* u = reinterpret_cast<unsigned*>(p);
    unsigned old = __hip_atomic_load(u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    for (;;) {
        const unsigned nv = __float_as_uint(__uint_as_float(old) + v);
        if (__hip_atomic_compare_exchange_strong(u, &old, nv, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_WORKGROUP))
            break;
    }
}

// Two adjacent floats (8-byte aligned) added by one 64-bit compare-and-swap
// loop: half the serial LDS round trips of two single adds.
__device__ __forceinline__ void lds_add2(float* p, float a, float b)
{
    unsigned long long* u = reinterpret_cast<unsigned long long*>(p);
    unsigned long long old = __hip_atomic_load(u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    for (;;) {
        const float lo = __uint_as_float((unsigned)old) + a;
        const float hi = __uint_as_float((unsigned)(old >> 32)) + b;
        const unsigned long long nv = (unsigned long long)__float_as_uint(lo) |
                                      ((unsigned long long)__float_as_uint(hi) << 32);
        if (__hip_atomic_compare_exchange_strong(u, &old, nv, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_WORKGROUP))
            break;
    }
}

__device__ __forceinline__ void lds_add(double* p, double v)
{
    unsigned long long* u = reinterpret_cast<unsigned long long*>(p);
    unsigned long long old = __hip_atomic_load(u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    for (;;) {
        const unsigned long long nv =
            (unsigned long long)__double_as_longlong(__longlong_as_double((long long)old) + v);
        if (__hip_atomic_compare_exchange_strong(u, &old, nv, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_WORKGROUP))
            break;
    }
}

// Adds VEC consecutive columns to LDS; float column pairs (8-byte aligned:
// row strides and column offsets are multiples of VEC) go through one 64-bit
// compare-and-swap each.
template <typename T, int VEC>
__device__ __forceinline__ void lds_add_cols(T* dst, const T (&c)[VEC])
{
    static_assert(VEC == 1 || VEC == 2 || VEC == 4, "columns per lane");
    if constexpr (sizeof(T) == 4 && VEC >= 2) {
        lds_add2(dst, c[0], c[1]);
        if constexpr (VEC == 4) lds_add2(dst + 2, c[2], c[3]);
    } else {
        lds_add(dst, c[0]);
        if constexpr (VEC >= 2) lds_add(dst + 1, c[1]);
        if constexpr (VEC == 4) {
            lds_add(dst + 2, c[2]);
            lds_add(dst + 3, c[3]);
        }
    }
}

// Element offset of column 0 of model row `row` (row < 2^32, checked when the
// tensor is created): one 32 x 32 -> 64-bit multiply.
__device__ __forceinline__ uint64_t row_elem(uint64_t row, int R)
{
    return (uint64_t)(uint32_t)row * (uint32_t)R;
}

template <typename T>
__device__ __forceinline__ uint4 pack_entry(uint64_t key, T y)
{
    uint4 e;
    e.x = (uint32_t)key;
    e.y = (uint32_t)(key >> 32);
    if constexpr (sizeof(T) == 4) {
        e.z = __float_as_uint(y);
        e.w = 0;
    } else {
        const uint64_t b = (uint64_t)__double_as_longlong(y);
        e.z = (uint32_t)b;
        e.w = (uint32_t)(b >> 32);
    }
    return e;
}

template <typename T>
__device__ __forceinline__ T entry_y(uint4 e)
{
    if constexpr (sizeof(T) == 4) return __uint_as_float(e.z);
    else return __longlong_as_double((long long)(((uint64_t)e.w << 32) | e.z));
}

// Butterfly exchange across lanes (lane ^ mask).  Doubles move as two 32-bit
// halves: the 64-bit form of the cross-half exchange trips a gfx950 code
// generation error in this toolchain.
__device__ __forceinline__ float xor_shfl(float v, int mask) { return __shfl_xor(v, mask, 64); }
__device__ __forceinline__ double xor_shfl(double v, int mask)
{
    const long long b = __double_as_longlong(v);
    const int lo = __shfl_xor((int)(b & 0xffffffffll), mask, 64);
    const int hi = __shfl_xor((int)(b >> 32), mask, 64);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Exclusive prefix sum of cnt[0, n) into off[0, n) by one wavefront.
__device__ inline void wave_exclusive_scan(const int* cnt, int* off, int n, int lane)
{
    const int per = (n + 63) / 64;
    const int b0 = lane * per;
    int local = 0;
    for (int i = 0; i < per; ++i)
        if (b0 + i < n) local += cnt[b0 + i];
    int incl = local;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int o = __shfl_up(incl, d, 64);
        if (lane >= d) incl += o;
    }
    int run = incl - local;
    for (int i = 0; i < per; ++i) {
        if (b0 + i < n) {
            off[b0 + i] = run;
            run += cnt[b0 + i];
        }
    }
}

// Samples per lane group whose factor-row gathers are issued together.  It
// must divide LANES: a pass covers samples it*S+g .. (it+U-1)*S+g of the
// wave's 64 staged samples, so a U that does not divide LANES would read past
// the staging slice on the last pass.
#ifndef GCP_UNROLL_WIDE
#define GCP_UNROLL_WIDE 2
#endif
template <typename T, int D, int LANES, int VEC>
constexpr int samples_in_flight()
{
    constexpr int U = (D == 0 || LANES < 4) ? 1 : sizeof(T) == 8 ? 2 : VEC == 4 ? GCP_UNROLL_WIDE : 4;
    static_assert(U >= 1 && LANES % U == 0, "samples in flight must divide the lanes per sample");
    return U;
}

// Entries in flight per lane group in the owner pass of the bucketed scatter
// (float, four columns per lane: GCP_OWNER_UNROLL_WIDE).
#ifndef GCP_OWNER_UNROLL_WIDE
#define GCP_OWNER_UNROLL_WIDE GCP_UNROLL_WIDE
#endif
template <typename T, int D, int LANES, int VEC>
constexpr int owner_in_flight()
{
    constexpr int U = (D == 0 || LANES < 4) ? 1 : sizeof(T) == 8 ? 2 : VEC == 4 ? GCP_OWNER_UNROLL_WIDE : 4;
    static_assert(U >= 1 && LANES % U == 0, "entries in flight must divide the lanes per entry");
    return U;
}

// One chunk of 64 samples: phase 1 (one lane per sample: draw or read the
// sample, stage it in the wave's LDS slice) and phase 2 (LANES lanes per
// sample: gather rows, model value, loss derivative, scatter).  Shared by the
// sampled-gradient kernel and the batched GCP-FedAdam kernel.
//   SRC = 0  draw the samples (the fused sampled gradient);
//   SRC = 1  read a materialised sample list (coordinates, x, w);
//   SRC = 2  draw the samples and write the sampled tensor (coordinates and
//            y = w f'(x, m)) instead of scattering: the sampling step of the
//            non-fused gradient;
//   SRC = 3  read a sampled tensor whose values are already y (w = 1 unless a
//            weight list is given): the MTTKRP step of the non-fused gradient.
template <typename T, int D, int LANES, int VEC, int SRC>
__device__ __forceinline__ void lg_chunk(const LGParams<T>& P, int64_t chunk, int lane, uint64_t* skey, T* sx,
                                         T* sw, T* priv, uint64_t* bkey, T* by, int64_t block_s0, bool tiled,
                                         T scale, double& lacc, uint64_t step)
{
    constexpr int S = 64 / LANES;                  // samples per pass
    constexpr int U = samples_in_flight<T, D, LANES, VEC>();
    constexpr int DM = D > 0 ? D : kMaxModes;
    const int dd = D > 0 ? D : P.sc.d;
    const int R = P.R;
    const int g = lane / LANES, cl = lane % LANES;
    const int col0 = cl * VEC;
    const bool col_ok = col0 < R;          // VEC divides R
    const int64_t s0 = chunk * 64;
    {   // phase 1: one lane per sample
        const int64_t s = s0 + lane;
        uint64_t key = 0;
        T x = T(0), w = T(0);
        if (s < P.n) {
            if constexpr (SRC == 0 || SRC == 2) {
                draw_sample<T, D>(P.sc, step, s, key, x, w);
            } else {
                bool ok = true;
#pragma unroll
                for (int k = 0; k < DM; ++k) {
                    if (k < dd) {
                        int64_t c = P.m_coords[s * dd + k];
                        if (c < 0 || c >= P.sc.L.dims[k]) ok = false;
                        else key += pack_coord<D == 0>(P.sc.L, (uint64_t)c, k);
                    }
                }
                x = P.m_x[s];
                w = P.m_w ? P.m_w[s] : T(1);
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
    // phase 2: LANES lanes per sample, U samples per lane group in flight
    for (int it = 0; it < LANES; it += U) {
        uint64_t key[U];
        T a[U][DM][VEC];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int slot = (it + u) * S + g;
            const bool valid = s0 + slot < P.n;
            key[u] = skey[slot];
            uint32_t ci[DM];
            unpack_all<D == 0>(P.sc.L, dd, key[u], ci);
#pragma unroll
            for (int k = 0; k < DM; ++k) {
                if (k < dd) {
                    const uint64_t row = (uint64_t)P.rowoff[k] + ci[k];
                    if (col_ok && valid) {
                        load_cols<T, VEC>(P.A + row_elem(row, R) + col0, a[u][k]);
                    } else {
#pragma unroll
                        for (int v = 0; v < VEC; ++v) a[u][k][v] = T(0);
                    }
                }
            }
        }
        T m[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            T part = T(0);
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                T prod = a[u][0][v];
#pragma unroll
                for (int k = 1; k < DM; ++k)
                    if (k < dd) prod *= a[u][k][v];
                part += prod;
            }
            m[u] = part;
        }
#pragma unroll
        for (int off = LANES / 2; off >= 1; off >>= 1) {
#pragma unroll
            for (int u = 0; u < U; ++u) m[u] += xor_shfl(m[u], off);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int slot = (it + u) * S + g;
            const int64_t s = s0 + slot;
            if (s >= P.n) continue;
            const T x = sx[slot], w = sw[slot];
            T y;
            if constexpr (SRC == 3) {
                y = w * x;
            } else {
                const bool semi_nz = P.semi && s < P.sc.p;
                y = w * loss_df<T>(P.loss, x, m[u]);
                if (semi_nz) y -= w * loss_df<T>(P.loss, T(0), m[u]);
                if (P.loss_out && cl == 0) {
                    T l = w * loss_f<T>(P.loss, x, m[u]);
                    if (semi_nz) l -= w * loss_f<T>(P.loss, T(0), m[u]);
                    lacc += (double)l;
                }
            }
            if constexpr (SRC == 2) {
                // the sampled tensor Y~ goes to memory; nothing is scattered
                if (cl == 0) {
                    uint32_t ci[DM];
                    unpack_all<D == 0>(P.sc.L, dd, key[u], ci);
#pragma unroll
                    for (int k = 0; k < DM; ++k)
                        if (k < dd) P.c_out[s * dd + k] = (int64_t)ci[k];
                    P.y_out[s] = y;
                }
                continue;
            }
            if (P.loss_only) continue;
            y *= scale;
            if (tiled && cl == 0) {
                bkey[s - block_s0] = key[u];
                by[s - block_s0] = y;
            }
            // all modes bucketed: the owner pass forms the products
            if (!col_ok || P.bucket_mask == (1u << dd) - 1) continue;
            // coordinates again from the key (a few shifts when bit-packed),
            // rather than holding them live across the gathers
            uint32_t ci[DM];
            unpack_all<D == 0>(P.sc.L, dd, key[u], ci);
            if constexpr (sizeof(T) == 4 && VEC >= 2) {
                // leave-one-out products y prod_{n != k} A_n[i_n, :] by prefix
                // and suffix running products, then per mode not bucketed:
                // added to the LDS-private copy (column pairs) or to G by
                // global atomics
                T cv[DM][VEC];
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    T pre[DM];
                    pre[0] = y;
#pragma unroll
                    for (int k = 1; k < DM; ++k)
                        if (k < dd) pre[k] = pre[k - 1] * a[u][k - 1][v];
                    T suf = T(1);
#pragma unroll
                    for (int k = DM - 1; k >= 0; --k) {
                        if (k < dd) {
                            cv[k][v] = pre[k] * suf;
                            suf *= a[u][k][v];
                        }
                    }
                }
#pragma unroll
                for (int k = DM - 1; k >= 0; --k) {
                    if (k < dd && !((P.bucket_mask >> k) & 1u)) {
                        const uint32_t i = ci[k];
                        if ((P.lds_mask >> k) & 1u) {
                            lds_add_cols<T, VEC>(priv + P.lds_off[k] + i * (uint32_t)R + col0, cv[k]);
                        } else {
#pragma unroll
                            for (int v = 0; v < VEC; ++v)
                                global_add(P.G + row_elem((uint64_t)P.rowoff[k] + i, R) + col0 + v, cv[k][v]);
                        }
                    }
                }
            } else {
                // no column pairs: each product goes out as soon as it is formed
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    T pre[DM];
                    pre[0] = y;
#pragma unroll
                    for (int k = 1; k < DM; ++k)
                        if (k < dd) pre[k] = pre[k - 1] * a[u][k - 1][v];
                    T suf = T(1);
#pragma unroll
                    for (int k = DM - 1; k >= 0; --k) {
                        if (k < dd) {
                            const T c = pre[k] * suf;
                            suf *= a[u][k][v];
                            if ((P.bucket_mask >> k) & 1u) continue;
                            const uint32_t i = ci[k];
                            if ((P.lds_mask >> k) & 1u) {
                                lds_add(priv + P.lds_off[k] + i * (uint32_t)R + col0 + v, c);
                            } else {
                                global_add(P.G + row_elem((uint64_t)P.rowoff[k] + i, R) + col0 + v, c);
                            }
                        }
                    }
                }
            }
        }
    }
    wave_sync();
}

// Bucketed scatter, sampling side: sorts the (key, y) of the workgroup's
// nvalid staged samples (bkey, by in LDS) by (mode, row block) into segment
// list `seg` of the bucket workspace -- count, scan, place -- and records the
// list's per-bucket counts and starts.  Every thread of the workgroup calls it.
template <typename T, int D>
__device__ __forceinline__ void bucket_write_out(const LGParams<T>& P, int64_t seg, int nvalid, const uint64_t* bkey,
                                                 const T* by, int* bcnt, int* boff)
{
    constexpr int DM = D > 0 ? D : kMaxModes;
    const int dd = D > 0 ? D : P.sc.d;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    for (int b = threadIdx.x; b < P.nb; b += blockDim.x) bcnt[b] = 0;
    __syncthreads();
    for (int e = threadIdx.x; e < nvalid; e += blockDim.x) {
        uint32_t ci[DM];
        unpack_all<D == 0>(P.sc.L, dd, bkey[e], ci);
#pragma unroll
        for (int k = 0; k < DM; ++k)
            if (k < dd && ((P.bucket_mask >> k) & 1u)) atomicAdd(bcnt + P.bucket_base[k] + (int)(ci[k] >> P.br_shift), 1);
    }
    __syncthreads();
    if (wave == 0) wave_exclusive_scan(bcnt, boff, P.nb, lane);
    __syncthreads();
    for (int b = threadIdx.x; b < P.nb; b += blockDim.x) {
        P.hist[(int64_t)b * P.nblocks + seg] = bcnt[b];
        P.start[(int64_t)b * P.nblocks + seg] = boff[b];
    }
    __syncthreads();
    uint4* out = P.entries + seg * P.entry_cap;
    for (int e = threadIdx.x; e < nvalid; e += blockDim.x) {
        const uint64_t key = bkey[e];
        const uint4 ent = pack_entry<T>(key, by[e]);
        uint32_t ci[DM];
        unpack_all<D == 0>(P.sc.L, dd, key, ci);
#pragma unroll
        for (int k = 0; k < DM; ++k) {
            if (k < dd && ((P.bucket_mask >> k) & 1u)) {
                const int pos = atomicAdd(boff + P.bucket_base[k] + (int)(ci[k] >> P.br_shift), 1);
                out[pos] = ent;
            }
        }
    }
    __syncthreads();
}

// Bucketed scatter, owner side: accumulates into `part` (LDS, rows x R) the
// contributions y prod_{n != k} A_n[i_n, :] of every entry of bucket b (rows
// [r0, r0 + rows) of mode k) in segment lists [j0, j1).  Each wave takes whole
// segments in turn, loading the next pass's entries while it gathers the
// other modes' rows; adds go through LDS compare-and-swap.  seg_cnt is LDS
// scratch for 2 (j1 - j0) ints.  Every thread of the workgroup calls it; part
// is complete when it returns.
template <typename T, int D, int LANES, int VEC>
__device__ __forceinline__ void bucket_accumulate(const LGParams<T>& P, int k, int b, int64_t r0, int64_t rows,
                                                  int64_t j0, int64_t j1, T* part, int* seg_cnt)
{
    constexpr int S = 64 / LANES;
    constexpr int U = owner_in_flight<T, D, LANES, VEC>();
    constexpr int DM = D > 0 ? D : kMaxModes;
    static_assert(VEC == 1 || VEC == 2 || VEC == 4, "columns per lane");
    const int nwaves = blockDim.x >> 6;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane / LANES, cl = lane % LANES;
    const int col0 = cl * VEC;
    const int R = P.R;
    const bool col_ok = col0 < R;
    const int dd = D > 0 ? D : P.sc.d;
    // mode k's key field, selected with compile-time indices: a run-time
    // index into the parameter block would force a register copy of it
    // (the persistent FedAdam kernel holds one) out to scratch memory
    int shift_k = 0;
    uint64_t mask_k = 0;
#pragma unroll
    for (int kk = 0; kk < DM; ++kk)
        if (kk == k) {
            shift_k = P.sc.L.shift[kk];
            mask_k = P.sc.L.mask[kk];
        }
    int* seg_start = seg_cnt + (j1 - j0);
    for (int64_t e = threadIdx.x; e < rows * R; e += blockDim.x) part[e] = T(0);
    for (int64_t j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
        seg_cnt[j - j0] = P.hist[(int64_t)b * P.nblocks + j];
        seg_start[j - j0] = P.start[(int64_t)b * P.nblocks + j];
    }
    __syncthreads();

    if constexpr (D > 0) {
        // Bit-packed keys: every load below is unconditional.  The D - 1 modes
        // other than k are enumerated at compile time (shift, mask, row offset
        // picked with compile-time indices), lanes past column R read column 0
        // and lanes past the segment's end re-read its last entry, so each load
        // has an in-bounds address and no branch around it.  Loads under a
        // branch make the compiler wait for all outstanding loads before each
        // one, which serialises the gathers of a pass.
        static_assert(D >= 2, "orders with their own kernels");
        constexpr int DO = D - 1;
        int sh_o[DO];
        uint32_t mk_o[DO], ro_o[DO];
#pragma unroll
        for (int o = 0; o < DO; ++o) {
            const int m = o + (o >= k ? 1 : 0);
            sh_o[o] = 0;
            mk_o[o] = 0;
            ro_o[o] = 0;
#pragma unroll
            for (int kk = 0; kk < D; ++kk)
                if (kk == m) {
                    sh_o[o] = P.sc.L.shift[kk];
                    mk_o[o] = (uint32_t)P.sc.L.mask[kk];
                    ro_o[o] = (uint32_t)P.rowoff[kk];
                }
        }
        const int colL = col_ok ? col0 : 0;
        for (int64_t j = j0 + wave; j < j1; j += nwaves) {
            const int cnt = seg_cnt[j - j0];
            if (cnt == 0) continue;
            const uint4* seg = P.entries + j * P.entry_cap + seg_start[j - j0];
            uint4 nxt[U];
#pragma unroll
            for (int u = 0; u < U; ++u) nxt[u] = seg[min(u * S + g, cnt - 1)];
            for (int base = 0; base < cnt; base += S * U) {
                uint64_t key[U];
                T y[U];
                T a[U][DO][VEC];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    key[u] = (uint64_t)nxt[u].x | ((uint64_t)nxt[u].y << 32);
                    y[u] = entry_y<T>(nxt[u]);
#pragma unroll
                    for (int o = 0; o < DO; ++o) {
                        const uint32_t row = ro_o[o] + ((uint32_t)(key[u] >> sh_o[o]) & mk_o[o]);
                        load_cols<T, VEC>(P.A + row_elem(row, R) + colL, a[u][o]);
                    }
                }
                // the next pass's entries stay in flight through this pass's
                // scatter
#pragma unroll
                for (int u = 0; u < U; ++u) nxt[u] = seg[min(base + S * U + u * S + g, cnt - 1)];
                // keeps the gathers here: sunk into the scatter branch below
                // they would issue after the prefetch, and waiting for them
                // would wait for the prefetch as well
                __asm__ volatile("" ::: "memory");
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (base + u * S + g >= cnt || !col_ok) continue;
                    const uint32_t i = (uint32_t)((key[u] >> shift_k) & mask_k) - (uint32_t)r0;
                    T c[VEC];
#pragma unroll
                    for (int v = 0; v < VEC; ++v) {
                        c[v] = y[u];
#pragma unroll
                        for (int o = 0; o < DO; ++o) c[v] *= a[u][o][v];
                    }
                    lds_add_cols<T, VEC>(part + i * (uint32_t)R + col0, c);
                }
            }
        }
        __syncthreads();
        return;
    }
    // General order (run-time d, either key form), with the loads as
    // unconditional as above: the d - 1 modes other than k fill slots
    // 0 .. d - 2 in mode order (slot o holds mode o, or o + 1 from k on, both
    // compile-time indices), slots past d - 2 re-read column block 0 of the
    // first model row and count as ones, lanes past column R read column 0,
    // and lanes past the segment's end re-read its last entry.
    constexpr int SO = DM - 1;
    const int colL = col_ok ? col0 : 0;
    for (int64_t j = j0 + wave; j < j1; j += nwaves) {
        const int cnt = seg_cnt[j - j0];
        if (cnt == 0) continue;
        const uint4* seg = P.entries + j * P.entry_cap + seg_start[j - j0];
        // entries of the next pass are loaded while this pass gathers rows
        uint4 nxt[U];
#pragma unroll
        for (int u = 0; u < U; ++u) nxt[u] = seg[min(u * S + g, cnt - 1)];
        for (int base = 0; base < cnt; base += S * U) {
            uint32_t ik[U];
            T y[U];
            T a[U][SO][VEC];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint4 ent = nxt[u];
                const uint64_t key = (uint64_t)ent.x | ((uint64_t)ent.y << 32);
                uint32_t ci[DM];
                unpack_all<true>(P.sc.L, dd, key, ci);
                // the owned mode's row, picked with compile-time indices
                ik[u] = ci[0];
#pragma unroll
                for (int kk = 1; kk < DM; ++kk)
                    if (kk == k) ik[u] = ci[kk];
                y[u] = entry_y<T>(ent);
#pragma unroll
                for (int o = 0; o < SO; ++o) {
                    const bool after = o >= k;
                    const uint64_t row = after ? (uint64_t)P.rowoff[o + 1] + ci[o + 1] : (uint64_t)P.rowoff[o] + ci[o];
                    const T* src = P.A + (o < dd - 1 ? row_elem(row, R) : 0) + colL;
                    load_cols<T, VEC>(src, a[u][o]);
                }
            }
            // the next pass's entries stay in flight through this pass's
            // scatter
#pragma unroll
            for (int u = 0; u < U; ++u) nxt[u] = seg[min(base + S * U + u * S + g, cnt - 1)];
            __asm__ volatile("" ::: "memory");
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (base + u * S + g >= cnt || !col_ok) continue;
                const uint32_t i = ik[u] - (uint32_t)r0;
                T c[VEC];
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    c[v] = y[u];
#pragma unroll
                    for (int o = 0; o < SO; ++o)
                        if (o < dd - 1) c[v] *= a[u][o][v];
                }
                lds_add_cols<T, VEC>(part + i * (uint32_t)R + col0, c);
            }
        }
    }
    __syncthreads();
}

}  // namespace gcp
