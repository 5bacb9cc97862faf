// Internal declarations shared by the HIP translation units of libgcp.
//
// Device-side building blocks of the sampled stochastic gradient:
//   * Philox4x64-10 counter-based RNG and the exact [0, n) range map
//     (the paper leaves the RNG open; counters make samples reproducible);
//   * cell keys (bit-packed or mixed radix) and the open-addressing membership table
//     (the O(1) hash search for zero samples, Sec. 3.1.1);
//   * the three losses and their derivatives.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/gcp.h"

namespace gcp {

// ----------------------------------------------------------------- errors --

gcp_status set_error(gcp_status st, const char* fmt, ...);
gcp_status hip_error(hipError_t e, const char* what);
void clear_error();

#define GCP_HIP(call)                                        \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return ::gcp::hip_error(e_, #call); \
    } while (0)

// Bits of the device status word.
enum : uint32_t {
    kStatusSampling = 1u,   // a zero sample exhausted its rejection attempts
    kStatusData = 2u,       // repeated or out-of-range coordinate
};

constexpr int kMaxModes = 8;
constexpr uint64_t kEmptySlot = ~0ull;      // never a cell key (see KeyLayout)

// One 64-bit key per cell.  Bit-packed when the modes' bit widths sum to at
// most 63: mode k occupies bits [shift_k, shift_k + bits_k), the last mode the
// lowest bits.  Otherwise mixed radix: the row-major linear index
// sum_k i_k stride_k with stride_k = prod_{j > k} I_j, for any M < 2^64 - 1.
// Neither form ever equals all ones, the empty hash slot.  Every I_k < 2^32.
struct KeyLayout {
    int d;
    int radix;                    // 0 bit-packed, 1 mixed radix
    int shift[kMaxModes];
    uint64_t mask[kMaxModes];
    int64_t dims[kMaxModes];
    uint64_t stride[kMaxModes];   // mixed radix: prod_{j > k} I_j
    double inv[kMaxModes];        // mixed radix: 1 / I_k, rounded to nearest
};

struct gcp_tensor_impl;

}  // namespace gcp

struct gcp_tensor_s {
    int device = 0;
    int d = 0;
    int64_t dims[gcp::kMaxModes] = {};
    int64_t rowoff[gcp::kMaxModes + 1] = {};  // first model row of each mode
    int64_t nnz = 0;
    uint64_t cells = 0;       // prod_k I_k (< 2^64)
    gcp_dtype dt = GCP_F32;
    bool dense = false;
    gcp::KeyLayout layout{};
    void* rec = nullptr;               // sparse: nnz 16-byte records {key, value}
    uint64_t* table = nullptr;         // sparse: hash slots
    uint64_t table_mask = 0;           // slots - 1
    int table_log2 = 0;
    const void* dense_vals = nullptr;  // dense: borrowed values
    uint32_t* status = nullptr;        // device status word
    int64_t owned_bytes = 0;
    // workspace of the bucketed scatter (gcp_tensor_reserve)
    void* ws = nullptr;
    int64_t ws_entries = 0;            // 16-byte sample entries
    int64_t ws_hist = 0;               // ints in each of the count and start arrays
    int64_t ws_bytes = 0;
    int64_t ws_max_samples = 0;        // samples per call the workspace was sized for
};

namespace gcp {
// Order the kernels are specialised for: 3 and 4 have their own builds, every
// other order -- and every mixed-radix key layout -- runs the general one (0).
inline int kernel_order(const gcp_tensor_s* t)
{
    return (t->layout.radix || (t->d != 3 && t->d != 4)) ? 0 : t->d;
}
}  // namespace gcp

namespace gcp {

// --------------------------------------------------------------- records --

template <typename T>
struct alignas(16) Record {
    uint64_t key;
    T val;
};
static_assert(sizeof(Record<float>) == 16, "record size");
static_assert(sizeof(Record<double>) == 16, "record size");

// -------------------------------------------------------------- Philox RNG --
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 64x64->128 multiplies with the published multipliers, key bumped by the
// published Weyl constants between rounds.

struct U64x4 {
    uint64_t v[4];
};

__host__ __device__ __forceinline__ void mul_hilo64(uint64_t a, uint64_t b, uint64_t& hi, uint64_t& lo)
{
#if defined(__HIP_DEVICE_COMPILE__)
    lo = a * b;
    hi = __umul64hi(a, b);
#else
    unsigned __int128 p = (unsigned __int128)a * b;
    lo = (uint64_t)p;
    hi = (uint64_t)(p >> 64);
#endif
}

__host__ __device__ __forceinline__ U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                                         uint64_t k0, uint64_t k1)
{
    constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t hi0, lo0, hi1, lo1;
        mul_hilo64(M0, c0, hi0, lo0);
        mul_hilo64(M1, c2, hi1, lo1);
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += W0;
        k1 += W1;
    }
    return U64x4{{c0, c1, c2, c3}};
}

// floor(u * n / 2^64): exact, unbiased to within 2^-64 per value.
__host__ __device__ __forceinline__ uint64_t range_map(uint64_t u, uint64_t n)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __umul64hi(u, n);
#else
    return (uint64_t)(((unsigned __int128)u * n) >> 64);
#endif
}

enum : uint64_t { kStreamNonzero = 0, kStreamZero = 1, kStreamUniform = 2 };

// ------------------------------------------------------------- cell keys --

// q = n / dv with r = n % dv, for n < 2^64 and 1 <= dv < 2^32 (inv = 1 / dv
// rounded to nearest).  Each 32-bit digit of the quotient is estimated in
// double precision, whose error stays below one unit, and corrected once
// with exact integer arithmetic.
__host__ __device__ __forceinline__ uint64_t divmod_u64_u32(uint64_t n, uint32_t dv, double inv, uint32_t& r)
{
    const uint32_t hi = (uint32_t)(n >> 32), lo = (uint32_t)n;
    uint32_t qh = (uint32_t)((double)hi * inv);
    int64_t rh = (int64_t)hi - (int64_t)qh * (int64_t)dv;
    if (rh < 0) {
        --qh;
        rh += dv;
    } else if (rh >= (int64_t)dv) {
        ++qh;
        rh -= dv;
    }
    const uint64_t x = ((uint64_t)rh << 32) | lo;     // < dv * 2^32: the low digit fits 32 bits
    const double e = (double)x * inv;
    uint32_t ql = e >= 4294967295.0 ? 0xffffffffu : (uint32_t)e;
    int64_t rl = (int64_t)(x - (uint64_t)ql * dv);
    if (rl < 0) {
        --ql;
        rl += dv;
    } else if (rl >= (int64_t)dv) {
        ++ql;
        rl -= dv;
    }
    r = (uint32_t)rl;
    return ((uint64_t)qh << 32) | ql;
}

// Key term of coordinate c of mode k; a cell's key is the sum of its terms.
// Code built with RADIX = false handles bit-packed layouts only (see unpack_all).
template <bool RADIX = true>
__host__ __device__ __forceinline__ uint64_t pack_coord(const KeyLayout& L, uint64_t c, int k)
{
    return (RADIX && L.radix) ? c * L.stride[k] : c << L.shift[k];
}

// All coordinates of a key (modes 0 .. dd-1 of at most DM).  Only code built
// with RADIX = true reads mixed-radix keys: tensors whose layout is mixed
// radix run the general-order kernels, so the order-specialised ones carry no
// division code (and none of its registers).
template <bool RADIX, int DM>
__host__ __device__ __forceinline__ void unpack_all(const KeyLayout& L, int dd, uint64_t key, uint32_t (&c)[DM])
{
    if (!RADIX || !L.radix) {
#pragma unroll
        for (int k = 0; k < DM; ++k)
            c[k] = k < dd ? (uint32_t)((key >> L.shift[k]) & L.mask[k]) : 0u;
    } else {
#pragma unroll
        for (int k = DM - 1; k >= 1; --k) {
            c[k] = 0;
            if (k < dd) key = divmod_u64_u32(key, (uint32_t)L.dims[k], L.inv[k], c[k]);
        }
        c[0] = (uint32_t)key;
    }
}

// Candidate cell of sample s / attempt a drawn straight into a cell key.
template <int D>
__device__ __forceinline__ uint64_t draw_cell_key(const KeyLayout& L, int d, uint64_t seed, uint64_t client,
                                                  uint64_t s, uint64_t step, uint64_t stream, uint64_t attempt)
{
    const int dd = D > 0 ? D : d;
    uint64_t key = 0;
    U64x4 o = philox4x64_10(s, step, stream | (attempt << 8), 0, seed, client);
#pragma unroll
    for (int k = 0; k < (D > 0 ? (D < 4 ? D : 4) : 4); ++k)
        if (k < dd) key += pack_coord<D == 0>(L, range_map(o.v[k], (uint64_t)L.dims[k]), k);
    if (dd > 4) {
        U64x4 o2 = philox4x64_10(s, step, stream | (attempt << 8), 1, seed, client);
#pragma unroll
        for (int k = 4; k < kMaxModes; ++k)
            if (k < dd) key += pack_coord<D == 0>(L, range_map(o2.v[k - 4], (uint64_t)L.dims[k]), k);
    }
    return key;
}

// ------------------------------------------------------ membership table --
// Open addressing with linear probing over 2^b slots holding cell keys;
// the home slot is the top b bits of a 64-bit finalising mix of the key
// (the murmur3 fmix64 finaliser).

__host__ __device__ __forceinline__ uint64_t mix64(uint64_t k)
{
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return k;
}

typedef unsigned long long u64x2_vec __attribute__((ext_vector_type(2)));

// Linear-probing membership test.  Each probe is one 16-byte load of the
// aligned slot pair holding the current slot, scanned from that slot on, so a
// lookup whose home slot is even and occupied can still end on its first
// load.  The table is an allocation of its own with at least 2^10 slots, so a
// pair never runs past its end.
__device__ __forceinline__ bool table_contains(const uint64_t* __restrict__ table, uint64_t mask, int log2n,
                                               uint64_t key)
{
    uint64_t h = log2n > 0 ? (mix64(key) >> (64 - log2n)) : 0;
    for (;;) {
        const uint64_t pair = h & ~uint64_t(1);
        const u64x2_vec t = __builtin_nontemporal_load(reinterpret_cast<const u64x2_vec*>(table + pair));
        if ((h & 1) == 0) {
            if (t.x == key) return true;
            if (t.x == kEmptySlot) return false;
        }
        if (t.y == key) return true;
        if (t.y == kEmptySlot) return false;
        h = (pair + 2) & mask;
    }
}

// ------------------------------------------------------------------ losses --

// Internal loss code of the sampled MTTKRP over a given sampled tensor: its
// values are already the derivative values, so y = w x (the kernels take
// that branch at compile time).
constexpr int kLossGivenValues = 3;

template <typename T>
__device__ __forceinline__ T loss_df(int loss, T x, T m)
{
    if (loss == GCP_LOSS_GAUSSIAN) return m - x;
    if (loss == GCP_LOSS_POISSON) return T(1) - x / (m + T(1e-10));
    // Bernoulli-logit: sigmoid(m) - x, each branch free of overflow
    if (m >= T(0)) return T(1) / (T(1) + exp(-m)) - x;
    T e = exp(m);
    return e / (T(1) + e) - x;
}

template <typename T>
__device__ __forceinline__ T loss_f(int loss, T x, T m)
{
    if (loss == GCP_LOSS_GAUSSIAN) return T(0.5) * (m - x) * (m - x);
    if (loss == GCP_LOSS_POISSON) return m - x * log(m + T(1e-10));
    return (m > T(0) ? m : T(0)) + log1p(exp(-fabs(m))) - x * m;
}

// ------------------------------------------------------------------- Adam --
// One element of Alg. adam-update; c1 = 1 - beta1^t and c2 = 1 - beta2^t.
template <typename T>
__device__ __forceinline__ void adam_update(T& p, T g, T& b, T& c, T lr, T b1, T b2, T one_m_b1, T one_m_b2, T c1,
                                            T c2, T eps, T lower)
{
    b = b1 * b + one_m_b1 * g;
    c = b2 * c + one_m_b2 * g * g;
    const T bhat = b / c1;
    const T chat = c / c2;
    p = fmax(p - lr * (bhat / sqrt(chat + eps)), lower);
}

// -------------------------------------------------------------- host misc --

int device_cu_count(int device);
int64_t ceil_div(int64_t a, int64_t b);
// Checks a launch's dynamic LDS against the device limit and opts the kernel
// in to more than 64 KiB when needed.
gcp_status prepare_lds(const void* fn, size_t bytes, int device);

// Device memory the row-bucketed scatter of gcp_loss_grad may use for its
// sample entries and per-(row block, workgroup) counts and starts.  Either a
// reservation of gcp_tensor_reserve (entries / hist / max_samples fixed when
// it was sized) or, when scratch_bytes > 0, a fixed scratch region of that
// many bytes carved up afresh by each call.
struct LGWorkspace {
    void* base = nullptr;
    int64_t entries = 0;        // reservation: 16-byte entries
    int64_t hist = 0;           // reservation: ints in each of counts and starts
    int64_t max_samples = 0;    // reservation: p + q it was sized for
    int64_t scratch_bytes = 0;  // > 0: fixed scratch region of this size
};

// The non-fused forms of the sampled gradient (Sec. 3.1.2): the sampling
// kernel may write the sampled tensor Y~ -- each sample's coordinates and its
// derivative value y = w f'(x, m) -- instead of scattering, and the MTTKRP
// may read such a tensor (its values are then y, loss kLossGivenValues).
struct LGOutputs {
    void* y_out = nullptr;          // [n] tensor dtype
    int64_t* coords_out = nullptr;  // [n x d]
    double* loss_parts = nullptr;   // per-wave objective partials (deterministic objective)
    int64_t loss_parts_cap = 0;     // slots available
    int64_t* parts_used = nullptr;  // receives the number of slots the launch fills
};

// Bytes of workspace the deterministic sampled gradient needs for up to
// max_samples samples (deterministic.hip); -1 on failure.
int64_t det_workspace_bytes(const gcp_tensor_s* t, int64_t max_samples);

// gcp_loss_grad with GCP_DETERMINISTIC (deterministic.hip).
gcp_status loss_grad_deterministic(gcp_tensor_s* t, const gcp_sample_params* sp, const gcp_samples* smp,
                                   const void* A, int R, gcp_loss loss, unsigned flags, const void* scale_dev,
                                   void* G_out, double* loss_out, const gcp_tile* tile, hipStream_t stream);

// gcp_loss_grad with an explicit bucketed-scatter workspace (the argument
// checks and launches of loss_grad.hip).
gcp_status loss_grad_with_workspace(gcp_tensor_s* t, const gcp_sample_params* sp, const gcp_samples* smp,
                                    const void* A, int R, gcp_loss loss, unsigned flags, const void* scale_dev,
                                    void* G_out, double* loss_out, const gcp_tile* tile, const LGWorkspace& ws,
                                    hipStream_t stream, const LGOutputs* xo = nullptr);

}  // namespace gcp
