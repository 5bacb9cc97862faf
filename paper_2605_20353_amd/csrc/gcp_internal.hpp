// Internal declarations shared by the HIP translation units of libgcp.
//
// Device-side building blocks of the sampled stochastic gradient:
//   * Philox4x64-10 counter-based RNG and the exact [0, n) range map
//     (the paper leaves the RNG open; counters make samples reproducible);
//   * bit-packed coordinate keys and the open-addressing membership table
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
constexpr uint64_t kEmptySlot = ~0ull;      // never a packed key (keys use <= 63 bits)

// Bit-packed coordinates: mode k occupies bits [shift_k, shift_k + bits_k);
// the last mode sits in the lowest bits.
struct KeyLayout {
    int d;
    int shift[kMaxModes];
    uint64_t mask[kMaxModes];
    int64_t dims[kMaxModes];
};

struct gcp_tensor_impl;

}  // namespace gcp

struct gcp_tensor_s {
    int device = 0;
    int d = 0;
    int64_t dims[gcp::kMaxModes] = {};
    int64_t rowoff[gcp::kMaxModes + 1] = {};  // first model row of each mode
    int64_t nnz = 0;
    int64_t cells = 0;        // prod_k I_k
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

// --------------------------------------------------------- packed coords --

__host__ __device__ __forceinline__ uint64_t unpack(const KeyLayout& L, uint64_t key, int k)
{
    return (key >> L.shift[k]) & L.mask[k];
}

// Candidate cell of sample s / attempt a drawn straight into a packed key.
template <int D>
__device__ __forceinline__ uint64_t draw_cell_key(const KeyLayout& L, int d, uint64_t seed, uint64_t client,
                                                  uint64_t s, uint64_t step, uint64_t stream, uint64_t attempt)
{
    const int dd = D > 0 ? D : d;
    uint64_t key = 0;
    U64x4 o = philox4x64_10(s, step, stream | (attempt << 8), 0, seed, client);
#pragma unroll
    for (int k = 0; k < (D > 0 ? (D < 4 ? D : 4) : 4); ++k)
        if (k < dd) key |= range_map(o.v[k], (uint64_t)L.dims[k]) << L.shift[k];
    if (dd > 4) {
        U64x4 o2 = philox4x64_10(s, step, stream | (attempt << 8), 1, seed, client);
#pragma unroll
        for (int k = 4; k < kMaxModes; ++k)
            if (k < dd) key |= range_map(o2.v[k - 4], (uint64_t)L.dims[k]) << L.shift[k];
    }
    return key;
}

// ------------------------------------------------------ membership table --
// Open addressing with linear probing over 2^b slots holding packed keys;
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

__device__ __forceinline__ bool table_contains(const uint64_t* __restrict__ table, uint64_t mask, int log2n,
                                               uint64_t key)
{
    uint64_t h = log2n > 0 ? (mix64(key) >> (64 - log2n)) : 0;
    for (;;) {
        uint64_t v = __builtin_nontemporal_load(table + h);
        if (v == key) return true;
        if (v == kEmptySlot) return false;
        h = (h + 1) & mask;
    }
}

// ------------------------------------------------------------------ losses --

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

}  // namespace gcp
