// GCP-FedAdam (Alg. gcp-fed-iter) on one GPU: every client's local GCP-Adam
// steps in one persistent launch, then one server kernel that averages the
// deltas per row and takes the server Adam step.
//
// Persistent launch: client c owns W consecutive workgroups.  Per round they
// copy the client's rows of the server model into M_c, then for each of the
// tau local steps: the sampled gradient of the client's block (the same
// per-chunk body as gcp_loss_grad; small modes accumulate in LDS, large ones
// with hardware atomics into G_c), a group barrier, Adam on M_c (which also
// re-zeroes G_c), a group barrier.
//
// Batched rounds with the row-bucketed scatter instead run, per local step,
// three launches that each cover every client (blockIdx.y = client): sample
// and sort by row block (k_fed_sample), row-block owners that accumulate in
// LDS and store their rows of G_c (k_fed_owner), and Adam (k_fed_adam); the
// kernel boundaries take the place of the group barriers.  The
// barrier is a per-client arrival counter in global memory with a wait
// bounded in device wall-clock time: all K*W workgroups must be resident
// (checked at create), and a barrier that waits too long records an error
// and ends the round instead of hanging.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "lg_core.hpp"

namespace gcp {

constexpr uint32_t kStatusBarrier = 4u;
constexpr double kBarrierTimeoutS = 10.0;      // default wait bound of a group barrier
constexpr int kFedLdsBudget = 64 * 1024;   // bytes of private client gradient per workgroup
constexpr int kFedBucketRowBytes = 32 * 1024;   // LDS of one row block in the bucketed scatter
constexpr int64_t kFedBucketMinSamples = 1 << 14;   // automatic bucketing from this many samples per client step

template <typename T>
struct FedClientDev {
    LGParams<T> P;                 // P.A = M_c, P.G = G_c, P.sc = the block's sampler
    T* B;
    T* C;
    int64_t nparams;               // sum_k I_k^c * R
    int64_t seg_src[kMaxModes];    // first server element of the block's rows in mode k
    int64_t seg_dst[kMaxModes];    // first client element of mode k
    int64_t seg_len[kMaxModes];    // elements of mode k (I_k^c * R)
};

template <typename T>
struct FedArgs {
    const FedClientDev<T>* clients;
    int K, W, tau, d, R;
    T* U;
    T* Bs;
    T* Cs;
    int64_t nserver;               // server elements
    T lr, meta, b1, b2, one_m_b1, one_m_b2, eps, lower;
    double b1d, b2d;
    int* barrier;                  // [K] arrival counters, zero between rounds
    uint64_t barrier_ticks;        // wait bound of a group barrier, device wall-clock ticks
    const int64_t* round;          // device round number
    uint32_t* status;
    const int64_t* cov_ptr;        // per server row: clients covering it (CSR)
    const int* cov_client;
    const int* cov_lrow;           // the row's index in the client's model
    T* const* Mptrs;               // per client model
    int staging_bytes;             // LDS before the private gradient copies
};

__device__ __forceinline__ bool barrier_failed(const uint32_t* status)
{
    return (__hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kStatusBarrier) != 0;
}

// Group barrier of one client's W workgroups.  Returns false when this or
// any other barrier of the launch has given up (waited longer than `ticks`
// of the device wall clock); the caller then ends the round.
__device__ __forceinline__ bool fed_barrier(int* ctr, int target, uint32_t* status, uint64_t ticks)
{
    __threadfence();               // this thread's atomics and stores are performed
    __syncthreads();
    int bad = 0;
    if (threadIdx.x == 0) {
        atomicAdd(ctr, 1);
        const uint64_t t0 = wall_clock64();
        while (__hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (barrier_failed(status)) {
                bad = 1;
                break;
            }
            if (wall_clock64() - t0 > ticks) {
                atomicOr(status, kStatusBarrier);
                bad = 1;
                break;
            }
            __builtin_amdgcn_s_sleep(4);
        }
    }
    bad = __syncthreads_or(bad);
    __threadfence();               // see the other workgroups' writes
    return bad == 0;
}

template <typename T>
__device__ __forceinline__ T bias_correction(double beta, int64_t t)
{
    return (T)(1.0 - pow(beta, (double)t));
}

template <typename T, int D, int LANES, int VEC>
__global__ void __launch_bounds__(1024) k_fed_clients(const FedArgs<T> F)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int c = blockIdx.x / F.W, w = blockIdx.x % F.W;
    const FedClientDev<T>& C = F.clients[c];
    // a private copy: read once, then held in registers -- read through the
    // global reference, every field would be reloaded after each atomic.  It
    // stays in registers only while every index into it is a compile-time one
    constexpr int DM = D > 0 ? D : kMaxModes;
    const LGParams<T> P = C.P;
    T* M = const_cast<T*>(P.A);
    T* G = P.G;
    T* const Bc = C.B;
    T* const Cc = C.C;
    const int64_t nparams = C.nparams;
    const int nwaves = blockDim.x >> 6;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint64_t* skey = reinterpret_cast<uint64_t*>(smem) + wave * 64;
    T* sx = reinterpret_cast<T*>(smem + (size_t)nwaves * 64 * 8) + wave * 64;
    T* sw = reinterpret_cast<T*>(smem + (size_t)nwaves * 64 * (8 + sizeof(T))) + wave * 64;
    T* priv = reinterpret_cast<T*>(smem + F.staging_bytes);
    const int64_t round = *F.round;
    const int64_t tid = (int64_t)w * blockDim.x + threadIdx.x;
    const int64_t nthreads = (int64_t)F.W * blockDim.x;
    const int dd = D > 0 ? D : P.sc.d;
    int arrivals = 0;
    // a barrier failure of an earlier round stands until the host clears it
    if (barrier_failed(F.status)) return;

    // M_c <- the client's rows of the server model
    for (int k = 0; k < F.d; ++k)
        for (int64_t e = tid; e < C.seg_len[k]; e += nthreads) M[C.seg_dst[k] + e] = F.U[C.seg_src[k] + e];
    if (!fed_barrier(F.barrier + c, (++arrivals) * F.W, F.status, F.barrier_ticks)) return;

    for (int j = 0; j < F.tau; ++j) {
        const uint64_t step = (uint64_t)(round * F.tau + j);
        double lacc = 0.0;
        if (P.lds_mask) {
            for (int64_t e = threadIdx.x; e < P.lds_elems; e += blockDim.x) priv[e] = T(0);
            __syncthreads();
        }
        for (int64_t chunk = (int64_t)w * nwaves + wave; chunk < P.nchunks; chunk += (int64_t)F.W * nwaves)
            lg_chunk<T, D, LANES, VEC, 0>(P, chunk, lane, skey, sx, sw, priv, nullptr, nullptr, 0, false, T(1),
                                          lacc, step);
        if (P.lds_mask) {
            // flush this workgroup's share of the small modes' gradient once
            __syncthreads();
#pragma unroll
            for (int k = 0; k < DM; ++k) {
                if (k >= dd || !((P.lds_mask >> k) & 1u)) continue;
                const int64_t elems = P.sc.L.dims[k] * (int64_t)P.R;
                T* dst = G + P.rowoff[k] * P.R;
                const T* src = priv + P.lds_off[k];
                for (int64_t e = threadIdx.x; e < elems; e += blockDim.x) {
                    const T v = src[e];
                    if (v != T(0)) global_add(dst + e, v);
                }
            }
        }
        if (!fed_barrier(F.barrier + c, (++arrivals) * F.W, F.status, F.barrier_ticks)) return;
        const int64_t t = round * F.tau + j + 1;
        const T c1 = bias_correction<T>(F.b1d, t), c2 = bias_correction<T>(F.b2d, t);
        for (int64_t e = tid; e < nparams; e += nthreads) {
            T p = M[e], b = Bc[e], cc = Cc[e];
            adam_update<T>(p, G[e], b, cc, F.lr, F.b1, F.b2, F.one_m_b1, F.one_m_b2, c1, c2, F.eps, F.lower);
            M[e] = p;
            Bc[e] = b;
            Cc[e] = cc;
            G[e] = T(0);
        }
        if (j + 1 < F.tau && !fed_barrier(F.barrier + c, (++arrivals) * F.W, F.status, F.barrier_ticks)) return;
    }
}

// Bucketed batched round, sampling side.  Workgroup (x, c) takes client c's
// sample blocks x, x + gridDim.x, ...: draws and stages each block's
// samples, forms model values and derivatives, accumulates the small modes in
// its LDS, and sorts the block by row block into the client's segment list
// of the same index; the small modes are flushed into G_c once at the end.
template <typename T, int D, int LANES, int VEC>
__global__ void __launch_bounds__(1024) k_fed_sample(const FedArgs<T> F, int j)
{
    constexpr int DM = D > 0 ? D : kMaxModes;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const LGParams<T> P = F.clients[blockIdx.y].P;
    const int nwaves = blockDim.x >> 6;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint64_t* skey = reinterpret_cast<uint64_t*>(smem) + wave * 64;
    T* sx = reinterpret_cast<T*>(smem + (size_t)nwaves * 64 * 8) + wave * 64;
    T* sw = reinterpret_cast<T*>(smem + (size_t)nwaves * 64 * (8 + sizeof(T))) + wave * 64;
    T* priv = reinterpret_cast<T*>(smem + F.staging_bytes);
    uint64_t* bkey = reinterpret_cast<uint64_t*>(smem + P.bucket_lds);
    T* by = reinterpret_cast<T*>(smem + P.bucket_lds + (size_t)P.spb * 8);
    int* bcnt = reinterpret_cast<int*>(smem + P.bucket_lds + (size_t)P.spb * (8 + sizeof(T)));
    int* boff = bcnt + P.nb;
    const int dd = D > 0 ? D : P.sc.d;
    const uint64_t step = (uint64_t)(*F.round * F.tau + j);
    double lacc = 0.0;
    if (P.lds_mask) {
        for (int64_t e = threadIdx.x; e < P.lds_elems; e += blockDim.x) priv[e] = T(0);
        __syncthreads();
    }
    for (int64_t jb = blockIdx.x; jb < P.nblocks; jb += gridDim.x) {
        const int64_t s0 = jb * P.spb;
        const int64_t c_end = std::min<int64_t>(P.nchunks, (s0 + P.spb) / 64);
        for (int64_t chunk = s0 / 64 + wave; chunk < c_end; chunk += nwaves)
            lg_chunk<T, D, LANES, VEC, 0>(P, chunk, lane, skey, sx, sw, priv, bkey, by, s0, true, T(1), lacc, step);
        bucket_write_out<T, D>(P, jb, (int)std::min<int64_t>(P.spb, P.n - s0), bkey, by, bcnt, boff);
    }
    if (P.lds_mask) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < DM; ++k) {
            if (k < dd && ((P.lds_mask >> k) & 1u)) {
                const int64_t elems = P.sc.L.dims[k] * (int64_t)P.R;
                T* dst = P.G + P.rowoff[k] * P.R;
                const T* src = priv + P.lds_off[k];
                for (int64_t e = threadIdx.x; e < elems; e += blockDim.x) {
                    const T v = src[e];
                    if (v != T(0)) global_add(dst + e, v);
                }
            }
        }
    }
}

// Bucketed batched round, owner side.  Workgroup (rb, c) owns row block rb of
// client c's bucketed modes: it accumulates the entries of every segment list
// for the block in LDS and stores the rows into G_c -- no other workgroup
// writes them.
template <typename T, int D, int LANES, int VEC>
__global__ void __launch_bounds__(1024) k_fed_owner(const FedArgs<T> F)
{
    constexpr int DM = D > 0 ? D : kMaxModes;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const LGParams<T> P = F.clients[blockIdx.y].P;
    const int rb = blockIdx.x;
    if (rb >= P.nb) return;
    const int dd = D > 0 ? D : P.sc.d;
    // the row block's mode and rows, read with compile-time indices
    int k = 0;
    int64_t r0 = 0, rows = 0, roff = 0;
#pragma unroll
    for (int kk = 0; kk < DM; ++kk) {
        if (kk < dd && P.bucket_base[kk] <= rb && rb < P.bucket_base[kk + 1]) {
            k = kk;
            r0 = (int64_t)(rb - P.bucket_base[kk]) << P.br_shift;
            rows = std::min<int64_t>((int64_t)1 << P.br_shift, P.sc.L.dims[kk] - r0);
            roff = P.rowoff[kk];
        }
    }
    T* part = reinterpret_cast<T*>(smem);
    int* seg_cnt = reinterpret_cast<int*>(smem + ((((size_t)1 << P.br_shift) * P.R * sizeof(T) + 15) & ~(size_t)15));
    bucket_accumulate<T, D, LANES, VEC>(P, k, rb, r0, rows, 0, P.nblocks, part, seg_cnt);
    T* dst = P.G + (roff + r0) * P.R;
    for (int64_t e = threadIdx.x; e < rows * P.R; e += blockDim.x) dst[e] = part[e];
}

// Adam on every client's model (blockIdx.y = client) for local step j,
// re-zeroing G_c.
template <typename T>
__global__ void __launch_bounds__(256) k_fed_adam(const FedArgs<T> F, int j)
{
    const FedClientDev<T>& C = F.clients[blockIdx.y];
    T* M = const_cast<T*>(C.P.A);
    T* G = C.P.G;
    const int64_t t = *F.round * F.tau + j + 1;
    const T c1 = bias_correction<T>(F.b1d, t), c2 = bias_correction<T>(F.b2d, t);
    const int64_t n = C.nparams;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        T p = M[e], b = C.B[e], cc = C.C[e];
        adam_update<T>(p, G[e], b, cc, F.lr, F.b1, F.b2, F.one_m_b1, F.one_m_b2, c1, c2, F.eps, F.lower);
        M[e] = p;
        C.B[e] = b;
        C.C[e] = cc;
        G[e] = T(0);
    }
}

// Server step: D = per-row mean over covering clients of U - M_c, then Adam
// on U with rate meta; also clears the clients' barrier counters.  Skipped
// (counters still cleared) when a group barrier of the round gave up.
template <typename T>
__global__ void __launch_bounds__(256) k_fed_server(const FedArgs<T> F)
{
    const int64_t t = *F.round + 1;
    const T c1 = bias_correction<T>(F.b1d, t), c2 = bias_correction<T>(F.b2d, t);
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t nserver = barrier_failed(F.status) ? 0 : F.nserver;
    for (int64_t e = gid; e < nserver; e += stride) {
        const int64_t row = e / F.R, col = e - row * F.R;
        const int64_t b = F.cov_ptr[row], end = F.cov_ptr[row + 1];
        T u = F.U[e];
        T g = T(0);
        for (int64_t i = b; i < end; ++i) g += u - F.Mptrs[F.cov_client[i]][(int64_t)F.cov_lrow[i] * F.R + col];
        if (end > b) g /= T(end - b);
        T bs = F.Bs[e], cs = F.Cs[e];
        adam_update<T>(u, g, bs, cs, F.meta, F.b1, F.b2, F.one_m_b1, F.one_m_b2, c1, c2, F.eps, F.lower);
        F.U[e] = u;
        F.Bs[e] = bs;
        F.Cs[e] = cs;
    }
    if (gid < F.K) F.barrier[gid] = 0;
}

// Per-client launches: M_c <- rows of U (blockIdx.y = client).
template <typename T>
__global__ void __launch_bounds__(256) k_fed_copy(const FedArgs<T> F)
{
    const FedClientDev<T>& C = F.clients[blockIdx.y];
    T* M = const_cast<T*>(C.P.A);
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = (int64_t)gridDim.x * blockDim.x;
    for (int k = 0; k < F.d; ++k)
        for (int64_t e = tid; e < C.seg_len[k]; e += n) M[C.seg_dst[k] + e] = F.U[C.seg_src[k] + e];
}

__global__ void k_fed_set_round(int64_t* round, int64_t value) { *round = value; }

template <typename T>
using FedKernel = void (*)(const FedArgs<T>);
template <typename T>
using FedStepKernel = void (*)(const FedArgs<T>, int);

#define GCP_FED_SHAPES_F32(X) X(8, 1) X(16, 1) X(32, 1) X(64, 1) X(16, 2) X(32, 2) X(64, 2) X(8, 4) X(16, 4) X(64, 4)
#define GCP_FED_SHAPES_F64(X) X(8, 1) X(16, 1) X(32, 1) X(64, 1) X(16, 2) X(32, 2) X(64, 2) X(64, 4)

template <typename T, int D>
static FedKernel<T> pick_fed(int lanes, int vec)
{
#define GCP_CASE(LN, VC) \
    if (lanes == LN && vec == VC) return k_fed_clients<T, D, LN, VC>;
    if constexpr (sizeof(T) == 4) {
        GCP_FED_SHAPES_F32(GCP_CASE)
    } else {
        GCP_FED_SHAPES_F64(GCP_CASE)
    }
#undef GCP_CASE
    return nullptr;
}

template <typename T, int D>
static FedStepKernel<T> pick_fed_sample(int lanes, int vec)
{
#define GCP_CASE(LN, VC) \
    if (lanes == LN && vec == VC) return k_fed_sample<T, D, LN, VC>;
    if constexpr (sizeof(T) == 4) {
        GCP_FED_SHAPES_F32(GCP_CASE)
    } else {
        GCP_FED_SHAPES_F64(GCP_CASE)
    }
#undef GCP_CASE
    return nullptr;
}

template <typename T, int D>
static FedKernel<T> pick_fed_owner(int lanes, int vec)
{
#define GCP_CASE(LN, VC) \
    if (lanes == LN && vec == VC) return k_fed_owner<T, D, LN, VC>;
    if constexpr (sizeof(T) == 4) {
        GCP_FED_SHAPES_F32(GCP_CASE)
    } else {
        GCP_FED_SHAPES_F64(GCP_CASE)
    }
#undef GCP_CASE
    return nullptr;
}

}  // namespace gcp

using namespace gcp;

struct gcp_fed_s {
    int device = 0;
    gcp_dtype dt = GCP_F32;
    gcp_fed_desc desc{};
    std::vector<gcp_fed_client> clients;
    int d = 0;
    int W = 1, block = 256, lanes = 0, vec = 0;
    int64_t nserver = 0;
    uint32_t lds_mask = 0;         // batched: modes accumulated in LDS per workgroup
    uint32_t bucket_mask = 0;      // batched: row-bucketed modes
    int spb = 0;                   // row-bucketed: samples per sorted block
    uint32_t* status_host = nullptr;   // pinned copy of the status word, refreshed after each batched round
    void* dev_clients = nullptr;   // FedClientDev<T>[K]
    void* dev_mptrs = nullptr;
    int* barrier = nullptr;
    int64_t* round = nullptr;
    uint32_t* status = nullptr;
    int64_t* cov_ptr = nullptr;
    int* cov_client = nullptr;
    int* cov_lrow = nullptr;
    unsigned char args[sizeof(FedArgs<double>)] = {};   // FedArgs<T> for the tensor dtype
    const void* client_kernel = nullptr;
    size_t client_lds = 0;
    size_t lds_bytes = 0;          // private gradient copies of the batched kernel
    // row-bucketed batched rounds: per local step one sampling, one owner and
    // one Adam launch over all clients
    bool want_bucket = false;      // the description asks for (or defaults to) bucketing
    bool bucketed = false;
    void* bucket_ws = nullptr;     // sample entries, counts and starts of every client
    const void* sample_kernel = nullptr;
    const void* owner_kernel = nullptr;
    size_t sample_lds = 0, owner_lds = 0;
    int nb_max = 0;                // row blocks of the largest client
    int64_t max_params = 0;        // parameters of the largest client
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t graph_stream = nullptr;
};

namespace gcp {

template <typename T>
static gcp_status fed_build(gcp_fed_s* f)
{
    const gcp_fed_desc& D = f->desc;
    const int K = D.nclients, R = D.R, d = f->d;
    int64_t goff[kMaxModes + 1] = {0};
    for (int k = 0; k < d; ++k) goff[k + 1] = goff[k] + D.global_dims[k];
    f->nserver = goff[d] * R;
    std::vector<FedClientDev<T>> host(K);
    std::vector<T*> mptrs(K);
    // coverage lists per server row
    std::vector<int64_t> cnt(goff[d] + 1, 0);
    for (int c = 0; c < K; ++c) {
        const gcp_fed_client& cl = f->clients[c];
        const gcp_tensor_s* t = cl.tensor;
        for (int k = 0; k < d; ++k)
            for (int64_t r = 0; r < t->dims[k]; ++r) cnt[goff[k] + cl.row_base[k] + r + 1]++;
    }
    for (size_t i = 1; i < cnt.size(); ++i) cnt[i] += cnt[i - 1];
    std::vector<int64_t> ptr = cnt;
    std::vector<int> cov_c(cnt.back()), cov_l(cnt.back());
    std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
    for (int c = 0; c < K; ++c) {
        const gcp_fed_client& cl = f->clients[c];
        const gcp_tensor_s* t = cl.tensor;
        for (int k = 0; k < d; ++k)
            for (int64_t r = 0; r < t->dims[k]; ++r) {
                const int64_t g = goff[k] + cl.row_base[k] + r;
                cov_c[fill[g]] = c;
                cov_l[fill[g]] = (int)(t->rowoff[k] + r);
                ++fill[g];
            }
    }
    // small modes of the batched kernel accumulate in LDS (per workgroup and
    // local step) when the largest client block of the mode fits the budget
    uint32_t lds_mask = 0;
    int64_t lds_max_elems = 0;
    if (D.batched && D.lds_modes != 0) {
        int64_t used = 0;
        for (int k = 0; k < d; ++k) {
            int64_t mx = 0;
            for (int c = 0; c < K; ++c) mx = std::max<int64_t>(mx, f->clients[c].tensor->dims[k]);
            const int64_t bytes = mx * R * (int64_t)sizeof(T);
            const bool want = D.lds_modes > 0 ? ((D.lds_modes >> k) & 1) : true;
            if (want && used + bytes <= kFedLdsBudget) {
                lds_mask |= 1u << k;
                used += bytes;
            } else if (D.lds_modes > 0 && want) {
                return set_error(GCP_ERR_ARG, "LDS-private mode %d does not fit in %d bytes", k, kFedLdsBudget);
            }
        }
        lds_max_elems = used / (int64_t)sizeof(T);
    }
    f->lds_mask = lds_mask;
    f->lds_bytes = (size_t)lds_max_elems * sizeof(T);
    const size_t staging = (size_t)(f->block / 64) * 64 * (8 + 2 * sizeof(T));

    // row-bucketed modes of the batched kernel: a row block of 2^br_shift rows
    // fills kFedBucketRowBytes of LDS; each client sorts its samples in blocks
    // of spb into its own segment lists
    uint32_t bucket_mask = 0;
    int br_shift = 0, spb = 0;
    int64_t nblocks_c = 0;
    if (f->want_bucket) {
        const uint32_t all = (1u << d) - 1;
        bucket_mask = (D.bucket_modes > 0 ? (uint32_t)D.bucket_modes : all) & all & ~lds_mask;
    }
    std::vector<int64_t> ws_off(K + 1, 0);
    std::vector<int> nb_c(K, 0);
    int nbm = 0, nb_max = 0;
    if (bucket_mask) {
        while (((int64_t)2 << br_shift) * R * (int64_t)sizeof(T) <= kFedBucketRowBytes && br_shift < 30) ++br_shift;
        spb = D.bucket_block_samples > 0 ? D.bucket_block_samples : 2048;
        if (spb % 64 != 0 || spb < 512 || spb > 8192)
            return set_error(GCP_ERR_ARG, "bucket_block_samples = %d", spb);
        nblocks_c = ceil_div(D.p + D.q, spb);
        for (int k = 0; k < d; ++k) nbm += (int)((bucket_mask >> k) & 1u);
        for (int c = 0; c < K; ++c) {
            const gcp_tensor_s* t = f->clients[c].tensor;
            for (int k = 0; k < d; ++k)
                if ((bucket_mask >> k) & 1u) nb_c[c] += (int)ceil_div(t->dims[k], int64_t(1) << br_shift);
            nb_max = std::max(nb_max, nb_c[c]);
            // entries, then counts and starts, 16-byte aligned per client
            const int64_t bytes = nblocks_c * spb * nbm * 16 + (((int64_t)2 * nb_c[c] * nblocks_c * 4 + 15) & ~int64_t(15));
            ws_off[c + 1] = ws_off[c] + bytes;
        }
        GCP_HIP(hipMalloc(&f->bucket_ws, (size_t)std::max<int64_t>(16, ws_off[K])));
        f->bucketed = true;
        f->bucket_mask = bucket_mask;
        f->spb = spb;
        f->nb_max = nb_max;
        f->sample_lds = ((staging + f->lds_bytes + 15) & ~(size_t)15) + (size_t)spb * (8 + sizeof(T)) + (size_t)nb_max * 8;
        f->owner_lds = ((((size_t)1 << br_shift) * R * sizeof(T) + 15) & ~(size_t)15) + (size_t)nblocks_c * 8;
    }
    for (int c = 0; c < K; ++c) {
        const gcp_fed_client& cl = f->clients[c];
        const gcp_tensor_s* t = cl.tensor;
        FedClientDev<T>& h = host[c];
        gcp_sample_params sp{};
        sp.kind = GCP_SAMPLE_STRATIFIED;
        sp.max_attempts = D.max_attempts;
        sp.p = D.p;
        sp.q = D.q;
        sp.seed = D.seed;
        sp.step = 0;
        sp.client = (uint64_t)c;
        int64_t n = 0;
        gcp_status st = make_sample_ctx<T>(t, &sp, h.P.sc, n);
        if (st != GCP_OK) return st;
        h.P.n = n;
        h.P.nchunks = ceil_div(n, 64);
        h.P.A = (const T*)cl.M;
        h.P.G = (T*)cl.G;
        h.P.R = R;
        h.P.loss = D.loss;
        for (int k = 0; k < kMaxModes; ++k) h.P.rowoff[k] = k < d ? t->rowoff[k] : t->rowoff[d];
        for (int k = 0; k <= kMaxModes; ++k) h.P.bucket_base[k] = 0;
        h.P.lds_mask = lds_mask;
        int64_t off = 0;
        for (int k = 0; k < d; ++k) {
            if ((lds_mask >> k) & 1u) {
                h.P.lds_off[k] = off;
                off += t->dims[k] * R;
            }
        }
        h.P.lds_elems = off;
        if (bucket_mask) {
            h.P.bucket_mask = bucket_mask;
            h.P.n_bucket_modes = nbm;
            h.P.br_shift = br_shift;
            h.P.nb = nb_c[c];
            h.P.spb = spb;
            h.P.nblocks = nblocks_c;
            h.P.entry_cap = (int64_t)spb * nbm;
            h.P.bucket_lds = (int)((staging + f->lds_bytes + 15) & ~(size_t)15);
            int nb = 0;
            for (int k = 0; k < d; ++k) {
                h.P.bucket_base[k] = nb;
                if ((bucket_mask >> k) & 1u) nb += (int)ceil_div(t->dims[k], int64_t(1) << br_shift);
            }
            for (int k = d; k <= kMaxModes; ++k) h.P.bucket_base[k] = nb;
            unsigned char* base = (unsigned char*)f->bucket_ws + ws_off[c];
            h.P.entries = (uint4*)base;
            h.P.hist = (int*)(base + nblocks_c * spb * nbm * 16);
            h.P.start = h.P.hist + (int64_t)nb_c[c] * nblocks_c;
        }
        h.B = (T*)cl.B;
        h.C = (T*)cl.C;
        h.nparams = t->rowoff[d] * R;
        f->max_params = std::max<int64_t>(f->max_params, h.nparams);
        for (int k = 0; k < kMaxModes; ++k) {
            h.seg_src[k] = k < d ? (goff[k] + cl.row_base[k]) * R : 0;
            h.seg_dst[k] = k < d ? t->rowoff[k] * R : 0;
            h.seg_len[k] = k < d ? t->dims[k] * R : 0;
        }
        mptrs[c] = (T*)cl.M;
    }
    GCP_HIP(hipMalloc(&f->dev_clients, sizeof(FedClientDev<T>) * K));
    GCP_HIP(hipMemcpy(f->dev_clients, host.data(), sizeof(FedClientDev<T>) * K, hipMemcpyHostToDevice));
    GCP_HIP(hipMalloc(&f->dev_mptrs, sizeof(T*) * K));
    GCP_HIP(hipMemcpy(f->dev_mptrs, mptrs.data(), sizeof(T*) * K, hipMemcpyHostToDevice));
    GCP_HIP(hipMalloc((void**)&f->cov_ptr, sizeof(int64_t) * ptr.size()));
    GCP_HIP(hipMemcpy(f->cov_ptr, ptr.data(), sizeof(int64_t) * ptr.size(), hipMemcpyHostToDevice));
    const size_t ncov = std::max<size_t>(1, cov_c.size());
    GCP_HIP(hipMalloc((void**)&f->cov_client, sizeof(int) * ncov));
    GCP_HIP(hipMalloc((void**)&f->cov_lrow, sizeof(int) * ncov));
    if (!cov_c.empty()) {
        GCP_HIP(hipMemcpy(f->cov_client, cov_c.data(), sizeof(int) * cov_c.size(), hipMemcpyHostToDevice));
        GCP_HIP(hipMemcpy(f->cov_lrow, cov_l.data(), sizeof(int) * cov_l.size(), hipMemcpyHostToDevice));
    }
    GCP_HIP(hipMalloc((void**)&f->barrier, sizeof(int) * K));
    GCP_HIP(hipMemset(f->barrier, 0, sizeof(int) * K));
    GCP_HIP(hipMalloc((void**)&f->round, sizeof(int64_t)));
    GCP_HIP(hipMemset(f->round, 0, sizeof(int64_t)));
    GCP_HIP(hipMalloc((void**)&f->status, sizeof(uint32_t)));
    GCP_HIP(hipMemset(f->status, 0, sizeof(uint32_t)));
    GCP_HIP(hipHostMalloc((void**)&f->status_host, sizeof(uint32_t), hipHostMallocDefault));
    *f->status_host = 0;
    int clock_khz = 0;
    if (hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, f->device) != hipSuccess || clock_khz <= 0)
        clock_khz = 100000;         // gfx9 wall clock: 100 MHz
    const double timeout_s = D.barrier_timeout_s > 0 ? D.barrier_timeout_s : kBarrierTimeoutS;

    FedArgs<T> a{};
    a.clients = (const FedClientDev<T>*)f->dev_clients;
    a.K = K;
    a.W = f->W;
    a.tau = D.tau;
    a.d = d;
    a.R = R;
    a.U = (T*)D.U;
    a.Bs = (T*)D.Bs;
    a.Cs = (T*)D.Cs;
    a.nserver = f->nserver;
    a.lr = (T)D.lr;
    a.meta = (T)D.meta_lr;
    a.b1 = (T)D.beta1;
    a.b2 = (T)D.beta2;
    a.one_m_b1 = (T)(1.0 - D.beta1);
    a.one_m_b2 = (T)(1.0 - D.beta2);
    a.eps = (T)D.eps;
    a.lower = (T)D.lower;
    a.b1d = D.beta1;
    a.b2d = D.beta2;
    a.barrier = f->barrier;
    a.barrier_ticks = (uint64_t)(timeout_s * 1000.0 * (double)clock_khz);
    a.round = f->round;
    a.status = f->status;
    a.cov_ptr = f->cov_ptr;
    a.cov_client = f->cov_client;
    a.cov_lrow = f->cov_lrow;
    a.Mptrs = (T* const*)f->dev_mptrs;
    memcpy(f->args, &a, sizeof(a));

    bool order3 = d == 3;
    for (const gcp_fed_client& cl : f->clients) order3 = order3 && kernel_order(cl.tensor) == 3;
    if (D.batched && f->bucketed) {
        reinterpret_cast<FedArgs<T>*>(f->args)->staging_bytes = (int)staging;
        FedStepKernel<T> sk = order3 ? pick_fed_sample<T, 3>(f->lanes, f->vec) : pick_fed_sample<T, 0>(f->lanes, f->vec);
        FedKernel<T> ok = order3 ? pick_fed_owner<T, 3>(f->lanes, f->vec) : pick_fed_owner<T, 0>(f->lanes, f->vec);
        if (!sk || !ok)
            return set_error(GCP_ERR_UNSUPPORTED, "batched lane shape lanes = %d, vec = %d not built", f->lanes, f->vec);
        f->sample_kernel = reinterpret_cast<const void*>(sk);
        f->owner_kernel = reinterpret_cast<const void*>(ok);
        gcp_status st = prepare_lds(f->sample_kernel, f->sample_lds, f->device);
        if (st != GCP_OK) return st;
        st = prepare_lds(f->owner_kernel, f->owner_lds, f->device);
        if (st != GCP_OK) return st;
        if (D.workgroups_per_client <= 0) {
            // automatic: the sampling launch fills the GPU once
            int per_cu = 0;
            GCP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f->sample_kernel, f->block, f->sample_lds));
            const int64_t resident = (int64_t)std::max(1, per_cu) * device_cu_count(f->device);
            f->W = (int)std::max<int64_t>(1, std::min<int64_t>(nblocks_c, resident / K));
            reinterpret_cast<FedArgs<T>*>(f->args)->W = f->W;
        }
        return GCP_OK;
    }
    if (D.batched) {
        gcp_status st = GCP_OK;
        FedKernel<T> kern = nullptr;
        if (order3) kern = pick_fed<T, 3>(f->lanes, f->vec);
        else kern = pick_fed<T, 0>(f->lanes, f->vec);
        if (!kern) return set_error(GCP_ERR_UNSUPPORTED, "batched lane shape lanes = %d, vec = %d not built", f->lanes,
                                    f->vec);
        f->client_kernel = reinterpret_cast<const void*>(kern);
        f->client_lds = staging + f->lds_bytes;
        reinterpret_cast<FedArgs<T>*>(f->args)->staging_bytes = (int)staging;
        st = prepare_lds(f->client_kernel, f->client_lds, f->device);
        if (st != GCP_OK) return st;
        int per_cu = 0;
        GCP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f->client_kernel, f->block, f->client_lds));
        const int64_t resident = (int64_t)per_cu * device_cu_count(f->device);
        if (D.workgroups_per_client <= 0) {
            // automatic: as many workgroups per client as stay resident, but
            // no more than leave each wavefront about four 64-sample chunks
            // of a local step (beyond that the extra workgroups only add
            // barrier arrivals and LDS flushes)
            const int64_t busy = ceil_div(ceil_div(D.p + D.q, 64), 4 * (int64_t)(f->block / 64));
            f->W = (int)std::max<int64_t>(1, std::min<int64_t>(busy, resident / K));
            reinterpret_cast<FedArgs<T>*>(f->args)->W = f->W;
        }
        if ((int64_t)K * f->W > resident)
            return set_error(GCP_ERR_UNSUPPORTED,
                             "%d clients x %d workgroups exceed the %lld workgroups the GPU holds at once", K, f->W,
                             (long long)resident);
    }
    return GCP_OK;
}

template <typename T>
static gcp_status fed_launch_batched(gcp_fed_s* f, hipStream_t stream)
{
    const FedArgs<T>& a = *reinterpret_cast<const FedArgs<T>*>(f->args);
    const unsigned K = (unsigned)f->desc.nclients;
    if (f->bucketed) {
        int64_t maxlen = 0;
        for (const gcp_fed_client& cl : f->clients) maxlen = std::max<int64_t>(maxlen, cl.tensor->rowoff[f->d] * f->desc.R);
        const unsigned cb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(maxlen, 256), 1024));
        k_fed_copy<T><<<dim3(cb, K), 256, 0, stream>>>(a);
        GCP_HIP(hipGetLastError());
        const unsigned ab = (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(f->max_params, 256 * 4), 256));
        for (int j = 0; j < f->desc.tau; ++j) {
            hipLaunchKernelGGL(reinterpret_cast<FedStepKernel<T>>(const_cast<void*>(f->sample_kernel)),
                               dim3((unsigned)f->W, K), dim3(f->block), f->sample_lds, stream, a, j);
            GCP_HIP(hipGetLastError());
            hipLaunchKernelGGL(reinterpret_cast<FedKernel<T>>(const_cast<void*>(f->owner_kernel)),
                               dim3((unsigned)f->nb_max, K), dim3(1024), f->owner_lds, stream, a);
            GCP_HIP(hipGetLastError());
            k_fed_adam<T><<<dim3(ab, K), 256, 0, stream>>>(a, j);
            GCP_HIP(hipGetLastError());
        }
    } else {
        hipLaunchKernelGGL(reinterpret_cast<FedKernel<T>>(const_cast<void*>(f->client_kernel)),
                           dim3(K * (unsigned)f->W), dim3(f->block), f->client_lds, stream, a);
        GCP_HIP(hipGetLastError());
    }
    const int64_t sb = std::max<int64_t>(1, std::min<int64_t>(ceil_div(f->nserver, 256), 2048));
    k_fed_server<T><<<(unsigned)sb, 256, 0, stream>>>(a);
    GCP_HIP(hipGetLastError());
    return GCP_OK;
}

template <typename T>
static gcp_status fed_round_plain(gcp_fed_s* f, int64_t round, hipStream_t stream)
{
    const FedArgs<T>& a = *reinterpret_cast<const FedArgs<T>*>(f->args);
    const gcp_fed_desc& D = f->desc;
    int64_t maxlen = 0;
    for (const gcp_fed_client& cl : f->clients) maxlen = std::max<int64_t>(maxlen, cl.tensor->rowoff[f->d] * D.R);
    const unsigned cb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(maxlen, 256), 1024));
    k_fed_copy<T><<<dim3(cb, (unsigned)D.nclients), 256, 0, stream>>>(a);
    GCP_HIP(hipGetLastError());
    gcp_tile tile{};
    // with the automatic scatter, each call also picks its own lane shape
    // (four columns per lane when it row-buckets), unless one was asked for
    const bool auto_shape = D.bucket_modes != 0 && D.lanes <= 0 && D.vec <= 0;
    tile.lanes = auto_shape ? 0 : f->lanes;
    tile.vec = auto_shape ? 0 : f->vec;
    tile.lds_modes = -1;       // the per-launch automatic choice
    tile.bucket_modes = D.bucket_modes;
    for (int j = 0; j < D.tau; ++j) {
        for (int c = 0; c < D.nclients; ++c) {
            const gcp_fed_client& cl = f->clients[c];
            gcp_sample_params sp{};
            sp.kind = GCP_SAMPLE_STRATIFIED;
            sp.max_attempts = D.max_attempts;
            sp.p = D.p;
            sp.q = D.q;
            sp.seed = D.seed;
            sp.step = (uint64_t)(round * D.tau + j);
            sp.client = (uint64_t)c;
            gcp_status st = gcp_loss_grad(cl.tensor, &sp, nullptr, cl.M, D.R, (gcp_loss)D.loss, GCP_ACCUMULATE,
                                          nullptr, cl.G, nullptr, &tile, stream);
            if (st != GCP_OK) return st;
            st = gcp_adam_step(cl.M, cl.G, cl.B, cl.C, cl.tensor->rowoff[f->d] * D.R, f->dt, round * D.tau + j + 1,
                               D.lr, D.beta1, D.beta2, D.eps, D.lower, GCP_ADAM_ZERO_GRAD, stream);
            if (st != GCP_OK) return st;
        }
    }
    const int64_t sb = std::max<int64_t>(1, std::min<int64_t>(ceil_div(f->nserver, 256), 2048));
    k_fed_server<T><<<(unsigned)sb, 256, 0, stream>>>(a);
    GCP_HIP(hipGetLastError());
    return GCP_OK;
}

static void fed_free(gcp_fed_s* f)
{
    if (!f) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(f->device);
    (void)hipDeviceSynchronize();
    if (f->exec) (void)hipGraphExecDestroy(f->exec);
    if (f->graph) (void)hipGraphDestroy(f->graph);
    void* ptrs[] = {f->dev_clients, f->dev_mptrs, f->barrier, f->round, f->status, f->cov_ptr, f->cov_client,
                    f->cov_lrow, f->bucket_ws};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (f->status_host) (void)hipHostFree(f->status_host);
    (void)hipSetDevice(cur);
    delete f;
}

}  // namespace gcp

extern "C" {

gcp_status gcp_fedadam_create(gcp_fed* out, const gcp_fed_desc* desc, hipStream_t stream)
{
    clear_error();
    (void)stream;
    if (!out || !desc) return set_error(GCP_ERR_ARG, "NULL argument");
    *out = nullptr;
    const gcp_fed_desc& D = *desc;
    if (D.nclients < 1 || !D.clients) return set_error(GCP_ERR_ARG, "no clients");
    if (D.R < 1 || D.R > 256) return set_error(GCP_ERR_ARG, "R = %d outside [1, 256]", D.R);
    if (D.tau < 1) return set_error(GCP_ERR_ARG, "tau = %d < 1", D.tau);
    if (D.loss < GCP_LOSS_GAUSSIAN || D.loss > GCP_LOSS_BERNOULLI_LOGIT) return set_error(GCP_ERR_ARG, "loss");
    if (D.p < 0 || D.q < 0) return set_error(GCP_ERR_ARG, "negative sample count");
    if (!D.U || !D.Bs || !D.Cs) return set_error(GCP_ERR_ARG, "server buffers are NULL");
    if (!(D.beta1 >= 0 && D.beta1 < 1) || !(D.beta2 >= 0 && D.beta2 < 1) || !(D.eps >= 0))
        return set_error(GCP_ERR_ARG, "Adam constants");
    gcp_fed_s* f = new (std::nothrow) gcp_fed_s();
    if (!f) return set_error(GCP_ERR_OOM, "host allocation");
    f->desc = D;
    f->clients.assign(D.clients, D.clients + D.nclients);
    f->desc.clients = nullptr;
    (void)hipGetDevice(&f->device);
    const gcp_tensor_s* t0 = D.clients[0].tensor;
    if (!t0) { delete f; return set_error(GCP_ERR_ARG, "client 0 has no tensor"); }
    f->dt = t0->dt;
    f->d = t0->d;
    for (int c = 0; c < D.nclients; ++c) {
        const gcp_fed_client& cl = D.clients[c];
        const gcp_tensor_s* t = cl.tensor;
        if (!t || t->dense || t->dt != f->dt || t->d != f->d) {
            delete f;
            return set_error(GCP_ERR_ARG, "client %d: tensor missing, dense, or of another dtype or order", c);
        }
        if (!cl.M || !cl.B || !cl.C || !cl.G) { delete f; return set_error(GCP_ERR_ARG, "client %d: NULL buffer", c); }
        if (D.q > 0 && (uint64_t)t->nnz >= t->cells) {
            delete f;
            return set_error(GCP_ERR_ARG, "client %d: q > 0 but the block has no zero cells", c);
        }
        for (int k = 0; k < f->d; ++k) {
            if (cl.row_base[k] < 0 || cl.row_base[k] + t->dims[k] > D.global_dims[k]) {
                delete f;
                return set_error(GCP_ERR_ARG, "client %d: block outside the global dims in mode %d", c, k);
            }
        }
    }
    const int esize = f->dt == GCP_F32 ? 4 : 8;
    // row-bucketed batched rounds: on request, or automatically at enough
    // samples per client step
    f->want_bucket = D.batched && (D.bucket_modes > 0 || (D.bucket_modes < 0 && D.p + D.q >= kFedBucketMinSamples));
    f->block = D.block > 0 ? D.block : (f->want_bucket ? 1024 : 256);
    if (f->block % 64 != 0 || f->block > 1024) { delete f; return set_error(GCP_ERR_ARG, "block = %d", f->block); }
    // lane shape: one column per lane up to R = 64 (coalesced gradient
    // atomics), else the fewest columns per lane that let 64 lanes cover R;
    // with the row-bucketed scatter, which issues no gradient atomics for its
    // modes, four columns per lane in FP32
    const bool wide = f->want_bucket && f->dt == GCP_F32 && D.R % 4 == 0 && D.R <= 64;
    int vec_auto = 1;
    while (vec_auto < 4 && 64 * vec_auto < D.R) vec_auto *= 2;
    f->vec = D.vec > 0 ? D.vec : wide ? 4 : vec_auto;
    if (D.lanes > 0) f->lanes = D.lanes;
    else if (wide && D.vec <= 0) f->lanes = D.R <= 32 ? 8 : 16;
    else {
        const int need = (D.R + f->vec - 1) / f->vec;
        f->lanes = 8;
        while (f->lanes < need && f->lanes < 64) f->lanes <<= 1;
    }
    if (D.R % f->vec != 0 || f->lanes * f->vec < D.R) {
        delete f;
        return set_error(GCP_ERR_ARG, "lane shape %d x %d does not cover R = %d", f->lanes, f->vec, D.R);
    }
    // the automatic count is set once the kernel is chosen (its occupancy)
    if (D.batched) f->W = D.workgroups_per_client > 0 ? D.workgroups_per_client : 1;
    (void)esize;
    gcp_status st = f->dt == GCP_F32 ? fed_build<float>(f) : fed_build<double>(f);
    if (st != GCP_OK) {
        fed_free(f);
        return st;
    }
    *out = f;
    return GCP_OK;
}

gcp_status gcp_fedadam_round(gcp_fed f, int64_t round, hipStream_t stream)
{
    clear_error();
    if (!f) return set_error(GCP_ERR_ARG, "handle is NULL");
    if (round < 0) return set_error(GCP_ERR_ARG, "round < 0");
    // a barrier failure of an earlier batched round, once copied back
    if (__atomic_load_n(f->status_host, __ATOMIC_RELAXED) & kStatusBarrier)
        return set_error(GCP_ERR_HIP, "an earlier round's group barrier timed out; gcp_fedadam_status clears it");
    k_fed_set_round<<<1, 1, 0, stream>>>(f->round, round);
    GCP_HIP(hipGetLastError());
    if (!f->desc.batched) return f->dt == GCP_F32 ? fed_round_plain<float>(f, round, stream)
                                                  : fed_round_plain<double>(f, round, stream);
    if (!f->desc.use_graph) {
        gcp_status st = f->dt == GCP_F32 ? fed_launch_batched<float>(f, stream) : fed_launch_batched<double>(f, stream);
        if (st != GCP_OK) return st;
        GCP_HIP(hipMemcpyAsync(f->status_host, f->status, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
        return GCP_OK;
    }
    if (!stream) return set_error(GCP_ERR_ARG, "use_graph needs a non-default stream");
    if (f->exec && f->graph_stream != stream) return set_error(GCP_ERR_ARG, "the graph was captured on another stream");
    if (!f->exec) {
        GCP_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
        gcp_status st = f->dt == GCP_F32 ? fed_launch_batched<float>(f, stream) : fed_launch_batched<double>(f, stream);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(stream, &g);
        if (st != GCP_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return hip_error(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&f->exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g);
            f->exec = nullptr;
            return hip_error(e, "hipGraphInstantiate");
        }
        f->graph = g;
        f->graph_stream = stream;
    }
    GCP_HIP(hipGraphLaunch(f->exec, stream));
    GCP_HIP(hipMemcpyAsync(f->status_host, f->status, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
    return GCP_OK;
}

gcp_status gcp_fedadam_status(gcp_fed f, hipStream_t stream)
{
    clear_error();
    if (!f) return set_error(GCP_ERR_ARG, "handle is NULL");
    GCP_HIP(hipStreamSynchronize(stream));
    uint32_t hs = 0;
    GCP_HIP(hipMemcpy(&hs, f->status, sizeof(hs), hipMemcpyDeviceToHost));
    if (hs) GCP_HIP(hipMemset(f->status, 0, sizeof(uint32_t)));
    __atomic_store_n(f->status_host, 0u, __ATOMIC_RELAXED);
    gcp_status worst = GCP_OK;
    for (const gcp_fed_client& cl : f->clients) {
        gcp_status st = gcp_device_status(cl.tensor, stream);
        if (st != GCP_OK) worst = st;
    }
    if (hs & kStatusBarrier)
        return set_error(GCP_ERR_HIP, "a batched round's group barrier timed out (workgroups not co-resident)");
    if (worst != GCP_OK) return set_error(worst, "a client tensor reported a device error");
    return GCP_OK;
}

int64_t gcp_struct_size(const char* name)
{
    if (!name) return -1;
    if (!strcmp(name, "gcp_sample_params")) return sizeof(gcp_sample_params);
    if (!strcmp(name, "gcp_samples")) return sizeof(gcp_samples);
    if (!strcmp(name, "gcp_tile")) return sizeof(gcp_tile);
    if (!strcmp(name, "gcp_fed_client")) return sizeof(gcp_fed_client);
    if (!strcmp(name, "gcp_fed_desc")) return sizeof(gcp_fed_desc);
    if (!strcmp(name, "gcp_fed_info")) return sizeof(gcp_fed_info);
    return -1;
}

gcp_status gcp_fedadam_info(gcp_fed f, gcp_fed_info* out)
{
    clear_error();
    if (!f || !out) return set_error(GCP_ERR_ARG, "NULL argument");
    gcp_fed_info i{};
    const gcp_fed_desc& D = f->desc;
    const int64_t K = D.nclients;
    if (!D.batched) {
        i.form = GCP_FED_PER_CLIENT;
        i.lds_modes = -1;
        i.bucket_modes = D.bucket_modes;
        if (D.bucket_modes != 0 && D.lanes <= 0 && D.vec <= 0) {
            // the lane shape is each call's own choice
            *out = i;
            out->workgroups_per_client = 0;
            out->block = 0;
            out->lanes = 0;
            out->vec = 0;
            out->launches_per_round = 3 + K * D.tau * 3;
            return GCP_OK;
        }
        // round number, copy, server; per client and step the gradient (one
        // launch, two when it row-buckets) and Adam
        i.launches_per_round = 3 + K * D.tau * (D.bucket_modes != 0 ? 3 : 2);
    } else if (f->bucketed) {
        i.form = GCP_FED_ROW_BUCKETED;
        i.lds_modes = (int32_t)f->lds_mask;
        i.bucket_modes = (int32_t)f->bucket_mask;
        i.bucket_block_samples = f->spb;
        i.launches_per_round = 1 + 1 + 3 * (int64_t)D.tau + 1;
    } else {
        i.form = GCP_FED_PERSISTENT;
        i.lds_modes = (int32_t)f->lds_mask;
        i.bucket_modes = 0;
        i.launches_per_round = 1 + 1 + 1;
    }
    i.workgroups_per_client = D.batched ? f->W : 0;
    i.block = f->block;
    i.lanes = f->lanes;
    i.vec = f->vec;
    *out = i;
    return GCP_OK;
}

gcp_status gcp_fedadam_destroy(gcp_fed f)
{
    clear_error();
    if (!f) return set_error(GCP_ERR_ARG, "handle is NULL");
    fed_free(f);
    return GCP_OK;
}

}  // extern "C"
