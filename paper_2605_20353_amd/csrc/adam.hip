// gcp_adam_step: Alg. adam-update in one launch over the single contiguous
// parameter vector of all modes (Sec. 3.1.3).  Streaming, HBM bound: 16-byte
// vector accesses, grid-stride, the bias corrections folded into two scalars
// computed on the host.
#include <math.h>

#include <algorithm>

#include "gcp_internal.hpp"

namespace gcp {

template <typename T>
struct AdamArgs {
    T* A;
    T* G;
    T* B;
    T* C;
    int64_t n;
    T lr, b1, b2, one_m_b1, one_m_b2, c1, c2, eps, lower;
    int zero_grad;
};

template <typename T>
__device__ __forceinline__ void adam_elem(const AdamArgs<T>& a, T& p, T g, T& b, T& c)
{
    adam_update<T>(p, g, b, c, a.lr, a.b1, a.b2, a.one_m_b1, a.one_m_b2, a.c1, a.c2, a.eps, a.lower);
}

template <typename T>
__global__ void __launch_bounds__(256) k_adam(const AdamArgs<T> a)
{
    constexpr int V = 16 / sizeof(T);
    const int64_t nv = a.n / V;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool aligned = ((uintptr_t)a.A | (uintptr_t)a.G | (uintptr_t)a.B | (uintptr_t)a.C) % 16 == 0;
    if (aligned) {
        typedef T vec_t __attribute__((ext_vector_type(V)));
        for (int64_t i = t0; i < nv; i += stride) {
            vec_t p = reinterpret_cast<vec_t*>(a.A)[i];
            vec_t g = reinterpret_cast<const vec_t*>(a.G)[i];
            vec_t b = reinterpret_cast<vec_t*>(a.B)[i];
            vec_t c = reinterpret_cast<vec_t*>(a.C)[i];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                T pv = p[v], bv = b[v], cv = c[v];
                adam_elem(a, pv, g[v], bv, cv);
                p[v] = pv; b[v] = bv; c[v] = cv;
            }
            reinterpret_cast<vec_t*>(a.A)[i] = p;
            reinterpret_cast<vec_t*>(a.B)[i] = b;
            reinterpret_cast<vec_t*>(a.C)[i] = c;
            if (a.zero_grad) reinterpret_cast<vec_t*>(a.G)[i] = vec_t(0);
        }
    }
    for (int64_t i = (aligned ? nv * V : 0) + t0; i < a.n; i += stride) {
        T p = a.A[i], b = a.B[i], c = a.C[i];
        adam_elem(a, p, a.G[i], b, c);
        a.A[i] = p;
        a.B[i] = b;
        a.C[i] = c;
        if (a.zero_grad) a.G[i] = T(0);
    }
}

template <typename T>
static gcp_status launch_adam(void* A, void* G, void* B, void* C, int64_t n, int64_t t, double lr, double beta1,
                              double beta2, double eps, double lower, unsigned flags, hipStream_t stream)
{
    AdamArgs<T> a;
    a.A = (T*)A;
    a.G = (T*)G;
    a.B = (T*)B;
    a.C = (T*)C;
    a.n = n;
    a.lr = (T)lr;
    a.b1 = (T)beta1;
    a.b2 = (T)beta2;
    a.one_m_b1 = (T)(1.0 - beta1);
    a.one_m_b2 = (T)(1.0 - beta2);
    a.c1 = (T)(1.0 - pow(beta1, (double)t));
    a.c2 = (T)(1.0 - pow(beta2, (double)t));
    a.eps = (T)eps;
    a.lower = (T)lower;
    a.zero_grad = (flags & GCP_ADAM_ZERO_GRAD) ? 1 : 0;
    int dev = 0;
    (void)hipGetDevice(&dev);
    const int64_t work = ceil_div(n, 16 / (int64_t)sizeof(T));
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(ceil_div(work, 256), (int64_t)device_cu_count(dev) * 8));
    k_adam<T><<<(unsigned)blocks, 256, 0, stream>>>(a);
    GCP_HIP(hipGetLastError());
    return GCP_OK;
}

}  // namespace gcp

extern "C" gcp_status gcp_adam_step(void* A, void* G, void* B, void* C, int64_t n, gcp_dtype dt, int64_t t,
                                    double lr, double beta1, double beta2, double eps, double lower, unsigned flags,
                                    hipStream_t stream)
{
    gcp::clear_error();
    if (n < 0) return gcp::set_error(GCP_ERR_ARG, "n < 0");
    if (n == 0) return GCP_OK;
    if (!A || !G || !B || !C) return gcp::set_error(GCP_ERR_ARG, "NULL array");
    if (t < 1) return gcp::set_error(GCP_ERR_ARG, "t = %lld < 1", (long long)t);
    if (!(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0))
        return gcp::set_error(GCP_ERR_ARG, "betas outside [0, 1)");
    if (!(eps >= 0.0)) return gcp::set_error(GCP_ERR_ARG, "eps < 0");
    if (flags & ~GCP_ADAM_ZERO_GRAD) return gcp::set_error(GCP_ERR_ARG, "unknown flags 0x%x", flags);
    if (dt == GCP_F32) return gcp::launch_adam<float>(A, G, B, C, n, t, lr, beta1, beta2, eps, lower, flags, stream);
    if (dt == GCP_F64) return gcp::launch_adam<double>(A, G, B, C, n, t, lr, beta1, beta2, eps, lower, flags, stream);
    return gcp::set_error(GCP_ERR_ARG, "dtype %d", (int)dt);
}
