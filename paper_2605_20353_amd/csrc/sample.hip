// gcp_sample: materialise the sampled tensor (Sec. 3.1.1) -- coordinates,
// values and weights of the p + q samples, nonzero samples first.  One lane
// per sample; preallocated output written without synchronisation, as the
// paper describes for its sampler.
#include "sampling.hpp"

namespace gcp {

template <typename T, int D>
__global__ void __launch_bounds__(256) k_sample(SampleCtx<T> c, int64_t n, int64_t* __restrict__ coords,
                                                T* __restrict__ xo, T* __restrict__ wo)
{
    const int dd = D > 0 ? D : c.d;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (int64_t)gridDim.x * blockDim.x) {
        uint64_t key;
        T x, w;
        draw_sample<T, D>(c, c.step, s, key, x, w);
        constexpr int DM = D > 0 ? D : kMaxModes;
        uint32_t ci[DM];
        unpack_all<D == 0>(c.L, dd, key, ci);
#pragma unroll
        for (int k = 0; k < DM; ++k)
            if (k < dd) coords[s * dd + k] = (int64_t)ci[k];
        xo[s] = x;
        wo[s] = w;
    }
}

template <typename T>
static gcp_status launch_sample(const gcp_tensor_s* t, const gcp_sample_params* sp, int64_t* coords, void* x,
                                void* w, hipStream_t stream)
{
    SampleCtx<T> c;
    int64_t n = 0;
    gcp_status st = make_sample_ctx<T>(t, sp, c, n);
    if (st != GCP_OK) return st;
    if (n == 0) return GCP_OK;
    if (!coords || !x || !w) return set_error(GCP_ERR_ARG, "output pointer is NULL");
    int64_t blocks = std::min<int64_t>(ceil_div(n, 256), (int64_t)device_cu_count(t->device) * 16);
    const int order = kernel_order(t);
    if (order == 3)
        k_sample<T, 3><<<(unsigned)blocks, 256, 0, stream>>>(c, n, coords, (T*)x, (T*)w);
    else if (order == 4)
        k_sample<T, 4><<<(unsigned)blocks, 256, 0, stream>>>(c, n, coords, (T*)x, (T*)w);
    else
        k_sample<T, 0><<<(unsigned)blocks, 256, 0, stream>>>(c, n, coords, (T*)x, (T*)w);
    GCP_HIP(hipGetLastError());
    return GCP_OK;
}

}  // namespace gcp

extern "C" gcp_status gcp_sample(gcp_tensor t, const gcp_sample_params* sp, int64_t* coords_out, void* x_out,
                                 void* w_out, hipStream_t stream)
{
    gcp::clear_error();
    if (!t) return gcp::set_error(GCP_ERR_ARG, "tensor is NULL");
    if (t->dt == GCP_F32) return gcp::launch_sample<float>(t, sp, coords_out, x_out, w_out, stream);
    return gcp::launch_sample<double>(t, sp, coords_out, x_out, w_out, stream);
}
