// gcp_loss_grad_noalloc: gcp_loss_grad for callers that cannot allocate
// device memory (code under HIP graph capture, serving loops, harnesses that
// forbid hipMalloc).  The row-bucketed scatter's sample entries and
// per-(row block, workgroup) counts and starts live in one file-scope device
// array, `scratch`, instead of a gcp_tensor_reserve workspace.
//
// Host code never passes `scratch` itself to a kernel: on the host that name
// is a stand-in, not the device address.  The address is looked up once per
// device with hipGetSymbolAddress (with that device current) and kept; each
// GPU holds its own copy of the array at its own address until the process
// ends.  Every call on one GPU shares that GPU's copy.  Nothing in it needs to
// start at zero: the sampling kernel writes every count and start the owner
// pass reads, and every entry it points at, before they are read.
#include <mutex>

#include "gcp_internal.hpp"

namespace gcp {
namespace {

constexpr int64_t kScratchBytes = int64_t(128) << 20;
constexpr int kMaxDevices = 64;

__device__ __attribute__((used)) __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device`, looked up on the first call for
// that device.
gcp_status scratch_on(int device, void** out)
{
    if (device < 0 || device >= kMaxDevices) return set_error(GCP_ERR_UNSUPPORTED, "device %d", device);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = 0;
        GCP_HIP(hipGetDevice(&cur));
        if (cur != device) GCP_HIP(hipSetDevice(device));
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != device) GCP_HIP(hipSetDevice(cur));
        if (e != hipSuccess) return hip_error(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return set_error(GCP_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return GCP_OK;
}

}  // namespace
}  // namespace gcp

extern "C" int64_t gcp_noalloc_scratch_bytes(void) { return gcp::kScratchBytes; }

extern "C" gcp_status gcp_loss_grad_noalloc(gcp_tensor t, const gcp_sample_params* sp, const gcp_samples* smp,
                                            const void* A, int R, gcp_loss loss, unsigned flags,
                                            const void* scale_dev, void* G_out, double* loss_out,
                                            const gcp_tile* tile, hipStream_t stream)
{
    gcp::clear_error();
    if (!t) return gcp::set_error(GCP_ERR_ARG, "tensor is NULL");
    if (flags & GCP_DETERMINISTIC)
        return gcp::set_error(GCP_ERR_UNSUPPORTED, "GCP_DETERMINISTIC needs the workspace of gcp_tensor_reserve");
    gcp::LGWorkspace ws;
    gcp_status st = gcp::scratch_on(t->device, &ws.base);
    if (st != GCP_OK) return st;
    ws.scratch_bytes = gcp::kScratchBytes;
    return gcp::loss_grad_with_workspace(t, sp, smp, A, R, loss, flags, scale_dev, G_out, loss_out, tile, ws, stream);
}
