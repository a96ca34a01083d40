// Allocation-free variant of poly_simplify: the workspace is a fixed array in
// device memory that the library owns, so the caller allocates nothing.
//
// `scratch` is a file-scope device array.  Its name in host code is only a
// stand-in for the registration of the symbol, not a device address: every
// use from host code goes through the address hipGetSymbolAddress returns
// for the current device, fetched once per device and kept.
#include <mutex>

#include "kernels.h"

using namespace polyhip;

namespace {

constexpr size_t kScratchBytes = POLY_NOALLOC_SCRATCH_BYTES;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {nullptr};

// Device address of `scratch` on the current device (set-up on the first
// call made with that device current).
poly_status scratch_address(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return POLY_ERR_HIP;
    if (dev < 0 || dev >= kMaxDevices) return POLY_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return POLY_ERR_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return POLY_OK;
}

// The device status word (first bytes of the workspace) to the caller.
__global__ void k_copy_status(const int32_t *ws_status, int32_t *out)
{
    if (threadIdx.x == 0) *out = *ws_status;
}

}  // namespace

extern "C" poly_status poly_simplify_noalloc(const poly_csr *in, poly_csr *out, double zero_tol, int32_t *status,
                                             void *stream)
{
    // every size check runs on the host before the device is touched
    size_t need = 0;
    poly_status st = poly_simplify_workspace(in, &need);
    if (st != POLY_OK) return st;
    if (need > kScratchBytes) return POLY_ERR_SCRATCH;
    void *ws = nullptr;
    if ((st = scratch_address(&ws)) != POLY_OK) return st;
    st = poly_simplify(in, out, zero_tol, ws, kScratchBytes, stream);
    if (st != POLY_OK) return st;
    if (status) {
        hipLaunchKernelGGL(k_copy_status, dim3(1), dim3(64), 0, (hipStream_t)stream, (const int32_t *)ws, status);
        if (hipGetLastError() != hipSuccess) return POLY_ERR_HIP;
    }
    return POLY_OK;
}
