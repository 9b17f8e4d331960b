// gfq_noalloc.hip -- gfq_matmul_noalloc: the product of gfq_matmul_config for callers that
// cannot allocate device memory.  Where the inner dimension is split, the slices' partial
// products go to `scratch`, a fixed array of this library in every device's memory, instead
// of the workspace gfq_matmul allocates.
#include <hip/hip_runtime.h>

#include <mutex>

#include "gfq.h"
#include "gfq_host.h"
#include "gfq_internal.h"

using namespace gfq;

namespace {

// One copy per device, at its own address on each; host code never uses the name itself
// (in host code it stands for a host-side placeholder, not a device address) but the
// address hipGetSymbolAddress returns for the current device.
__device__ __align__(256) unsigned char scratch[GFQ_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void *g_scratch_ptr[MAX_DEVICES];   // device address of `scratch`, per device, once looked up

// The current device's address of `scratch`; looked up on the first call on a device,
// with that device current.
int scratch_address(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= MAX_DEVICES) return GFQ_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return GFQ_EHIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return GFQ_OK;
}

}  // namespace

extern "C" int gfq_matmul_noalloc(int q, int64_t m, int64_t l, int64_t n, const void *A, const void *B, void *C,
                                  const gfq_config *cfg) {
    // validation first, so that no call with bad arguments touches the device
    int st = validate_mm(q, m, l, n, A, B, C);
    if (st != GFQ_OK) return st;
    if (cfg) {
        st = check_config(q, *cfg);
        if (st != GFQ_OK) return st;
    }
    void *ws = nullptr;
    st = scratch_address(&ws);
    if (st != GFQ_OK) return st;
    return matmul_into(q, m, l, n, A, B, C, cfg, ws, (size_t)GFQ_NOALLOC_SCRATCH_BYTES);
}
