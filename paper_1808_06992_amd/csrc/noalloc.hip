// Allocation-free form of the batched LASSO solves (uoi_lasso_solve_batch):
// the scratch memory is a fixed static device array instead of the library's
// grow-only pool, and the host side uses no pinned memory, events or second
// stream, so a call allocates nothing.  Meant for callers that cannot allocate
// (code under stream capture, tight serving loops, harnesses that forbid it).
//
// The array lives in this code object; every device the library runs on holds
// its own copy until the process ends.  In host code its name is only a
// stand-in symbol, so the device address of each copy is looked up once per
// device (hipGetSymbolAddress, with that device current) and only that address
// is handed to kernels.  Calls on one device share the array: the solve clears
// or overwrites every part of it that it reads, and calls that overlap on one
// device race.
#include <map>
#include <mutex>

#include "common.hpp"

namespace uoi {

constexpr size_t kNoAllocScratchBytes = UOI_NOALLOC_SCRATCH_BYTES;  // per device

static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;  // device -> address of its copy of `scratch`

// Device address of the current device's copy, looked up on the first call.
void *scratch_device_ptr() {
    int dev = 0;
    UOI_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) return it->second;
    void *ptr = nullptr;
    UOI_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    UOI_REQUIRE(ptr != nullptr, "no device address for the static scratch buffer");
    g_scratch_ptr[dev] = ptr;
    return ptr;
}
}  // namespace

}  // namespace uoi

using namespace uoi;

extern "C" int uoi_lasso_solve_batch_noalloc(int32_t nb, int32_t p, const double *G, const double *c,
                                             const uoi_opts *o, const double *z0, const double *u0,
                                             double *z_out, double *u_out, int32_t *iters, double *kkt) {
    return guarded([&] {
        return solve_batch(nb, p, G, c, o, z0, u0, z_out, u_out, iters, kkt, scratch_device_ptr,
                           kNoAllocScratchBytes);
    });
}
