// The entry point that allocates nothing: imin_solve_static, an enqueued
// solve (imin_solve with a workspace) whose workspace is a fixed array of
// device memory that the library itself declares.
//
// The array, `scratch`, exists once per device (the loader places a copy on
// every GPU the library runs on, held until the process ends).  Host code
// never uses its name as an address: on a device's first call its address on
// that device is looked up with hipGetSymbolAddress, with that device
// current, and kept in a per-device table.  Every call on a device uses that
// device's one copy, so calls that overlap on one GPU would race; each call
// clears or overwrites everything it reads from the array with kernels of
// its own before reading it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "imin.h"
#include "imin_internal.hpp"

namespace {

constexpr size_t kStaticScratchBytes = (size_t)256 << 20;  // 256 MiB
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// the address of `scratch` on device dev (the current device), looked up
// once per device
imin_status_t scratch_on(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return IMIN_ERR_INVALID;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return IMIN_ERR_DEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return IMIN_OK;
}

}  // namespace

extern "C" imin_status_t imin_solve_static(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, int32_t k,
                                           int64_t theta, uint64_t rng_seed, void* stream, int32_t* blockers,
                                           int64_t* gains, int64_t* spread_totals, int32_t* n_selected,
                                           int32_t* device_status) {
    if (!g) return IMIN_ERR_INVALID;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return IMIN_ERR_DEVICE;
    }
    if (dev != imin::graph_device(g)) return IMIN_ERR_INVALID;  // the graph's device must be current
    void* ws = nullptr;
    const imin_status_t st = scratch_on(dev, &ws);
    if (st != IMIN_OK) return st;
    return imin::solve_enqueued(g, seeds, n_seeds, k, theta, rng_seed, ws, kStaticScratchBytes, stream, blockers,
                                gains, spread_totals, n_selected, device_status);
}
