// noalloc.hip -- compression for callers that cannot allocate device memory
// (code under stream capture, tight serving loops, hosts that forbid it).
//
// ebc_compress_async_noalloc is ebc_compress_async with its workspace taken
// from a fixed device array of this library instead of a caller's buffer.
// The kernels are the same; only where the scratch lives differs.
//
// The array is a device symbol: host code must not use its name as an
// address.  Its device address is resolved once per device, with that device
// current, by hipGetSymbolAddress, and only that address reaches the kernels.
// Every call on a device shares the one array and leaves its contents behind;
// the pipeline initialises everything it reads, so stale contents are harmless,
// but two calls that overlap in time on one device (different streams, no
// ordering between them) race on the array.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ebc.h"
#include "ebc_launch.h"

namespace {

constexpr uint64_t kScratchBytes = EBC_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices];  // device address of `scratch` on each device, once resolved

// Address of the array on the current device (nullptr after a HIP error,
// which is recorded for ebc_last_error).
void* scratch_ptr(int* status)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        *status = ebc::set_error(EBC_ERR_HIP, "hipGetDevice failed: %s", hipGetErrorString(e));
        return nullptr;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        *status = ebc::set_error(EBC_ERR_UNSUPPORTED, "device %d beyond the %d the fixed scratch tracks",
                                 dev, kMaxDevices);
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            *status = ebc::set_error(EBC_ERR_HIP, "hipGetSymbolAddress(scratch) failed on device %d: %s",
                                     dev, hipGetErrorString(e));
            return nullptr;
        }
        g_scratch[dev] = p;
    }
    return g_scratch[dev];
}

}  // namespace

extern "C" int ebc_compress_async_noalloc(const void* d_field, int rank, const uint64_t dims[3],
                                          const ebc_params* p, void* d_out, uint64_t out_cap,
                                          uint64_t* d_result, void* stream)
{
    if (!dims || !p) return ebc::set_error(EBC_ERR_ARG, "NULL argument");
    uint64_t need = 0;
    int st = ebc_compress_workspace_size(rank, dims, p, &need);
    if (st) return st;
    if (need > kScratchBytes)
        return ebc::set_error(EBC_ERR_WS_TOO_SMALL,
                              "field needs %llu bytes of scratch; the fixed array holds %llu "
                              "(use ebc_compress_async with a workspace)",
                              (unsigned long long)need, (unsigned long long)kScratchBytes);
    void* ws = scratch_ptr(&st);
    if (!ws) return st;
    return ebc_compress_async(d_field, rank, dims, p, d_out, out_cap, d_result, ws, kScratchBytes, stream);
}
