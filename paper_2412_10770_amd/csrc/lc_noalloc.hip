// lc_compress_noalloc: lc_compress with its workspace in a static device
// array of the library instead of a caller buffer, for callers that cannot
// allocate device memory (code under graph capture, tight serving loops,
// harnesses that forbid hipMalloc).  The array is a file-scope __device__
// variable: every GPU the library runs on holds its own copy, at its own
// address, until the process ends.  In host code the array's name is only a
// host-side stand-in, so its device address is looked up once per device
// with hipGetSymbolAddress and only that address is ever handed to kernels.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "lc.h"

#define LC_API extern "C" __attribute__((visibility("default")))

namespace {

static_assert(LC_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size must keep 256-byte alignment");

// The workspace of every lc_compress_noalloc call on this device.  Nothing in
// it needs to start at zero: the compress kernels write every workspace byte
// they read (block infos, tile sums, segment records) earlier in the same call.
static __device__ __align__(256) uint8_t scratch[LC_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices];  // device address of `scratch` per device (null until looked up)

// Device address of this device's scratch array, looked up on the first call
// made with the device current and kept for the rest of the process.
lc_status scratch_address(void** out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return LC_EDEVICE;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return LC_EDEVICE;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return LC_OK;
}

}  // namespace

LC_API lc_status lc_compress_noalloc(const void* d_keys, uint64_t n, const lc_params* p, void* d_blob,
                                     uint64_t blob_cap, uint64_t* d_blob_bytes, uint32_t* d_flags, void* stream)
{
    uint64_t ws_bytes = 0;
    lc_status st = lc_compress_bound(n, p, nullptr, &ws_bytes);
    if (st != LC_OK) return st;
    if (ws_bytes > LC_NOALLOC_SCRATCH_BYTES) return LC_ETOOBIG;
    void* ws = nullptr;
    st = scratch_address(&ws);
    if (st != LC_OK) return st;
    return lc_compress(d_keys, n, p, d_blob, blob_cap, ws, LC_NOALLOC_SCRATCH_BYTES, d_blob_bytes, d_flags, stream);
}
