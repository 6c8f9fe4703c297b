// gres_compute_noalloc: gres_compute with its workspace in a fixed device array of this library,
// for callers that cannot allocate device memory (code under graph capture, serving loops,
// harnesses that forbid allocation).
//
// The array lives in device memory for as long as the library is loaded; every device the
// library runs on holds its own copy at its own address. Host code never passes the array's
// name to a kernel (on the host it is only a stand-in for the symbol): the device address is
// taken once per device with hipGetSymbolAddress and kept in g_scratch_ptr.
#include <mutex>

#include "sky_plan.hpp"

namespace {

__device__ __align__(256) unsigned char scratch[SKY_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch` (looked up on the first call per
// device, with that device current).
sky_status scratch_of_current_device(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return SKY_ERR_HIP;
    if (dev >= kMaxDevices) return SKY_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SKY_ERR_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SKY_OK;
}

}  // namespace

extern "C" sky_status gres_compute_noalloc(const float* x_soa, int64_t n, int32_t d, int64_t ld,
                                           const int64_t* sky_idx, int64_t s, int32_t g_max,
                                           int32_t* g_exit, float* gres, int32_t* dev_status,
                                           const sky_gres_opts* opts, void* stream) {
    if (s < 0 || s > sky::kMaxBuildRows || d < 1 || d > SKY_MAX_D || g_max < 2 || g_max > SKY_MAX_G ||
        !dev_status)
        return SKY_ERR_INVALID_ARG;
    if (s == 0) return gres_compute(x_soa, n, d, ld, sky_idx, s, g_max, g_exit, gres, nullptr, 0,
                                    dev_status, opts, stream);
    // the packed key table of the tile search when it fits beside the rest, else without it
    const size_t need = sky::gres_ws_bytes(s, d, g_max, false);
    if (need == 0) return SKY_ERR_INVALID_ARG;
    if (need > (size_t)SKY_NOALLOC_SCRATCH_BYTES) return SKY_ERR_UNSUPPORTED;
    const bool keys = sky::gres_ws_bytes(s, d, g_max, true) <= (size_t)SKY_NOALLOC_SCRATCH_BYTES;
    void* ws = nullptr;
    SKY_TRY(scratch_of_current_device(&ws));
    // gres_compute writes every workspace word it reads (the search's work counters are
    // cleared by a kernel before each launch, the key table is rebuilt by every search), so the
    // previous call's contents do not matter
    return sky::gres_compute_ws(x_soa, n, d, ld, sky_idx, s, g_max, g_exit, gres, ws,
                                (size_t)SKY_NOALLOC_SCRATCH_BYTES, keys, dev_status, opts, (hipStream_t)stream);
}
