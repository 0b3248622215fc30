// Subband dedispersion without caller scratch: step one's sums go to a
// file-scope device array instead of a caller-provided work buffer, for
// callers that cannot allocate device memory.
//
// The array is part of the library's code object: every GPU the library runs
// on holds its own copy (kStaticWorkBytes) until the process ends.  Host code
// never passes the array's name to a kernel (on the host it is only a stand-in
// for the symbol); the device address of each GPU's copy is looked up once per
// device with hipGetSymbolAddress, with that device current, and kept.  Every
// call on a GPU shares that GPU's copy, so calls that overlap on one GPU (on
// different streams, or from different threads) race on it.  Step one writes
// every element step two reads, so nothing needs clearing between calls.
#include <mutex>

#include "internal.h"

namespace amber {
namespace {
constexpr int64_t kStaticWorkBytes = (int64_t)32 << 20;
}  // namespace
}  // namespace amber

static __device__ __align__(256) uint32_t scratch[amber::kStaticWorkBytes / 4];

namespace amber {
namespace {

constexpr int kMaxDevices = 64;

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The current device's copy of `scratch`.
amber_status scratch_address(void **out)
{
    int dev = -1;
    AMBER_HIP(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(AMBER_E_DEVICE, "device index %d outside [0, %d)", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        AMBER_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!p) return fail(AMBER_E_DEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return AMBER_OK;
}

}  // namespace
}  // namespace amber

using namespace amber;

extern "C" {

int64_t amber_subband_static_bytes(void) { return kStaticWorkBytes; }

amber_status amber_subband_dedisperse_noalloc(const int32_t *d_delay1, const int32_t *d_delay2,
                                              const amber_subband_info *info, const uint8_t *d_in,
                                              int64_t in_stride, int64_t n_in, int32_t *d_dd, int64_t dd_stride,
                                              int64_t n_out, const uint8_t *d_keep, const amber_tiles *tiles1,
                                              const amber_tiles *tiles2, void *stream)
{
    clear_error();
    if (!info) return fail(AMBER_E_ARG, "NULL pointer argument");
    if (n_out < 0 || n_out > (int64_t)1 << 30 || info->max_delay2 < 0)
        return fail(AMBER_E_ARG, "n_out=%lld must be in [0, 2^30]", (long long)n_out);
    void *work = nullptr;
    amber_status s = scratch_address(&work);
    if (s != AMBER_OK) return s;
    // rows of 128-byte multiples, as the Python binding's work buffers
    const int64_t n1 = n_out + info->max_delay2;
    int64_t work_stride = (n1 + 63) / 64 * 64;
    if (work_stride < 64) work_stride = 64;
    return subband_run(d_delay1, d_delay2, info, d_in, in_stride, n_in, static_cast<uint16_t *>(work), work_stride,
                       kStaticWorkBytes / 2, d_dd, dd_stride, n_out, d_keep, tiles1, tiles2, (hipStream_t)stream);
}

}  // extern "C"
