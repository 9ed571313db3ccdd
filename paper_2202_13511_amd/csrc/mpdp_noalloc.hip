// The no-allocation entry point, mpdp_optimize_noalloc: the exact DP of
// mpdp_optimize_ws for queries of up to kNoAllocMaxRel relations, with its
// workspace in a fixed device array of this library instead of caller or
// runtime allocations.
//
// The array is a file-scope __device__ variable: every GPU the library runs
// on holds its own copy until the process ends.  Host code never passes the
// variable's name to a kernel (on the host it is only a stand-in for the
// symbol); on the first call on a device its device address is looked up
// with hipGetSymbolAddress, with that device current, and kept per device.
// Every call on one device shares that device's array, so calls that overlap
// on one device (other threads, other streams) race; the memo, counters and
// lists are rewritten by every call before they are read, so nothing has to
// start at zero.
#include <hip/hip_runtime.h>

#include <mutex>

#include "mpdp.h"
#include "mpdp_host_internal.h"

namespace {

constexpr uint32_t kNoAllocMaxRel = MPDP_NOALLOC_MAX_REL;
// 2^20 memo entries of 21 bytes, two lists of C(20, 10) sets, query
// information, counters and plan: 22.5 MiB, rounded up
constexpr size_t kScratchBytes = size_t(24) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_scratch[kMaxDevices];  // device address of `scratch`, per device (null until looked up)

// Device address of this device's array, looked up once per device.
mpdp_status scratch_for_current_device(void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        return MPDP_EDEVICE;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        if (mpdp_host::noalloc_workspace_bytes(kNoAllocMaxRel) > kScratchBytes) return MPDP_EDEVICE;
        (void)mpdp_host::noalloc_setup();
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return MPDP_EDEVICE;
        }
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return MPDP_OK;
}

}  // namespace

extern "C" {

size_t mpdp_noalloc_scratch_bytes(void) { return kScratchBytes; }

mpdp_status mpdp_optimize_noalloc(uint32_t n, uint32_t m, const mpdp_edge *edges, const double *cardinalities,
                                  const double *selectivities, mpdp_cost_model cost_model, void *hip_stream,
                                  uint32_t flags, mpdp_plan_node *plan_out, double *cost_out,
                                  mpdp_stats *stats_out) {
    if (n > kNoAllocMaxRel) return MPDP_ETOOLARGE;
    // the input is validated on the host before the array is looked up
    return mpdp_host::optimize_noalloc(n, m, edges, cardinalities, selectivities, cost_model,
                                       scratch_for_current_device, kScratchBytes,
                                       static_cast<hipStream_t>(hip_stream), flags, plan_out, cost_out, stats_out);
}

}  // extern "C"
