// The library's static device workspace for tp_solve_static: the solve's
// per-workgroup partial summaries and its reduced summary live in a
// file-scope device array instead of plan-owned allocations, so that solve
// calls need no allocation at all.  Each GPU holds its own copy of the array
// (at its own address) until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"

namespace tpfdm {

namespace {

// Partial summaries the workspace holds (24 bytes each), then the summary.
constexpr int64_t kStaticParts = 16384;
constexpr size_t kSummaryOffset = static_cast<size_t>(kStaticParts) * sizeof(SolvePartial);
static_assert(kSummaryOffset % 256 == 0, "summary must stay 256-byte aligned");
constexpr size_t kScratchBytes = kSummaryOffset + 256;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` per device, looked up once per device.  In
// host code the name of the array only stands for the symbol; its memory
// is reached through these addresses.
constexpr int kMaxDevices = 64;
std::mutex g_mutex;
unsigned char* g_addr[kMaxDevices] = {};

}  // namespace

tp_status static_solve_work(SolveWork* out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_error(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return set_error(TP_ERR_UNSUPPORTED, "device index beyond the static workspace table");
    unsigned char* base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mutex);
        if (!g_addr[dev]) {
            void* ptr = nullptr;
            e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess) return hip_error(e, "hipGetSymbolAddress of the static solve workspace");
            g_addr[dev] = static_cast<unsigned char*>(ptr);
        }
        base = g_addr[dev];
    }
    out->parts = reinterpret_cast<SolvePartial*>(base);
    out->cap = kStaticParts;
    out->summary = reinterpret_cast<SolveSummary*>(base + kSummaryOffset);
    return TP_OK;
}

}  // namespace tpfdm
