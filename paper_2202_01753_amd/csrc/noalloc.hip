// mc_integrate_noalloc: the whole m-Cubes run on a fixed per-device scratch
// array instead of a caller-provided workspace, for callers that cannot
// allocate memory on the device (code under stream capture, serving loops
// that must not allocate).
//
// The array is a file-scope device global, one copy per GPU, held from the
// library's load until the process ends.  Host code never passes the array's
// name to a kernel or a copy: it asks the runtime for the array's address on
// each device once, with that device current, and uses that pointer.
#include <hip/hip_runtime.h>

#include <mutex>

#include "host.hpp"
#include "internal.hpp"
#include "mcubes.h"

namespace {

constexpr size_t kScratchBytes = MC_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

// Per device: the scratch array's device address (null until looked up) and
// the lock that serialises this entry point's calls on the device, which all
// share the one array.
std::mutex g_lock[kMaxDevices];
void *g_scratch[kMaxDevices] = {};

}  // namespace

extern "C" mc_status mc_integrate_noalloc(const mc_problem *prob, void *stream, mc_result *out,
                                          double *h_iters, double *h_grid) {
    if (!out) return MC_EINVAL;
    size_t need = 0;
    const mc_status st = mc_workspace_bytes(prob, &need);  // validates the problem first
    if (st != MC_OK) return st;
    if (need > kScratchBytes) return MC_EWORKSPACE;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return MC_EDEVICE;
    std::lock_guard<std::mutex> hold(g_lock[dev]);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return MC_EDEVICE;
        g_scratch[dev] = p;
    }
    return mcubes::host::integrate_unpinned(prob, g_scratch[dev], kScratchBytes, stream, out, h_iters,
                                            h_grid);
}
