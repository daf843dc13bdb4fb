// noalloc.hip -- vrs_scan_topk_noalloc: the filtered exact top-k scan with
// its workspace in a static device array instead of a caller's buffer, for
// callers that cannot allocate device memory (HIP graph capture, serving
// loops, harnesses that forbid allocation).
//
// The array lives in this file's device code, one copy per GPU the library
// runs on, held until the process ends.  In host code its name is only a
// host-side stand-in, never a device address: the device address is taken
// once per device with hipGetSymbolAddress (the device current) and kept,
// and only that address is handed to the kernels.  Every call on a GPU uses
// that GPU's copy, so calls that overlap on one GPU (on two streams, or from
// two threads) race and must be serialised by the caller.  The scan
// initialises everything it reads from the workspace (query preparation
// clears the counters, bounds and flags), so the contents left by the
// previous call do not matter.
#include <mutex>

#include "internal.h"
#include "planner.h"

namespace vrs {

namespace {

constexpr size_t SCRATCH_BYTES = VRS_NOALLOC_SCRATCH_BYTES;
constexpr int MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES];  // device address of `scratch`, per device (null: not yet taken)

// The current device's copy of `scratch` (taken on the first call there).
hipError_t scratch_address(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

}  // namespace vrs

extern "C" {

vrs_status vrs_scan_topk_noalloc(vrs_table t, const float *q, int32_t B, const vrs_pred *pred,
                                 int32_t k, vrs_metric metric, int64_t *out_idx, float *out_dist,
                                 const vrs_opts *opts, void *stream) {
    size_t need = 0;
    vrs_status st = vrs_scan_workspace_bytes(t, B, k, opts, &need);  // validates t, B, k
    if (st != VRS_OK) return st;
    if (need > vrs::SCRATCH_BYTES) {
        char msg[160];
        snprintf(msg, sizeof msg, "this scan needs %zu bytes of workspace; the static scratch holds %zu",
                 need, vrs::SCRATCH_BYTES);
        return vrs::set_error(VRS_E_WORKSPACE, msg);
    }
    void *ws = nullptr;
    hipError_t e = vrs::scratch_address(&ws);
    if (e != hipSuccess) {
        char msg[160];
        snprintf(msg, sizeof msg, "static scratch address: %s", hipGetErrorString(e));
        return vrs::set_error(VRS_E_HIP, msg);
    }
    return vrs_scan_topk(t, q, B, pred, k, metric, out_idx, out_dist, ws, vrs::SCRATCH_BYTES, opts, stream);
}

}  // extern "C"
