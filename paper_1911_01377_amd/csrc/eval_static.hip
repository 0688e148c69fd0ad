// useries_eval_static: the evaluation of useries_eval_parts with its
// per-charge workspace (encoded and sorted positions, permutation, cluster
// table, near forces, energy partials) taken from a fixed device array of
// this library instead of memory that the plan allocates on demand, so that
// the call itself allocates nothing.
//
// `scratch` is a file-scope device array.  Each GPU that loads the library
// holds its own copy, at its own address, until the process ends; host code
// must not pass the array's name to a kernel (on the host it only stands for
// the symbol), so its device address is looked up once per device with
// hipGetSymbolAddress, with that device current, and that address is what
// the kernels receive.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdio>
#include <mutex>
#include <string>

#include "useries_internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(16) << 20;   // 16 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};        // device address of `scratch`, per device
hipError_t g_err[kMaxDevices] = {};   // result of the lookup, per device
bool g_done[kMaxDevices] = {};

// device address of this library's scratch array on `dev` (current device)
hipError_t scratch_address(int dev, void** out) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_done[dev]) {
        void* ptr = nullptr;
        g_err[dev] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        g_ptr[dev] = g_err[dev] == hipSuccess ? ptr : nullptr;
        g_done[dev] = true;
    }
    *out = g_ptr[dev];
    return g_err[dev];
}

}  // namespace

extern "C" int useries_eval_static(useries_plan_t p, int64_t n, const float* xyz, const float* q,
                                   float* forces, double* energy, double* parts, void* stream) {
    using namespace useries;
    if (!p) return set_last_error(USERIES_EINVAL, "NULL plan");
    if (!energy && !parts) return set_last_error(USERIES_EINVAL, "NULL energy and parts");
    if (n < 0 || n > INT_MAX / 4) return set_last_error(USERIES_EINVAL, "n out of range");
    const size_t need = atom_workspace_bytes(p, n);
    if (need > kScratchBytes) {
        char buf[200];
        std::snprintf(buf, sizeof buf,
                      "useries_eval_static: %lld charges need %zu bytes of workspace, above the "
                      "library's fixed %zu bytes (use useries_eval)",
                      (long long)n, need, kScratchBytes);
        return set_last_error(USERIES_EINVAL, buf);
    }
    const int dev = plan_device(p);
    if (dev < 0 || dev >= kMaxDevices)
        return set_last_error(USERIES_EINVAL, "useries_eval_static: device index out of range");
    // the lookup runs with the plan's device current
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev && hipSetDevice(dev) != hipSuccess)
        return set_last_error(USERIES_EHIP, "useries_eval_static: hipSetDevice failed");
    void* base = nullptr;
    const hipError_t e = scratch_address(dev, &base);
    if (prev >= 0 && prev != dev) hipSetDevice(prev);
    if (e != hipSuccess || !base)
        return set_last_error(USERIES_EHIP, std::string("useries_eval_static: hipGetSymbolAddress: ") +
                                                hipGetErrorString(e));
    const AtomWs ws = atom_workspace_at(p, n, static_cast<char*>(base));
    return plan_eval(p, n, xyz, q, forces, energy, parts, stream, &ws);
}
