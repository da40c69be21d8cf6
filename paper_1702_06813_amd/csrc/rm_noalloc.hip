// Allocation-free variant of rm_align_cost_grad: the call's scratch (visible
// cluster lists, bin counters, tile bins, per-tile partial records, cluster
// bounds) lives in a fixed device array of this file instead of the
// context's growable arena, so the call never allocates device memory.
#include <mutex>

#include "rm_internal.h"

namespace {

constexpr size_t kNoAllocBytes = (size_t)256 << 20;

// The scratch array.  Host code never uses this name as a device address:
// each device's copy is found once with hipGetSymbolAddress and that address
// is what the kernels receive.
static __device__ __align__(256) char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices];                 // the array's address on each device
hipError_t g_status[kMaxDevices];
bool g_looked_up[kMaxDevices];

}  // namespace

namespace rm {

void noalloc_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_looked_up[device]) return;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) (void)hipGetLastError();
    g_status[device] = e;
    g_addr[device] = e == hipSuccess ? p : nullptr;
    g_looked_up[device] = true;
}

}  // namespace rm

extern "C" int rm_align_cost_grad_noalloc(rm_ctx* ctx, const rm_mesh* mesh, const rm_scan* scans, int32_t n_scans,
                                          const int32_t* pose_off, const double* T_wc, rm_cost_params params,
                                          double* out) {
    if (!ctx) return rm::align_common(nullptr, mesh, scans, n_scans, pose_off, T_wc, params, out, rm::kGrad, nullptr,
                                      nullptr);
    const int dev = rm::ctx_device(ctx);
    void* addr = nullptr;
    hipError_t st = hipErrorInvalidDevice;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (dev >= 0 && dev < kMaxDevices && g_looked_up[dev]) {
            addr = g_addr[dev];
            st = g_status[dev];
        }
    }
    if (!addr) {
        char msg[160];
        snprintf(msg, sizeof(msg), "allocation-free scratch unavailable on device %d: %s", dev,
                 hipGetErrorString(st));
        return rm::ctx_fail(ctx, RM_ERR_DEVICE, msg);
    }
    rm::Arena arena;
    arena.fixed = static_cast<char*>(addr);
    arena.fixed_size = kNoAllocBytes;
    return rm::align_common(ctx, mesh, scans, n_scans, pose_off, T_wc, params, out, rm::kGrad, nullptr, &arena);
}
