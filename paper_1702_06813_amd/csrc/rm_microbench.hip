// Throughput peaks of the two atomic operations the pose-scoring path relies
// on, measured on the device itself: the LDS 64-bit minimum that resolves
// the per-tile depth keys (no return value, each lane on its own slot of a
// tile-sized table), and the global 32-bit add with return that reserves
// bin space during binning (low contention, a small counter array shared by
// every compute unit).  These are the secondary ceilings the benchmark
// reports beside the HBM roofline; the library itself does not use this
// file.  Separate shared object, C ABI:
//
//   int rm_mb_lds_min_u64(int blocks, int iters, double* seconds, double* lane_ops)
//   int rm_mb_global_atomic_add(int blocks, int iters, int slots_log2, double* seconds, double* ops)
//
// Each allocates its own buffers, runs one warm-up launch and one timed
// launch (HIP events on the null stream), frees the buffers and returns 0,
// or -1 for arguments out of range, or -2 for a HIP error.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kWG = 256;
constexpr int kSlots = 2048;               // u64 keys: 16 KB, the depth table of a 64x32 tile
constexpr int kPerIter = kSlots / kWG;     // atomics per lane per iteration, one per table row

__global__ void __launch_bounds__(kWG) k_lds_min_u64(int iters, unsigned long long* __restrict__ sink) {
    __shared__ unsigned long long z[kSlots];
    for (int i = threadIdx.x; i < kSlots; i += kWG) z[i] = ~0ull;
    __syncthreads();
    // strictly decreasing keys, so that every minimum stores
    unsigned long long key = ~0ull - 1ull - (unsigned long long)threadIdx.x;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < kPerIter; ++k) atomicMin(&z[threadIdx.x + k * kWG], key - (unsigned long long)k);
        key -= kPerIter;
    }
    __syncthreads();
    unsigned long long m = ~0ull;
    for (int i = threadIdx.x; i < kSlots; i += kWG) m = z[i] < m ? z[i] : m;
    if (m == 0ull) sink[blockIdx.x] = m;   // keys stay far above 0: keeps the table observable
}

__global__ void __launch_bounds__(kWG) k_global_add(uint32_t* __restrict__ cnt, uint32_t mask, int iters,
                                                    uint32_t* __restrict__ sink) {
    const uint32_t gid = blockIdx.x * kWG + threadIdx.x;
    uint32_t acc = 0;
    for (int it = 0; it < iters; ++it) {
        const uint32_t a = (gid * 2654435761u + (uint32_t)it * 40503u) & mask;
        acc += atomicAdd(cnt + a, 1u);
    }
    if (acc == 0xffffffffu) sink[0] = acc;
}

template <typename F>
int timed(F launch, double* seconds) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -2;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return -2; }
    launch();                                                  // warm-up
    (void)hipEventRecord(e0, nullptr);
    launch();
    (void)hipEventRecord(e1, nullptr);
    int rc = hipEventSynchronize(e1) == hipSuccess && hipGetLastError() == hipSuccess ? 0 : -2;
    float ms = 0.0f;
    if (rc == 0 && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = -2;
    *seconds = ms * 1e-3;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

}  // namespace

extern "C" int rm_mb_lds_min_u64(int blocks, int iters, double* seconds, double* lane_ops) {
    if (blocks < 1 || blocks > 65535 || iters < 1 || iters > (1 << 20) || !seconds || !lane_ops) return -1;
    unsigned long long* sink = nullptr;
    if (hipMalloc(&sink, sizeof(unsigned long long) * blocks) != hipSuccess) return -2;
    const int rc = timed([&] { hipLaunchKernelGGL(k_lds_min_u64, dim3(blocks), dim3(kWG), 0, nullptr, iters, sink); },
                         seconds);
    (void)hipFree(sink);
    *lane_ops = (double)blocks * kWG * (double)iters * kPerIter;
    return rc;
}

extern "C" int rm_mb_global_atomic_add(int blocks, int iters, int slots_log2, double* seconds, double* ops) {
    if (blocks < 1 || blocks > 65535 || iters < 1 || iters > (1 << 20) || slots_log2 < 6 || slots_log2 > 24 ||
        !seconds || !ops)
        return -1;
    const size_t n = (size_t)1 << slots_log2;
    uint32_t* cnt = nullptr;
    uint32_t* sink = nullptr;
    if (hipMalloc(&cnt, n * sizeof(uint32_t)) != hipSuccess) return -2;
    if (hipMalloc(&sink, sizeof(uint32_t)) != hipSuccess) { (void)hipFree(cnt); return -2; }
    int rc = hipMemset(cnt, 0, n * sizeof(uint32_t)) == hipSuccess ? 0 : -2;
    if (rc == 0)
        rc = timed([&] {
            hipLaunchKernelGGL(k_global_add, dim3(blocks), dim3(kWG), 0, nullptr, cnt, (uint32_t)(n - 1), iters, sink);
        }, seconds);
    (void)hipFree(sink);
    (void)hipFree(cnt);
    *ops = (double)blocks * kWG * (double)iters;
    return rc;
}
