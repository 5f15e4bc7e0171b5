// Streaming-copy ceiling: the HBM bandwidth a plain device copy reaches,
// the practical bound next to the published peak that the step kernels are
// compared with.  Kept apart from the step kernels so that it never changes
// their code objects.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "hemelb_hip.h"

namespace {

typedef unsigned int u4 __attribute__((ext_vector_type(4)));

// One 16-byte element per lane; both streams bypass the caches' reuse
// policy (each line is touched once).
__global__ void __launch_bounds__(256) k_copy16(const u4 *__restrict__ src, u4 *__restrict__ dst, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

}  // namespace

extern "C" int hl_copy_bandwidth(void *dst, const void *src, int64_t bytes, int32_t reps, void *stream,
                                 double *gbps) {
    if (!dst || !src || !gbps || bytes <= 0 || (bytes & 15) || reps < 1 || reps > 1000) return HL_E_INVAL;
    const uintptr_t d = (uintptr_t)dst, s = (uintptr_t)src;
    if ((d & 15) || (s & 15)) return HL_E_INVAL;
    if (d < s + (uintptr_t)bytes && s < d + (uintptr_t)bytes) return HL_E_INVAL;  // overlapping ranges
    const int64_t n = bytes / 16;
    const int64_t blocks = (n + 255) / 256;
    if (blocks > INT32_MAX) return HL_E_RANGE;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = HL_OK;
    float ms = 0.0f;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        rc = HL_E_DEVICE;
    } else {
        // one untimed launch, then reps timed back to back
        for (int r = 0; r <= reps && rc == HL_OK; ++r) {
            if (r == 1 && hipEventRecord(e0, st) != hipSuccess) rc = HL_E_DEVICE;
            hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(256), 0, st, (const u4 *)src, (u4 *)dst, n);
            if (hipGetLastError() != hipSuccess) rc = HL_E_DEVICE;
        }
        if (rc == HL_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                            hipEventElapsedTime(&ms, e0, e1) != hipSuccess || !(ms > 0.0f)))
            rc = HL_E_DEVICE;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (rc == HL_OK) *gbps = 2.0 * (double)bytes * reps / ((double)ms * 1e-3) / 1e9;
    return rc;
}
