// probe_read.hip -- the achievable HBM streaming-read rate of the device, the
// measured roof that the benchmark quotes next to the nominal 8 TB/s.  Not
// part of the cost-model path: a separate library (libcm_probe.so) that only
// the benchmark loads.
//
// Every thread reads 16-byte words in a grid-stride loop (four loads in
// flight per iteration, whole 128-byte lines per 8 lanes) and folds them into
// one register; a word is written only if the fold hits a constant no
// buffer of the probe's pattern produces, which keeps the loads without
// adding traffic.  The loads are non-temporal and the grid is 32 workgroups
// of 4 waves per compute unit: on MI355X these read about 10% faster than
// cached loads from 8 workgroups per compute unit (6.5 against 5.5-5.9 TB/s
// over 4 GiB).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <vector>

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_stream_read(const u32x4 *__restrict__ p, uint64_t n,
                                                     uint32_t *__restrict__ out)
{
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    uint32_t acc = 0;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const u32x4 a = __builtin_nontemporal_load(p + i);
        const u32x4 b = __builtin_nontemporal_load(p + i + stride);
        const u32x4 c = __builtin_nontemporal_load(p + i + 2 * stride);
        const u32x4 d = __builtin_nontemporal_load(p + i + 3 * stride);
        acc ^= (a[0] + b[1]) ^ (c[2] + d[3]) ^ (a[3] + b[2]) ^ (c[0] + d[1]) ^
               (a[1] ^ b[0] ^ c[3] ^ d[2]) ^ (a[2] ^ b[3] ^ c[1] ^ d[0]);
    }
    for (; i < n; i += stride) {
        const u32x4 a = __builtin_nontemporal_load(p + i);
        acc ^= a[0] ^ a[1] ^ a[2] ^ a[3];
    }
    if (acc == 0x9e3779b9u) out[blockIdx.x] = acc;
}

}  // namespace

extern "C" {

// Streaming-read rate over a buffer of `bytes` (rounded down to 16) on the
// current device: `reps` timed launches after two untimed ones, each timed
// with HIP events; writes the median and best GB/s (10^9 bytes per second).
// Allocates and frees its own buffer.  Returns 0, or a negative HIP error.
int cm_probe_read_gbs(int64_t bytes, int32_t reps, double *median_gbs, double *best_gbs)
{
    if (bytes < (1 << 20) || reps < 1 || !median_gbs || !best_gbs) return -1;
    const uint64_t n = (uint64_t)bytes / 16;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return -2;
    u32x4 *buf = nullptr;
    uint32_t *out = nullptr;
    const int grid = prop.multiProcessorCount * 32;
    if (hipMalloc((void **)&buf, n * 16) != hipSuccess) return -3;
    if (hipMalloc((void **)&out, (size_t)grid * 4) != hipSuccess) {
        (void)hipFree(buf);
        return -3;
    }
    int rc = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    std::vector<float> ms;
    if (hipMemset(buf, 0x5a, n * 16) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess) {
        rc = -4;
    }
    for (int r = -2; rc == 0 && r < reps; ++r) {
        if (hipEventRecord(e0, nullptr) != hipSuccess) rc = -5;
        hipLaunchKernelGGL(k_stream_read, dim3(grid), dim3(256), 0, nullptr, buf, n, out);
        if (hipGetLastError() != hipSuccess || hipEventRecord(e1, nullptr) != hipSuccess ||
            hipEventSynchronize(e1) != hipSuccess)
            rc = -5;
        float t = 0.f;
        if (rc == 0 && hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = -5;
        if (rc == 0 && r >= 0) ms.push_back(t);
    }
    if (rc == 0) {
        std::sort(ms.begin(), ms.end());
        *median_gbs = (double)(n * 16) / (ms[ms.size() / 2] * 1e-3) / 1e9;
        *best_gbs = (double)(n * 16) / (ms.front() * 1e-3) / 1e9;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(out);
    (void)hipFree(buf);
    return rc;
}

}  // extern "C"
