// Integer VALU throughput probe: independent chains of 32-bit XOR, 3-input
// bit logic (v_bitop3) and AND-OR, on every CU, so the integer peak used for
// roofline fractions can be checked on the device at hand.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace wpm {

namespace {
template <int OP>
__global__ __launch_bounds__(256) void valu_probe(const uint32_t *__restrict__ in, uint32_t *out,
                                                  int iters) {
    uint32_t a[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = in[(threadIdx.x + i) & 255];
    uint32_t b = in[256 + (threadIdx.x & 63)], c = in[320 + (threadIdx.x & 63)];
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                if (OP == 0)
                    a[i] = a[i] ^ b;
                else if (OP == 1)
                    a[i] = __builtin_amdgcn_bitop3_b32(a[i], b, c, 0x96);
                else
                    a[i] = (a[i] & b) | c;
            }
            b += 0x9E3779B9u;  // keeps the operands live: 2 ops per 8 chain ops
            c ^= b;
        }
    }
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) s ^= a[i];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}
}  // namespace

int valu_probe_run(int op, int waves_per_simd, int iters, double *lane_ops_per_s) {
    if (op < 0 || op > 2 || waves_per_simd < 1 || waves_per_simd > 8 || iters < 1 || !lane_ops_per_s)
        return WPM_EINVAL;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return WPM_EHIP;
    const int grid = cus * waves_per_simd;  // 256 threads = one wave per SIMD per workgroup
    uint32_t *din = nullptr, *dout = nullptr;
    uint32_t h[512];
    for (int i = 0; i < 512; ++i) h[i] = (uint32_t)i * 2654435761u;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = WPM_OK;
    float ms = 0.0f;
    auto launch = [&]() {
        if (op == 0) hipLaunchKernelGGL(valu_probe<0>, dim3(grid), dim3(256), 0, 0, din, dout, iters);
        else if (op == 1) hipLaunchKernelGGL(valu_probe<1>, dim3(grid), dim3(256), 0, 0, din, dout, iters);
        else hipLaunchKernelGGL(valu_probe<2>, dim3(grid), dim3(256), 0, 0, din, dout, iters);
    };
    if (hipMalloc(&din, sizeof(h)) != hipSuccess || hipMalloc(&dout, sizeof(uint32_t) * 256 * grid) != hipSuccess ||
        hipMemcpy(din, h, sizeof(h), hipMemcpyHostToDevice) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        rc = WPM_EHIP;
    } else {
        launch();
        if (hipDeviceSynchronize() != hipSuccess) rc = WPM_EHIP;
        if (!rc) {
            (void)hipEventRecord(e0, 0);
            launch();
            (void)hipEventRecord(e1, 0);
            if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                rc = WPM_EHIP;
        }
    }
    if (!rc) *lane_ops_per_s = (double)grid * 256.0 * iters * 16.0 * 10.0 / (ms * 1e-3);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (din) (void)hipFree(din);
    if (dout) (void)hipFree(dout);
    return rc;
}

}  // namespace wpm
