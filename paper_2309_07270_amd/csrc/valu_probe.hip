// Measured int32 vector-ALU throughput of one GPU: independent add / max
// chains (the operation mix of the X-drop recurrence) at full occupancy.
// A measuring tool for the roofline of the window kernels; not part of the
// alignment path.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kChains = 8;          // independent dependency chains per lane
constexpr int kOpsPerChainStep = 2; // one add, one max

__global__ void __launch_bounds__(256) valu_chains(int *out, int iters, int b, int c)
{
    int a[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = (int)threadIdx.x * (k + 3) + (int)blockIdx.x;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) a[k] = max(a[k] + b, c - k);
    }
    int s = 0;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s ^= a[k];
    // never true for the arguments the host passes; keeps the chains live
    if (s == 0x7fffffff) out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

// Runs the probe on `device` and stores the int32 lane-operations per second
// and the timed launch in milliseconds.  Returns 0, or -1 on a HIP error.
extern "C" int xdrop_probe_valu_ops(int device, int iters, double *ops_per_s, double *launch_ms)
{
    if (hipSetDevice(device) != hipSuccess) return -1;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return -1;
    const int blocks = prop.multiProcessorCount * 16;   // 16 x 256 lanes per CU: full occupancy
    const int threads = 256;
    int *out = nullptr;
    if (hipMalloc(&out, (size_t)blocks * threads * sizeof(int)) != hipSuccess) return -1;
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    hipLaunchKernelGGL(valu_chains, dim3(blocks), dim3(threads), 0, 0, out, iters / 8, 1, -5);   // warm-up
    hipEventRecord(e0, 0);
    hipLaunchKernelGGL(valu_chains, dim3(blocks), dim3(threads), 0, 0, out, iters, 1, -5);
    hipEventRecord(e1, 0);
    const hipError_t st = hipEventSynchronize(e1);
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    hipFree(out);
    if (st != hipSuccess || hipGetLastError() != hipSuccess || ms <= 0.f) return -1;
    const double ops = (double)blocks * threads * (double)iters * kChains * kOpsPerChainStep;
    *ops_per_s = ops / (ms * 1e-3);
    *launch_ms = ms;
    return 0;
}
