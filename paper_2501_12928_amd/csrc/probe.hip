// Measured FP64 matrix peak of the device: back-to-back 16x16x4 FP64 MFMAs
// on independent accumulators, two workgroups of four waves per CU, no
// memory traffic in the loop. Reported beside the specification peak, since
// the clock a part sustains under a long MFMA load is below its nominal one.
#include "common.h"

namespace eor {

namespace {

constexpr int CHAINS = 8;

__global__ __launch_bounds__(256, 2) void mfma_probe_kernel(double *__restrict__ out, int64_t iters, double a0) {
    d4 acc[CHAINS];
#pragma unroll
    for (int i = 0; i < CHAINS; ++i) acc[i] = d4{0, 0, 0, 0};
    const double a = a0 + threadIdx.x * 1e-9, b = a0 * 0.5;
    for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < CHAINS; ++i) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[i], 0, 0, 0);
    }
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < CHAINS; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;  // keeps the chains live
}

}  // namespace

}  // namespace eor

extern "C" eor_status eor_probe_fp64_mfma(int device, int64_t iters, double *tflops, double *ms) {
    if (!tflops || iters < 1 || iters > ((int64_t)1 << 32))
        return eor::fail_status(EOR_ERR_ARG, "eor_probe_fp64_mfma: need tflops and 1 <= iters <= 2^32");
    int prev = -1;
    (void)hipGetDevice(&prev);
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return eor::hip_status(e, "eor_probe_fp64_mfma: hipSetDevice");
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    const int64_t blocks = 2 * (int64_t)(cus > 0 ? cus : 1);
    double *out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipStream_t s = nullptr;
    float t_ms = 0.f;
    if (e == hipSuccess) e = hipMalloc(&out, (size_t)blocks * 256 * sizeof(double));
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(eor::mfma_probe_kernel, dim3((unsigned)blocks), dim3(256), 0, s, out, (int64_t)100, 1.0);
        e = hipEventRecord(e0, s);
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(eor::mfma_probe_kernel, dim3((unsigned)blocks), dim3(256), 0, s, out, iters, 1.0);
        e = hipEventRecord(e1, s);
    }
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&t_ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    if (out) (void)hipFree(out);
    if (prev >= 0) (void)hipSetDevice(prev);
    if (e != hipSuccess) return eor::hip_status(e, "eor_probe_fp64_mfma");
    const double flop = (double)blocks * 4 * (double)iters * eor::CHAINS * 2048.0;
    *tflops = flop / ((double)t_ms * 1e-3) / 1e12;
    if (ms) *ms = t_ms;
    return EOR_OK;
}
