// Measured device ceilings, reported beside the published peaks: the FP32
// FMA rate of register-resident chains (non-packed, as all code here is
// built), the rate of the hardware exp2, and device-to-device copy bandwidth.
#include "internal.h"

namespace rgs {
namespace {

constexpr int kChains = 8;

__global__ __launch_bounds__(256) void k_fma_loop(float *__restrict__ out, int iters, float a, float b)
{
    float x[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) x[k] = (float)(threadIdx.x + k);
#pragma unroll 4
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int k = 0; k < kChains; ++k) x[k] = __builtin_fmaf(x[k], a, b);
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += x[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// y <- 2^-y converges to a fixed point near 0.64, so every iteration is one
// exp2 on a finite argument
__global__ __launch_bounds__(256) void k_exp_loop(float *__restrict__ out, int iters)
{
    float y[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) y[k] = 0.01f * (float)(threadIdx.x % 7 + k);
#pragma unroll 4
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int k = 0; k < kChains; ++k) y[k] = __builtin_amdgcn_exp2f(-y[k]);
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += y[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

hipError_t measure_ceilings(int num_cus, hipStream_t stream, double *fma_tflops, double *exp_tops, double *copy_gbs)
{
    const int blocks = num_cus * 8, threads = 256, iters = 8192;
    const size_t copy_bytes = size_t(512) << 20;
    float *out = nullptr;
    void *a = nullptr, *b = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t err = hipSuccess;
    float ms = 0.0f;
    auto timed = [&](auto &&launch) -> double {
        launch();  // warm-up
        if ((err = hipEventRecord(e0, stream)) != hipSuccess) return 0.0;
        launch();
        if ((err = hipEventRecord(e1, stream)) != hipSuccess) return 0.0;
        if ((err = hipEventSynchronize(e1)) != hipSuccess) return 0.0;
        if ((err = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) return 0.0;
        return ms;
    };
    do {
        if ((err = hipMalloc(&out, sizeof(float) * blocks * threads)) != hipSuccess) break;
        if ((err = hipMalloc(&a, copy_bytes)) != hipSuccess) break;
        if ((err = hipMalloc(&b, copy_bytes)) != hipSuccess) break;
        if ((err = hipEventCreate(&e0)) != hipSuccess) break;
        if ((err = hipEventCreate(&e1)) != hipSuccess) break;
        const double n_threads = (double)blocks * threads;
        double t = timed([&] { k_fma_loop<<<blocks, threads, 0, stream>>>(out, iters, 0.999f, 0.001f); });
        if (err != hipSuccess) break;
        *fma_tflops = n_threads * iters * kChains * 2.0 / (t * 1e-3) / 1e12;
        t = timed([&] { k_exp_loop<<<blocks, threads, 0, stream>>>(out, iters / 4); });
        if (err != hipSuccess) break;
        *exp_tops = n_threads * (iters / 4) * kChains / (t * 1e-3) / 1e12;
        t = timed([&] { (void)hipMemcpyAsync(b, a, copy_bytes, hipMemcpyDeviceToDevice, stream); });
        if (err != hipSuccess) break;
        *copy_gbs = 2.0 * (double)copy_bytes / (t * 1e-3) / 1e9;
    } while (false);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (out) (void)hipFree(out);
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    return err;
}

}  // namespace rgs
