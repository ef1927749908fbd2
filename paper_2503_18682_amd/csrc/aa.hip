// Box downsampling for anti-aliasing evaluation: a view rendered at f times
// the resolution (f x f rays per output pixel on an ordered grid, centres at
// offsets (k + 1/2) / f) averaged back to the output grid.  With f = 2 this
// is the 4-ray multisampling baseline of Sec. 6.2; larger f gives
// supersampled references.
#include "internal.h"

namespace rgs {
namespace {

// One thread per output pixel and plane; reads of a wave cover f contiguous
// rows of 64 f contiguous source floats.
__global__ __launch_bounds__(256) void k_downsample_box(const float *__restrict__ src, int width, int height,
                                                        int factor, int planes, float *__restrict__ dst)
{
    const int64_t n = (int64_t)width * height * planes;
    const float inv = 1.0f / (float)(factor * factor);
    const int sw = width * factor;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % width);
        const int64_t t = i / width;
        const int y = (int)(t % height);
        const int64_t p = t / height;
        const float *s = src + (p * height * factor + (int64_t)y * factor) * sw + (int64_t)x * factor;
        float acc = 0.0f;
        for (int r = 0; r < factor; ++r)
            for (int c = 0; c < factor; ++c) acc += s[(int64_t)r * sw + c];
        dst[i] = acc * inv;
    }
}

}  // namespace

hipError_t launch_downsample_box(const float *src, int width, int height, int factor, int planes, float *dst,
                                 hipStream_t stream)
{
    const int64_t n = (int64_t)width * height * planes;
    if (n == 0) return hipSuccess;
    const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
    k_downsample_box<<<grid, 256, 0, stream>>>(src, width, height, factor, planes, dst);
    return hipGetLastError();
}

}  // namespace rgs
