// Primary-ray generation on the device: one pinhole ray (or `samples`
// jittered rays) per pixel, in the paper's per-pixel form (Fig. 5: one
// pixel/ray), written in the 32-byte ray layout the trace kernel reads.
//
// Ray order: pixels in 8x8 tiles (tile rows top to bottom, tiles left to
// right, pixels row-major inside a tile; partial tiles at the right and
// bottom edges hold only in-image pixels), `samples` consecutive rays per
// pixel.  Jitter comes from a counter-based hash of (seed, pixel, sample).
#include <hip/hip_runtime.h>

#include "svo_internal.h"

namespace svo {

namespace {

// 32-bit integer finaliser (the "lowbias32" mix of Wellons' hash prospector):
// a bijective, counter-based mix used only for sub-pixel jitter.
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

__device__ __forceinline__ float unit24(uint32_t h) { return (float)(h >> 8) * 0x1p-24f; }

__global__ __launch_bounds__(256) void primary_rays_kernel(CameraArgs c, float4* __restrict__ out) {
    const uint64_t n = (uint64_t)c.width * c.height * c.samples;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t pix = (uint32_t)(i / c.samples);
        const uint32_t smp = (uint32_t)(i % c.samples);
        uint32_t x, y;
        if (c.tiled) {
            const uint32_t W = c.width, H = c.height;
            const uint32_t ty = pix / (8u * W);
            uint32_t rem = pix - ty * 8u * W;
            const uint32_t h = min(8u, H - 8u * ty);
            const uint32_t tx = rem / (8u * h);
            rem -= tx * 8u * h;
            const uint32_t w = min(8u, W - 8u * tx);
            y = 8u * ty + rem / w;
            x = 8u * tx + rem % w;
        } else {
            y = pix / c.width;
            x = pix % c.width;
        }
        float fx = 0.5f, fy = 0.5f;
        if (c.jitter) {
            const uint32_t k = mix32(c.seed ^ mix32(pix * 0x9e3779b9u + smp));
            fx = unit24(mix32(k ^ 0x68e31da4u));
            fy = unit24(mix32(k ^ 0xb5297a4du));
        }
        const float sx = (((float)x + fx) / (float)c.width * 2.0f - 1.0f) * c.tan_half_fov * c.aspect;
        const float sy = (1.0f - ((float)y + fy) / (float)c.height * 2.0f) * c.tan_half_fov;
        float dx = fmaf(sy, c.up[0], fmaf(sx, c.right[0], c.fwd[0]));
        float dy = fmaf(sy, c.up[1], fmaf(sx, c.right[1], c.fwd[1]));
        float dz = fmaf(sy, c.up[2], fmaf(sx, c.right[2], c.fwd[2]));
        const float inv = 1.0f / sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
        dx *= inv;
        dy *= inv;
        dz *= inv;
        out[2 * i] = make_float4(c.eye[0], c.eye[1], c.eye[2], 0.0f);
        out[2 * i + 1] = make_float4(dx, dy, dz, INFINITY);
    }
}

}  // namespace

hipError_t launch_primary_rays(const CameraArgs& c, float* out, hipStream_t stream) {
    const uint64_t n = (uint64_t)c.width * c.height * c.samples;
    if (n == 0) return hipSuccess;
    const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 65535);
    hipLaunchKernelGGL(primary_rays_kernel, dim3((uint32_t)blocks), dim3(256), 0, stream, c,
                       reinterpret_cast<float4*>(out));
    return hipGetLastError();
}

}  // namespace svo
