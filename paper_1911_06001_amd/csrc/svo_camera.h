// Pinhole primary rays, one per pixel sample (the paper's per-pixel form,
// Fig. 5: one pixel/ray), for device code: the ray generation kernel writes
// them out, and the trace kernel makes them where it would otherwise read
// them (a job with a camera).  Both use camera_ray, so a camera trace sees
// exactly the rays svo_generate_primary_rays writes.
//
// Ray order: pixels in 8x8 tiles (tile rows top to bottom, tiles left to
// right, pixels row-major inside a tile; partial tiles at the right and
// bottom edges hold only in-image pixels) or row-major, `samples`
// consecutive rays per pixel.  Jitter comes from a counter-based hash of
// (seed, pixel, sample).
#pragma once

#include <hip/hip_runtime.h>

#include "svo_internal.h"

namespace svo {

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

// Pixel (x, y) of the pix-th pixel in ray order.
__device__ __forceinline__ void pixel_of(uint32_t pix, uint32_t W, uint32_t H, uint32_t tiled, uint32_t& x,
                                         uint32_t& y) {
    if (tiled) {
        const uint32_t ty = pix / (8u * W);
        uint32_t rem = pix - ty * 8u * W;
        const uint32_t h = min(8u, H - 8u * ty);
        const uint32_t tx = rem / (8u * h);
        rem -= tx * 8u * h;
        const uint32_t w = min(8u, W - 8u * tx);
        y = 8u * ty + rem / w;
        x = 8u * tx + rem % w;
    } else {
        y = pix / W;
        x = pix % W;
    }
}

// Ray i of camera c: origin at the eye, tmin 0, tmax +inf, direction through
// the pixel sample, normalised.  With whole 8x8 tiles and one sample per
// pixel (c.full_tiles) the ray's 64-ray tile is its pixel tile, found with
// one FP64 multiply instead of integer divisions.
__device__ __forceinline__ void camera_ray(const CameraArgs& c, uint32_t i, float4& r0, float4& r1) {
    uint32_t x, y, pix, smp;
    if (c.full_tiles) {
        const uint32_t T = i >> 6, k = i & 63u;
        uint32_t ty = (uint32_t)((double)T * c.inv_tiles_x);
        if (ty * c.tiles_x > T) --ty;
        else if ((ty + 1u) * c.tiles_x <= T) ++ty;
        const uint32_t tx = T - ty * c.tiles_x;
        x = 8u * tx + (k & 7u);
        y = 8u * ty + (k >> 3);
        pix = i;
        smp = 0;
    } else {
        pix = i / c.samples;
        smp = i - pix * c.samples;
        pixel_of(pix, c.width, c.height, c.tiled, x, y);
    }
    float fx = 0.5f, fy = 0.5f;
    if (c.jitter) {
        const uint32_t h = mix32(c.seed ^ mix32(pix * 0x9e3779b9u + smp));
        fx = unit24(mix32(h ^ 0x68e31da4u));
        fy = unit24(mix32(h ^ 0xb5297a4du));
    }
    const float sx = (((float)x + fx) / (float)c.width * 2.0f - 1.0f) * c.tan_half_fov * c.aspect;
    const float sy = (1.0f - ((float)y + fy) / (float)c.height * 2.0f) * c.tan_half_fov;
    float dx = fmaf(sy, c.up[0], fmaf(sx, c.right[0], c.fwd[0]));
    float dy = fmaf(sy, c.up[1], fmaf(sx, c.right[1], c.fwd[1]));
    float dz = fmaf(sy, c.up[2], fmaf(sx, c.right[2], c.fwd[2]));
    const float inv = 1.0f / sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
    r0 = make_float4(c.eye[0], c.eye[1], c.eye[2], 0.0f);
    r1 = make_float4(dx * inv, dy * inv, dz * inv, INFINITY);
}

}  // namespace svo
