// Image-space kernels around the trace.  Primary-ray generation on the
// device: one pinhole ray (or `samples` jittered rays) per pixel, in the
// paper's per-pixel form (Fig. 5: one pixel/ray), written in the 32-byte ray
// layout the trace kernel reads (camera_ray, in the order svo_camera.h
// states); ambient-occlusion rays from primary hits; and compositing hits
// into an RGBA8 image (the colour field of the paper's hit buffer, Sec. 4.3).
#include <hip/hip_runtime.h>

#include "svo_camera.h"
#include "svo_internal.h"

namespace svo {

namespace {

__global__ __launch_bounds__(256) void primary_rays_kernel(CameraArgs c, float4* __restrict__ out) {
    const uint64_t n = (uint64_t)c.width * c.height * c.samples;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        float4 r0, r1;
        camera_ray(c, (uint32_t)i, r0, r1);
        out[2 * i] = r0;
        out[2 * i + 1] = r1;
    }
}

// Ambient-occlusion rays: for primary ray i with a hit at p = o + t d and
// normal n, k rays from p + offset * max(1, |p|inf) * n in cosine-weighted
// directions about n (Malley's method: a uniform point of the unit disc
// lifted to the hemisphere), tmax = radius.  The tangent frame is the
// branchless orthonormal basis of Duff et al. (JCGT 2017).  Primary misses
// and starts inside a voxel (zero normal) give rays with tmin > tmax, which
// the trace reports as misses.
__global__ __launch_bounds__(256) void ao_rays_kernel(AoArgs a) {
    const uint64_t total = a.n * a.k;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t src = i / a.k;
        const uint32_t j = (uint32_t)(i % a.k);
        const float t = a.t[src];
        const float nx = a.normal[3 * src], ny = a.normal[3 * src + 1], nz = a.normal[3 * src + 2];
        if (!isfinite(t) || (nx == 0.f && ny == 0.f && nz == 0.f)) {
            a.out[2 * i] = make_float4(0.f, 0.f, 0.f, 1.f);
            a.out[2 * i + 1] = make_float4(0.f, 0.f, 1.f, 0.f);
            continue;
        }
        const float4 r0 = a.rays[2 * src];
        const float4 r1 = a.rays[2 * src + 1];
        const float px = fmaf(t, r1.x, r0.x), py = fmaf(t, r1.y, r0.y), pz = fmaf(t, r1.z, r0.z);
        const float lift = a.offset * fmaxf(1.f, fmaxf(fabsf(px), fmaxf(fabsf(py), fabsf(pz))));
        const float sg = copysignf(1.f, nz);
        const float aa = -1.f / (sg + nz);
        const float bb = nx * ny * aa;
        const float b1x = 1.f + sg * nx * nx * aa, b1y = sg * bb, b1z = -sg * nx;
        const float b2x = bb, b2y = sg + ny * ny * aa, b2z = -ny;
        const uint32_t h = mix32(a.seed ^ mix32((uint32_t)src * 0x9e3779b9u + j));
        const float u1 = unit24(mix32(h ^ 0x68e31da4u));
        const float u2 = unit24(mix32(h ^ 0xb5297a4du));
        const float rr = sqrtf(u1);
        float sn, cs;
        sincosf(6.2831853071795864f * u2, &sn, &cs);
        const float lx = rr * cs, ly = rr * sn, lz = sqrtf(fmaxf(0.f, 1.f - u1));
        float dx = lx * b1x + ly * b2x + lz * nx;
        float dy = lx * b1y + ly * b2y + lz * ny;
        float dz = lx * b1z + ly * b2z + lz * nz;
        const float inv = 1.0f / sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
        a.out[2 * i] = make_float4(fmaf(lift, nx, px), fmaf(lift, ny, py), fmaf(lift, nz, pz), 0.f);
        a.out[2 * i + 1] = make_float4(dx * inv, dy * inv, dz * inv, a.radius);
    }
}

// Composite one pixel per thread, in integers: sample i of the pixel has
// leaf colour c (RGB of the hit leaf's word1; the background for a miss,
// which is any id outside the pool)
// and `occ` of its k AO rays blocked; it contributes c * (F k + (1000 - F)
// (k - occ)) / (1000 k) (weight 1 for a miss), and the pixel is the rounded
// mean of its samples.  Alpha is 255.
__global__ __launch_bounds__(256) void shade_kernel(ShadeArgs a) {
    const uint64_t npix = (uint64_t)a.width * a.height;
    const uint64_t den = 1000ull * (a.k ? a.k : 1u);
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t acc[3] = {0, 0, 0};
        for (uint32_t s = 0; s < a.samples; ++s) {
            const uint64_t i = p * a.samples + s;
            const uint32_t id = a.prim_id[i];
            uint32_t col = a.background;
            uint64_t w = den;
            if ((uint64_t)id < a.n_nodes) {
                col = (uint32_t)(a.nodes[id] >> 32);
                uint32_t occ = 0;
                for (uint32_t j = 0; j < a.k; ++j) occ += (a.ao_id[i * a.k + j] != 0xFFFFFFFFu) ? 1u : 0u;
                w = (uint64_t)a.ambient * a.k + (uint64_t)(1000u - a.ambient) * (a.k - occ);
                if (a.k == 0) w = den;
            }
            for (int c = 0; c < 3; ++c) acc[c] += (uint64_t)((col >> (8 * c)) & 0xFFu) * w;
        }
        const uint64_t total = den * a.samples;
        uint32_t x, y;
        pixel_of((uint32_t)p, a.width, a.height, a.tiled, x, y);
        uint32_t out = 0xFF000000u;
        for (int c = 0; c < 3; ++c) out |= (uint32_t)((acc[c] + total / 2) / total) << (8 * c);
        a.out[(uint64_t)y * a.width + x] = out;
    }
}

}  // namespace

hipError_t launch_shade(const ShadeArgs& a, hipStream_t stream) {
    const uint64_t n = (uint64_t)a.width * a.height;
    if (n == 0) return hipSuccess;
    const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 65535);
    hipLaunchKernelGGL(shade_kernel, dim3((uint32_t)blocks), dim3(256), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_ao_rays(const AoArgs& a, hipStream_t stream) {
    const uint64_t n = a.n * a.k;
    if (n == 0) return hipSuccess;
    const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 65535);
    hipLaunchKernelGGL(ao_rays_kernel, dim3((uint32_t)blocks), dim3(256), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_primary_rays(const CameraArgs& c, float* out, hipStream_t stream) {
    const uint64_t n = (uint64_t)c.width * c.height * c.samples;
    if (n == 0) return hipSuccess;
    const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 65535);
    hipLaunchKernelGGL(primary_rays_kernel, dim3((uint32_t)blocks), dim3(256), 0, stream, c,
                       reinterpret_cast<float4*>(out));
    return hipGetLastError();
}

}  // namespace svo
