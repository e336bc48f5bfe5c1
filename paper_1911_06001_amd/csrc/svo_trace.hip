// First-hit traversal of sparse voxel octrees with transformed subtrees, for
// gfx950 (wave64, no matrix cores: the work is dependent 8-byte gathers).
//
// Per ray (one lane each):
//   1. map the world ray into a frame's grid coordinates (paper Eq. 2-3 with
//      the scale folded into the affine map, Sec. 3.2); t is not rescaled;
//   2. mirror axes with negative direction so every direction component is
//      positive; a plane crossing is then t(v) = v * invd + bias, one FMA,
//      evaluated by the same formula for every cell sharing that plane;
//   3. walk the frame's octree front to back, top-down (the role Revelles'
//      parametric traversal plays in the paper, Sec. 5): integer cell
//      corners, a per-level stack of (child start, mask) in LDS, and an exit
//      by the highest changed coordinate bit, so popping needs no search;
//   4. frames whose moved content leaves their static cell are candidates,
//      tried in order of root-cell entry and skipped once their entry lies
//      beyond the best hit (the depth sort of Sec. 4.2 with an exact slab
//      cull in place of the bounding sphere of Sec. 4.1);
//   5. write id, slot, t and the normal (entry face mapped by the inverse
//      transpose).
//
// Work distribution: a persistent grid; each wave claims 64-ray tiles from
// a global counter, and the last work-group to finish resets the counter so
// the next launch on the stream starts from zero.
#include <hip/hip_runtime.h>

#include "svo_internal.h"

namespace svo {

namespace {

constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint32_t kStepLimitId = 0xFFFFFFFEu;

struct Ray {
    float ox, oy, oz, tmin, dx, dy, dz, tmax;
};

// A ray in one frame's mirrored grid coordinates.
struct FrameRay {
    float ix, iy, iz;   // 1 / |d_a|
    float bx, by, bz;   // t(v) = v * i_a + b_a for the mirrored plane v
    uint32_t flip;      // bit a: d_a < 0 in the frame (axis mirrored)
    uint32_t K;
};

__device__ __forceinline__ float min3f(float a, float b, float c) { return fminf(fminf(a, b), c); }
__device__ __forceinline__ float max3f(float a, float b, float c) { return fmaxf(fmaxf(a, b), c); }

// Map the ray into frame F and clip it to the root cell [0, 2^K)^3.
// Returns false when the clipped interval [t0, t1] is empty.  eaxis = axis
// of the entry face, 3 when the ray starts inside (t0 = tmin).
__device__ __forceinline__ bool frame_setup(const FrameRec& F, const Ray& r, float tlimit, FrameRay& fr, float& t0,
                                            int& eaxis) {
    const float gx = fmaf(F.m[0], r.ox, fmaf(F.m[1], r.oy, fmaf(F.m[2], r.oz, F.m[3])));
    const float gy = fmaf(F.m[4], r.ox, fmaf(F.m[5], r.oy, fmaf(F.m[6], r.oz, F.m[7])));
    const float gz = fmaf(F.m[8], r.ox, fmaf(F.m[9], r.oy, fmaf(F.m[10], r.oz, F.m[11])));
    float dx = fmaf(F.m[0], r.dx, fmaf(F.m[1], r.dy, F.m[2] * r.dz));
    float dy = fmaf(F.m[4], r.dx, fmaf(F.m[5], r.dy, F.m[6] * r.dz));
    float dz = fmaf(F.m[8], r.dx, fmaf(F.m[9], r.dy, F.m[10] * r.dz));
    const uint32_t K = (F.info >> FR_K_SHIFT) & FR_K_MASK;
    const float N = (float)(1u << K);
    // A zero component would make 0 * inf; a tiny one of the same sign keeps
    // every plane crossing finite and far outside the root cell.
    const float eps = max3f(fabsf(dx), fabsf(dy), fabsf(dz)) * 0x1p-21f;
    if (fabsf(dx) < eps) dx = copysignf(eps, dx);
    if (fabsf(dy) < eps) dy = copysignf(eps, dy);
    if (fabsf(dz) < eps) dz = copysignf(eps, dz);
    fr.flip = (dx < 0.f ? 1u : 0u) | (dy < 0.f ? 2u : 0u) | (dz < 0.f ? 4u : 0u);
    fr.ix = 1.0f / fabsf(dx);
    fr.iy = 1.0f / fabsf(dy);
    fr.iz = 1.0f / fabsf(dz);
    fr.bx = -((dx < 0.f) ? (N - gx) : gx) * fr.ix;
    fr.by = -((dy < 0.f) ? (N - gy) : gy) * fr.iy;
    fr.bz = -((dz < 0.f) ? (N - gz) : gz) * fr.iz;
    fr.K = K;
    // root entry: the low mirrored planes are at 0, so t(0) = bias
    float te = max3f(fr.bx, fr.by, fr.bz);
    eaxis = (fr.bx >= fr.by && fr.bx >= fr.bz) ? 0 : ((fr.by >= fr.bz) ? 1 : 2);
    const float tx = min3f(fmaf(N, fr.ix, fr.bx), fmaf(N, fr.iy, fr.by), fmaf(N, fr.iz, fr.bz));
    if (te < r.tmin) {
        te = r.tmin;
        eaxis = 3;
    }
    t0 = te;
    return te <= fminf(tx, tlimit);
}

// Front-to-back walk of one frame.  Returns 1 on a hit (t_hit, id_hit,
// axis_hit set), 0 when the frame has no hit before tlimit, 2 when the step
// limit is reached.  stk points at this lane's column of the wave's stack
// (entry for level l at stk[l * 64]).
__device__ __forceinline__ int frame_walk(const uint64_t* __restrict__ nodes, const uint64_t* lds_nodes,
                                          uint32_t n_lds, uint2* stk, const FrameRec& F, const FrameRay& fr,
                                          float t0, int eaxis, float tlimit, uint32_t step_limit, uint32_t& steps,
                                          float& t_hit, uint32_t& id_hit, int& axis_hit) {
    const uint32_t K = fr.K;
    uint32_t pmask = F.info & FR_MASK;
    uint32_t pchild = F.child;
    uint32_t lvl = 1;
    uint32_t size = 1u << (K - 1);
    // first child: upper half on every axis whose mid plane is crossed before entry
    uint32_t px = (fmaf((float)size, fr.ix, fr.bx) <= t0) ? size : 0u;
    uint32_t py = (fmaf((float)size, fr.iy, fr.by) <= t0) ? size : 0u;
    uint32_t pz = (fmaf((float)size, fr.iz, fr.bz) <= t0) ? size : 0u;
    float tc0 = t0;
    for (;;) {
        if (++steps > step_limit) return 2;
        const float ex = fmaf((float)(px + size), fr.ix, fr.bx);
        const float ey = fmaf((float)(py + size), fr.iy, fr.by);
        const float ez = fmaf((float)(pz + size), fr.iz, fr.bz);
        const float tc1 = min3f(ex, ey, ez);
        const uint32_t oct = (((px & size) ? 1u : 0u) | ((py & size) ? 2u : 0u) | ((pz & size) ? 4u : 0u)) ^ fr.flip;
        if ((pmask >> oct) & 1u) {
            const uint32_t cidx = pchild + __popc(pmask & ((1u << oct) - 1u));
            const uint64_t w = (cidx < n_lds) ? lds_nodes[cidx] : nodes[cidx];
            const uint32_t w0 = (uint32_t)w;
            const uint32_t w1 = (uint32_t)(w >> 32);
            const uint32_t cm = w0 & 0xFFu;
            if (cm == 0u) {
                t_hit = tc0;
                id_hit = cidx;
                axis_hit = eaxis;
                return 1;
            }
            if (!(w1 & 0x80000000u)) {
                stk[lvl * 64] = make_uint2(pchild, pmask);
                const uint32_t c24 = w0 >> 8;
                pchild = (c24 == 0xFFFFFFu) ? w1 : cidx + c24;
                pmask = cm;
                ++lvl;
                size >>= 1;
                px += (fmaf((float)(px + size), fr.ix, fr.bx) <= tc0) ? size : 0u;
                py += (fmaf((float)(py + size), fr.iy, fr.by) <= tc0) ? size : 0u;
                pz += (fmaf((float)(pz + size), fr.iz, fr.bz) <= tc0) ? size : 0u;
                continue;
            }
            // a transformed child belongs to another frame: empty here
        }
        // leave the current cell through its nearest exit plane(s)
        if (tc1 > tlimit) return 0;
        const uint32_t step = (ex == tc1 ? 1u : 0u) | (ey == tc1 ? 2u : 0u) | (ez == tc1 ? 4u : 0u);
        if (step == 0u) return 0;  // non-finite crossing: nothing more to find
        const uint32_t nx = px + ((step & 1u) ? size : 0u);
        const uint32_t ny = py + ((step & 2u) ? size : 0u);
        const uint32_t nz = pz + ((step & 4u) ? size : 0u);
        const uint32_t diff = (nx ^ px) | (ny ^ py) | (nz ^ pz);
        const uint32_t h = 31u - __clz(diff);
        if (h >= K) return 0;  // left the frame's root cell
        const uint32_t nsize = 1u << h;
        const uint32_t keep = ~(nsize - 1u);
        px = nx & keep;
        py = ny & keep;
        pz = nz & keep;
        const uint32_t nlvl = K - h;
        if (nlvl < lvl) {
            const uint2 e = stk[nlvl * 64];
            pchild = e.x;
            pmask = e.y;
        }
        lvl = nlvl;
        size = nsize;
        tc0 = tc1;
        eaxis = __ffs(step) - 1;
    }
}

__device__ __forceinline__ bool ray_valid(const Ray& r) {
    const bool fin = isfinite(r.ox) && isfinite(r.oy) && isfinite(r.oz) && isfinite(r.dx) && isfinite(r.dy) &&
                     isfinite(r.dz);
    const bool nonzero = (r.dx != 0.f) || (r.dy != 0.f) || (r.dz != 0.f);
    return fin && nonzero && !isnan(r.tmin) && !isnan(r.tmax) && r.tmin <= r.tmax && r.tmin < INFINITY;
}

}  // namespace

__global__ __launch_bounds__(512) void trace_kernel(TraceArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint64_t* lds_nodes = reinterpret_cast<uint64_t*>(smem);
    FrameRec* lds_frames = reinterpret_cast<FrameRec*>(smem + (size_t)a.lds_nodes * 8);
    uint2* lds_stack = reinterpret_cast<uint2*>(smem + (size_t)a.lds_nodes * 8 + (size_t)a.n_frames * 64);

    for (uint32_t i = threadIdx.x; i < a.lds_nodes; i += blockDim.x) lds_nodes[i] = a.nodes[i];
    {
        const uint4* src = reinterpret_cast<const uint4*>(a.frames);
        uint4* dst = reinterpret_cast<uint4*>(lds_frames);
        for (uint32_t i = threadIdx.x; i < a.n_frames * 4u; i += blockDim.x) dst[i] = src[i];
    }
    __syncthreads();

    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = threadIdx.x >> 6;
    uint2* stk = lds_stack + (size_t)wave * a.stack_levels * 64 + lane;

    for (;;) {
        uint32_t tile = 0;
        if (lane == 0) tile = atomicAdd(&a.queue[0], 1u);
        tile = __shfl(tile, 0);
        const uint64_t base = (uint64_t)tile * 64u;
        if (base >= a.n_rays) break;
        const uint64_t i = base + lane;
        if (i >= a.n_rays) continue;

        const float4 r0 = a.rays[2 * i];
        const float4 r1 = a.rays[2 * i + 1];
        const Ray r{r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w};

        float best_t = INFINITY;
        uint32_t best_id = kNone, best_inst = kNone;
        int best_frame = -1, best_axis = 3;
        uint32_t steps = 0;
        bool limit = false;

        if (ray_valid(r)) {
            // world frame
            const FrameRec& W = lds_frames[0];
            if (!(W.info & FR_EMPTY)) {
                FrameRay fr;
                float t0;
                int ea;
                if (frame_setup(W, r, r.tmax, fr, t0, ea)) {
                    if (W.info & FR_ROOT_LEAF) {
                        best_t = t0;
                        best_id = W.root;
                        best_inst = W.inst;
                        best_axis = ea;
                        best_frame = 0;
                    } else {
                        float th;
                        uint32_t ih;
                        int ah;
                        const int res = frame_walk(a.nodes, lds_nodes, a.lds_nodes, stk, W, fr, t0, ea, r.tmax,
                                                   a.step_limit, steps, th, ih, ah);
                        if (res == 1) {
                            best_t = th;
                            best_id = ih;
                            best_inst = W.inst;
                            best_axis = ah;
                            best_frame = 0;
                        } else if (res == 2) {
                            limit = true;
                        }
                    }
                }
            }
            // candidate frames, nearest root-cell entry first
            uint64_t done = 0;
            while (!limit) {
                const float tl = fminf(r.tmax, best_t);
                float bestc = INFINITY;
                int pick = -1;
                for (uint32_t c = 0; c < a.n_cand; ++c) {
                    if ((done >> c) & 1ull) continue;
                    FrameRay fr;
                    float t0;
                    int ea;
                    if (frame_setup(lds_frames[1 + c], r, tl, fr, t0, ea) && (pick < 0 || t0 < bestc)) {
                        bestc = t0;
                        pick = (int)c;
                    }
                }
                if (pick < 0) break;
                done |= 1ull << pick;
                const FrameRec& F = lds_frames[1 + pick];
                FrameRay fr;
                float t0;
                int ea;
                frame_setup(F, r, tl, fr, t0, ea);
                float th;
                uint32_t ih;
                int ah;
                const int res = frame_walk(a.nodes, lds_nodes, a.lds_nodes, stk, F, fr, t0, ea, tl, a.step_limit,
                                           steps, th, ih, ah);
                if (res == 1) {
                    const uint32_t inst = F.inst;
                    if (th < best_t || (th == best_t && (inst < best_inst || (inst == best_inst && ih < best_id)))) {
                        best_t = th;
                        best_id = ih;
                        best_inst = inst;
                        best_axis = ah;
                        best_frame = 1 + pick;
                    }
                } else if (res == 2) {
                    limit = true;
                }
            }
        }

        float nx = 0.f, ny = 0.f, nz = 0.f;
        if (limit) {
            best_id = kStepLimitId;
            best_inst = kNone;
            best_t = INFINITY;
        } else if (best_frame >= 0 && best_axis < 3) {
            // outward normal: -sgn(d_a) e_a in the frame, mapped by M^T (row a of M)
            const FrameRec& F = lds_frames[best_frame];
            const float* row = &F.m[4 * best_axis];
            const float da = fmaf(row[0], r.dx, fmaf(row[1], r.dy, row[2] * r.dz));
            const float s = (da < 0.f) ? 1.f : -1.f;
            const float inv = s / sqrtf(fmaf(row[0], row[0], fmaf(row[1], row[1], row[2] * row[2])));
            nx = row[0] * inv;
            ny = row[1] * inv;
            nz = row[2] * inv;
        }
        a.out_id[i] = best_id;
        if (a.out_inst) a.out_inst[i] = best_inst;
        a.out_t[i] = best_t;
        if (a.out_n) {
            a.out_n[3 * i] = nx;
            a.out_n[3 * i + 1] = ny;
            a.out_n[3 * i + 2] = nz;
        }
    }

    // the last work-group out resets the queue for the next launch
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t prev = atomicAdd(&a.queue[1], 1u);
        if (prev == gridDim.x - 1) {
            atomicExch(&a.queue[0], 0u);
            atomicExch(&a.queue[1], 0u);
        }
    }
}

size_t trace_lds_bytes(uint32_t lds_nodes, uint32_t n_frames, uint32_t stack_levels, uint32_t waves_per_block) {
    return (size_t)lds_nodes * 8 + (size_t)n_frames * 64 + (size_t)waves_per_block * stack_levels * 64 * 8;
}

hipError_t launch_trace(const TraceArgs& a, const LaunchCfg& c, hipStream_t stream) {
    hipLaunchKernelGGL(trace_kernel, dim3(c.blocks), dim3(c.waves_per_block * 64), c.lds_bytes, stream, a);
    return hipGetLastError();
}

}  // namespace svo
