// First-hit traversal of sparse voxel octrees with transformed subtrees, for
// gfx950 (wave64; no matrix cores: the work is dependent 8-byte gathers).
//
// Per ray (one lane each):
//   1. map the world ray into a frame's grid coordinates (paper Eq. 2-3 with
//      the scale folded into the affine map, Sec. 3.2); t is not rescaled;
//   2. mirror axes with a negative direction so every component is positive;
//      a plane crossing is then t(v) = v * invd + bias, one FMA, evaluated by
//      the same formula for every cell sharing that plane;
//   3. walk the frame's octree front to back, top-down (the role of the
//      parametric traversal in the paper, Sec. 5): integer cell corners, a
//      per-level LDS stack of (child start, mask), and an exit by the highest
//      changed coordinate bit, so popping needs no search (5 bytes per
//      level and lane: a 32-bit child start and an 8-bit mask);
//   4. at a transformed node whose moved content stays inside its static
//      cell, switch into that node's frame in place (Sec. 3, Fig. 1: the ray,
//      not the model, is transformed) and resume the enclosing walk after it;
//   5. transformed subtrees that leave their static cell are candidates,
//      traced from their own roots and skipped once their entry lies beyond
//      the best hit (the depth sort of Sec. 4.2): up to 16 in order of exact
//      root-cell entry after the bounding-sphere test of Sec. 4.1, more
//      through a hierarchy of their world boxes, nearer boxes first;
//   6. at the hit, recompute its entry t and face from the frame's FP64 map
//      (the walk's FP32 entry t carries an error that grows with the
//      coordinates); write id, slot, t and the normal (entry face, inverse
//      transpose).
//
// Work distribution: a persistent grid.  Each wave keeps 64 rays in flight
// and refills lanes once `refill` of them are idle (64 = whole tiles), from
// a range of `claim` rays it takes at once from one of kQueueParts counters
// (claims interleaved over the counters, each wave starting on its own), so
// that no single address serialises the claims.  Claims visit the 64-ray
// tiles in a stride permutation, so that expensive regions of an image (rays
// grazing a surface) spread over time and over waves instead of reaching a
// few waves back to back.  The last work-group to finish resets the counters
// so the next launch on the stream starts from zero.
//
// Slow tiles first (one-job launches with whole tiles): a launch ends when
// its longest chains of walk steps do, and the same rays traced again (an
// animation under a fixed camera) have their costliest tiles in nearly the
// same places.  Each launch lists the tiles whose longest ray took the most
// advances in its work queue's state (kHot*), and the next launch on the same
// rays deals those tiles to its waves before any regular claim, while the
// regular order skips them; results never depend on the order.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <type_traits>

#include "svo_camera.h"
#include "svo_internal.h"

namespace svo {

namespace {

constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint32_t kStepLimitId = 0xFFFFFFFEu;
constexpr uint32_t kXform = 0x80000000u;

enum : uint32_t { M_DONE = 0, M_WALK = 1, M_SELECT = 2 };
enum : uint32_t { EV_NONE = 0, EV_HIT = 1, EV_ENTER = 2, EV_END = 3, EV_LIMIT = 4 };
enum : uint32_t { PEND_RESUME = 1, PEND_ROOT_HIT = 2 };

struct Ray {
    float ox, oy, oz, tmin, dx, dy, dz, tmax;
};

// A ray in one frame's mirrored grid coordinates.
struct FrameRay {
    float ix, iy, iz;   // 1 / |d_a|
    float bx, by, bz;   // t(v) = v * i_a + b_a for the mirrored plane v
    uint32_t flip;      // bit a: d_a < 0 in the frame (axis mirrored)
    uint32_t K;         // frame height
};

__device__ __forceinline__ float min3f(float a, float b, float c) { return fminf(fminf(a, b), c); }

// Reciprocal, square root and reciprocal square root on the hardware units
// (v_rcp_f32, v_sqrt_f32, v_rsq_f32: about 1 ulp) instead of the correctly
// rounded sequences.  Uses: the walk's plane parameters (one reciprocal per
// axis, used for every plane, so the walk stays self-consistent and
// monotone), the inflated bounding-sphere test and normals.  Arguments stay
// in the normal range: rays whose direction is below 2^-100 in every
// component miss (ray_valid), and a frame's clamped components are at least
// 2^-21 of its largest.
__device__ __forceinline__ float rcp_fast(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float sqrt_fast(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float rsq_fast(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float max3f(float a, float b, float c) { return fmaxf(fmaxf(a, b), c); }

// Map the ray into frame F and clip it to the root cell [0, 2^K)^3 and
// [tmin, tlimit].  Returns false when that interval is empty.  kPrecise:
// the plane parameters take correctly rounded reciprocals (a walk runs on
// them, and the error of every plane crossing it compares includes theirs:
// on the depth-12 terrain this takes the share of rays whose voxel differs
// from the exact one by about a tenth); otherwise the hardware reciprocal
// (entry tests that only order or cull).
template <bool kPrecise>
__device__ __forceinline__ bool frame_setup(const FrameRec& F, const Ray& r, float tlimit, FrameRay& fr, float& t0) {
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
    if constexpr (kPrecise) {
        fr.ix = 1.0f / fabsf(dx);
        fr.iy = 1.0f / fabsf(dy);
        fr.iz = 1.0f / fabsf(dz);
    } else {
        fr.ix = rcp_fast(fabsf(dx));
        fr.iy = rcp_fast(fabsf(dy));
        fr.iz = rcp_fast(fabsf(dz));
    }
    fr.bx = -((dx < 0.f) ? (N - gx) : gx) * fr.ix;
    fr.by = -((dy < 0.f) ? (N - gy) : gy) * fr.iy;
    fr.bz = -((dz < 0.f) ? (N - gz) : gz) * fr.iz;
    fr.K = K;
    // root entry: the low mirrored planes are at 0, so t(0) = bias
    float te = max3f(fr.bx, fr.by, fr.bz);
    const float tx = min3f(fmaf(N, fr.ix, fr.bx), fmaf(N, fr.iy, fr.by), fmaf(N, fr.iz, fr.bz));
    if (te < r.tmin) te = r.tmin;
    t0 = te;
    return te <= fminf(tx, tlimit);
}

// Slow-tiles-first state (see kHotHdr): which list is the input, the
// threshold, a list's tiles and its bitmap.  The header stays fixed during a
// launch until its last work-group rewrites it.
__device__ __forceinline__ uint32_t hot_in(const uint32_t* hot) { return hot[0] & 1u; }
__device__ __forceinline__ uint32_t hot_thr(const uint32_t* hot) { return hot[1] ? hot[1] : kHotInitialThreshold; }
__device__ __forceinline__ uint32_t* hot_cnt(uint32_t* hot, uint32_t b, uint32_t s) {
    return hot + kHotCntBase + (b * kHotSub + s) * kHotLine;
}
__device__ __forceinline__ uint32_t* hot_sum(uint32_t* hot, uint32_t s) { return hot + kHotSumBase + s * kHotLine; }
__device__ __forceinline__ uint32_t* hot_max(uint32_t* hot, uint32_t s) { return hot + kHotMaxBase + s * kHotLine; }
__device__ __forceinline__ uint32_t* hot_list(uint32_t* hot, uint32_t b) { return hot + kHotHdr + b * kHotCap; }
__device__ __forceinline__ uint32_t* hot_bits(uint32_t* hot, uint32_t b) {
    return hot + kHotHdr + 2 * kHotCap + b * kHotBitsWords;
}

// The largest of a wave's 64 values, wave-uniform: within each row of 16
// lanes by DPP moves (swap neighbours, swap pairs, mirror the half-rows,
// mirror the rows), then over the four rows by lane reads.  Every lane must
// be active.
__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));  // row_half_mirror
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));  // row_mirror
    const uint32_t r = max(max((uint32_t)__builtin_amdgcn_readlane((int)v, 0), (uint32_t)__builtin_amdgcn_readlane((int)v, 16)),
                           max((uint32_t)__builtin_amdgcn_readlane((int)v, 32), (uint32_t)__builtin_amdgcn_readlane((int)v, 48)));
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)r);
}

// The slow-tile state's address from a work-group's LDS header.
__device__ __forceinline__ uint32_t* lds_hot_ptr(const uint32_t* lds_hot) {
    return reinterpret_cast<uint32_t*>((uint64_t)lds_hot[kHotLdsPtr] | ((uint64_t)lds_hot[kHotLdsPtr + 1] << 32));
}
// A wave-uniform value in scalar registers of its own.
__device__ __forceinline__ uint32_t uniform_u32(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
template <typename T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    return reinterpret_cast<T*>((uint64_t)uniform_u32((uint32_t)v) | ((uint64_t)uniform_u32((uint32_t)(v >> 32)) << 32));
}

// The hit the walk found, checked and measured in FP64.  The walk decides
// in FP32 which cell the ray meets first; its plane crossings carry an
// error that grows with the coordinates (frame map, reciprocal direction,
// rounding at the scale of t), so near an edge or a corner it may take a
// cell the ray passes by, and its entry t is off by that much.  Here the
// cell [p, p + size)^3 (p in frame F's mirrored grid coordinates) is
// intersected with the ray mapped by F's exact map X in FP64 (Eq. 2: the
// frame's ray keeps the world t): per axis the closed slab between the
// cell's two face planes.  Returns whether max(t_near, tmin) <= min(t_far,
// tmax) holds in FP64; then t = max(t_near, tmin) and axis = the entry face
// (the largest t_near, ties to the lowest axis), 3 when the ray starts
// inside the cell (t = tmin).
__device__ __forceinline__ bool exact_hit(const double* X, const Ray& r, const FrameRay& fr, uint32_t px,
                                          uint32_t py, uint32_t pz, uint32_t size, float& t, int& axis) {
    const double N = (double)(1ull << fr.K), S = (double)size;
    double tn = -INFINITY, tf = INFINITY;
    int ea = 3;
    // one axis at a time: a row's four doubles are the only FP64 values live
#pragma unroll 1
    for (int k = 0; k < 3; ++k) {
        const double* row = X + 4 * k;
        const double go = fma(row[0], (double)r.ox, fma(row[1], (double)r.oy, fma(row[2], (double)r.oz, row[3])));
        const double gd = fma(row[0], (double)r.dx, fma(row[1], (double)r.dy, row[2] * (double)r.dz));
        const uint32_t pk = (k == 0) ? px : ((k == 1) ? py : pz);
        const double lo = ((fr.flip >> k) & 1u) ? N - (double)pk - S : (double)pk;
        const double hi = lo + S;
        double a, b;
        if (gd == 0.0) {
            // parallel: the whole line or nothing
            a = (go >= lo && go <= hi) ? -INFINITY : INFINITY;
            b = (go >= lo && go <= hi) ? INFINITY : -INFINITY;
        } else {
            // reciprocal: hardware estimate and two Newton steps (within an
            // ulp or two of 1 / gd; gd is far from the subnormal range)
            double inv = __builtin_amdgcn_rcp(gd);
            inv = fma(inv, fma(-gd, inv, 1.0), inv);
            inv = fma(inv, fma(-gd, inv, 1.0), inv);
            const double t1 = (lo - go) * inv, t2 = (hi - go) * inv;
            a = fmin(t1, t2);
            b = fmax(t1, t2);
        }
        if (a > tn) {
            tn = a;
            ea = k;
        }
        tf = fmin(tf, b);
    }
    double te = tn;
    if (!(te >= (double)r.tmin)) {
        te = (double)r.tmin;
        ea = 3;
    }
    t = (float)te;
    axis = ea;
    return te <= fmin(tf, (double)r.tmax);
}

// Bounding-sphere test of the paper's Sec. 4.1 (Eq. 4), made conservative
// for FP32: false only when the ray segment [tmin, tlimit] certainly misses
// the sphere (its perpendicular distance exceeds the radius, or the sphere
// lies wholly before tmin or after tlimit).  To absorb rounding the radius
// is inflated by a relative 1e-4, and its square by 1e-6 of the squared
// centre distance (about 1e-3 of the distance).
__device__ __forceinline__ bool sphere_may_hit(const float4 sp, const Ray& r, float tlimit) {
    const float lx = sp.x - r.ox, ly = sp.y - r.oy, lz = sp.z - r.oz;
    const float dd = fmaf(r.dx, r.dx, fmaf(r.dy, r.dy, r.dz * r.dz));
    const float ll = fmaf(lx, lx, fmaf(ly, ly, lz * lz));
    const float tca = fmaf(lx, r.dx, fmaf(ly, r.dy, lz * r.dz));
    const float rr = sp.w * 1.0001f;
    const float r2 = fmaf(rr, rr, 1e-6f * ll);
    const float idd = rcp_fast(dd);
    const float perp2 = ll - tca * tca * idd;           // squared distance of the line from the centre
    if (perp2 > r2) return false;
    const float half = sqrt_fast(fmaxf(r2 - perp2, 0.f) * idd);  // half chord, in t
    const float tc = tca * idd;                                    // t of the closest approach
    return (tc - half <= tlimit) && (tc + half >= r.tmin);
}

// Entry t of the ray into a hierarchy box over [tmin, tlimit], +inf when the
// box is missed or entered beyond tlimit (i*: inverse world direction).
__device__ __forceinline__ float box_entry(const BvhNode& B, const Ray& r, float ix, float iy, float iz,
                                           float tlimit) {
    const float ax = (B.lo[0] - r.ox) * ix, bx = (B.hi[0] - r.ox) * ix;
    const float ay = (B.lo[1] - r.oy) * iy, by = (B.hi[1] - r.oy) * iy;
    const float az = (B.lo[2] - r.oz) * iz, bz = (B.hi[2] - r.oz) * iz;
    const float t0 = fmaxf(max3f(fminf(ax, bx), fminf(ay, by), fminf(az, bz)), r.tmin);
    const float t1 = fminf(min3f(fmaxf(ax, bx), fmaxf(ay, by), fmaxf(az, bz)), tlimit);
    return (t0 <= t1) ? t0 : INFINITY;
}

// Inverse world direction for the hierarchy's box tests, tiny components
// clamped as in frame_setup (so no 0 * inf).
__device__ __forceinline__ void inv_world_dir(const Ray& r, float& ix, float& iy, float& iz) {
    const float eps = max3f(fabsf(r.dx), fabsf(r.dy), fabsf(r.dz)) * 0x1p-21f;
    ix = rcp_fast(fabsf(r.dx) < eps ? copysignf(eps, r.dx) : r.dx);
    iy = rcp_fast(fabsf(r.dy) < eps ? copysignf(eps, r.dy) : r.dy);
    iz = rcp_fast(fabsf(r.dz) < eps ? copysignf(eps, r.dz) : r.dz);
}

__device__ __forceinline__ bool ray_valid(const Ray& r) {
    const bool fin = isfinite(r.ox) && isfinite(r.oy) && isfinite(r.oz) && isfinite(r.dx) && isfinite(r.dy) &&
                     isfinite(r.dz);
    const bool nonzero = max3f(fabsf(r.dx), fabsf(r.dy), fabsf(r.dz)) >= 0x1p-100f;
    return fin && nonzero && !isnan(r.tmin) && !isnan(r.tmax) && r.tmin <= r.tmax && r.tmin < INFINITY;
}

__host__ __device__ __forceinline__ size_t align16(size_t v) { return (v + 15) & ~(size_t)15; }

// Pointers read out of LDS job records lose their address space; these
// accessors restore it so the compiler emits global (not generic) loads and
// stores.
typedef float v4f __attribute__((ext_vector_type(4)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

template <typename T>
__device__ __forceinline__ T gld(const T* p, uint64_t i) {
    return ((const __attribute__((address_space(1))) T*)p)[i];
}
template <typename T>
__device__ __forceinline__ void gst(T* p, uint64_t i, T v) {
    ((__attribute__((address_space(1))) T*)p)[i] = v;
}

}  // namespace

// Per-lane candidate state in LDS: the entry table (sorted path) or the
// hierarchy stack of box indices, one more than its levels.
__host__ __device__ __forceinline__ size_t cand_lane_bytes(const TraceArgs& a) {
    return a.sort_cand ? (size_t)a.max_cand * 4 : (a.max_cand ? (size_t)(a.bvh_depth + 1) * 4 : 0);
}

size_t trace_lds_bytes(const TraceArgs& a, uint32_t waves_per_block) {
    const size_t shared = align16((size_t)a.lds_nodes * 8) + (size_t)a.n_frames * 80 +
                          align16((size_t)a.n_cand_total * 4) + (size_t)a.n_jobs * sizeof(JobRec) +
                          (size_t)a.n_bvh_total * sizeof(BvhNode) + (a.jobs ? 0 : kHotLdsBytes) +
                          (a.has_cam0 ? sizeof(CameraArgs) : 0);
    const size_t per_wave = cand_lane_bytes(a) * 64 + (size_t)a.stack_levels * 64 * 5 + (size_t)a.nest_levels * 64 * 16;
    return shared + per_wave * waves_per_block;
}

// kSorted: every job's candidates go through the per-lane entry table (at
// most 16 of them); otherwise through the per-frame box hierarchy.  A launch
// uses one of the two, and each instantiation carries only its own path,
// which keeps the sorted one at fewer registers.  The sorted one is compiled
// for 6 resident waves per SIMD (80 VGPRs): the few values that then go to
// scratch are per-ray state outside the walk loop, and the extra waves hide
// more of the node-load latency.  The hierarchy one keeps its natural
// count (102 VGPRs single-job, 110 batched): forcing it lower spills inside
// its candidate search.
// kSingle: a one-job launch (the job in the arguments), whose pool, cache
// size and table offsets are then launch-wide values (scalar registers)
// rather than per-lane ones.
// kInline: the frame table comes in the arguments (TraceArgsInline).
// kCount: the counting build (TraceArgs::counts and trail), for tests and
// measurement only.
template <bool kSorted, bool kSingle, bool kInline = false, bool kCount = false>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(kSorted ? 6 : 1, 8))) void trace_kernel(
    typename std::conditional<kInline, TraceArgsInline, TraceArgs>::type a) {
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned char* p = smem;
    uint64_t* lds_nodes = reinterpret_cast<uint64_t*>(p);
    p += align16((size_t)a.lds_nodes * 8);
    FrameRec* lds_frames = reinterpret_cast<FrameRec*>(p);
    p += (size_t)a.n_frames * 64;
    float4* lds_sph = reinterpret_cast<float4*>(p);
    p += (size_t)a.n_frames * 16;
    uint32_t* lds_cand = reinterpret_cast<uint32_t*>(p);
    p += align16((size_t)a.n_cand_total * 4);
    JobRec* lds_jobs = reinterpret_cast<JobRec*>(p);
    p += (size_t)a.n_jobs * sizeof(JobRec);
    BvhNode* lds_bvh = reinterpret_cast<BvhNode*>(p);
    p += (size_t)a.n_bvh_total * sizeof(BvhNode);
    // slow tiles first (single-job launches): the work-group's header and the
    // tiles it lists
    uint32_t* lds_hot = reinterpret_cast<uint32_t*>(p);
    if (kSingle) p += kHotLdsBytes;
    // a single job's camera (read once per claim; kept in LDS rather than in
    // scalar registers for the whole launch)
    CameraArgs* lds_cam = reinterpret_cast<CameraArgs*>(p);
    if (a.has_cam0) p += sizeof(CameraArgs);
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = threadIdx.x >> 6;
    const size_t ent_bytes = cand_lane_bytes(a) * 64;
    const size_t per_wave = ent_bytes + (size_t)a.stack_levels * 64 * 5 + (size_t)a.nest_levels * 64 * 16;
    const uint32_t bst_cap = a.bvh_depth + 1;
    unsigned char* wp = p + per_wave * wave;
    float* ent = reinterpret_cast<float*>(wp) + lane;                                   // candidate c at ent[c * 64]
    // hierarchy stack entry k at bst[k * 64]: a box index; its entry is tested
    // again when popped, against the best hit by then
    uint32_t* bst = reinterpret_cast<uint32_t*>(wp) + lane;
    // traversal stack, slot l: child start at stkc[l * 64], child mask at stkm[l * 64]
    uint32_t* stkc = reinterpret_cast<uint32_t*>(wp + ent_bytes) + lane;
    uint8_t* stkm = reinterpret_cast<uint8_t*>(wp + ent_bytes + (size_t)a.stack_levels * 256) + lane;
    uint4* fst = reinterpret_cast<uint4*>(wp + ent_bytes + (size_t)a.stack_levels * 320) + lane;  // nest n at fst[n * 64]

    // launch-wide counts: the arguments, or a plan's header (capacities
    // above bound them, so every LDS copy below stays in its region)
    uint64_t n_rays = a.n_rays;
    uint32_t n_jobs = a.n_jobs, n_frames = a.n_frames, n_cand_total = a.n_cand_total, fill_nodes = a.lds_nodes;
    uint32_t n_bvh = a.n_bvh_total;
    const uint64_t* cache_src = a.cache_src;
    uint64_t tstride = a.tile_stride;
    if (a.hdr) {
        const LaunchHdr& h = *a.hdr;
        n_rays = h.n_rays;
        tstride = h.tile_stride;
        n_jobs = min(h.n_jobs, a.n_jobs);
        n_frames = min(h.n_frames, a.n_frames);
        n_cand_total = min(h.n_cand_total, a.n_cand_total);
        fill_nodes = min(h.lds_nodes, a.lds_nodes);
        n_bvh = min(h.n_bvh_total, a.n_bvh_total);
        cache_src = h.cache_src;
        if (!cache_src) fill_nodes = 0;
        if (n_jobs == 0) n_rays = 0;
    }
    // work-groups beyond what this launch's rays need (a plan's grid is
    // fixed) fill no LDS and claim nothing
    const uint32_t wpb = blockDim.x >> 6;
    const uint32_t n_active = (uint32_t)min((uint64_t)gridDim.x, (((n_rays + 63) >> 6) + wpb - 1) / wpb);
    const bool active = blockIdx.x < n_active;
    if (!active) {
        fill_nodes = 0;
        n_frames = 0;
        n_cand_total = 0;
        n_bvh = 0;
        n_jobs = 0;
    }
    for (uint32_t i = threadIdx.x; i < fill_nodes; i += blockDim.x) lds_nodes[i] = cache_src[i];
    // the frame table: in the arguments (small one-job launches) or in
    // device memory
    const FrameRec* src_frames = a.frames;
    const float4* src_sph = a.spheres;
    const uint32_t* src_cand = a.cand;
    const double* xmaps = a.xmaps;   // read only at hits: stays in global memory
    if constexpr (kInline) {
        src_frames = reinterpret_cast<const FrameRec*>(a.inline_tab);
        src_sph = reinterpret_cast<const float4*>(a.inline_tab + a.inline_off_sph);
        src_cand = reinterpret_cast<const uint32_t*>(a.inline_tab + a.inline_off_cand);
        xmaps = reinterpret_cast<const double*>(a.inline_tab + a.inline_off_x);
    }
    {
        const uint4* src = reinterpret_cast<const uint4*>(src_frames);
        uint4* dst = reinterpret_cast<uint4*>(lds_frames);
        for (uint32_t i = threadIdx.x; i < n_frames * 4u; i += blockDim.x) dst[i] = src[i];
    }
    for (uint32_t i = threadIdx.x; i < n_frames; i += blockDim.x) lds_sph[i] = src_sph[i];
    for (uint32_t i = threadIdx.x; i < n_cand_total; i += blockDim.x) lds_cand[i] = src_cand[i];
    {
        const uint4* src = reinterpret_cast<const uint4*>(a.bvh);
        uint4* dst = reinterpret_cast<uint4*>(lds_bvh);
        for (uint32_t i = threadIdx.x; i < n_bvh * 2u; i += blockDim.x) dst[i] = src[i];
    }
    if (a.jobs) {
        const uint4* src = reinterpret_cast<const uint4*>(a.jobs);
        uint4* dst = reinterpret_cast<uint4*>(lds_jobs);
        for (uint32_t i = threadIdx.x; i < n_jobs * (uint32_t)(sizeof(JobRec) / 16); i += blockDim.x) dst[i] = src[i];
    } else if (threadIdx.x == 0) {
        lds_jobs[0] = a.job0;
    }
    if (kSingle && a.has_cam0 && threadIdx.x == 0) *lds_cam = a.cam0;
    // slow tiles first: the previous launch's list is this launch's input if
    // it traced the same rays (same signature); this launch's own slow tiles
    // go to the other list.  The state's header words stay fixed until the
    // last work-group out rewrites them, so each work-group reads them once
    // into its LDS header; the main loop reads the header there and the
    // state's pointer from the arguments, which keeps them out of its scalar
    // registers.
    const uint64_t n_tiles = (n_rays + 63) >> 6;
    if (kSingle && threadIdx.x < kHotLdsHdr) {
        const uint32_t* hot = a.hot;
        const uint32_t t = threadIdx.x;
        uint32_t v = 0;
        if (hot && !a.hdr && n_tiles <= kHotMaxTiles) {
            // one round of loads: the words of both lists, then the input's
            const uint32_t b = hot_in(hot);
            if (t == kHotLdsOn) {
                const bool same = ((uint64_t)hot[4 + 2 * b] | ((uint64_t)hot[5 + 2 * b] << 32)) == a.hot_sig;
                v = (!same || hot[10 + b] || a.hot_seq % kHotResample == 0) ? 1u : 0u;
            } else if (t == kHotLdsIn) {
                v = b;
            } else if (t == kHotLdsThr) {
                v = hot_thr(hot);
            } else if (t == kHotLdsDeal) {
                uint32_t c0 = 0, c1 = 0;
                for (uint32_t k = 0; k < kHotSub; ++k) {
                    c0 = max(c0, hot[kHotCntBase + k * kHotLine]);
                    c1 = max(c1, hot[kHotCntBase + (kHotSub + k) * kHotLine]);
                }
                const bool d0 = hot[10] && ((uint64_t)hot[4] | ((uint64_t)hot[5] << 32)) == a.hot_sig;
                const bool d1 = hot[11] && ((uint64_t)hot[6] | ((uint64_t)hot[7] << 32)) == a.hot_sig;
                // entry e is sub-list e mod kHotSub's (e / kHotSub)-th
                if (b ? d1 : d0) v = min(b ? c1 : c0, kHotSubCap) * kHotSub;
            } else if (t >= kHotLdsCnt && t < kHotLdsCnt + kHotSub) {
                const uint32_t k = t - kHotLdsCnt;
                const uint32_t c0 = hot[kHotCntBase + k * kHotLine], c1 = hot[kHotCntBase + (kHotSub + k) * kHotLine];
                v = min(b ? c1 : c0, kHotSubCap);
            } else if (t == kHotLdsPtr || t == kHotLdsPtr + 1) {
                v = (uint32_t)(reinterpret_cast<uint64_t>(hot) >> (t == kHotLdsPtr ? 0 : 32));
            }
        }
        lds_hot[t] = v;
    }
    __syncthreads();

    const uint32_t refill = a.refill;
    const uint32_t claim = a.claim;
    // partition-local ray indices run to part_len (whole tiles); a wave owns
    // the claimed range [rlo, rhi) of partition q (wave-uniform state)
    const uint32_t part_len = (uint32_t)((n_tiles + kQueueParts - 1) / kQueueParts) * 64u;
    uint32_t q = (blockIdx.x * wpb + wave) % kQueueParts, rlo = 0, rhi = 0;
    uint64_t known_dry = 0;  // partitions this wave knows to be dry

    // per-lane state
    uint32_t mode = M_DONE;
    uint32_t ri = 0;           // ray index within its job (a launch holds at most 0xff000000 rays)
    uint32_t gray = 0, c_nodes = 0, c_frames = 0, c_trail = 0;   // counting build only
    uint32_t job = 0;
    // a single job's constants come from its LDS copy, made wave-uniform:
    // read from the arguments, they would share one wide scalar load with
    // fields the loop never uses, and be kept or spilled with them
    const uint64_t* nodes = kSingle ? uniform_ptr(lds_jobs[0].nodes) : nullptr;
    uint32_t n_lds = kSingle ? min(uniform_u32(lds_jobs[0].lds_nodes), fill_nodes) : 0u;
    uint32_t fbase = kSingle ? uniform_u32(lds_jobs[0].frame_base) : 0u;
    uint32_t cbase = kSingle ? uniform_u32(lds_jobs[0].cand_base) : 0u;
    uint32_t ncand = kSingle ? uniform_u32(lds_jobs[0].n_cand) : 0u;
    Ray r{};
    float best_t = INFINITY, tl = 0.f;
    uint32_t best_id = kNone, best_inst = kNone;
    int best_f = -1, best_axis = 3;
    uint32_t steps = 0;
    // the hierarchy walk over the candidates, packed (a job has at most 1023
    // candidates): bits 0-10 next item of the current leaf, 11-21 the
    // leaf's end, 22-31 stack depth
    uint32_t bws = 0;
    FrameRay fr{};
    uint32_t cur_f = 0, pmask = 0, pchild = 0, px = 0, py = 0, pz = 0, size = 1, nest = 0;
    // stack slots: the current frame's levels start at sbase; slot = sbase +
    // level of the current cell, top = sbase + K (so size = 2^(top - slot)).
    // Slot s holds the child start and mask of the node on the current path
    // whose children are the cells of level s - sbase: pchild and pmask are
    // always a copy of the current slot, so leaving cells up to any level is
    // a plain read.
    uint32_t slot = 1, sbase = 0, top = 0;
    uint32_t lds_last = n_lds ? n_lds - 1u : 0u;  // the last cached node index (0 with no cache: reads stay in bounds)
    float tc0 = 0.f;
    // what the next walk step does first: PEND_RESUME continue just past a
    // transformed cell the walk came back from; PEND_ROOT_HIT the frame root
    // is itself a solid leaf (recorded where every walk hit is)
    uint32_t pend = 0;
    bool exhausted = !active;  // wave-uniform
    // slow tiles first: the tile the wave's lanes are tracing (whole-tile
    // refill; set only while the launch keeps the slow-tile state)
    uint32_t cur_tile = 0xFFFFFFFFu;

    auto record_hit = [&](float t, uint32_t id, uint32_t f, int axis) {
        const uint32_t inst = lds_frames[f].inst;
        if (t < best_t || (t == best_t && (inst < best_inst || (inst == best_inst && id < best_id)))) {
            best_t = t;
            best_id = id;
            best_inst = inst;
            best_f = (int)f;
            best_axis = axis;
            tl = fminf(r.tmax, best_t);
        }
    };

    // Enter top-level frame f from its root.  Returns true when a walk starts.
    auto start_frame = [&](uint32_t f) -> bool {
        const FrameRec& F = lds_frames[f];
        if (F.info & FR_EMPTY) return false;
        float t0;
        if (!frame_setup<true>(F, r, tl, fr, t0)) return false;
        if constexpr (kCount) {
            ++c_frames;
            ++c_nodes;   // the frame's root record
        }
        cur_f = f;
        if (F.info & FR_ROOT_LEAF) {
            px = py = pz = 0u;
            size = 1u << fr.K;
            pend = PEND_ROOT_HIT;
            return true;
        }
        pmask = F.info & FR_MASK;
        pchild = F.child;
        sbase = 0;
        slot = 1;
        top = fr.K;
        stkc[slot * 64] = pchild;
        stkm[slot * 64] = (uint8_t)pmask;
        nest = 0;
        size = 1u << (fr.K - 1);
        px = (fmaf((float)size, fr.ix, fr.bx) <= t0) ? size : 0u;
        py = (fmaf((float)size, fr.iy, fr.by) <= t0) ? size : 0u;
        pz = (fmaf((float)size, fr.iz, fr.bz) <= t0) ? size : 0u;
        tc0 = t0;
        pend = 0;
        return true;
    };

    // Hit buffer (Sec. 4.3, for transforms on nodes): the outputs hold the
    // previous trace of this ray.  A previous hit in the static world frame
    // (or a miss) is still the answer unless some moved frame -- in place or
    // candidate -- now lies in front of it; the world frame itself never
    // changes.  Every moved frame (through the candidate hierarchy's boxes
    // when there is one) is tested up to the previous hit.
    auto previous_stands = [&]() -> bool {
        // a moved frame can hold a hit no later than tlim only if the ray
        // enters its root cell by then: the sphere first, then the exact
        // root-cell entry the walk itself uses (leaf entries never precede it)
        auto may_reach = [&](uint32_t f, float tlim) -> bool {
            if (!sphere_may_hit(lds_sph[f], r, tlim)) return false;
            FrameRay cfr;
            float t0;
            // the walk's own entry test rounds differently: widened so that
            // no frame a full trace would walk is ruled out here
            return frame_setup<false>(lds_frames[f], r, tlim + fabsf(tlim) * 0x1p-18f, cfr, t0);
        };
        const JobRec& J = lds_jobs[job];
        if (!J.out_inst) return false;
        const uint32_t pid = gld(J.out_id, ri);
        const uint32_t pinst = gld(J.out_inst, ri);
        const float pt = gld(J.out_t, ri);
        if (pinst != kNone || pid == kStepLimitId || isnan(pt)) return false;
        const float tlim = fminf(pt, r.tmax);
        const uint32_t nin = J.n_inline;
        for (uint32_t i = 0; i < nin; ++i)
            if (may_reach(lds_cand[cbase + ncand + i], tlim)) return false;
        if (ncand == 0) return true;
        if (kSorted) {
            for (uint32_t c = 0; c < ncand; ++c)
                if (may_reach(lds_cand[cbase + c], tlim)) return false;
            return true;
        }
        // any candidate box in front of the previous hit?
        float ix, iy, iz;
        inv_world_dir(r, ix, iy, iz);
        const uint32_t bbase = J.bvh_base;
        uint32_t sp = 0;
        if (box_entry(lds_bvh[bbase], r, ix, iy, iz, tlim) < INFINITY) bst[(sp++) * 64] = 0u;
        while (sp > 0u) {
            const BvhNode& N = lds_bvh[bbase + bst[(--sp) * 64]];
            if (N.b & kBvhLeaf) {
                for (uint32_t c = N.a; c < N.a + (N.b & 0xFFFFu); ++c)
                    if (may_reach(lds_cand[cbase + c], tlim)) return false;
                continue;
            }
            if (sp + 2u > bst_cap) return false;   // cannot happen (depth bound); trace it then
            if (box_entry(lds_bvh[bbase + N.a], r, ix, iy, iz, tlim) < INFINITY) bst[(sp++) * 64] = N.a;
            if (box_entry(lds_bvh[bbase + N.b], r, ix, iy, iz, tlim) < INFINITY) bst[(sp++) * 64] = N.b;
        }
        return true;
    };

    auto finish = [&]() {
        float nx = 0.f, ny = 0.f, nz = 0.f;
        if (best_id == kStepLimitId) {
            best_inst = kNone;
            best_t = INFINITY;
        } else if (best_f >= 0 && best_axis < 3) {
            // outward normal: -sgn(d_a) e_a in the frame, mapped by M^T (row a of M)
            const float* row = &lds_frames[best_f].m[4 * best_axis];
            const float da = fmaf(row[0], r.dx, fmaf(row[1], r.dy, row[2] * r.dz));
            const float s = (da < 0.f) ? 1.f : -1.f;
            const float inv = s * rsq_fast(fmaf(row[0], row[0], fmaf(row[1], row[1], row[2] * row[2])));
            nx = row[0] * inv;
            ny = row[1] * inv;
            nz = row[2] * inv;
        }
        const JobRec& J = lds_jobs[job];
        if constexpr (kCount) {
            gst(a.counts, (uint64_t)gray, c_nodes);
            gst(a.counts, n_rays + gray, c_frames);
            atomicAdd(a.counts + 2 * n_rays + gray, 1u);
        }
        gst(J.out_id, ri, best_id);
        if (J.out_inst) gst(J.out_inst, ri, best_inst);
        gst(J.out_t, ri, best_t);
        if (J.out_n) {
            gst(J.out_n, 3 * (uint64_t)ri, nx);
            gst(J.out_n, 3 * (uint64_t)ri + 1, ny);
            gst(J.out_n, 3 * (uint64_t)ri + 2, nz);
        }
        mode = M_DONE;
    };

    for (;;) {
        // ---------------------------------------------------------- refill
        const uint64_t idle = __ballot(mode == M_DONE);
        const uint32_t nidle = (uint32_t)__popcll(idle);
        if (nidle == 64u && cur_tile != 0xFFFFFFFFu) {
            // the wave's tile is done (whole tiles): listed when its slowest
            // ray took at least the threshold's advances
            const uint32_t m = wave_max(steps);
            steps = 0;   // lanes left without a ray in the next tile count nothing
            if (lane == 0u) {
                atomicAdd(lds_hot + kHotLdsSum, min(m, kHotCostClamp));
                atomicMax(lds_hot + kHotLdsMax, min(m, kHotCostClamp));
                if (m >= lds_hot[kHotLdsThr]) {
                    const uint32_t i = atomicAdd(lds_hot + kHotLdsListed, 1u);
                    if (i < kHotPerBlock) lds_hot[kHotLdsHdr + i] = cur_tile | (min(m, kHotEntryCostMax) << kHotTileBits);
                }
            }
            cur_tile = 0xFFFFFFFFu;
        }
        if (exhausted && nidle == 64u) break;
        if (!exhausted && nidle >= refill) {
            const uint32_t leader = (uint32_t)__ffsll((unsigned long long)idle) - 1u;
            bool retrace = false;
            // slow tiles first: whether this launch keeps the state, and
            // the input entries to deal out
            bool got_hot = false;
            uint32_t htile = 0, hcost = 0, hon = 0, hin = 0;
            if constexpr (kSingle) {
                hon = lds_hot[kHotLdsOn];
                hin = lds_hot[kHotLdsDeal];
            }
            if (hin && rlo >= rhi) {
                // the work-group's next entry, claimed by the leader for the
                // wave (hin and the counts stay fixed during the launch):
                // its k-th claim takes entry (k / wpb) W + blockIdx.x wpb +
                // k mod wpb, W = n_active wpb, so that the first W entries
                // go one to each wave of the grid in work-group order
                uint32_t k = 0;
                if (lane == leader) k = atomicAdd(lds_hot + kHotLdsTaken, 1u);
                k = (uint32_t)__shfl((int)k, (int)leader);
                const uint64_t e = (uint64_t)(k / wpb) * n_active * wpb + (uint64_t)blockIdx.x * wpb + k % wpb;
                const uint32_t sub = (uint32_t)(e % kHotSub), i = (uint32_t)(e / kHotSub);
                if (e < hin && i < lds_hot[kHotLdsCnt + sub]) {
                    got_hot = true;
                    const uint32_t ent = gld(hot_list(lds_hot_ptr(lds_hot), lds_hot[kHotLdsIn]), (uint64_t)sub * kHotSubCap + i);
                    htile = ent & kHotTileMask;
                    hcost = ent >> kHotTileBits;
                }
            }
            if constexpr (kSorted && kSingle) {
                // a dealt tile among the previous launch's costliest: its
                // wave issues ahead of the others on its SIMD while it runs
                // (a scalar branch: s_setprio ignores the lane mask)
                const bool up = got_hot && 10ull * hcost >= (uint64_t)kHotPrioTenths * lds_hot[kHotLdsThr];
                if (uniform_u32(up ? 1u : 0u)) __builtin_amdgcn_s_setprio(3);
                else __builtin_amdgcn_s_setprio(0);
            }
            if (!got_hot && rlo >= rhi) {
                // claim the next range of partition q.  A dry partition is
                // marked in the shared bitmap by the first wave to overflow
                // it, so a set bit always means dry (an unset one may be
                // stale); the wave moves on to the next partition it does not
                // know to be dry, and is done once it knows all of them are.
                uint32_t base = part_len;
                while (known_dry != ~0ull) {
                    uint32_t* ctr = a.queue + q * kQueueStride;
                    if (lane == leader) base = atomicAdd(ctr, claim);
                    base = __shfl(base, (int)leader);
                    if (base < part_len) break;
                    uint64_t dry = 0;
                    if (lane == leader) {
                        uint32_t* bm = a.queue + kQueueDry;
                        if (base < part_len + claim) atomicOr(bm + (q >> 5), 1u << (q & 31u));   // first to overflow
                        dry = (uint64_t)__hip_atomic_load(bm, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) |
                              ((uint64_t)__hip_atomic_load(bm + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) << 32);
                    }
                    known_dry |= __shfl(dry, (int)leader) | (1ull << q);
                    if (known_dry == ~0ull) break;
                    // the next partition after q not known to be dry, cyclically
                    const uint64_t open = ~known_dry;
                    const uint64_t above = open & ~((2ull << q) - 1ull);
                    q = (uint32_t)__ffsll((unsigned long long)(above ? above : open)) - 1u;
                }
                if (known_dry == ~0ull) {
                    exhausted = true;
                } else {
                    rlo = base;
                    rhi = min(base + claim, part_len);
                }
            }
            const uint32_t take = got_hot ? min(nidle, 64u) : ((rlo < rhi) ? min(nidle, rhi - rlo) : 0u);
            const uint32_t first = rlo;
            if (!got_hot) rlo += take;
            // a regular claim's tile (whole tiles: the same for every lane)
            // and the input bitmap's word for it, tested once the rays'
            // loads are on their way
            const uint64_t csl = (uint64_t)(first >> 6) * kQueueParts + q;
            const uint64_t ctile = (csl * tstride) % n_tiles;
            uint32_t cword = 0;
            if (take && !got_hot && hin) cword = gld(hot_bits(lds_hot_ptr(lds_hot), lds_hot[kHotLdsIn]), ctile >> 5);
            if (mode == M_DONE) {
                const uint32_t rank =
                    __builtin_amdgcn_mbcnt_hi((uint32_t)(idle >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)idle, 0u));
                const uint32_t j = first + rank;
                const uint64_t slot = (uint64_t)(j >> 6) * kQueueParts + q;     // claim order
                uint64_t gidx = n_rays;
                if (got_hot) {
                    if (rank < take && htile < n_tiles) gidx = (uint64_t)htile * 64u + rank;
                } else if (rank < take && slot < n_tiles) {
                    // a lane in the claim's first tile (every lane, with
                    // whole tiles) takes its tile from ctile
                    gidx = ((j >> 6) == (first >> 6) ? ctile : (slot * tstride) % n_tiles) * 64u + (j & 63u);
                }
                if (gidx < n_rays) {
                    if constexpr (kCount) {
                        gray = (uint32_t)gidx;
                        c_nodes = c_frames = c_trail = 0;
                    }
                    const float4* rays;
                    const CameraArgs* cam = nullptr;
                    if constexpr (kSingle) {
                        ri = (uint32_t)(gidx - lds_jobs[0].ray_begin);
                        rays = lds_jobs[0].rays;
                    } else {
                        // the job holding this launch-wide ray index (jobs are in ray order)
                        uint32_t lo = 0, hi = n_jobs;
                        while (hi - lo > 1u) {
                            const uint32_t mid = (lo + hi) >> 1;
                            if (lds_jobs[mid].ray_begin <= gidx) lo = mid; else hi = mid;
                        }
                        job = lo;
                        const JobRec& J = lds_jobs[job];
                        ri = (uint32_t)(gidx - J.ray_begin);
                        nodes = J.nodes;
                        n_lds = min(J.lds_nodes, fill_nodes);
                        lds_last = n_lds ? n_lds - 1u : 0u;
                        fbase = J.frame_base;
                        cbase = J.cand_base;
                        ncand = J.n_cand;
                        rays = J.rays;
                        cam = J.cam;
                    }
                    // the ray: read, or made from the job's camera (Fig. 5:
                    // one pixel sample per ray)
                    bool made = false;
                    if constexpr (kSingle) {
                        if (a.has_cam0) {
                            uint32_t w[sizeof(CameraArgs) / 4];
                            const uint32_t* src = reinterpret_cast<const uint32_t*>(lds_cam);
                            for (int k = 0; k < (int)(sizeof(CameraArgs) / 4); ++k) w[k] = uniform_u32(src[k]);
                            CameraArgs C;
                            std::memcpy(&C, w, sizeof C);
                            float4 c0, c1;
                            camera_ray(C, ri, c0, c1);
                            r = Ray{c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
                            made = true;
                        }
                    } else {
                        if (cam) {
                            // 96 bytes from global memory (six 16-byte loads)
                            v4u w[6];
                            for (int k = 0; k < 6; ++k) w[k] = gld(reinterpret_cast<const v4u*>(cam), k);
                            CameraArgs C;
                            std::memcpy(&C, w, sizeof C);
                            float4 c0, c1;
                            camera_ray(C, ri, c0, c1);
                            r = Ray{c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
                            made = true;
                        }
                    }
                    if (!made) {
                        const v4f* rp = reinterpret_cast<const v4f*>(rays);
                        const v4f r0 = gld(rp, 2 * (uint64_t)ri);
                        const v4f r1 = gld(rp, 2 * (uint64_t)ri + 1);
                        r = Ray{r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w};
                    }
                    best_t = INFINITY;
                    best_id = kNone;
                    best_inst = kNone;
                    best_f = -1;
                    best_axis = 3;
                    steps = 0;
                    bws = 0;
                    // a tile of the input list was traced by the wave it was dealt to
                    const bool dealt = !got_hot && ((cword >> (ctile & 31u)) & 1u);
                    bool keep = false;
                    if (!dealt && a.reuse && ray_valid(r)) keep = previous_stands();
                    if (dealt || keep) {
                        // nothing to trace or write: dealt to another wave, or
                        // the previous result stands
                    } else if (!ray_valid(r)) {
                        finish();
                    } else {
                        retrace = true;
                        tl = r.tmax;
                        if (kSorted) {
                            for (uint32_t c = 0; c < ncand; ++c) {
                                const uint32_t f = lds_cand[cbase + c];
                                float e = INFINITY;
                                if (sphere_may_hit(lds_sph[f], r, tl)) {
                                    FrameRay cfr;
                                    float t0;
                                    if (frame_setup<false>(lds_frames[f], r, tl, cfr, t0)) e = t0;
                                }
                                ent[c * 64] = e;
                            }
                        } else if (ncand) {
                            float wix, wiy, wiz;
                            inv_world_dir(r, wix, wiy, wiz);
                            const float e = box_entry(lds_bvh[lds_jobs[job].bvh_base], r, wix, wiy, wiz, tl);
                            if (e < INFINITY) {
                                bst[0] = 0u;
                                bws = 1u << 22;
                            }
                        }
                        mode = start_frame(fbase) ? M_WALK : M_SELECT;
                    }
                }
            }
            if (hon && take) {
                // wave-uniform
                const uint32_t t = got_hot ? (htile < n_tiles ? htile : 0xFFFFFFFFu)
                                           : ((csl < n_tiles && !((cword >> (ctile & 31u)) & 1u)) ? (uint32_t)ctile
                                                                                                  : 0xFFFFFFFFu);
                cur_tile = (uint32_t)__builtin_amdgcn_readfirstlane((int)t);
            }
            if (a.reuse && a.retraced) {
                const uint64_t re = __ballot(retrace);
                if (lane == leader && re) atomicAdd(a.retraced, (unsigned long long)__popcll(re));
            }
        }

        // ---------------------------------------------------------- walk
        if (mode == M_WALK) {
            // Leave the current cell through its nearest exit plane(s); EV_END
            // when the ray leaves the frame's root cell or passes tl.
            auto advance = [&](float ex, float ey, float ez, float tc1) -> uint32_t {
                const bool sx = ex == tc1, sy = ey == tc1, sz = ez == tc1;
                const uint32_t nx = px + (sx ? size : 0u);
                const uint32_t ny = py + (sy ? size : 0u);
                const uint32_t nz = pz + (sz ? size : 0u);
                // the new cell's size is 2^h, h the highest changed corner bit;
                // no plane at tc1 (a NaN) leaves diff = 0 and h = 2^32 - 1
                const uint32_t diff = (nx ^ px) | (ny ^ py) | (nz ^ pz);
                const uint32_t h = 31u - __clz(diff);
                // descents between two advances are bounded by the depth, so
                // counting advances bounds the walk
                ++steps;
                const uint32_t ev = (tc1 > tl || h >= fr.K) ? EV_END : (steps > a.step_limit ? EV_LIMIT : EV_NONE);
                if (ev != EV_NONE) return ev;
                const uint32_t nsize = 1u << h;
                const uint32_t keep = ~(nsize - 1u);
                px = nx & keep;
                py = ny & keep;
                pz = nz & keep;
                slot = top - h;  // at or above the current level
                pchild = stkc[slot * 64];
                pmask = stkm[slot * 64];
                size = nsize;
                tc0 = tc1;
                return EV_NONE;
            };
            uint32_t ev = EV_NONE;
            uint32_t hit_id = 0, xf = 0;
            float xf_tc1 = 0.f;
            const bool hit_root = pend == PEND_ROOT_HIT;
            if (hit_root) {
                pend = 0;
                ev = EV_HIT;
                hit_id = lds_frames[cur_f].root;
            } else if (pend == PEND_RESUME) {
                // continue just past a transformed cell the walk came back from
                pend = 0;
                const float ex = fmaf((float)(px + size), fr.ix, fr.bx);
                const float ey = fmaf((float)(py + size), fr.iy, fr.by);
                const float ez = fmaf((float)(pz + size), fr.iz, fr.bz);
                ev = advance(ex, ey, ez, min3f(ex, ey, ez));
            }
            // the hot loop: visit, descend or advance until something happens
            while (ev == EV_NONE) {
                const float ex = fmaf((float)(px + size), fr.ix, fr.bx);
                const float ey = fmaf((float)(py + size), fr.iy, fr.by);
                const float ez = fmaf((float)(pz + size), fr.iz, fr.bz);
                const float tc1 = min3f(ex, ey, ez);
                // the cell's octant in its parent: bit h of each corner (size = 2^h)
                const uint32_t h = top - slot;
                const uint32_t oct = (__builtin_amdgcn_ubfe(px, h, 1) | (__builtin_amdgcn_ubfe(py, h, 1) << 1) |
                                      (__builtin_amdgcn_ubfe(pz, h, 1) << 2)) ^ fr.flip;
                if (__builtin_amdgcn_ubfe(pmask, oct, 1)) {
                    const uint32_t cidx = pchild + __popc(pmask & ((1u << oct) - 1u));
                    // the child's corner does not depend on the node: computed
                    // while its load is in flight
                    const uint32_t hs = size >> 1;
                    const uint32_t cx = px + ((fmaf((float)(px + hs), fr.ix, fr.bx) <= tc0) ? hs : 0u);
                    const uint32_t cy = py + ((fmaf((float)(py + hs), fr.iy, fr.by) <= tc0) ? hs : 0u);
                    const uint32_t cz = pz + ((fmaf((float)(pz + hs), fr.iz, fr.bz) <= tc0) ? hs : 0u);
                    // separate LDS and global reads (a select between the two
                    // would become one generic load waiting on both counters)
                    const uint64_t wl = lds_nodes[min(cidx, lds_last)];
                    uint64_t wg = 0;
                    if (cidx >= n_lds) wg = gld(nodes, cidx);
                    const uint64_t w = (cidx < n_lds) ? wl : wg;
                    if constexpr (kCount) {
                        if (a.trail && c_trail < a.trail_cap)
                            gst(a.trail, (uint64_t)c_trail * n_rays + gray, cidx | ((cidx < n_lds) ? 0x80000000u : 0u));
                        ++c_trail;
                        ++c_nodes;
                    }
                    const uint32_t w0 = (uint32_t)w;
                    const uint32_t w1 = (uint32_t)(w >> 32);
                    const uint32_t cm = w0 & 0xFFu;
                    if (cm == 0u) {
                        ev = EV_HIT;
                        hit_id = cidx;
                        break;
                    }
                    if (!(w1 & kXform)) {
                        const uint32_t c24 = w0 >> 8;
                        pchild = (c24 == 0xFFFFFFu) ? w1 : cidx + c24;
                        pmask = cm;
                        ++slot;
                        stkc[slot * 64] = pchild;
                        stkm[slot * 64] = (uint8_t)pmask;
                        size = hs;
                        px = cx;
                        py = cy;
                        pz = cz;
                        continue;
                    }
                    const uint32_t f = fbase + 1u + (w1 & 0x7FFFFFFFu);
                    if (lds_frames[f].info & FR_INLINE) {
                        ev = EV_ENTER;
                        xf = f;
                        xf_tc1 = tc1;
                        break;
                    }
                    // a candidate frame: traced on its own, empty here
                }
                ev = advance(ex, ey, ez, tc1);
            }
            if (ev == EV_HIT) {
                // the first solid leaf front to back ends this top-level frame;
                // a leaf the ray passes by in FP64 is empty for this ray (the
                // walk goes on past it; a frame root leaf ends the frame)
                int ha;
                float th;
                if (exact_hit(xmaps + (size_t)kExactMapDoubles * cur_f, r, fr, px, py, pz, size, th, ha)) {
                    record_hit(th, hit_id, cur_f, ha);
                    mode = M_SELECT;
                    nest = 0;
                } else if (hit_root) {
                    mode = M_SELECT;
                    nest = 0;
                } else {
                    pend = PEND_RESUME;
                }
            } else if (ev == EV_LIMIT) {
                best_id = kStepLimitId;
                finish();
            } else if (ev == EV_ENTER) {
                const FrameRec& C = lds_frames[xf];
                FrameRay cfr;
                float t0;
                if (frame_setup<true>(C, r, fminf(tl, xf_tc1), cfr, t0)) {
                    if constexpr (kCount) {
                        ++c_frames;
                        ++c_nodes;   // the frame's root record
                    }
                    // save where the enclosing walk stands (its current slot
                    // keeps its node), then enter in place
                    fst[nest * 64] =
                        make_uint4(cur_f | ((slot - sbase) << 11) | (sbase << 16), px, py, pz);
                    ++nest;
                    sbase = slot;
                    cur_f = xf;
                    fr = cfr;
                    pmask = C.info & FR_MASK;
                    pchild = C.child;
                    slot = sbase + 1u;
                    top = sbase + fr.K;
                    stkc[slot * 64] = pchild;
                    stkm[slot * 64] = (uint8_t)pmask;
                    size = 1u << (fr.K - 1);
                    px = (fmaf((float)size, fr.ix, fr.bx) <= t0) ? size : 0u;
                    py = (fmaf((float)size, fr.iy, fr.by) <= t0) ? size : 0u;
                    pz = (fmaf((float)size, fr.iz, fr.bz) <= t0) ? size : 0u;
                    tc0 = t0;
                } else {
                    pend = PEND_RESUME;  // missed it: the cell is empty for this ray
                }
            } else if (ev == EV_END) {
                if (nest > 0) {
                    // back to the enclosing frame, just past the transformed cell
                    --nest;
                    const uint4 e = fst[nest * 64];
                    cur_f = e.x & 0x7FFu;
                    const uint32_t lvl = (e.x >> 11) & 31u;
                    sbase = (e.x >> 16) & 127u;
                    slot = sbase + lvl;
                    px = e.y;
                    py = e.z;
                    pz = e.w;
                    float t0;
                    frame_setup<true>(lds_frames[cur_f], r, tl, fr, t0);
                    size = 1u << (fr.K - lvl);
                    top = sbase + fr.K;
                    pchild = stkc[slot * 64];
                    pmask = stkm[slot * 64];
                    pend = PEND_RESUME;
                } else {
                    mode = M_SELECT;
                }
            }
        }
        if (mode == M_SELECT) {
            // the walk's state is dead here (start_frame sets all of it before
            // the next walk step); saying so frees its registers for the
            // candidate search
            fr = FrameRay{};
            px = py = pz = 0;
            size = 1;
            pchild = pmask = 0;
            slot = 1;
            sbase = top = 0;
            cur_f = nest = 0;
            tc0 = 0.f;
            pend = 0;
            if (++steps > a.step_limit) {
                best_id = kStepLimitId;
                finish();
                continue;
            }
            // ------------------------------------------------------ next candidate frame
            if (kSorted) {
                float bc = INFINITY;
                int pick = -1;
                for (uint32_t c = 0; c < ncand; ++c) {
                    // consumed and missed candidates hold +inf, which must never
                    // pass the test even when tl is +inf (no hit yet, tmax = inf)
                    const float e = ent[c * 64];
                    if (e < INFINITY && e <= tl && (pick < 0 || e < bc)) {
                        bc = e;
                        pick = (int)c;
                    }
                }
                if (pick < 0) {
                    finish();
                } else {
                    ent[pick * 64] = INFINITY;
                    if (start_frame(lds_cand[cbase + pick])) mode = M_WALK;
                }
            } else {
                // candidates through the job's hierarchy of their world
                // boxes, nearer child first, each box skipped once its entry
                // lies beyond the best hit; a leaf's candidates then pass the
                // sphere test (Sec. 4.1) before their exact root-cell entry
                const uint32_t bbase = lds_jobs[job].bvh_base;
                float wix, wiy, wiz;
                inv_world_dir(r, wix, wiy, wiz);
                uint32_t leaf_i = bws & 0x7FFu, leaf_end = (bws >> 11) & 0x7FFu, bsp = bws >> 22;
                bool started = false;
                while (!started) {
                    if (leaf_i < leaf_end) {
                        const uint32_t f = lds_cand[cbase + leaf_i++];
                        if (sphere_may_hit(lds_sph[f], r, tl)) started = start_frame(f);
                        continue;
                    }
                    if (bsp == 0u) break;
                    --bsp;
                    // the box may now lie beyond the best hit
                    const BvhNode& N = lds_bvh[bbase + bst[bsp * 64]];
                    if (!(box_entry(N, r, wix, wiy, wiz, tl) < INFINITY)) continue;
                    if (N.b & kBvhLeaf) {
                        leaf_i = N.a;
                        leaf_end = N.a + (N.b & 0xFFFFu);
                        continue;
                    }
                    const float eL = box_entry(lds_bvh[bbase + N.a], r, wix, wiy, wiz, tl);
                    const float eR = box_entry(lds_bvh[bbase + N.b], r, wix, wiy, wiz, tl);
                    const bool left_near = eL <= eR;
                    const float en = left_near ? eL : eR, ef = left_near ? eR : eL;
                    const uint32_t nn = left_near ? N.a : N.b, nf = left_near ? N.b : N.a;
                    // the far child first, so the near one is popped next
                    if (ef < INFINITY && bsp < bst_cap) {
                        bst[bsp * 64] = nf;
                        ++bsp;
                    }
                    if (en < INFINITY && bsp < bst_cap) {
                        bst[bsp * 64] = nn;
                        ++bsp;
                    }
                }
                bws = leaf_i | (leaf_end << 11) | (bsp << 22);
                if (started) {
                    mode = M_WALK;
                } else {
                    finish();
                }
            }
        }
    }

    // the last work-group out resets the queue for the next launch; only
    // work-groups that may claim count (an idle one of a plan's fixed grid
    // touches no counter, and skipping its atomic spares the others a
    // same-address queue)
    __syncthreads();
    uint32_t* const hot = (kSingle && lds_hot[kHotLdsOn]) ? a.hot : nullptr;
    const uint32_t hp = hot ? lds_hot[kHotLdsIn] : 0u, ob = hp ^ 1u;
    if (hot && active && threadIdx.x == 0) {
        // this work-group's slow tiles into the output list and its bitmap
        const uint32_t sub = blockIdx.x % kHotSub;
        atomicAdd(hot_sum(hot, sub), lds_hot[kHotLdsSum]);
        atomicMax(hot_max(hot, sub), lds_hot[kHotLdsMax]);
        const uint32_t n = min(lds_hot[kHotLdsListed], kHotPerBlock);
        if (n) {
            const uint32_t base = atomicAdd(hot_cnt(hot, ob, sub), n);
            uint32_t* olist = hot_list(hot, ob) + sub * kHotSubCap;
            uint32_t* obits = hot_bits(hot, ob);
            for (uint32_t i = 0; i < n && base + i < kHotSubCap; ++i) {
                const uint32_t ent = lds_hot[kHotLdsHdr + i], t = ent & kHotTileMask;
                olist[base + i] = ent;
                atomicOr(obits + (t >> 5), 1u << (t & 31u));
            }
        }
    }
    if (active && threadIdx.x == 0) {
        __threadfence();
        uint32_t* fin = a.queue + kQueueFinished;
        const uint32_t prev = atomicAdd(fin, 1u);
        const bool last = prev == n_active - 1;
        if (last) {
            for (uint32_t p = 0; p < kQueueParts; ++p) atomicExch(a.queue + p * kQueueStride, 0u);
            atomicExch(a.queue + kQueueDry, 0u);
            atomicExch(a.queue + kQueueDry + 1, 0u);
            atomicExch(fin, 0u);
        }
        if (hot) lds_hot[kHotLdsListed] = last ? 1u : 0u;
    }
    if (hot) {
        __syncthreads();
        if (active && lds_hot[kHotLdsListed]) {
            // last out (every other work-group has written its list): clear
            // the input list's bitmap, the words of the tiles of the launch
            // that wrote it
            const uint32_t iw = (min(hot[12 + hp], kHotMaxTiles) + 31u) >> 5;
            uint32_t* ibits = hot_bits(hot, hp);
            for (uint32_t i = threadIdx.x; i < iw; i += blockDim.x) ibits[i] = 0u;
            if (threadIdx.x < 64u) {
                // the lines' counts and cost statistics, one line per lane
                const uint32_t k = threadIdx.x;
                uint32_t c = 0, csum = 0, cmax = 0;
                if (k < kHotSub) {
                    c = atomicAdd(hot_cnt(hot, ob, k), 0u);
                    csum = atomicExch(hot_sum(hot, k), 0u);
                    cmax = atomicExch(hot_max(hot, k), 0u);
                    atomicExch(hot_cnt(hot, hp, k), 0u);
                }
                for (int off = kHotSub / 2; off > 0; off >>= 1) {
                    c += (uint32_t)__shfl_xor((int)c, off);
                    csum += (uint32_t)__shfl_xor((int)csum, off);
                    cmax = max(cmax, (uint32_t)__shfl_xor((int)cmax, off));
                }
                if (k == 0u) {
                    // the threshold follows the target count of listed tiles
                    const uint32_t tg = a.hot_target, hthr = lds_hot[kHotLdsThr];
                    uint32_t nt = hthr;
                    if (c > tg + tg / 2u) nt = hthr + max(1u, hthr / 8u);
                    else if (2u * c < tg && hthr > 1u) nt = hthr - max(1u, hthr / 8u);
                    atomicExch(hot + 4 + 2 * ob, (uint32_t)a.hot_sig);
                    atomicExch(hot + 5 + 2 * ob, (uint32_t)(a.hot_sig >> 32));
                    // deal the new list out only if this launch was bound by
                    // its slowest tiles: largest cost >= 0.7 x (sum of costs /
                    // waves)
                    atomicExch(hot + 10 + ob, (10ull * cmax * n_active * wpb >= 7ull * csum) ? 1u : 0u);
                    atomicExch(hot + 12 + ob, (uint32_t)n_tiles);
                    atomicExch(hot + 1, nt);
                    atomicExch(hot + 0, ob);
                }
            }
        }
    }
}

// The allocation-free entry point's scratch (see static_scratch).  In host
// code this name is not a device address: host code reaches the array only
// through the pointer static_scratch returns.
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

hipError_t static_scratch(int device, unsigned char** out) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static unsigned char* addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices || !out) return hipErrorInvalidValue;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[device] = static_cast<unsigned char*>(p);
    }
    *out = addr[device];
    return hipSuccess;
}

__global__ __launch_bounds__(256) void zero_words_kernel(uint32_t* p, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

hipError_t launch_zero_words(uint32_t* p, uint32_t n, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(zero_words_kernel, dim3((n + 255) / 256 < 64 ? (n + 255) / 256 : 64), dim3(256), 0, stream, p, n);
    return hipGetLastError();
}

hipError_t prepare_trace(size_t max_lds) {
    const void* kernels[] = {reinterpret_cast<const void*>(&trace_kernel<true, true>),
                             reinterpret_cast<const void*>(&trace_kernel<true, false>),
                             reinterpret_cast<const void*>(&trace_kernel<false, true>),
                             reinterpret_cast<const void*>(&trace_kernel<false, false>),
                             reinterpret_cast<const void*>(&trace_kernel<true, true, true>),
                             reinterpret_cast<const void*>(&trace_kernel<true, true, false, true>),
                             reinterpret_cast<const void*>(&trace_kernel<false, true, false, true>),
                             reinterpret_cast<const void*>(&trace_kernel<true, true, true, true>)};
    for (const void* k : kernels) {
        const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_trace(const TraceArgs& a, const LaunchCfg& c, hipStream_t stream, const unsigned char* inline_tab,
                        size_t inline_bytes) {
    const dim3 grid(c.blocks), block(c.waves_per_block * 64);
    if (inline_tab) {
        if (!a.sort_cand || a.jobs || inline_bytes > kInlineTableBytes) return hipErrorInvalidValue;
        TraceArgsInline ai{};
        static_cast<TraceArgs&>(ai) = a;
        std::memcpy(ai.inline_tab, inline_tab, inline_bytes);
        hipLaunchKernelGGL((trace_kernel<true, true, true>), grid, block, c.lds_bytes, stream, ai);
        return hipGetLastError();
    }
    if (a.sort_cand) {
        if (!a.jobs)
            hipLaunchKernelGGL((trace_kernel<true, true>), grid, block, c.lds_bytes, stream, a);
        else
            hipLaunchKernelGGL((trace_kernel<true, false>), grid, block, c.lds_bytes, stream, a);
    } else {
        if (!a.jobs)
            hipLaunchKernelGGL((trace_kernel<false, true>), grid, block, c.lds_bytes, stream, a);
        else
            hipLaunchKernelGGL((trace_kernel<false, false>), grid, block, c.lds_bytes, stream, a);
    }
    return hipGetLastError();
}

hipError_t launch_trace_counted(const TraceArgs& a, const LaunchCfg& c, hipStream_t stream,
                                const unsigned char* inline_tab, size_t inline_bytes) {
    const dim3 grid(c.blocks), block(c.waves_per_block * 64);
    if (!a.counts || a.jobs || a.hdr) return hipErrorInvalidValue;
    if (inline_tab) {
        if (!a.sort_cand || inline_bytes > kInlineTableBytes) return hipErrorInvalidValue;
        TraceArgsInline ai{};
        static_cast<TraceArgs&>(ai) = a;
        std::memcpy(ai.inline_tab, inline_tab, inline_bytes);
        hipLaunchKernelGGL((trace_kernel<true, true, true, true>), grid, block, c.lds_bytes, stream, ai);
    } else if (a.sort_cand) {
        hipLaunchKernelGGL((trace_kernel<true, true, false, true>), grid, block, c.lds_bytes, stream, a);
    } else {
        hipLaunchKernelGGL((trace_kernel<false, true, false, true>), grid, block, c.lds_bytes, stream, a);
    }
    return hipGetLastError();
}

}  // namespace svo
