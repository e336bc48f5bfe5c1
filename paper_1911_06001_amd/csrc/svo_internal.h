// Internal layout shared by the host library and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace svo {

// One frame of a scene, as the device reads it: 64 bytes, cached in LDS.
// The map takes a world point to the frame's grid coordinates, where the frame's root cell is [0, 2^K)^3 and a leaf at depth
// l spans 2^(K-l) units: g = M x + c (paper Eq. 3 with the scale of
// Sec. 3.2 and the grid scaling folded into one affine map).
struct alignas(16) FrameRec {
    float m[12];        // rows r = 0..2: m[4r..4r+2] = row r of M, m[4r+3] = c_r
    uint32_t child;     // child group start of the frame root
    uint32_t info;      // see FR_* below
    uint32_t inst;      // slot id reported on hits (SVO_NONE for the world)
    uint32_t root;      // node index of the frame root
};
static_assert(sizeof(FrameRec) == 64, "frame record must be 64 bytes");

enum : uint32_t {
    FR_MASK = 0xFFu,          // child mask of the frame root
    FR_K_SHIFT = 8,           // bits 8..12: height K (levels below the frame root)
    FR_K_MASK = 0x1Fu,
    FR_ROOT_LEAF = 1u << 13,  // the frame root itself is a solid leaf (world only)
    FR_EMPTY = 1u << 14,      // nothing to trace in this frame
    FR_CONTAINED = 1u << 15,  // moved content stays inside the static cell
};

struct TraceArgs {
    const uint64_t* nodes;
    const FrameRec* frames;   // [0] = world, [1 .. n_cand] = candidate frames
    uint32_t n_frames;        // records copied to LDS
    uint32_t n_cand;          // candidate (overflowing) frames, <= 64
    const float4* rays;       // 2 x float4 per ray
    uint64_t n_rays;
    uint32_t* out_id;
    uint32_t* out_inst;       // nullable
    float* out_t;
    float* out_n;             // nullable, 3 floats per ray
    uint32_t* queue;          // [0] next tile, [1] finished work-groups
    uint32_t lds_nodes;       // pool prefix cached in LDS
    uint32_t stack_levels;    // stack entries per lane (>= max frame height)
    uint32_t step_limit;
};

struct LaunchCfg {
    uint32_t blocks;
    uint32_t waves_per_block;
    size_t lds_bytes;
};

size_t trace_lds_bytes(uint32_t lds_nodes, uint32_t n_frames, uint32_t stack_levels, uint32_t waves_per_block);
hipError_t launch_trace(const TraceArgs& a, const LaunchCfg& c, hipStream_t stream);

}  // namespace svo
