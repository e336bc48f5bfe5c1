// Internal layout shared by the host library and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

namespace svo {

// One frame of a scene as the device reads it: 64 bytes, held in LDS.  The
// map takes a world point to the frame's grid coordinates, where the frame's
// root cell is [0, 2^K)^3 and a leaf at depth l spans 2^(K-l) units:
// g = M x + c (paper Eq. 3, with the scale of Sec. 3.2 and the grid scaling
// folded into one affine map).  Record 0 is the world, record 1 + s slot s.
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
    FR_EMPTY = 1u << 14,      // nothing to trace in this frame (unused slot, empty world)
    FR_INLINE = 1u << 15,     // moved content stays in its static cell: entered in place
};

// Frames entered in place may nest this deep inside one top-level frame.
constexpr uint32_t kMaxInlineNest = 4;
// Per-lane candidate entry tables are kept in LDS up to this many candidates;
// beyond, candidates are found through a bounding-box hierarchy.
constexpr uint32_t kMaxSortedCand = 16;

// One node of a frame table's hierarchy over its candidate frames: the
// world-space box of the moved root cells below it (widened outward so that
// FP32 slab tests never lose a hit).  Interior: a = left child, b = right
// child (node indices within the table's hierarchy).  Leaf: b = kBvhLeaf |
// count, a = first entry in the table's candidate list.  32 bytes.
struct alignas(16) BvhNode {
    float lo[3];
    uint32_t a;
    float hi[3];
    uint32_t b;
};
static_assert(sizeof(BvhNode) == 32, "hierarchy node must be 32 bytes");
constexpr uint32_t kBvhLeaf = 0x80000000u;
constexpr uint32_t kBvhLeafMax = 2;     // candidates per leaf

// Pinhole camera for primary rays made on the device (see svo_camera.h):
// by the ray generation kernel, or by the trace kernel for a job that has
// a camera instead of a ray buffer.  96 bytes.
struct alignas(16) CameraArgs {
    float eye[3], fwd[3], right[3], up[3];
    float tan_half_fov, aspect;
    uint32_t width, height, samples, seed;
    uint32_t jitter;      // 0: pixel centres
    uint32_t tiled;       // 1: 8x8 tile order
    uint32_t full_tiles;  // tiled, one sample, width and height multiples of 8
    uint32_t tiles_x;     // width / 8
    double inv_tiles_x;   // 1 / tiles_x
};
static_assert(sizeof(CameraArgs) == 96, "camera record must be 96 bytes");

// One job of a launch: a ray range traced against one scene under one set
// of transforms (96 bytes, held in LDS).
struct alignas(16) JobRec {
    const uint64_t* nodes;    // the scene's pool
    const float4* rays;       // 2 x float4 per ray
    uint32_t* out_id;
    uint32_t* out_inst;       // nullable
    float* out_t;
    float* out_n;             // nullable, 3 floats per ray
    uint64_t ray_begin;       // first launch-wide ray index of this job
    uint32_t frame_base;      // the job's world record in the launch's frame array
    uint32_t cand_base;       // the job's first entry in the launch's candidate list
    uint32_t n_cand;
    uint32_t lds_nodes;       // pool prefix of this job's scene held in LDS (0: none)
    uint32_t bvh_base;        // the job's hierarchy root in the launch's node array
    uint32_t n_inline;        // in-place frames, listed after the job's candidates
    const CameraArgs* cam;    // device camera making the job's rays (rays unused), or nullptr
    uint64_t pad;
};
static_assert(sizeof(JobRec) == 96, "job record must be 96 bytes");

constexpr uint32_t kMaxJobs = 256;

// Work queue of one launch: kQueueParts claim counters, each on its own
// 128-byte line, then a bitmap of exhausted partitions, then the
// finished-work-group counter.  Claims are interleaved over the partitions
// (claim slot s belongs to partition s mod kQueueParts) so that no single
// address serialises them; a wave starts on its own partition, and a wave
// that finds a partition dry marks it in the bitmap and moves on to the next
// partition the bitmap still shows as open.
constexpr uint32_t kQueueParts = 64;
constexpr uint32_t kQueueStride = 32;                              // uint32 words between counters
constexpr uint32_t kQueueDry = kQueueParts * kQueueStride;         // 2 words: bitmap of dry partitions
constexpr uint32_t kQueueFinished = kQueueDry + kQueueStride;      // finished work-groups
constexpr uint32_t kQueueWords = kQueueFinished + kQueueStride;

// Scratch of the allocation-free batched entry point: one work queue, then
// a table area for the launch's job, frame, candidate, sphere, exact-map and
// hierarchy records.  One copy per device, in the library's code object.
// Slow tiles first: per work queue, device state that carries the tiles one
// launch found slow to the next launch on the same queue (the same rays traced
// again, as in an animation with a fixed camera).  A tile's cost is the most
// advances (moves from a cell to the next, the counter the step limit already
// keeps) any of its rays took; a launch lists the tiles whose cost is at or
// above a threshold, and the next launch deals them out to its waves first (no
// shared counter: wave w takes entries w, w + waves, ...) while its regular
// claim order skips them.  The threshold follows a target count.  A list is
// only dealt out when the launch that wrote it was bound by its slowest tiles:
// when its costliest tile cost at least 0.7 times the mean work of a wave (all
// tile costs over the active waves); launches of many short tiles per wave
// keep the plain order.  Work-groups add to the counts on kHotSub separate
// cache lines (work-group g on line g mod kHotSub), so that no address takes
// every work-group's atomic at the end of a launch; each line has its own
// sub-list.
// Words: [0] which of the two lists is the input, [1] the threshold (0: not
// yet set), [4 + 2b, 5 + 2b] the signature of the launch that wrote list b,
// [10 + b] whether list b is to be dealt out, [12 + b] the tile count of the
// launch that wrote it; then per line s: list b's count (raw, may pass
// kHotSubCap) at hot_cnt(b, s), this launch's sum and largest of tile costs
// at hot_sum(s) and hot_max(s); then list 0, list 1 (kHotSub sub-lists of
// kHotSubCap entries each), bitmap 0, bitmap 1 (a bit per tile of the launch
// that wrote it).
constexpr uint32_t kHotSub = 8;
constexpr uint32_t kHotLine = 32;                // words per cache line (128 B)
constexpr uint32_t kHotSubCap = 1024;
constexpr uint32_t kHotCap = kHotSub * kHotSubCap;
constexpr uint32_t kHotTileBits = 18;
constexpr uint32_t kHotMaxTiles = 1u << kHotTileBits;   // launches with more tiles keep the plain order
// A list entry is a tile index in its low kHotTileBits bits and the tile's
// cost, clamped, above them.
constexpr uint32_t kHotTileMask = kHotMaxTiles - 1u;
constexpr uint32_t kHotEntryCostMax = (1u << (32 - kHotTileBits)) - 1u;
// The sorted instantiation raises the issue priority of a wave on a dealt
// tile whose cost is at least this many tenths of the listing threshold.
constexpr uint32_t kHotPrioTenths = 20;
// A launch whose input list is of its own rays but was not to be dealt out
// gathers no tile statistics (and leaves the state as it is), except every
// kHotResample-th launch on the state, which decides again.
constexpr uint32_t kHotResample = 8;
constexpr uint32_t kHotBitsWords = kHotMaxTiles / 32;
constexpr uint32_t kHotCntBase = kHotLine;                                  // 2 kHotSub lines
constexpr uint32_t kHotSumBase = kHotCntBase + 2 * kHotSub * kHotLine;      // kHotSub lines
constexpr uint32_t kHotMaxBase = kHotSumBase + kHotSub * kHotLine;          // kHotSub lines
constexpr uint32_t kHotHdr = kHotMaxBase + kHotSub * kHotLine;
constexpr uint32_t kHotWords = kHotHdr + 2 * kHotCap + 2 * kHotBitsWords;
// A tile's cost enters the sum and the largest cost clamped to kHotCostClamp,
// so that a launch's sum (at most kHotMaxTiles tiles) fits 32 bits.
constexpr uint32_t kHotCostClamp = 4095;
// Per work-group LDS words (single-job launches): the tiles it listed, the
// sum and the largest of its tile costs, the input entries its waves have
// taken, the input sub-lists' counts, whether the launch keeps the state, the
// input list, the input entries to deal out (0: none), the threshold and the
// state's address; then up to kHotPerBlock listed tiles from kHotLdsHdr on
// (more are dropped).
constexpr uint32_t kHotLdsListed = 0;
constexpr uint32_t kHotLdsSum = 1;
constexpr uint32_t kHotLdsMax = 2;
constexpr uint32_t kHotLdsTaken = 3;
constexpr uint32_t kHotLdsCnt = 4;                        // kHotSub words
constexpr uint32_t kHotLdsOn = kHotLdsCnt + kHotSub;
constexpr uint32_t kHotLdsIn = kHotLdsOn + 1;
constexpr uint32_t kHotLdsDeal = kHotLdsOn + 2;
constexpr uint32_t kHotLdsThr = kHotLdsOn + 3;
constexpr uint32_t kHotLdsPtr = kHotLdsOn + 4;            // 2 words
constexpr uint32_t kHotLdsHdr = 20;
constexpr size_t kHotLdsBytes = 256;
constexpr uint32_t kHotPerBlock = kHotLdsBytes / 4 - kHotLdsHdr;
static_assert(kHotLdsPtr + 2 <= kHotLdsHdr, "slow-tile LDS header too small");
constexpr uint32_t kHotInitialThreshold = 64;

constexpr size_t kStaticQueueBytes = ((size_t)kQueueWords * 4 + 255) & ~(size_t)255;
constexpr size_t kStaticTableBytes = (size_t)256 << 10;
constexpr size_t kStaticScratchBytes = kStaticQueueBytes + kStaticTableBytes;

// Launch-wide counts of a plan launch, read by the kernel from the head of
// the plan's device table: a captured launch keeps its arguments across
// replays, so whatever changes between replays lives in device memory.
struct alignas(16) LaunchHdr {
    uint64_t n_rays;              // all jobs
    const uint64_t* cache_src;    // pool whose prefix is cached in LDS (nullptr: none)
    uint64_t tile_stride;         // as TraceArgs::tile_stride, for n_rays
    uint32_t n_jobs;              // <= TraceArgs::n_jobs (the capacity)
    uint32_t n_frames;            // <= TraceArgs::n_frames
    uint32_t n_cand_total;        // <= TraceArgs::n_cand_total
    uint32_t lds_nodes;           // <= TraceArgs::lds_nodes, even
    uint32_t n_bvh_total;         // <= TraceArgs::n_bvh_total
    uint32_t pad[5];
};
static_assert(sizeof(LaunchHdr) == 64, "launch header must be 64 bytes");

// A one-job launch of a small scene whose transforms changed since its last
// upload carries the frame table (records, candidates, spheres, exact maps;
// no hierarchy) in its kernel arguments (TraceArgsInline): no copy and no
// event per transform update, and the launch keeps the transforms it was
// enqueued with.  Larger arguments cost every launch a little, so launches
// that can read an up-to-date device table keep the plain arguments.
constexpr uint32_t kInlineTableBytes = 2048;

// The exact map of a frame: the FrameRec map before rounding to FP32 (FP64,
// rows r = 0..2 at [4r..4r+2], translation at [4r+3]).  The walk runs on the
// FP32 record; the entry t of the cell it hits is recomputed from this one.
constexpr uint32_t kExactMapDoubles = 12;

// In a plan launch (hdr != nullptr) n_jobs, n_frames, n_cand_total,
// n_bvh_total and lds_nodes are capacities that size the LDS layout, and the header holds
// the counts; n_rays, tile_stride and cache_src are ignored.
struct TraceArgs {
    const LaunchHdr* hdr;     // plan launches: counts in device memory; else nullptr
    const JobRec* jobs;       // device job table, or nullptr: the single job in job0
    JobRec job0;
    const FrameRec* frames;   // n_frames records; job j's slot s is frames[frame_base_j + 1 + s]
    const uint32_t* cand;     // candidate frames (absolute indices), per job contiguous
    const float4* spheres;    // n_frames world bounding spheres (centre, radius) of the moved root cells
    const double* xmaps;      // n_frames exact maps (kExactMapDoubles each), indexed like frames
    const BvhNode* bvh;       // n_bvh_total hierarchy nodes, per job contiguous (job j's root at bvh_base_j)
    uint32_t n_bvh_total;
    uint32_t bvh_depth;       // hierarchy stack entries per lane (used when sort_cand == 0)
    uint32_t n_jobs;
    uint32_t n_frames;
    uint32_t n_cand_total;
    uint32_t max_cand;        // largest per-job candidate count
    uint64_t n_rays;          // all jobs
    const uint64_t* cache_src;  // pool whose prefix is cached in LDS
    uint32_t* queue;          // kQueueWords: partition counters, then finished work-groups
    uint32_t lds_nodes;       // pool prefix cached in LDS (even)
    uint32_t stack_levels;    // traversal stack entries per lane
    uint32_t nest_levels;     // frame stack entries per lane (inline frames)
    uint32_t sort_cand;       // 1: candidates in entry order via a per-lane LDS table
    uint32_t refill;          // a wave claims new rays once this many lanes are idle (1..64)
    uint32_t claim;           // rays a wave takes from a partition counter at once (a multiple of 64)
    uint32_t reuse;           // 1: the outputs hold the previous trace of these rays (hit buffer)
    unsigned long long* retraced;  // reuse: rays traced again are added here (nullable)
    uint64_t tile_stride;     // claim i covers tile (i * tile_stride) mod tiles (coprime: a permutation)
    uint32_t step_limit;
    // slow tiles first (one-job launches with whole-tile refill; nullptr:
    // plain order): this queue's state (kHotWords), the target count of
    // listed tiles, and the signature of this launch's rays
    uint32_t* hot;
    uint32_t hot_target;
    uint32_t hot_seq;         // launches so far on this state (see kHotResample)
    uint64_t hot_sig;
    // TraceArgsInline launches: frames, cand, spheres and exact maps are read
    // from the inline table at these byte offsets instead of the pointers above
    uint32_t inline_off_cand, inline_off_sph, inline_off_x;
    // Counting launches (an instantiation of their own; ignored by the
    // others), per launch-wide ray index g of n_rays: counts[g] node records
    // read (each frame walked counts its root record), counts[n_rays + g]
    // frames walked, counts[2 n_rays + g] result writes (added atomically:
    // 1 when every ray is written exactly once); with trail, the index of
    // the k-th node record read, trail[k n_rays + g] for k < trail_cap, bit
    // 31 set when it came from the LDS copy of the pool prefix.
    uint32_t* counts;
    uint32_t* trail;
    uint32_t trail_cap;
    // single-job launches: when has_cam0, the job's rays are made from cam0
    // (job0.rays unused)
    uint32_t has_cam0;
    CameraArgs cam0;
};

struct TraceArgsInline : TraceArgs {
    alignas(16) unsigned char inline_tab[kInlineTableBytes];
};

struct LaunchCfg {
    uint32_t blocks;
    uint32_t waves_per_block;
    size_t lds_bytes;
};

hipError_t launch_primary_rays(const CameraArgs& c, float* out, hipStream_t stream);

// Ambient-occlusion rays from primary hits (see svo_raygen.hip).
struct AoArgs {
    const float4* rays;       // primary rays, 2 x float4 each
    const float* t;           // primary hit t (+inf: miss)
    const float* normal;      // 3 floats per primary ray
    uint64_t n;
    uint32_t k;               // AO rays per primary ray
    uint32_t seed;
    float radius;             // AO ray tmax
    float offset;             // origin lift along the normal, relative to max(1, |p|inf)
    float4* out;              // n * k rays
};

hipError_t launch_ao_rays(const AoArgs& a, hipStream_t stream);

// Compositing into an RGBA8 image (see svo_raygen.hip).
struct ShadeArgs {
    const uint64_t* nodes;    // the scene's pool: a leaf's word1 is its RGBA8 colour
    uint64_t n_nodes;         // ids at or beyond this count as misses
    const uint32_t* prim_id;  // width * height * samples, ray order
    const uint32_t* ao_id;    // k per primary ray (nullable when k == 0)
    uint32_t width, height, samples, tiled, k;
    uint32_t ambient;         // per mille of the colour kept when every AO ray is blocked
    uint32_t background;      // RGBA8 of a miss
    uint32_t* out;            // width * height, row-major
};

hipError_t launch_shade(const ShadeArgs& a, hipStream_t stream);

// Device address of this device's scratch (kStaticScratchBytes, 256-byte
// aligned), looked up once per device; the device must be current.
hipError_t static_scratch(int device, unsigned char** out);
// Zero n 32-bit words on `stream` with a small kernel (no memset node, so
// the clear may be captured into a graph).
hipError_t launch_zero_words(uint32_t* p, uint32_t n, hipStream_t stream);

size_t trace_lds_bytes(const TraceArgs& a, uint32_t waves_per_block);
// Allow the trace kernel up to max_lds bytes of dynamic LDS on the current
// device; done once when a context is created, so that no launch (eager or
// captured into a graph) changes the kernel's attributes.
hipError_t prepare_trace(size_t max_lds);
// inline_tab (nullable): the frame table to pass in the arguments (at most
// kInlineTableBytes; one-job launches with sorted candidates only).
hipError_t launch_trace(const TraceArgs& a, const LaunchCfg& c, hipStream_t stream,
                        const unsigned char* inline_tab = nullptr, size_t inline_bytes = 0);
// The counting instantiation (a.counts set; single-job launches only).
hipError_t launch_trace_counted(const TraceArgs& a, const LaunchCfg& c, hipStream_t stream,
                                const unsigned char* inline_tab = nullptr, size_t inline_bytes = 0);

}  // namespace svo
