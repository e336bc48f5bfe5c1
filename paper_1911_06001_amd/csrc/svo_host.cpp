// Host side of the C ABI: contexts, pool validation and upload, per-frame
// transform preparation (FP64 compose + invert, FP32 frame records) and
// kernel launches.  Every entry point returns a status code; nothing throws
// across the ABI.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <numeric>
#include <set>
#include <string>
#include <vector>

#include "svo.h"
#include "svo_internal.h"

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) return fail(SVO_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr uint32_t kFar = 0xFFFFFFu;
constexpr uint32_t kXform = 0x80000000u;
constexpr uint32_t kMaxStreams = 64;
constexpr uint32_t kMaxImageSide = 1u << 20;   // pixels per image row or column

inline uint32_t nd_mask(uint64_t w) { return (uint32_t)(w & 0xFFu); }
inline uint32_t nd_c24(uint64_t w) { return (uint32_t)((w >> 8) & 0xFFFFFFu); }
inline uint32_t nd_w1(uint64_t w) { return (uint32_t)(w >> 32); }
inline bool nd_leaf(uint64_t w) { return nd_mask(w) == 0; }
inline bool nd_xform(uint64_t w) { return nd_mask(w) != 0 && (nd_w1(w) & kXform); }
inline int popc(uint32_t v) { return __builtin_popcount(v); }

// ------------------------------------------------------------------ pool analysis

struct Analysis {
    uint32_t n_frames = 1, world_height = 0, max_height = 0, max_nesting = 0, n_shared = 0;
    std::vector<int32_t> slot_parent;   // -1 world, -2 unused, else slot
    std::vector<uint32_t> slot_node;
    std::vector<uint32_t> slot_height;  // levels below the slot's frame root
    std::vector<uint32_t> slot_level;   // level of the transformed node in its parent frame
    std::vector<std::array<uint32_t, 3>> slot_coord;
    std::vector<uint32_t> slot_mask;
    std::vector<uint32_t> order;        // used slots, parents before children
};

// Children of node i: start index and count; false if i is a leaf.
inline bool children_of(const uint64_t* nodes, uint64_t i, const uint32_t* slot_child, uint64_t& start, int& count) {
    const uint64_t w = nodes[i];
    if (nd_leaf(w)) return false;
    count = popc(nd_mask(w));
    if (nd_xform(w)) {
        start = slot_child[nd_w1(w) & 0x7FFFFFFFu];
    } else if (nd_c24(w) == kFar) {
        start = nd_w1(w);
    } else {
        start = i + nd_c24(w);
    }
    return true;
}

int analyse(const uint64_t* nodes, uint64_t n, uint32_t root, uint32_t max_depth, const uint32_t* slot_child,
            uint32_t n_slots, Analysis& A) {
    if (max_depth > SVO_MAX_DEPTH) return fail(SVO_ERANGE, "max_depth %u exceeds %u", max_depth, SVO_MAX_DEPTH);
    if (n_slots > SVO_MAX_SLOTS) return fail(SVO_ERANGE, "n_slots %u exceeds %u", n_slots, SVO_MAX_SLOTS);
    if (n >= 0xFFFFFFFEull) return fail(SVO_ERANGE, "n_nodes must be below 2^32 - 2");
    if (n && !nodes) return fail(SVO_EINVAL, "nodes is NULL");
    if (n_slots && !slot_child) return fail(SVO_EINVAL, "slot_child is NULL");
    A = Analysis();
    A.slot_parent.assign(n_slots, -2);
    A.slot_node.assign(n_slots, 0);
    A.slot_height.assign(n_slots, 0);
    A.slot_level.assign(n_slots, 0);
    A.slot_coord.assign(n_slots, {0, 0, 0});
    A.slot_mask.assign(n_slots, 0);
    if (root == SVO_NONE) return SVO_OK;
    if (root >= n) return fail(SVO_EINVAL, "root %u out of range (%llu nodes)", root, (unsigned long long)n);
    if (nd_xform(nodes[root])) return fail(SVO_EINVAL, "the world root may not be a transformed node");

    // check every node's child reference before any traversal uses it
    for (uint64_t i = 0; i < n; ++i) {
        const uint64_t w = nodes[i];
        if (nd_leaf(w)) continue;
        const uint64_t cnt = (uint64_t)popc(nd_mask(w));
        uint64_t start;
        if (nd_xform(w)) {
            const uint32_t s = nd_w1(w) & 0x7FFFFFFFu;
            if (s >= n_slots) return fail(SVO_EINVAL, "node %llu: slot %u out of range", (unsigned long long)i, s);
            start = slot_child[s];
        } else if (nd_c24(w) == kFar) {
            start = nd_w1(w);
        } else {
            if (nd_c24(w) == 0) return fail(SVO_EINVAL, "node %llu: child offset 0", (unsigned long long)i);
            if (nd_w1(w) != 0) return fail(SVO_EINVAL, "node %llu: word1 must be 0 with a relative offset", (unsigned long long)i);
            start = i + nd_c24(w);
        }
        if (start + cnt > n) return fail(SVO_EINVAL, "node %llu: child group out of range", (unsigned long long)i);
    }

    // post-order DFS: cycles, heights, "contains a transformed node", in-degree
    std::vector<uint8_t> color(n, 0), height(n, 0), has_xf(n, 0), refs(n, 0);
    std::vector<uint8_t> slot_h(n_slots, 0);
    std::vector<std::pair<uint32_t, uint32_t>> st;
    st.reserve(64);
    st.push_back({root, 0});
    color[root] = 1;
    while (!st.empty()) {
        auto& top = st.back();
        const uint32_t i = top.first;
        uint64_t start;
        int cnt = 0;
        const bool inner = children_of(nodes, i, slot_child, start, cnt);
        if (inner && (int)top.second < cnt) {
            const uint32_t c = (uint32_t)(start + top.second);
            ++top.second;
            if (refs[c] < 2) ++refs[c];
            if (color[c] == 1) return fail(SVO_EINVAL, "cycle through node %u", c);
            if (color[c] == 0) {
                color[c] = 1;
                st.push_back({c, 0});
            }
            continue;
        }
        // all children done
        uint32_t h = 0, x = 0;
        if (inner) {
            for (int k = 0; k < cnt; ++k) {
                const uint32_t c = (uint32_t)(start + k);
                h = std::max<uint32_t>(h, 1u + height[c]);
                x |= has_xf[c] | (nd_xform(nodes[c]) ? 1u : 0u);
            }
        }
        if (h > max_depth) return fail(SVO_ERANGE, "a frame is deeper than max_depth %u", max_depth);
        if (nd_xform(nodes[i])) {
            const uint32_t s = nd_w1(nodes[i]) & 0x7FFFFFFFu;
            slot_h[s] = (uint8_t)h;
            height[i] = 0;  // an empty cell for the frame around it
            has_xf[i] = 1;
        } else {
            height[i] = (uint8_t)h;
            has_xf[i] = (uint8_t)x;
        }
        color[i] = 2;
        st.pop_back();
    }
    for (uint64_t i = 0; i < n; ++i) {
        if (refs[i] >= 2) {
            ++A.n_shared;
            if (has_xf[i]) return fail(SVO_EINVAL, "node %llu is shared but contains a transformed node", (unsigned long long)i);
        }
    }
    A.world_height = height[root];
    A.max_height = A.world_height;

    // top-down walk along paths that lead to transformed nodes: parent
    // frame, level and cell of every transformed node (paths are unique)
    struct Item { uint32_t node; int32_t frame; uint32_t level, x, y, z, nest; };
    std::vector<Item> q;
    q.push_back({root, -1, 0, 0, 0, 0, 0});
    while (!q.empty()) {
        const Item it = q.back();
        q.pop_back();
        uint64_t start;
        int cnt;
        if (!children_of(nodes, it.node, slot_child, start, cnt)) continue;
        const uint32_t mask = nd_mask(nodes[it.node]);
        int k = 0;
        for (uint32_t o = 0; o < 8; ++o) {
            if (!(mask & (1u << o))) continue;
            const uint32_t c = (uint32_t)(start + k++);
            if (!has_xf[c]) continue;
            const uint32_t cx = 2 * it.x + (o & 1u), cy = 2 * it.y + ((o >> 1) & 1u), cz = 2 * it.z + ((o >> 2) & 1u);
            if (nd_xform(nodes[c])) {
                const uint32_t s = nd_w1(nodes[c]) & 0x7FFFFFFFu;
                if (A.slot_parent[s] != -2) return fail(SVO_EINVAL, "slot %u is used by two nodes", s);
                A.slot_parent[s] = it.frame;
                A.slot_node[s] = c;
                A.slot_level[s] = it.level + 1;
                A.slot_coord[s] = {cx, cy, cz};
                A.slot_mask[s] = nd_mask(nodes[c]);
                A.slot_height[s] = slot_h[s];
                A.max_height = std::max(A.max_height, (uint32_t)slot_h[s]);
                A.max_nesting = std::max(A.max_nesting, it.nest + 1);
                A.order.push_back(s);
                A.n_frames++;
                q.push_back({c, (int32_t)s, 0, 0, 0, 0, it.nest + 1});
            } else {
                q.push_back({c, it.frame, it.level + 1, cx, cy, cz, it.nest});
            }
        }
    }
    // parents before children
    std::vector<uint32_t> depth(n_slots, 0);
    for (uint32_t s : A.order) {
        uint32_t d = 0;
        for (int32_t p = A.slot_parent[s]; p >= 0; p = A.slot_parent[p]) ++d;
        depth[s] = d;
    }
    std::stable_sort(A.order.begin(), A.order.end(), [&](uint32_t a, uint32_t b) { return depth[a] < depth[b]; });
    return SVO_OK;
}

// ------------------------------------------------------------------ FP64 affine maps

struct Aff {
    double m[3][4];
};

Aff aff_identity() {
    Aff a;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 4; ++c) a.m[r][c] = (r == c) ? 1.0 : 0.0;
    return a;
}

// x -> P(C(x))
Aff aff_mul(const Aff& P, const Aff& C) {
    Aff o;
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 4; ++c) {
            double v = P.m[r][0] * C.m[0][c] + P.m[r][1] * C.m[1][c] + P.m[r][2] * C.m[2][c];
            if (c == 3) v += P.m[r][3];
            o.m[r][c] = v;
        }
    }
    return o;
}

// Inverse by elimination with partial pivoting; false if (near) singular.
bool aff_inverse(const Aff& A, Aff& I) {
    double a[3][6];
    double scale = 0.0;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) scale = std::max(scale, std::fabs(A.m[r][c]));
    if (!(scale > 0.0) || !std::isfinite(scale)) return false;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 6; ++c) a[r][c] = (c < 3) ? A.m[r][c] : ((c - 3 == r) ? 1.0 : 0.0);
    for (int col = 0; col < 3; ++col) {
        int p = col;
        for (int r = col + 1; r < 3; ++r)
            if (std::fabs(a[r][col]) > std::fabs(a[p][col])) p = r;
        if (std::fabs(a[p][col]) <= 1e-12 * scale) return false;
        if (p != col)
            for (int c = 0; c < 6; ++c) std::swap(a[p][c], a[col][c]);
        const double inv = 1.0 / a[col][col];
        for (int c = 0; c < 6; ++c) a[col][c] *= inv;
        for (int r = 0; r < 3; ++r) {
            if (r == col || a[r][col] == 0.0) continue;
            const double f = a[r][col];
            for (int c = 0; c < 6; ++c) a[r][c] -= f * a[col][c];
        }
    }
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) I.m[r][c] = a[r][3 + c];
        I.m[r][3] = -(I.m[r][0] * A.m[0][3] + I.m[r][1] * A.m[1][3] + I.m[r][2] * A.m[2][3]);
    }
    return true;
}

// ------------------------------------------------------------------ context / scenes

struct Scene {
    uint64_t n_nodes = 0;
    uint32_t root = SVO_NONE;
    float root_min[3] = {0, 0, 0};
    float root_size = 1;
    uint32_t n_slots = 0;
    Analysis an;
    std::vector<uint32_t> slot_child;
    std::vector<float> slot_cell;
    std::vector<Aff> fwd;               // parent-relative forward maps
    uint32_t world_child = 0;
    uint32_t world_mask = 0;
    uint64_t* d_nodes = nullptr;
    unsigned char* d_table[2] = {nullptr, nullptr};   // frame records, then the candidate list
    unsigned char* h_stage[2] = {nullptr, nullptr};
    hipEvent_t ev[2] = {nullptr, nullptr};
    size_t table_bytes = 0;
    bool inline_tab = false;            // small enough for the table to travel in a launch's arguments
    bool dev_current = true;            // the current device table holds the current transforms
    // traces that read device table k, one event per stream (re-recorded by
    // later traces on that stream): a copy into table k waits for them all
    std::vector<std::pair<hipStream_t, hipEvent_t>> readers[2];
    std::vector<hipEvent_t> spare_events;
    int cur = 0;                        // table the next trace reads
    uint32_t n_frames = 1;              // 1 + n_slots records per table
    // classification of the current table
    uint32_t n_cand = 0, stack_levels = 1, nest_levels = 0, n_inline = 0, n_bvh = 0, bvh_depth = 0;
    uint64_t bytes = 0;
    bool tuned = false;                 // svo_tune picked `cfg` for this scene
    svo_config cfg{};
};

}  // namespace

struct svo_ctx {
    int device = 0;
    int n_cu = 0;
    size_t max_lds = 0;       // LDS one work-group may use
    size_t lds_per_cu = 0;    // LDS of one compute unit
    svo_config cfg{};
    uint32_t next_scene = 1;
    std::map<uint32_t, std::unique_ptr<Scene>> scenes;
    uint32_t* d_queue = nullptr;                // kMaxStreams work queues of kQueueWords
    // slow tiles first: two states of kHotWords per work queue, each kept for
    // one ray set (signature); a state is used from the second trace of its
    // rays on, so rays traced once pay nothing for it
    uint32_t* d_hot = nullptr;
    struct HotRec {
        uint64_t sig[2] = {0, 0};
        uint32_t uses[2] = {0, 0};
        uint32_t seq[2] = {0, 0};   // launches on each state since its launch shape last changed
        uint32_t shape[2] = {0, 0}; // that shape (waves per work-group, work-groups per CU)
        bool fresh[2] = {false, false};  // handed to a new ray set: its threshold starts again
        uint32_t recent = 0;    // the state used last (the other one is replaced first)
    };
    HotRec hot_rec[kMaxStreams];
    std::map<hipStream_t, uint32_t> stream_slot;
    // ring of batch tables (job records, frames, candidates): pinned staging
    // + device copy, reused once the launch that read them has finished
    struct BatchBuf {
        unsigned char* dev = nullptr;
        unsigned char* host = nullptr;
        size_t cap = 0;
        hipEvent_t ev = nullptr;
    };
    BatchBuf batch[4];
    uint32_t next_batch = 0;
    // svo_trace_batch_static: this device's scratch (its queue, then its
    // table area), pinned staging for the table and the event after the
    // staging's last copy; all set up in svo_create
    unsigned char* d_static = nullptr;
    unsigned char* h_static = nullptr;
    hipEvent_t static_ev = nullptr;
    std::set<svo_plan*> plans;
};

// A reusable launch (svo_plan_*): fixed kernel arguments over a device
// table of fixed capacity, filled from pinned staging by each launch.
struct svo_plan {
    std::set<svo_scene> scenes;
    svo_config cfg{};
    svo::TraceArgs args{};
    svo::LaunchCfg launch_cfg{};
    uint32_t max_jobs = 0, max_frames = 0, max_cand = 0, stack_cap = 1, nest_cap = 0, max_bvh = 0, bvh_depth_cap = 0;
    size_t off_jobs = 0, off_frames = 0, off_cand = 0, off_sph = 0, off_x = 0, off_bvh = 0, off_cams = 0, bytes = 0;
    unsigned char* dev = nullptr;
    unsigned char* host = nullptr;
    uint32_t* d_queue = nullptr;
    hipEvent_t ev = nullptr;
    bool ev_pending = false;   // an eager launch's copy of the staging may still run
};

namespace {

void destroy_plan(svo_plan& p) {
    if (p.dev) (void)hipFree(p.dev);
    if (p.host) (void)hipHostFree(p.host);
    if (p.d_queue) (void)hipFree(p.d_queue);
    if (p.ev) (void)hipEventDestroy(p.ev);
    p.dev = nullptr;
    p.host = nullptr;
    p.d_queue = nullptr;
    p.ev = nullptr;
}

}  // namespace

namespace {

svo_config default_config() {
    svo_config c{};
    c.waves_per_block = 8;
    c.blocks_per_cu = 3;   // 24 waves per CU: what the sorted-candidate kernel's registers allow
    c.lds_cache_nodes = 1024;
    c.refill_lanes = 48;
    c.step_limit = 1u << 20;
    c.claim_tiles = 2;
    return c;
}

int check_config(const svo_config& c) {
    if (c.waves_per_block < 1 || c.waves_per_block > 16) return fail(SVO_EINVAL, "waves_per_block must be 1..16");
    if (c.blocks_per_cu < 1 || c.blocks_per_cu > 32) return fail(SVO_EINVAL, "blocks_per_cu must be 1..32");
    if (c.lds_cache_nodes > 16384) return fail(SVO_EINVAL, "lds_cache_nodes must be <= 16384");
    if (c.step_limit < 1) return fail(SVO_EINVAL, "step_limit must be >= 1");
    if (c.claim_tiles > 64) return fail(SVO_EINVAL, "claim_tiles must be <= 64");
    if (c.sorted_candidates > 64) return fail(SVO_EINVAL, "sorted_candidates must be <= 64");
    if (c.tile_order > 1) return fail(SVO_EINVAL, "tile_order must be 0 or 1");
    return SVO_OK;
}

// Candidates up to which a job takes the per-lane sorted entry table.
uint32_t sort_limit(const svo_config& c) {
    return c.sorted_candidates ? c.sorted_candidates : svo::kMaxSortedCand;
}

void free_scene(Scene& s) {
    if (s.d_nodes) (void)hipFree(s.d_nodes);
    for (int k = 0; k < 2; ++k) {
        if (s.d_table[k]) (void)hipFree(s.d_table[k]);
        if (s.h_stage[k]) (void)hipHostFree(s.h_stage[k]);
        if (s.ev[k]) (void)hipEventDestroy(s.ev[k]);
        for (auto& r : s.readers[k]) (void)hipEventDestroy(r.second);
        s.readers[k].clear();
    }
    for (hipEvent_t e : s.spare_events) (void)hipEventDestroy(e);
    s.spare_events.clear();
    s.d_nodes = nullptr;
}

Scene* find_scene(svo_ctx* ctx, svo_scene h) {
    auto it = ctx->scenes.find(h);
    return it == ctx->scenes.end() ? nullptr : it->second.get();
}

// Layout of a scene's frame table: n_frames records, then the candidate list
// (n_slots u32), then one bounding sphere (centre xyz, radius) per record,
// then one exact (FP64) map per record.
inline size_t cand_offset(uint32_t n_frames) { return (size_t)n_frames * sizeof(svo::FrameRec); }
inline size_t sphere_offset(uint32_t n_frames, uint32_t n_slots) {
    return (cand_offset(n_frames) + (size_t)n_slots * sizeof(uint32_t) + 15) & ~(size_t)15;
}
inline size_t xmap_offset(uint32_t n_frames, uint32_t n_slots) {
    return sphere_offset(n_frames, n_slots) + (size_t)n_frames * 16;
}
constexpr size_t kXmapBytes = svo::kExactMapDoubles * sizeof(double);
// ... then the hierarchy over the candidates (at most 2 n_slots nodes).
inline size_t bvh_offset(uint32_t n_frames, uint32_t n_slots) {
    return xmap_offset(n_frames, n_slots) + (size_t)n_frames * kXmapBytes;
}
inline uint32_t bvh_capacity(uint32_t n_slots) { return std::max<uint32_t>(1, 2 * n_slots); }
inline size_t table_size(uint32_t n_frames, uint32_t n_slots) {
    return bvh_offset(n_frames, n_slots) + (size_t)bvh_capacity(n_slots) * sizeof(svo::BvhNode);
}

struct TableInfo {
    uint32_t n_cand = 0, stack_levels = 1, nest_levels = 0, n_inline = 0, n_bvh = 0, bvh_depth = 0;
};

// Levels of the hierarchy bvh_build makes over n candidates (median splits,
// leaves of at most kBvhLeafMax).
uint32_t bvh_levels(uint32_t n) {
    if (n <= svo::kBvhLeafMax) return n ? 1u : 0u;
    return 1u + std::max(bvh_levels(n / 2), bvh_levels(n - n / 2));
}

struct BItem {
    double lo[3], hi[3], c[3];
    uint32_t frame;
};

float round_down_f32(double v) {
    float f = (float)v;
    return ((double)f > v) ? std::nextafter(f, -INFINITY) : f;
}
float round_up_f32(double v) {
    float f = (float)v;
    return ((double)f < v) ? std::nextafter(f, INFINITY) : f;
}

// Median-split hierarchy over items [begin, end), nodes in depth-first
// order from out[n]; returns the node index.  Boxes are widened by 1e-5 of
// their extent plus 1e-6 of their magnitude and rounded outward to FP32.
uint32_t bvh_build(std::vector<BItem>& it, uint32_t begin, uint32_t end, uint32_t level, svo::BvhNode* out,
                   uint32_t& n, uint32_t& depth) {
    const uint32_t me = n++;
    depth = std::max(depth, level);
    double lo[3], hi[3], clo[3], chi[3];
    for (int a = 0; a < 3; ++a) {
        lo[a] = clo[a] = INFINITY;
        hi[a] = chi[a] = -INFINITY;
    }
    for (uint32_t i = begin; i < end; ++i)
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], it[i].lo[a]);
            hi[a] = std::max(hi[a], it[i].hi[a]);
            clo[a] = std::min(clo[a], it[i].c[a]);
            chi[a] = std::max(chi[a], it[i].c[a]);
        }
    double ext = 0.0, mag = 1.0;
    for (int a = 0; a < 3; ++a) {
        ext = std::max(ext, hi[a] - lo[a]);
        mag = std::max(mag, std::max(std::fabs(lo[a]), std::fabs(hi[a])));
    }
    const double pad = 1e-5 * ext + 1e-6 * mag;
    svo::BvhNode& N = out[me];
    for (int a = 0; a < 3; ++a) {
        N.lo[a] = round_down_f32(lo[a] - pad);
        N.hi[a] = round_up_f32(hi[a] + pad);
    }
    if (end - begin <= svo::kBvhLeafMax) {
        N.a = begin;
        N.b = svo::kBvhLeaf | (end - begin);
        return me;
    }
    int axis = 0;
    for (int a = 1; a < 3; ++a)
        if (chi[a] - clo[a] > chi[axis] - clo[axis]) axis = a;
    const uint32_t mid = begin + (end - begin) / 2;
    std::nth_element(it.begin() + begin, it.begin() + mid, it.begin() + end,
                     [axis](const BItem& x, const BItem& y) { return x.c[axis] < y.c[axis]; });
    const uint32_t L = bvh_build(it, begin, mid, level + 1, out, n, depth);
    const uint32_t R = bvh_build(it, mid, end, level + 1, out, n, depth);
    out[me].a = L;
    out[me].b = R;
    return me;
}

// Compose, invert and pack the frame table into `out` (host): record 0 is
// the world, record 1 + s slot s; the candidate list follows the records.
// A slot whose moved cell stays inside its static cell is entered in place
// (FR_INLINE, nesting bounded by kMaxInlineNest); every other referenced slot
// is a candidate traced from its own root.
int build_frames(const Scene& S, const std::vector<Aff>& fwd, unsigned char* out, TableInfo& T) {
    const Analysis& A = S.an;
    svo::FrameRec* rec = reinterpret_cast<svo::FrameRec*>(out);
    uint32_t* cand = reinterpret_cast<uint32_t*>(out + cand_offset(S.n_frames));
    float* sph = reinterpret_cast<float*>(out + sphere_offset(S.n_frames, S.n_slots));
    double* xm = reinterpret_cast<double*>(out + xmap_offset(S.n_frames, S.n_slots));
    std::memset(out, 0, S.table_bytes);
    T = TableInfo();
    // world
    svo::FrameRec& W = rec[0];
    const uint32_t K0 = A.world_height;
    const double g0 = std::ldexp(1.0, (int)K0) / (double)S.root_size;
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) xm[4 * r + c] = (r == c) ? g0 : 0.0;
        xm[4 * r + 3] = -(double)S.root_min[r] * g0;
        for (int c = 0; c < 4; ++c) W.m[4 * r + c] = (float)xm[4 * r + c];
    }
    W.inst = SVO_NONE;
    W.root = S.root;
    if (S.root == SVO_NONE) {
        W.info = svo::FR_EMPTY;
    } else {
        W.info = (K0 << svo::FR_K_SHIFT) | S.world_mask;
        if (K0 == 0) W.info |= svo::FR_ROOT_LEAF;
        W.child = S.world_child;
    }
    T.stack_levels = std::max<uint32_t>(T.stack_levels, K0 + 1);
    for (uint32_t s = 0; s < S.n_slots; ++s) {
        rec[1 + s].info = svo::FR_EMPTY;
        rec[1 + s].inst = s;
        rec[1 + s].root = SVO_NONE;
    }
    std::vector<Aff> world(S.n_slots);
    std::vector<uint32_t> depth(S.n_slots, 0), sbase(S.n_slots, 0);
    std::vector<uint32_t> inline_frames;
    for (uint32_t s : A.order) {
        const int32_t p = A.slot_parent[s];
        world[s] = aff_mul(p < 0 ? aff_identity() : world[p], fwd[s]);
        Aff inv;
        if (!aff_inverse(world[s], inv)) return fail(SVO_EINVAL, "transform of slot %u is singular", s);
        const float* cell = &S.slot_cell[4 * s];
        const uint32_t K = A.slot_height[s];
        const double g = std::ldexp(1.0, (int)K) / (double)cell[3];
        svo::FrameRec& F = rec[1 + s];
        double* X = xm + (size_t)svo::kExactMapDoubles * (1 + s);
        for (int r = 0; r < 3; ++r) {
            for (int c = 0; c < 3; ++c) X[4 * r + c] = g * inv.m[r][c];
            X[4 * r + 3] = g * (inv.m[r][3] - (double)cell[r]);
            for (int c = 0; c < 4; ++c) F.m[4 * r + c] = (float)X[4 * r + c];
        }
        F.child = S.slot_child[s];
        F.info = A.slot_mask[s] | (K << svo::FR_K_SHIFT);
        F.inst = s;
        F.root = A.slot_node[s];
        {
            // world-space bounding sphere of the moved root cell (Sec. 4.1):
            // the image of the cell centre and the farthest image corner
            double c[3], h = 0.5 * cell[3];
            for (int r = 0; r < 3; ++r)
                c[r] = world[s].m[r][0] * (cell[0] + h) + world[s].m[r][1] * (cell[1] + h) +
                       world[s].m[r][2] * (cell[2] + h) + world[s].m[r][3];
            double rad = 0.0;
            for (int k = 0; k < 8; ++k) {
                double q = 0.0;
                for (int r = 0; r < 3; ++r) {
                    const double v = world[s].m[r][0] * (cell[0] + (((k >> 0) & 1) ? cell[3] : 0.0)) +
                                     world[s].m[r][1] * (cell[1] + (((k >> 1) & 1) ? cell[3] : 0.0)) +
                                     world[s].m[r][2] * (cell[2] + (((k >> 2) & 1) ? cell[3] : 0.0)) + world[s].m[r][3];
                    q += (v - c[r]) * (v - c[r]);
                }
                rad = std::max(rad, std::sqrt(q));
            }
            for (int r = 0; r < 3; ++r) sph[4 * (1 + s) + r] = (float)c[r];
            sph[4 * (1 + s) + 3] = (float)rad;
        }
        // does the moved cell stay inside its static cell (parent frame)?
        double pmin[3], psize;
        if (p < 0) {
            for (int a = 0; a < 3; ++a) pmin[a] = S.root_min[a];
            psize = S.root_size;
        } else {
            for (int a = 0; a < 3; ++a) pmin[a] = S.slot_cell[4 * p + a];
            psize = S.slot_cell[4 * p + 3];
        }
        const double csize = psize / std::ldexp(1.0, (int)A.slot_level[s]);
        const double margin = 1e-5 * csize;
        bool inside = true;
        for (int k = 0; k < 8 && inside; ++k) {
            double x[3];
            for (int a = 0; a < 3; ++a) x[a] = cell[a] + (((k >> a) & 1) ? cell[3] : 0.0);
            for (int r = 0; r < 3; ++r) {
                const double v = fwd[s].m[r][0] * x[0] + fwd[s].m[r][1] * x[1] + fwd[s].m[r][2] * x[2] +
                                 fwd[s].m[r][3];
                const double lo = pmin[r] + A.slot_coord[s][r] * csize;
                if (!(v >= lo + margin && v <= lo + csize - margin)) inside = false;
            }
        }
        const bool parent_inline = p >= 0 && (rec[1 + p].info & svo::FR_INLINE);
        const uint32_t d = parent_inline ? depth[p] + 1 : 1;
        if (inside && d <= svo::kMaxInlineNest) {
            F.info |= svo::FR_INLINE;
            depth[s] = d;
            sbase[s] = (parent_inline ? sbase[p] : 0) + A.slot_level[s];
            T.nest_levels = std::max(T.nest_levels, d);
            T.stack_levels = std::max(T.stack_levels, sbase[s] + K + 1);
            inline_frames.push_back(1 + s);
            ++T.n_inline;
        } else {
            cand[T.n_cand++] = 1 + s;
            T.stack_levels = std::max(T.stack_levels, K + 1);
        }
    }
    if (T.stack_levels > 127) return fail(SVO_ERANGE, "nested frames need %u stack levels (limit 127)", T.stack_levels);
    // the in-place frames follow the candidates in the list (the hit-buffer
    // test of svo_trace_rays_reuse checks every moved frame)
    for (uint32_t i = 0; i < T.n_inline; ++i) cand[T.n_cand + i] = inline_frames[i];
    // hierarchy over the candidates' world boxes (the image of each moved
    // root cell), leaves in candidate-list order
    if (T.n_cand) {
        std::vector<BItem> items(T.n_cand);
        for (uint32_t i = 0; i < T.n_cand; ++i) {
            const uint32_t s = cand[i] - 1;
            const float* cell = &S.slot_cell[4 * s];
            BItem& b = items[i];
            b.frame = cand[i];
            for (int r = 0; r < 3; ++r) {
                b.lo[r] = INFINITY;
                b.hi[r] = -INFINITY;
            }
            for (int k = 0; k < 8; ++k) {
                double x[3];
                for (int a = 0; a < 3; ++a) x[a] = cell[a] + (((k >> a) & 1) ? cell[3] : 0.0);
                for (int r = 0; r < 3; ++r) {
                    const double v = world[s].m[r][0] * x[0] + world[s].m[r][1] * x[1] + world[s].m[r][2] * x[2] +
                                     world[s].m[r][3];
                    b.lo[r] = std::min(b.lo[r], v);
                    b.hi[r] = std::max(b.hi[r], v);
                }
            }
            for (int r = 0; r < 3; ++r) b.c[r] = 0.5 * (b.lo[r] + b.hi[r]);
        }
        svo::BvhNode* bn = reinterpret_cast<svo::BvhNode*>(out + bvh_offset(S.n_frames, S.n_slots));
        uint32_t n = 0, depth = 0;
        bvh_build(items, 0, T.n_cand, 1, bn, n, depth);
        for (uint32_t i = 0; i < T.n_cand; ++i) cand[i] = items[i].frame;
        T.n_bvh = n;
        T.bvh_depth = depth;
    }
    return SVO_OK;
}

// Build the next table in the staging buffer not in use and make it current.
// With to_device the table is also copied into the device table not in use,
// on `stream`.  Without (transform updates of a scene whose table fits a
// launch's arguments) there is no device work: traces then copy the staging
// table into their arguments when they are enqueued.
int upload_frames(Scene& S, hipStream_t stream, bool to_device) {
    const int k = S.cur ^ 1;
    // the staging buffer may still feed an earlier copy
    HIP_TRY(hipEventSynchronize(S.ev[k]));
    TableInfo T;
    int rc = build_frames(S, S.fwd, S.h_stage[k], T);
    if (rc) return rc;
    if (to_device) {
        // traces on other streams may still read the table this copy
        // overwrites: the copy waits for them on the device
        for (auto& r : S.readers[k]) {
            if (r.first != stream) HIP_TRY(hipStreamWaitEvent(stream, r.second, 0));
            S.spare_events.push_back(r.second);
        }
        S.readers[k].clear();
        HIP_TRY(hipMemcpyAsync(S.d_table[k], S.h_stage[k], S.table_bytes, hipMemcpyHostToDevice, stream));
        HIP_TRY(hipEventRecord(S.ev[k], stream));
    }
    S.dev_current = to_device;
    S.cur = k;
    S.n_cand = T.n_cand;
    S.stack_levels = T.stack_levels;
    S.nest_levels = T.nest_levels;
    S.n_inline = T.n_inline;
    S.n_bvh = T.n_bvh;
    S.bvh_depth = T.bvh_depth;
    return SVO_OK;
}

}  // namespace

// ------------------------------------------------------------------ C ABI

extern "C" {

int svo_abi_version(void) { return SVO_ABI_VERSION; }

const char* svo_last_error(void) { return g_err.c_str(); }

int svo_validate(const uint64_t* nodes, uint64_t n_nodes, uint32_t root, uint32_t max_depth,
                 const uint32_t* slot_child, uint32_t n_slots, svo_pool_info* info) {
    try {
        Analysis A;
        const int rc = analyse(nodes, n_nodes, root, max_depth, slot_child, n_slots, A);
        if (rc) return rc;
        if (info) {
            std::memset(info, 0, sizeof *info);
            info->n_nodes = n_nodes;
            info->n_frames = A.n_frames;
            info->world_height = A.world_height;
            info->max_height = A.max_height;
            info->max_nesting = A.max_nesting;
            info->n_shared = A.n_shared;
        }
        return SVO_OK;
    } catch (const std::bad_alloc&) {
        return fail(SVO_ENOMEM, "out of host memory");
    } catch (...) {
        return fail(SVO_EINVAL, "unexpected error");
    }
}

int svo_create(svo_ctx** out, int device_ordinal) {
    if (!out) return fail(SVO_EINVAL, "out is NULL");
    *out = nullptr;
    int n = 0;
    HIP_TRY(hipGetDeviceCount(&n));
    if (device_ordinal < 0 || device_ordinal >= n) return fail(SVO_EINVAL, "device %d out of range (%d)", device_ordinal, n);
    HIP_TRY(hipSetDevice(device_ordinal));
    std::unique_ptr<svo_ctx> c(new (std::nothrow) svo_ctx());
    if (!c) return fail(SVO_ENOMEM, "out of host memory");
    c->device = device_ordinal;
    HIP_TRY(hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, device_ordinal));
    int lds = 0;
    HIP_TRY(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device_ordinal));
    c->max_lds = (size_t)lds;
    int lds_cu = 0;
    if (hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, device_ordinal) != hipSuccess ||
        lds_cu <= 0)
        lds_cu = lds;
    c->lds_per_cu = (size_t)std::max(lds_cu, lds);
    c->cfg = default_config();
    HIP_TRY(svo::prepare_trace(c->max_lds));
    auto undo = [&](int code, const char* what, hipError_t e) {
        if (c->d_queue) (void)hipFree(c->d_queue);
        if (c->d_hot) (void)hipFree(c->d_hot);
        if (c->h_static) (void)hipHostFree(c->h_static);
        if (c->static_ev) (void)hipEventDestroy(c->static_ev);
        return fail(code, "%s: %s", what, hipGetErrorString(e));
    };
    hipError_t e = hipMalloc((void**)&c->d_queue, kMaxStreams * svo::kQueueWords * sizeof(uint32_t));
    if (e != hipSuccess) return undo(SVO_ENOMEM, "work queue allocation", e);
    if ((e = hipMemset(c->d_queue, 0, kMaxStreams * svo::kQueueWords * sizeof(uint32_t))) != hipSuccess)
        return undo(SVO_EDEVICE, "work queue clear", e);
    if ((e = hipMalloc((void**)&c->d_hot, (size_t)kMaxStreams * 2 * svo::kHotWords * sizeof(uint32_t))) != hipSuccess)
        return undo(SVO_ENOMEM, "slow-tile state allocation", e);
    if ((e = hipMemset(c->d_hot, 0, (size_t)kMaxStreams * 2 * svo::kHotWords * sizeof(uint32_t))) != hipSuccess)
        return undo(SVO_EDEVICE, "slow-tile state clear", e);
    // the allocation-free entry point's scratch: found once per device, its
    // queue cleared here (its kernels leave the queue at zero on exit)
    if ((e = svo::static_scratch(device_ordinal, &c->d_static)) != hipSuccess) return undo(SVO_EDEVICE, "scratch lookup", e);
    if ((e = hipMemset(c->d_static, 0, svo::kStaticQueueBytes)) != hipSuccess) return undo(SVO_EDEVICE, "scratch clear", e);
    if ((e = hipHostMalloc((void**)&c->h_static, svo::kStaticTableBytes, hipHostMallocDefault)) != hipSuccess)
        return undo(SVO_ENOMEM, "pinned staging allocation", e);
    if ((e = hipEventCreateWithFlags(&c->static_ev, hipEventDisableTiming)) != hipSuccess)
        return undo(SVO_EDEVICE, "event creation", e);
    if ((e = hipDeviceSynchronize()) != hipSuccess) return undo(SVO_EDEVICE, "set-up", e);
    *out = c.release();
    return SVO_OK;
}

void svo_destroy(svo_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (svo_plan* p : ctx->plans) {
        destroy_plan(*p);
        delete p;
    }
    ctx->plans.clear();
    for (auto& kv : ctx->scenes) free_scene(*kv.second);
    ctx->scenes.clear();
    for (auto& b : ctx->batch) {
        if (b.dev) (void)hipFree(b.dev);
        if (b.host) (void)hipHostFree(b.host);
        if (b.ev) (void)hipEventDestroy(b.ev);
    }
    if (ctx->d_queue) (void)hipFree(ctx->d_queue);
    if (ctx->d_hot) (void)hipFree(ctx->d_hot);
    if (ctx->h_static) (void)hipHostFree(ctx->h_static);
    if (ctx->static_ev) (void)hipEventDestroy(ctx->static_ev);
    delete ctx;
}

int svo_upload(svo_ctx* ctx, const uint64_t* nodes, uint64_t n_nodes, uint32_t root, const float root_min[3],
               float root_size, uint32_t max_depth, const uint32_t* slot_child, const float* slot_cell,
               uint32_t n_slots, svo_scene* out) {
    if (!ctx || !out) return fail(SVO_EINVAL, "ctx and out must not be NULL");
    if (!root_min) return fail(SVO_EINVAL, "root_min is NULL");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(root_min[a])) return fail(SVO_EINVAL, "root_min must be finite");
    if (!(root_size > 0.0f) || !std::isfinite(root_size)) return fail(SVO_EINVAL, "root_size must be finite and > 0");
    if (n_slots && !slot_cell) return fail(SVO_EINVAL, "slot_cell is NULL");
    for (uint32_t s = 0; s < n_slots; ++s) {
        for (int a = 0; a < 4; ++a)
            if (!std::isfinite(slot_cell[4 * s + a])) return fail(SVO_EINVAL, "slot_cell[%u] must be finite", s);
        if (!(slot_cell[4 * s + 3] > 0.0f)) return fail(SVO_EINVAL, "slot_cell[%u] size must be > 0", s);
    }
    try {
        std::unique_ptr<Scene> S(new Scene());
        int rc = analyse(nodes, n_nodes, root, max_depth, slot_child, n_slots, S->an);
        if (rc) return rc;
        S->n_nodes = n_nodes;
        S->root = root;
        for (int a = 0; a < 3; ++a) S->root_min[a] = root_min[a];
        S->root_size = root_size;
        S->n_slots = n_slots;
        S->slot_child.assign(slot_child, slot_child + n_slots);
        S->slot_cell.assign(slot_cell, slot_cell + 4 * (size_t)n_slots);
        S->fwd.assign(n_slots, aff_identity());
        if (root != SVO_NONE && !nd_leaf(nodes[root])) {
            uint64_t st;
            int cnt;
            children_of(nodes, root, S->slot_child.data(), st, cnt);
            S->world_child = (uint32_t)st;
            S->world_mask = nd_mask(nodes[root]);
        }
        HIP_TRY(hipSetDevice(ctx->device));
        const size_t nb = std::max<uint64_t>(n_nodes, 1) * sizeof(uint64_t);
        if (hipMalloc((void**)&S->d_nodes, nb) != hipSuccess) {
            free_scene(*S);
            return fail(SVO_ENOMEM, "device allocation of %zu bytes failed", nb);
        }
        S->n_frames = 1 + n_slots;
        S->table_bytes = table_size(S->n_frames, n_slots);
        // at most 16 slots: every candidate takes the sorted path, which
        // needs no hierarchy, so records, candidates, spheres and exact maps suffice
        S->inline_tab = n_slots <= svo::kMaxSortedCand && bvh_offset(S->n_frames, n_slots) <= svo::kInlineTableBytes;
        const size_t fb = S->table_bytes;
        for (int k = 0; k < 2; ++k) {
            if (hipMalloc((void**)&S->d_table[k], fb) != hipSuccess ||
                hipHostMalloc((void**)&S->h_stage[k], fb, hipHostMallocDefault) != hipSuccess ||
                hipEventCreateWithFlags(&S->ev[k], hipEventDisableTiming) != hipSuccess) {
                free_scene(*S);
                return fail(SVO_ENOMEM, "allocation of frame tables failed");
            }
        }
        if (n_nodes) {
            hipError_t e = hipMemcpy(S->d_nodes, nodes, n_nodes * sizeof(uint64_t), hipMemcpyHostToDevice);
            if (e != hipSuccess) {
                free_scene(*S);
                return fail(SVO_EDEVICE, "pool copy failed: %s", hipGetErrorString(e));
            }
        }
        for (int k = 0; k < 2; ++k) (void)hipEventRecord(S->ev[k], 0);
        rc = upload_frames(*S, 0, true);
        if (rc == SVO_OK && hipStreamSynchronize(0) != hipSuccess) rc = fail(SVO_EDEVICE, "frame upload failed");
        if (rc) {
            free_scene(*S);
            return rc;
        }
        S->bytes = nb + 2 * fb;
        const uint32_t h = ctx->next_scene++;
        ctx->scenes[h] = std::move(S);
        *out = h;
        return SVO_OK;
    } catch (const std::bad_alloc&) {
        return fail(SVO_ENOMEM, "out of host memory");
    }
}

int svo_free_scene(svo_ctx* ctx, svo_scene scene) {
    if (!ctx) return fail(SVO_EINVAL, "ctx is NULL");
    auto it = ctx->scenes.find(scene);
    if (it == ctx->scenes.end()) return fail(SVO_EINVAL, "unknown scene %u", scene);
    for (const svo_plan* p : ctx->plans)
        if (p->scenes.count(scene)) return fail(SVO_EBUSY, "scene %u belongs to a live plan", scene);
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(hipDeviceSynchronize());
    free_scene(*it->second);
    ctx->scenes.erase(it);
    return SVO_OK;
}

int svo_scene_bytes(svo_ctx* ctx, svo_scene scene, uint64_t* bytes) {
    if (!ctx || !bytes) return fail(SVO_EINVAL, "ctx and bytes must not be NULL");
    Scene* S = find_scene(ctx, scene);
    if (!S) return fail(SVO_EINVAL, "unknown scene %u", scene);
    *bytes = S->bytes;
    return SVO_OK;
}

int svo_get_scene_stats(svo_ctx* ctx, svo_scene scene, svo_scene_stats* out) {
    if (!ctx || !out) return fail(SVO_EINVAL, "ctx and out must not be NULL");
    Scene* S = find_scene(ctx, scene);
    if (!S) return fail(SVO_EINVAL, "unknown scene %u", scene);
    std::memset(out, 0, sizeof *out);
    out->device_bytes = S->bytes;
    out->n_slots = S->n_slots;
    out->n_frames = S->an.n_frames;
    out->n_inline = S->n_inline;
    out->n_candidates = S->n_cand;
    out->stack_levels = S->stack_levels;
    out->nest_levels = S->nest_levels;
    return SVO_OK;
}

int svo_set_transforms(svo_ctx* ctx, svo_scene scene, uint32_t first_slot, uint32_t count, const float* fwd_3x4,
                       void* stream) {
    if (!ctx) return fail(SVO_EINVAL, "ctx is NULL");
    Scene* S = find_scene(ctx, scene);
    if (!S) return fail(SVO_EINVAL, "unknown scene %u", scene);
    if ((uint64_t)first_slot + count > S->n_slots) return fail(SVO_EINVAL, "slots [%u, %u) out of range (%u)", first_slot,
                                                               first_slot + count, S->n_slots);
    if (count && !fwd_3x4) return fail(SVO_EINVAL, "fwd_3x4 is NULL");
    // Every map is checked before any is stored: a rejected call leaves all
    // slots as they were.
    std::vector<Aff> next(count);
    for (uint32_t j = 0; j < count; ++j) {
        Aff& a = next[j];
        for (int r = 0; r < 3; ++r) {
            for (int c = 0; c < 4; ++c) {
                const float v = fwd_3x4[12 * j + 4 * r + c];
                if (!std::isfinite(v)) return fail(SVO_EINVAL, "transform of slot %u is not finite", first_slot + j);
                a.m[r][c] = v;
            }
        }
        Aff inv;
        if (!aff_inverse(a, inv)) return fail(SVO_EINVAL, "transform of slot %u is singular", first_slot + j);
    }
    std::vector<Aff> keep(S->fwd.begin() + first_slot, S->fwd.begin() + first_slot + count);
    std::copy(next.begin(), next.end(), S->fwd.begin() + first_slot);
    HIP_TRY(hipSetDevice(ctx->device));
    const int rc = upload_frames(*S, (hipStream_t)stream, !S->inline_tab);
    if (rc) {
        std::copy(keep.begin(), keep.end(), S->fwd.begin() + first_slot);
        return rc;
    }
    return SVO_OK;
}

int svo_get_config(svo_ctx* ctx, svo_config* cfg) {
    if (!ctx || !cfg) return fail(SVO_EINVAL, "ctx and cfg must not be NULL");
    *cfg = ctx->cfg;
    return SVO_OK;
}

int svo_set_config(svo_ctx* ctx, const svo_config* cfg) {
    if (!ctx || !cfg) return fail(SVO_EINVAL, "ctx and cfg must not be NULL");
    svo_config c = *cfg;
    const svo_config d = default_config();
    if (!c.waves_per_block) c.waves_per_block = d.waves_per_block;
    if (!c.blocks_per_cu) c.blocks_per_cu = d.blocks_per_cu;
    if (!c.step_limit) c.step_limit = d.step_limit;
    const int rc = check_config(c);
    if (rc) return rc;
    ctx->cfg = c;
    for (auto& kv : ctx->scenes) kv.second->tuned = false;
    return SVO_OK;
}

}  // extern "C"

namespace {

int queue_slot(svo_ctx* ctx, hipStream_t st, uint32_t& qslot) {
    auto it = ctx->stream_slot.find(st);
    if (it == ctx->stream_slot.end()) {
        if (ctx->stream_slot.size() >= kMaxStreams) return fail(SVO_ERANGE, "more than %u streams", kMaxStreams);
        qslot = (uint32_t)ctx->stream_slot.size();
        try {
            ctx->stream_slot[st] = qslot;
        } catch (const std::bad_alloc&) {
            return fail(SVO_ENOMEM, "out of host memory");
        }
    } else {
        qslot = it->second;
    }
    return SVO_OK;
}

// Work-groups of the persistent grid per CU: the configured count, capped by
// what can be resident at once (LDS per CU, 32 waves per CU), so that no
// work-group waits for another to exit before it starts.
uint32_t resident_blocks(const svo_ctx* ctx, const svo_config& c, size_t lds) {
    uint32_t b = c.blocks_per_cu;
    if (lds) b = std::min<uint32_t>(b, (uint32_t)(ctx->lds_per_cu / lds));
    b = std::min<uint32_t>(b, 32u / c.waves_per_block);
    return std::max<uint32_t>(b, 1u);
}

// A stride coprime with `tiles` near tiles / golden ratio: consecutive claims
// land far apart in the image.
uint64_t tile_stride(uint64_t tiles) {
    if (tiles <= 2) return 1;
    uint64_t s = (uint64_t)((double)tiles * 0.6180339887498949) | 1ull;
    while (s > 1 && std::gcd(s, tiles) != 1) s -= 2;
    return s ? s : 1;
}

// Fit a launch into the per-work-group LDS limit: halve the node cache,
// then take waves out of the work-group (to the next multiple of 4, so the
// four SIMDs stay evenly loaded, then one at a time).  Results never depend
// on either; a configuration tuned on one scene may meet a batch whose
// tables are larger.  Returns the LDS bytes, above the limit if nothing fits.
size_t fit_lds(const svo_ctx* ctx, svo::TraceArgs& a, uint32_t& waves) {
    size_t lds = svo::trace_lds_bytes(a, waves);
    while (lds > ctx->max_lds && a.lds_nodes > 0) {
        a.lds_nodes = (a.lds_nodes / 2) & ~1u;
        lds = svo::trace_lds_bytes(a, waves);
    }
    while (lds > ctx->max_lds && waves > 1) {
        waves = (waves > 4 && waves % 4) ? waves & ~3u : (waves > 4 ? waves - 4 : waves - 1);
        lds = svo::trace_lds_bytes(a, waves);
    }
    return lds;
}

// Size LDS (see fit_lds) and launch.
int launch(svo_ctx* ctx, const svo_config& cfg, svo::TraceArgs& a, hipStream_t st, const unsigned char* inline_tab = nullptr,
           size_t inline_bytes = 0) {
    a.tile_stride = tile_stride((a.n_rays + 63) / 64);
    svo_config c = cfg;
    const size_t lds = fit_lds(ctx, a, c.waves_per_block);
    if (lds > ctx->max_lds) return fail(SVO_ERANGE, "launch needs %zu bytes of LDS per work-group", lds);
    if (!a.jobs && a.job0.lds_nodes) a.job0.lds_nodes = a.lds_nodes;
    svo::LaunchCfg L{};
    L.waves_per_block = c.waves_per_block;
    const uint64_t tiles = (a.n_rays + 63) / 64;
    const uint64_t want = (tiles + c.waves_per_block - 1) / c.waves_per_block;
    const uint64_t cap = (uint64_t)ctx->n_cu * resident_blocks(ctx, c, lds);
    L.blocks = (uint32_t)std::max<uint64_t>(1, std::min(want, cap));
    L.lds_bytes = lds;
    const hipError_t e = a.counts ? svo::launch_trace_counted(a, L, st, inline_tab, inline_bytes)
                                  : svo::launch_trace(a, L, st, inline_tab, inline_bytes);
    if (e != hipSuccess) return fail(SVO_EDEVICE, "trace launch failed: %s", hipGetErrorString(e));
    return SVO_OK;
}

void fill_common(const svo_config& c, svo::TraceArgs& a) {
    a.refill = (c.refill_lanes == 0 || c.refill_lanes > 64) ? 64u : c.refill_lanes;
    a.claim = 64u * ((c.claim_tiles == 0) ? 2u : c.claim_tiles);
    a.step_limit = c.step_limit;
}

// Signature of a ray set, to tell whether a launch traces the rays of the
// previous one on its queue (FNV-1a over scene, ray pointer, count and
// camera record).
uint64_t ray_signature(svo_scene scene, const float* rays, uint64_t n, const svo::CameraArgs* cam) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](const void* p, size_t len) {
        const unsigned char* b = static_cast<const unsigned char*>(p);
        for (size_t i = 0; i < len; ++i) h = (h ^ b[i]) * 1099511628211ull;
    };
    const uintptr_t rp = (uintptr_t)rays;
    mix(&scene, sizeof scene);
    mix(&rp, sizeof rp);
    mix(&n, sizeof n);
    if (cam) mix(cam, sizeof *cam);
    return h | 1u;   // never the zero of a cleared state
}

// Validate a camera and fill the device record (svo_camera.h).
int camera_args(const svo_camera* cam, svo::CameraArgs& c) {
    if (!cam) return fail(SVO_EINVAL, "camera is NULL");
    if (cam->width == 0 || cam->height == 0 || cam->samples == 0) return fail(SVO_EINVAL, "empty image");
    if (cam->width > kMaxImageSide || cam->height > kMaxImageSide)
        return fail(SVO_ERANGE, "image sides must be at most %u", kMaxImageSide);
    if ((uint64_t)cam->width * cam->height * cam->samples > 0xFF000000ull) return fail(SVO_ERANGE, "too many rays");
    if (!(cam->tan_half_fov > 0.f) || !std::isfinite(cam->tan_half_fov)) return fail(SVO_EINVAL, "bad field of view");
    c = svo::CameraArgs{};
    for (int a = 0; a < 3; ++a) {
        c.eye[a] = cam->eye[a];
        c.fwd[a] = cam->forward[a];
        c.right[a] = cam->right[a];
        c.up[a] = cam->up[a];
    }
    c.tan_half_fov = cam->tan_half_fov;
    c.aspect = (float)cam->width / (float)cam->height;
    c.width = cam->width;
    c.height = cam->height;
    c.samples = cam->samples;
    c.seed = cam->seed;
    c.jitter = cam->jitter ? 1u : 0u;
    c.tiled = cam->tiled ? 1u : 0u;
    c.full_tiles = (c.tiled && c.samples == 1 && c.width % 8 == 0 && c.height % 8 == 0) ? 1u : 0u;
    c.tiles_x = (c.width + 7) / 8;
    c.inv_tiles_x = 1.0 / (double)c.tiles_x;
    return SVO_OK;
}

// Validated jobs of one launch, with their frame and candidate placement.
struct PackedJob {
    Scene* S;
    const svo_job* j;
    uint32_t frame_base, cand_base, bvh_base;
    std::vector<unsigned char> table;   // job-specific transforms (else the scene's current table)
    TableInfo T;
    bool has_cam = false;               // rays made from `cam` in the kernel
    svo::CameraArgs cam{};
};

struct Packing {
    std::vector<PackedJob> jobs;        // non-empty jobs, in order
    uint64_t total = 0;
    uint32_t frames = 0, cands = 0, max_cand = 0, stack_levels = 1, nest_levels = 0, bvh = 0, bvh_depth = 0;
    const uint64_t* cache_src = nullptr;  // the pool with the most rays
};

// Validate jobs (their scenes restricted to `allowed` when given), build the
// frame tables of jobs that bring their own transforms, and place every
// job's frame records and candidates.
int pack_jobs(svo_ctx* ctx, const svo_job* jobs, uint32_t n_jobs, const std::set<svo_scene>* allowed, Packing& P) {
    std::map<const uint64_t*, uint64_t> rays_per_pool;
    for (uint32_t i = 0; i < n_jobs; ++i) {
        const svo_job& J = jobs[i];
        Scene* S = find_scene(ctx, J.scene);
        if (!S) return fail(SVO_EINVAL, "job %u: unknown scene %u", i, J.scene);
        if (allowed && !allowed->count(J.scene)) return fail(SVO_EINVAL, "job %u: scene %u is not one of the plan's", i, J.scene);
        if (J.n == 0) continue;
        if (!J.out_id || !J.out_t) return fail(SVO_EINVAL, "job %u: out_id and out_t are required", i);
        svo::CameraArgs cam{};
        if (J.camera) {
            if (J.rays) return fail(SVO_EINVAL, "job %u: a camera job takes no ray buffer", i);
            const int rc = camera_args(J.camera, cam);
            if (rc) return rc;
            if (J.n != (uint64_t)cam.width * cam.height * cam.samples)
                return fail(SVO_EINVAL, "job %u: n must be width * height * samples of its camera", i);
        } else {
            if (!J.rays) return fail(SVO_EINVAL, "job %u: rays are required", i);
            if (((uintptr_t)J.rays) & 15u) return fail(SVO_EINVAL, "job %u: rays must be 16-byte aligned", i);
        }
        if (P.jobs.size() >= svo::kMaxJobs) return fail(SVO_ERANGE, "at most %u non-empty jobs per launch", svo::kMaxJobs);
        PackedJob Q{S, &J, P.frames, P.cands, P.bvh, {}, TableInfo(), J.camera != nullptr, cam};
        if (J.fwd_3x4) {
            std::vector<Aff> fwd(S->n_slots);
            for (uint32_t s = 0; s < S->n_slots; ++s) {
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 4; ++c) {
                        const float v = J.fwd_3x4[12 * s + 4 * r + c];
                        if (!std::isfinite(v)) return fail(SVO_EINVAL, "job %u: transform of slot %u is not finite", i, s);
                        fwd[s].m[r][c] = v;
                    }
            }
            Q.table.resize(S->table_bytes);
            const int rc = build_frames(*S, fwd, Q.table.data(), Q.T);
            if (rc) return rc;
        } else {
            Q.T.n_cand = S->n_cand;
            Q.T.stack_levels = S->stack_levels;
            Q.T.nest_levels = S->nest_levels;
            Q.T.n_bvh = S->n_bvh;
            Q.T.bvh_depth = S->bvh_depth;
            Q.T.n_inline = S->n_inline;
        }
        P.frames += S->n_frames;
        P.cands += Q.T.n_cand + Q.T.n_inline;
        P.bvh += Q.T.n_bvh;
        P.bvh_depth = std::max(P.bvh_depth, Q.T.bvh_depth);
        P.total += J.n;
        if (P.total > 0xFF000000ull) return fail(SVO_ERANGE, "at most 0xff000000 rays per launch");
        P.max_cand = std::max(P.max_cand, Q.T.n_cand);
        P.stack_levels = std::max(P.stack_levels, Q.T.stack_levels);
        P.nest_levels = std::max(P.nest_levels, Q.T.nest_levels);
        rays_per_pool[S->d_nodes] += J.n;
        P.jobs.push_back(std::move(Q));
    }
    uint64_t best = 0;
    for (auto& kv : rays_per_pool)
        if (kv.second > best) {
            best = kv.second;
            P.cache_src = kv.first;
        }
    return SVO_OK;
}

// Write job records, frame records, candidates (absolute frame indices),
// spheres, exact maps and hierarchy nodes (skipped when br is null: launches
// that take every candidate through the sorted path) of a packing into host
// memory; the jobs of the cached pool get `cache_nodes` LDS nodes.
// Camera jobs get their camera at cams[i] (host), which the launch reads at
// dev_cams + i.
void write_tables(const Packing& P, svo::JobRec* jr, svo::FrameRec* fr, uint32_t* cr, float* sr, double* xr,
                  svo::BvhNode* br, uint32_t cache_nodes, svo::CameraArgs* cams, const svo::CameraArgs* dev_cams) {
    uint64_t begin = 0;
    for (size_t i = 0; i < P.jobs.size(); ++i) {
        const PackedJob& Q = P.jobs[i];
        const Scene& S = *Q.S;
        const unsigned char* tab = Q.table.empty() ? S.h_stage[S.cur] : Q.table.data();
        std::memcpy(fr + Q.frame_base, tab, (size_t)S.n_frames * sizeof(svo::FrameRec));
        std::memcpy(sr + 4 * (size_t)Q.frame_base, tab + sphere_offset(S.n_frames, S.n_slots), (size_t)S.n_frames * 16);
        std::memcpy(xr + (size_t)svo::kExactMapDoubles * Q.frame_base, tab + xmap_offset(S.n_frames, S.n_slots),
                    (size_t)S.n_frames * kXmapBytes);
        const uint32_t* sc = reinterpret_cast<const uint32_t*>(tab + cand_offset(S.n_frames));
        for (uint32_t c = 0; c < Q.T.n_cand + Q.T.n_inline; ++c) cr[Q.cand_base + c] = Q.frame_base + sc[c];
        if (br)
            std::memcpy(br + Q.bvh_base, tab + bvh_offset(S.n_frames, S.n_slots), (size_t)Q.T.n_bvh * sizeof(svo::BvhNode));
        const svo_job& J = *Q.j;
        jr[i] = svo::JobRec{S.d_nodes, reinterpret_cast<const float4*>(J.rays), J.out_id, J.out_inst, J.out_t,
                            J.out_normal, begin, Q.frame_base, Q.cand_base, Q.T.n_cand,
                            S.d_nodes == P.cache_src ? cache_nodes : 0u, Q.bvh_base, Q.T.n_inline,
                            Q.has_cam ? dev_cams + i : nullptr, 0};
        if (Q.has_cam) cams[i] = Q.cam;
        begin += J.n;
    }
}

// Traversal-stack entries a scene can need under any transforms: the walk
// of an in-place frame stacks on top of its enclosing walks, so bound every
// frame by its root's depth below the world root plus its height.
uint32_t stack_bound(const Scene& S) {
    const Analysis& A = S.an;
    uint32_t bound = A.world_height + 1;
    std::vector<uint32_t> absdepth(S.n_slots, 0);
    for (uint32_t s : A.order) {
        const int32_t p = A.slot_parent[s];
        absdepth[s] = (p < 0 ? 0u : absdepth[p]) + A.slot_level[s];
        bound = std::max(bound, absdepth[s] + A.slot_height[s] + 1);
    }
    return bound;
}


}  // namespace

extern "C" {

}  // extern "C"

namespace {

int trace_rays(svo_ctx* ctx, svo_scene scene, const float* rays, uint64_t n, uint32_t* out_id, uint32_t* out_inst,
               float* out_t, float* out_normal, void* stream, bool reuse, unsigned long long* retraced,
               uint32_t* counts = nullptr, uint32_t* trail = nullptr, uint32_t trail_cap = 0,
               const svo::CameraArgs* cam = nullptr) {
    if (!ctx) return fail(SVO_EINVAL, "ctx is NULL");
    Scene* S = find_scene(ctx, scene);
    if (!S) return fail(SVO_EINVAL, "unknown scene %u", scene);
    if (n == 0) return SVO_OK;
    if ((!rays && !cam) || !out_id || !out_t) return fail(SVO_EINVAL, "rays, out_id and out_t are required");
    if (((uintptr_t)rays) & 15u) return fail(SVO_EINVAL, "rays must be 16-byte aligned");
    if (n > 0xFF000000ull) return fail(SVO_ERANGE, "at most 0xff000000 rays per call");
    hipStream_t st = (hipStream_t)stream;
    uint32_t qslot;
    int rc = queue_slot(ctx, st, qslot);
    if (rc) return rc;
    HIP_TRY(hipSetDevice(ctx->device));
    svo::TraceArgs a{};
    const svo_config& cfg = S->tuned ? S->cfg : ctx->cfg;
    const uint32_t cache = (uint32_t)std::min<uint64_t>(cfg.lds_cache_nodes, S->n_nodes) & ~1u;
    a.jobs = nullptr;
    a.job0 = svo::JobRec{S->d_nodes, reinterpret_cast<const float4*>(rays), out_id, out_inst, out_t, out_normal,
                         0, 0, 0, S->n_cand, cache, 0, S->n_inline};
    a.frames = reinterpret_cast<const svo::FrameRec*>(S->d_table[S->cur]);
    a.cand = reinterpret_cast<const uint32_t*>(S->d_table[S->cur] + cand_offset(S->n_frames));
    a.spheres = reinterpret_cast<const float4*>(S->d_table[S->cur] + sphere_offset(S->n_frames, S->n_slots));
    a.xmaps = reinterpret_cast<const double*>(S->d_table[S->cur] + xmap_offset(S->n_frames, S->n_slots));
    a.bvh = reinterpret_cast<const svo::BvhNode*>(S->d_table[S->cur] + bvh_offset(S->n_frames, S->n_slots));
    // the hierarchy is walked only past the configured number of
    // candidates; a table in the arguments has none, so it takes the sorted
    // path whatever the count (such scenes have at most 10 slots)
    const bool sorted = S->n_cand <= sort_limit(cfg) || !S->dev_current;
    a.n_bvh_total = sorted ? 0u : S->n_bvh;
    a.bvh_depth = S->bvh_depth;
    // transforms changed since the device table was written: the table
    // travels in the arguments
    const unsigned char* tab = nullptr;
    size_t tab_bytes = 0;
    if (!S->dev_current) {
        tab = S->h_stage[S->cur];
        tab_bytes = bvh_offset(S->n_frames, S->n_slots);
        a.inline_off_cand = (uint32_t)cand_offset(S->n_frames);
        a.inline_off_sph = (uint32_t)sphere_offset(S->n_frames, S->n_slots);
        a.inline_off_x = (uint32_t)xmap_offset(S->n_frames, S->n_slots);
    }
    a.n_jobs = 1;
    a.n_frames = S->n_frames;
    a.n_cand_total = S->n_cand + S->n_inline;
    a.max_cand = S->n_cand;
    a.n_rays = n;
    a.cache_src = S->d_nodes;
    a.queue = ctx->d_queue + svo::kQueueWords * qslot;
    a.lds_nodes = cache;
    a.stack_levels = S->stack_levels;
    a.nest_levels = S->nest_levels;
    a.sort_cand = sorted ? 1u : 0u;
    fill_common(cfg, a);
    a.reuse = reuse ? 1u : 0u;
    a.retraced = retraced;
    a.counts = counts;
    a.trail = trail;
    a.trail_cap = trail ? trail_cap : 0u;
    if (cam) {
        a.has_cam0 = 1;
        a.cam0 = *cam;
    }
    // slow tiles first (whole-tile claims): the queue's state carries them
    // from the previous launch of the same rays.  Hit-buffer launches keep
    // the plain order: the few rays they trace again change from frame to
    // frame, so the previous launch's slow tiles say little about theirs.
    const uint64_t tiles = (n + 63) / 64;
    if (cfg.tile_order == 0 && a.refill == 64 && !reuse && tiles <= svo::kHotMaxTiles) {
        const uint64_t sig = ray_signature(scene, rays, n, cam);
        auto& R = ctx->hot_rec[qslot];
        uint32_t k = R.sig[0] == sig ? 0u : (R.sig[1] == sig ? 1u : 2u);
        if (k == 2u) {
            k = R.recent ^ 1u;
            R.sig[k] = sig;
            R.uses[k] = 0;
            R.fresh[k] = true;
        }
        R.recent = k;
        if (R.uses[k] < 2u) ++R.uses[k];
        if (R.uses[k] >= 2u) {
            // whether a list is dealt out depends on the waves of the launch
            // that wrote it: a new shape starts a new count, so that its first
            // launch gathers statistics and decides for that shape
            const uint32_t shape = (cfg.waves_per_block << 16) | cfg.blocks_per_cu;
            if (R.shape[k] != shape) {
                R.shape[k] = shape;
                R.seq[k] = 0;
            }
            a.hot = ctx->d_hot + (size_t)svo::kHotWords * (2u * qslot + k);
            if (R.fresh[k]) {
                // the listing threshold was the previous ray set's: start from
                // the initial one (a fill kernel rather than a memset, so that
                // the trace can be captured in a graph)
                R.fresh[k] = false;
                if (svo::launch_zero_words(a.hot + 1, 1, st) != hipSuccess)
                    return fail(SVO_EDEVICE, "slow-tile state reset failed");
            }
            a.hot_target = (uint32_t)std::min<uint64_t>(svo::kHotCap, std::max<uint64_t>(16, tiles / 8));
            a.hot_seq = R.seq[k]++;
            a.hot_sig = sig;
        }
    }
    rc = launch(ctx, cfg, a, st, tab, tab_bytes);
    if (rc == SVO_OK && !tab) {
        // this launch reads the current device table: a later copy into it
        // must wait for the launch
        auto& rd = S->readers[S->cur];
        auto it = std::find_if(rd.begin(), rd.end(), [&](const std::pair<hipStream_t, hipEvent_t>& x) { return x.first == st; });
        if (it == rd.end()) {
            hipEvent_t e = nullptr;
            if (!S->spare_events.empty()) {
                e = S->spare_events.back();
                S->spare_events.pop_back();
            } else {
                HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            }
            rd.push_back({st, e});
            it = rd.end() - 1;
        }
        HIP_TRY(hipEventRecord(it->second, st));
    }
    return rc;
}

}  // namespace

extern "C" {

int svo_trace_rays(svo_ctx* ctx, svo_scene scene, const float* rays, uint64_t n, uint32_t* out_id,
                   uint32_t* out_inst, float* out_t, float* out_normal, void* stream) {
    return trace_rays(ctx, scene, rays, n, out_id, out_inst, out_t, out_normal, stream, false, nullptr);
}

int svo_trace_camera(svo_ctx* ctx, svo_scene scene, const svo_camera* cam, uint32_t* out_id, uint32_t* out_inst,
                     float* out_t, float* out_normal, void* stream) {
    svo::CameraArgs c;
    const int rc = camera_args(cam, c);
    if (rc) return rc;
    return trace_rays(ctx, scene, nullptr, (uint64_t)c.width * c.height * c.samples, out_id, out_inst, out_t, out_normal,
                      stream, false, nullptr, nullptr, nullptr, 0, &c);
}

int svo_trace_rays_counted(svo_ctx* ctx, svo_scene scene, const float* rays, uint64_t n, uint32_t* out_id,
                           uint32_t* out_inst, float* out_t, float* out_normal, uint32_t* counts, uint32_t* trail,
                           uint32_t trail_cap, void* stream) {
    if (n && !counts) return fail(SVO_EINVAL, "counts is required");
    if (n > 0x7FFFFFFFull) return fail(SVO_ERANGE, "at most 2^31 - 1 rays per counted trace");
    if (trail && (uint64_t)trail_cap * n > (1ull << 40)) return fail(SVO_ERANGE, "trail_cap * n is too large");
    return trace_rays(ctx, scene, rays, n, out_id, out_inst, out_t, out_normal, stream, false, nullptr, counts,
                      trail, trail_cap);
}

int svo_trace_rays_reuse(svo_ctx* ctx, svo_scene scene, const float* rays, uint64_t n, uint32_t* out_id,
                         uint32_t* out_inst, float* out_t, float* out_normal, uint64_t* retraced, void* stream) {
    if (n && !out_inst) return fail(SVO_EINVAL, "out_inst is required to reuse previous hits");
    return trace_rays(ctx, scene, rays, n, out_id, out_inst, out_t, out_normal, stream, true,
                      reinterpret_cast<unsigned long long*>(retraced));
}

}  // extern "C"

namespace {

// svo_trace_batch, and with use_static its allocation-free variant: the
// work queue and the launch's tables in the device's scratch instead of a
// per-stream queue and the ring of batch tables (allocated on first use).
int trace_batch(svo_ctx* ctx, const svo_job* jobs, uint32_t n_jobs, void* stream, bool use_static) {
    if (!ctx) return fail(SVO_EINVAL, "ctx is NULL");
    if (n_jobs && !jobs) return fail(SVO_EINVAL, "jobs is NULL");
    try {
        Packing P;
        int rc = pack_jobs(ctx, jobs, n_jobs, nullptr, P);
        if (rc) return rc;
        if (P.jobs.empty()) return SVO_OK;
        if (P.frames > 2047) return fail(SVO_ERANGE, "a batch may hold at most 2047 frame records (has %u)", P.frames);
        hipStream_t st = (hipStream_t)stream;
        uint32_t* queue = nullptr;
        if (use_static) {
            queue = reinterpret_cast<uint32_t*>(ctx->d_static);
        } else {
            uint32_t qslot;
            rc = queue_slot(ctx, st, qslot);
            if (rc) return rc;
            queue = ctx->d_queue + svo::kQueueWords * qslot;
        }
        HIP_TRY(hipSetDevice(ctx->device));

        // configuration and node cache: the pool with the most rays in this batch
        const svo_config* pcfg = &ctx->cfg;
        uint64_t cache_pool_nodes = 0;
        for (auto& J : P.jobs)
            if (J.S->d_nodes == P.cache_src) {
                cache_pool_nodes = J.S->n_nodes;
                if (J.S->tuned) pcfg = &J.S->cfg;
            }
        svo_config cfg = *pcfg;

        // pack [jobs][frames][candidates][spheres][exact maps][hierarchy nodes][cameras]
        const size_t jb = P.jobs.size() * sizeof(svo::JobRec);
        const size_t fb = (size_t)P.frames * sizeof(svo::FrameRec);
        const size_t sb = (jb + fb + (size_t)P.cands * sizeof(uint32_t) + 15) & ~(size_t)15;
        const size_t xb = sb + (size_t)P.frames * 16;
        const size_t bb = xb + (size_t)P.frames * kXmapBytes;
        const size_t cb = bb + (size_t)P.bvh * sizeof(svo::BvhNode);
        const size_t bytes = cb + P.jobs.size() * sizeof(svo::CameraArgs);
        svo::TraceArgs a{};
        const bool sorted = P.max_cand <= sort_limit(cfg);
        a.n_bvh_total = sorted ? 0u : P.bvh;
        a.bvh_depth = P.bvh_depth;
        a.n_jobs = (uint32_t)P.jobs.size();
        a.n_frames = P.frames;
        a.n_cand_total = P.cands;
        a.max_cand = P.max_cand;
        a.n_rays = P.total;
        a.cache_src = P.cache_src;
        a.queue = queue;
        a.lds_nodes = (uint32_t)std::min<uint64_t>(cfg.lds_cache_nodes, cache_pool_nodes) & ~1u;
        a.sort_cand = sorted ? 1u : 0u;
        a.stack_levels = P.stack_levels;
        a.nest_levels = P.nest_levels;
        fill_common(cfg, a);
        if (P.jobs.size() == 1 && P.jobs[0].has_cam) {
            // one job: its camera travels in the arguments
            a.has_cam0 = 1;
            a.cam0 = P.jobs[0].cam;
        }
        // size LDS now: a smaller node cache changes the jobs' lds_nodes
        const size_t lds = fit_lds(ctx, a, cfg.waves_per_block);
        if (lds > ctx->max_lds) return fail(SVO_ERANGE, "batch needs %zu bytes of LDS per work-group", lds);

        if (P.jobs.size() == 1 && P.jobs[0].S->inline_tab && a.sort_cand) {
            // one job of a small scene: its table (the scene's layout, frame
            // base 0) travels in the kernel arguments, with no table copy
            const PackedJob& Q = P.jobs[0];
            const Scene& S = *Q.S;
            const svo_job& J = *Q.j;
            a.jobs = nullptr;
            a.job0 = svo::JobRec{S.d_nodes, reinterpret_cast<const float4*>(J.rays), J.out_id, J.out_inst, J.out_t,
                                 J.out_normal, 0, 0, 0, Q.T.n_cand, a.lds_nodes, 0, Q.T.n_inline};
            a.inline_off_cand = (uint32_t)cand_offset(S.n_frames);
            a.inline_off_sph = (uint32_t)sphere_offset(S.n_frames, S.n_slots);
            a.inline_off_x = (uint32_t)xmap_offset(S.n_frames, S.n_slots);
            const unsigned char* tab = Q.table.empty() ? S.h_stage[S.cur] : Q.table.data();
            if (use_static) HIP_TRY(svo::launch_zero_words(queue, svo::kQueueWords, st));
            return launch(ctx, cfg, a, st, tab, bvh_offset(S.n_frames, S.n_slots));
        }

        if (use_static) {
            if (bytes > svo::kStaticTableBytes)
                return fail(SVO_ERANGE, "the batch's tables take %zu bytes; the allocation-free launch holds %zu", bytes,
                            svo::kStaticTableBytes);
            // the staging may still feed the previous call's copy
            HIP_TRY(hipEventSynchronize(ctx->static_ev));
            unsigned char* H = ctx->h_static;
            unsigned char* D = ctx->d_static + svo::kStaticQueueBytes;
            write_tables(P, reinterpret_cast<svo::JobRec*>(H), reinterpret_cast<svo::FrameRec*>(H + jb),
                         reinterpret_cast<uint32_t*>(H + jb + fb), reinterpret_cast<float*>(H + sb),
                         reinterpret_cast<double*>(H + xb), reinterpret_cast<svo::BvhNode*>(H + bb), a.lds_nodes,
                         reinterpret_cast<svo::CameraArgs*>(H + cb), reinterpret_cast<const svo::CameraArgs*>(D + cb));
            a.jobs = reinterpret_cast<const svo::JobRec*>(D);
            if (P.jobs.size() == 1) {
                a.job0 = *reinterpret_cast<const svo::JobRec*>(H);
                a.jobs = nullptr;
            }
            a.frames = reinterpret_cast<const svo::FrameRec*>(D + jb);
            a.cand = reinterpret_cast<const uint32_t*>(D + jb + fb);
            a.spheres = reinterpret_cast<const float4*>(D + sb);
            a.xmaps = reinterpret_cast<const double*>(D + xb);
            a.bvh = reinterpret_cast<const svo::BvhNode*>(D + bb);
            HIP_TRY(svo::launch_zero_words(queue, svo::kQueueWords, st));
            HIP_TRY(hipMemcpyAsync(D, H, bytes, hipMemcpyHostToDevice, st));
            rc = launch(ctx, cfg, a, st);
            // recorded even when the launch failed: the copy still reads H
            const hipError_t e = hipEventRecord(ctx->static_ev, st);
            if (rc) return rc;
            if (e != hipSuccess) return fail(SVO_EDEVICE, "event record failed: %s", hipGetErrorString(e));
            return SVO_OK;
        }

        auto& B = ctx->batch[ctx->next_batch];
        ctx->next_batch = (ctx->next_batch + 1) % 4;
        if (B.ev) HIP_TRY(hipEventSynchronize(B.ev));
        if (B.cap < bytes) {
            if (B.dev) (void)hipFree(B.dev);
            if (B.host) (void)hipHostFree(B.host);
            B.dev = nullptr;
            B.host = nullptr;
            B.cap = 0;
            const size_t cap = std::max<size_t>(bytes, 64 << 10);
            if (hipMalloc((void**)&B.dev, cap) != hipSuccess || hipHostMalloc((void**)&B.host, cap, hipHostMallocDefault) != hipSuccess)
                return fail(SVO_ENOMEM, "batch table allocation failed");
            B.cap = cap;
        }
        if (!B.ev) HIP_TRY(hipEventCreateWithFlags(&B.ev, hipEventDisableTiming));
        write_tables(P, reinterpret_cast<svo::JobRec*>(B.host), reinterpret_cast<svo::FrameRec*>(B.host + jb),
                     reinterpret_cast<uint32_t*>(B.host + jb + fb), reinterpret_cast<float*>(B.host + sb),
                     reinterpret_cast<double*>(B.host + xb), reinterpret_cast<svo::BvhNode*>(B.host + bb), a.lds_nodes,
                     reinterpret_cast<svo::CameraArgs*>(B.host + cb), reinterpret_cast<const svo::CameraArgs*>(B.dev + cb));
        a.jobs = reinterpret_cast<const svo::JobRec*>(B.dev);
        if (P.jobs.size() == 1) {
            // one job: passed in the arguments, which selects the single-job
            // kernel (the job's pool and table offsets launch-wide)
            a.job0 = *reinterpret_cast<const svo::JobRec*>(B.host);
            a.jobs = nullptr;
        }
        a.frames = reinterpret_cast<const svo::FrameRec*>(B.dev + jb);
        a.cand = reinterpret_cast<const uint32_t*>(B.dev + jb + fb);
        a.spheres = reinterpret_cast<const float4*>(B.dev + sb);
        a.xmaps = reinterpret_cast<const double*>(B.dev + xb);
        a.bvh = reinterpret_cast<const svo::BvhNode*>(B.dev + bb);
        HIP_TRY(hipMemcpyAsync(B.dev, B.host, bytes, hipMemcpyHostToDevice, st));
        rc = launch(ctx, cfg, a, st);
        // recorded even when the launch failed: the copy still reads B.host
        const hipError_t e = hipEventRecord(B.ev, st);
        if (rc) return rc;
        if (e != hipSuccess) return fail(SVO_EDEVICE, "batch event record failed: %s", hipGetErrorString(e));
        return SVO_OK;
    } catch (const std::bad_alloc&) {
        return fail(SVO_ENOMEM, "out of host memory");
    }
}

}  // namespace

extern "C" {

int svo_trace_batch(svo_ctx* ctx, const svo_job* jobs, uint32_t n_jobs, void* stream) {
    return trace_batch(ctx, jobs, n_jobs, stream, false);
}

int svo_trace_batch_static(svo_ctx* ctx, const svo_job* jobs, uint32_t n_jobs, void* stream) {
    return trace_batch(ctx, jobs, n_jobs, stream, true);
}

// ------------------------------------------------------------------ plans

int svo_plan_create(svo_ctx* ctx, const svo_scene* scenes, uint32_t n_scenes, const svo_plan_limits* limits,
                    svo_plan** out) {
    if (out) *out = nullptr;
    if (!ctx || !scenes || !limits || !out) return fail(SVO_EINVAL, "ctx, scenes, limits and out are required");
    if (n_scenes == 0) return fail(SVO_EINVAL, "a plan needs at least one scene");
    if (limits->reserved[0] || limits->reserved[1]) return fail(SVO_EINVAL, "reserved limit fields must be zero");
    if (limits->max_jobs < 1 || limits->max_jobs > svo::kMaxJobs)
        return fail(SVO_ERANGE, "max_jobs must be 1..%u", svo::kMaxJobs);
    if (limits->max_frames < 1 || limits->max_frames > 2047) return fail(SVO_ERANGE, "max_frames must be 1..2047");
    try {
        std::unique_ptr<svo_plan> pl(new svo_plan());
        uint32_t max_slots = 0;
        uint64_t max_pool = 0;
        for (uint32_t i = 0; i < n_scenes; ++i) {
            Scene* S = find_scene(ctx, scenes[i]);
            if (!S) return fail(SVO_EINVAL, "unknown scene %u", scenes[i]);
            pl->scenes.insert(scenes[i]);
            pl->stack_cap = std::max(pl->stack_cap, stack_bound(*S));
            pl->nest_cap = std::max(pl->nest_cap, std::min<uint32_t>(svo::kMaxInlineNest, S->an.max_nesting));
            max_slots = std::max(max_slots, S->n_slots);
            max_pool = std::max(max_pool, S->n_nodes);
        }
        if (pl->stack_cap > 127) return fail(SVO_ERANGE, "scenes need %u stack levels (limit 127)", pl->stack_cap);
        Scene* S0 = find_scene(ctx, scenes[0]);
        pl->cfg = S0->tuned ? S0->cfg : ctx->cfg;
        pl->max_jobs = limits->max_jobs;
        pl->max_frames = limits->max_frames;
        pl->max_cand = std::min(max_slots, limits->max_frames);
        // table layout: [header][jobs][frames][candidates][spheres][exact maps][hierarchy][cameras], capacities
        pl->off_jobs = sizeof(svo::LaunchHdr);
        pl->off_frames = pl->off_jobs + (size_t)pl->max_jobs * sizeof(svo::JobRec);
        pl->off_cand = pl->off_frames + (size_t)pl->max_frames * sizeof(svo::FrameRec);
        pl->off_sph = (pl->off_cand + (size_t)pl->max_frames * sizeof(uint32_t) + 15) & ~(size_t)15;
        pl->off_x = pl->off_sph + (size_t)pl->max_frames * 16;
        pl->off_bvh = pl->off_x + (size_t)pl->max_frames * kXmapBytes;
        pl->max_bvh = pl->max_cand > sort_limit(pl->cfg) ? 2 * pl->max_frames : 0u;
        pl->bvh_depth_cap = bvh_levels(pl->max_cand);
        pl->off_cams = pl->off_bvh + (size_t)pl->max_bvh * sizeof(svo::BvhNode);
        pl->bytes = pl->off_cams + (size_t)pl->max_jobs * sizeof(svo::CameraArgs);

        svo::TraceArgs& a = pl->args;
        a = svo::TraceArgs{};
        a.n_jobs = pl->max_jobs;
        a.n_frames = pl->max_frames;
        a.n_cand_total = pl->max_frames;
        a.n_bvh_total = pl->max_bvh;
        a.bvh_depth = pl->bvh_depth_cap;
        a.max_cand = pl->max_cand;
        a.sort_cand = pl->max_cand <= sort_limit(pl->cfg) ? 1u : 0u;
        a.stack_levels = pl->stack_cap;
        a.nest_levels = pl->nest_cap;
        a.lds_nodes = (uint32_t)std::min<uint64_t>(pl->cfg.lds_cache_nodes, max_pool) & ~1u;
        fill_common(pl->cfg, a);
        const size_t lds = fit_lds(ctx, a, pl->cfg.waves_per_block);
        if (lds > ctx->max_lds) return fail(SVO_ERANGE, "plan needs %zu bytes of LDS per work-group", lds);
        pl->launch_cfg.waves_per_block = pl->cfg.waves_per_block;
        pl->launch_cfg.blocks = (uint32_t)std::max<uint64_t>(1, (uint64_t)ctx->n_cu * resident_blocks(ctx, pl->cfg, lds));
        pl->launch_cfg.lds_bytes = lds;

        HIP_TRY(hipSetDevice(ctx->device));
        auto release = [&]() { destroy_plan(*pl); };
        if (hipMalloc((void**)&pl->dev, pl->bytes) != hipSuccess ||
            hipHostMalloc((void**)&pl->host, pl->bytes, hipHostMallocDefault) != hipSuccess ||
            hipMalloc((void**)&pl->d_queue, svo::kQueueWords * sizeof(uint32_t)) != hipSuccess) {
            release();
            return fail(SVO_ENOMEM, "plan allocation failed");
        }
        std::memset(pl->host, 0, pl->bytes);
        if (hipMemset(pl->d_queue, 0, svo::kQueueWords * sizeof(uint32_t)) != hipSuccess ||
            hipMemcpy(pl->dev, pl->host, pl->bytes, hipMemcpyHostToDevice) != hipSuccess ||
            hipEventCreateWithFlags(&pl->ev, hipEventDisableTiming) != hipSuccess ||
            hipDeviceSynchronize() != hipSuccess) {
            release();
            return fail(SVO_EDEVICE, "plan set-up failed");
        }
        a.hdr = reinterpret_cast<const svo::LaunchHdr*>(pl->dev);
        a.jobs = reinterpret_cast<const svo::JobRec*>(pl->dev + pl->off_jobs);
        a.frames = reinterpret_cast<const svo::FrameRec*>(pl->dev + pl->off_frames);
        a.cand = reinterpret_cast<const uint32_t*>(pl->dev + pl->off_cand);
        a.spheres = reinterpret_cast<const float4*>(pl->dev + pl->off_sph);
        a.xmaps = reinterpret_cast<const double*>(pl->dev + pl->off_x);
        a.bvh = reinterpret_cast<const svo::BvhNode*>(pl->dev + pl->off_bvh);
        a.queue = pl->d_queue;
        *out = pl.get();
        ctx->plans.insert(pl.release());
        return SVO_OK;
    } catch (const std::bad_alloc&) {
        return fail(SVO_ENOMEM, "out of host memory");
    }
}

int svo_plan_set_jobs(svo_ctx* ctx, svo_plan* plan, const svo_job* jobs, uint32_t n_jobs) {
    if (!ctx || !plan) return fail(SVO_EINVAL, "ctx and plan are required");
    if (!ctx->plans.count(plan)) return fail(SVO_EINVAL, "plan does not belong to this context");
    if (n_jobs && !jobs) return fail(SVO_EINVAL, "jobs is NULL");
    try {
        Packing P;
        int rc = pack_jobs(ctx, jobs, n_jobs, &plan->scenes, P);
        if (rc) return rc;
        if (P.jobs.size() > plan->max_jobs) return fail(SVO_ERANGE, "%zu jobs, the plan holds %u", P.jobs.size(), plan->max_jobs);
        if (P.frames > plan->max_frames)
            return fail(SVO_ERANGE, "%u frame records, the plan holds %u", P.frames, plan->max_frames);
        if (P.stack_levels > plan->stack_cap || P.nest_levels > plan->nest_cap || P.max_cand > plan->max_cand ||
            (plan->max_bvh && P.bvh > plan->max_bvh) || P.bvh_depth > plan->bvh_depth_cap)
            return fail(SVO_ERANGE, "jobs exceed the plan's stack, nesting or candidate capacity");
        if (plan->ev_pending) {
            HIP_TRY(hipSetDevice(ctx->device));
            HIP_TRY(hipEventSynchronize(plan->ev));
            plan->ev_pending = false;
        }
        unsigned char* H = plan->host;
        svo::LaunchHdr hdr{};
        hdr.n_rays = P.total;
        hdr.tile_stride = tile_stride((P.total + 63) / 64);
        hdr.n_jobs = (uint32_t)P.jobs.size();
        hdr.n_frames = P.frames;
        hdr.n_cand_total = P.cands;
        hdr.n_bvh_total = plan->max_bvh ? P.bvh : 0u;
        uint32_t fill = 0;
        for (auto& J : P.jobs)
            if (J.S->d_nodes == P.cache_src) fill = (uint32_t)std::min<uint64_t>(plan->args.lds_nodes, J.S->n_nodes) & ~1u;
        hdr.cache_src = fill ? P.cache_src : nullptr;
        hdr.lds_nodes = fill;
        std::memcpy(H, &hdr, sizeof hdr);
        write_tables(P, reinterpret_cast<svo::JobRec*>(H + plan->off_jobs), reinterpret_cast<svo::FrameRec*>(H + plan->off_frames),
                     reinterpret_cast<uint32_t*>(H + plan->off_cand), reinterpret_cast<float*>(H + plan->off_sph),
                     reinterpret_cast<double*>(H + plan->off_x), plan->max_bvh ? reinterpret_cast<svo::BvhNode*>(H + plan->off_bvh) : nullptr, fill,
                     reinterpret_cast<svo::CameraArgs*>(H + plan->off_cams),
                     reinterpret_cast<const svo::CameraArgs*>(plan->dev + plan->off_cams));
        return SVO_OK;
    } catch (const std::bad_alloc&) {
        return fail(SVO_ENOMEM, "out of host memory");
    }
}

int svo_plan_launch(svo_ctx* ctx, svo_plan* plan, void* stream) {
    if (!ctx || !plan) return fail(SVO_EINVAL, "ctx and plan are required");
    if (!ctx->plans.count(plan)) return fail(SVO_EINVAL, "plan does not belong to this context");
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(ctx->device));
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(st, &cs));
    HIP_TRY(hipMemcpyAsync(plan->dev, plan->host, plan->bytes, hipMemcpyHostToDevice, st));
    if (cs == hipStreamCaptureStatusNone) {
        HIP_TRY(hipEventRecord(plan->ev, st));
        plan->ev_pending = true;
    }
    const hipError_t e = svo::launch_trace(plan->args, plan->launch_cfg, st);
    if (e != hipSuccess) return fail(SVO_EDEVICE, "plan launch failed: %s", hipGetErrorString(e));
    return SVO_OK;
}

int svo_plan_destroy(svo_ctx* ctx, svo_plan* plan) {
    if (!plan) return SVO_OK;
    if (!ctx) return fail(SVO_EINVAL, "ctx is NULL");
    if (!ctx->plans.count(plan)) return fail(SVO_EINVAL, "plan does not belong to this context");
    (void)hipSetDevice(ctx->device);
    if (plan->ev_pending) (void)hipEventSynchronize(plan->ev);
    (void)hipDeviceSynchronize();
    ctx->plans.erase(plan);
    destroy_plan(*plan);
    delete plan;
    return SVO_OK;
}

int svo_tune(svo_ctx* ctx, svo_scene scene, const float* sample_rays, uint64_t n, void* stream, svo_config* best) {
    if (!ctx) return fail(SVO_EINVAL, "ctx is NULL");
    Scene* S = find_scene(ctx, scene);
    if (!S) return fail(SVO_EINVAL, "unknown scene %u", scene);
    if (n == 0 || !sample_rays) return fail(SVO_EINVAL, "svo_tune needs sample rays");
    if (n > 0xFF000000ull) return fail(SVO_ERANGE, "at most 0xff000000 sample rays");
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(ctx->device));
    uint32_t* d_id = nullptr;
    float* d_t = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
        if (d_id) (void)hipFree(d_id);
        if (d_t) (void)hipFree(d_t);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    if (hipMalloc((void**)&d_id, n * sizeof(uint32_t)) != hipSuccess || hipMalloc((void**)&d_t, n * sizeof(float)) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        cleanup();
        return fail(SVO_ENOMEM, "tuner scratch allocation failed");
    }
    const svo_config base = ctx->cfg;
    const bool was_tuned = S->tuned;
    const svo_config was_cfg = S->cfg;
    svo_config win = base;
    float win_ms = 1e30f;
    // Stages: the launch shape (waves per work-group, work-groups per CU,
    // LDS node cache) at whole-tile refill and 2-tile claims; refill, claim
    // size and candidate ordering for the winning shape; a longer timing of
    // the best three.
    static const uint32_t kWaves[] = {4, 8, 12, 16};
    static const uint32_t kBlocks[] = {1, 2, 3, 4, 5, 6, 8};
    static const uint32_t kCache[] = {1024, 2048, 4096};
    static const uint32_t kRefill[] = {0, 48};
    static const uint32_t kClaim[] = {1, 2, 4};
    auto time_cand = [&](const svo_config& cand, float& ms, int launches = 6) -> int {
        S->tuned = true;
        S->cfg = cand;
        int r = svo_trace_rays(ctx, scene, sample_rays, n, d_id, nullptr, d_t, nullptr, stream);
        if (r) return r;  // SVO_ERANGE: does not fit in LDS
        if (hipEventRecord(e0, st) != hipSuccess) return fail(SVO_EDEVICE, "tuner event record failed");
        for (int k = 0; k < launches && r == SVO_OK; ++k)
            r = svo_trace_rays(ctx, scene, sample_rays, n, d_id, nullptr, d_t, nullptr, stream);
        if (r) return r;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            return fail(SVO_EDEVICE, "tuner timing failed");
        return SVO_OK;
    };
    int rc = SVO_OK;
    std::vector<std::pair<float, svo_config>> shapes;   // stage 1 timings
    auto try_all = [&](const std::vector<svo_config>& cands, bool keep) {
        for (const svo_config& cand : cands) {
            float ms = 0.f;
            rc = time_cand(cand, ms);
            if (rc == SVO_ERANGE) continue;
            if (rc) return;
            if (keep) shapes.push_back({ms, cand});
            if (ms < win_ms) {
                win_ms = ms;
                win = cand;
            }
        }
    };
    std::vector<svo_config> cands;
    for (uint32_t w : kWaves)
        for (uint32_t b : kBlocks) {
            if (w * b > 32) continue;  // resident waves per CU
            for (uint32_t c : kCache) {
                svo_config cand = base;
                cand.waves_per_block = w;
                cand.blocks_per_cu = b;
                cand.lds_cache_nodes = c;
                cand.refill_lanes = 0;
                cand.claim_tiles = 2;
                cands.push_back(cand);
            }
        }
    try_all(cands, true);
    const svo_config shape1 = win;   // the first stage's winner
    if (rc == SVO_OK || rc == SVO_ERANGE) {
        const svo_config shape = win;
        cands.clear();
        for (uint32_t r : kRefill)
            for (uint32_t y : kClaim) {
                if (r == shape.refill_lanes && y == shape.claim_tiles) continue;
                svo_config cand = shape;
                cand.refill_lanes = r;
                cand.claim_tiles = y;
                cands.push_back(cand);
            }
        // the other candidate ordering: the box hierarchy for a scene that
        // takes the sorted table, the sorted table (up to 64) for one that
        // takes the hierarchy
        if (S->n_cand > 1 && S->n_cand <= 64) {
            svo_config other = shape;
            other.sorted_candidates = S->n_cand <= sort_limit(shape) ? S->n_cand - 1 : 64u;
            cands.push_back(other);
        }
        try_all(cands, false);
    }
    // Short timings are noisy: the winner, the first stage's winner (when the
    // second stage changed it) and the next two shapes of the first stage are
    // timed again with five times the launches, and the fastest is kept.
    if ((rc == SVO_OK || rc == SVO_ERANGE) && win_ms < 1e30f) {
        std::sort(shapes.begin(), shapes.end(), [](const std::pair<float, svo_config>& x,
                                                   const std::pair<float, svo_config>& y) { return x.first < y.first; });
        std::vector<svo_config> finalists{win};
        if (std::memcmp(&shape1, &win, sizeof win) != 0) finalists.push_back(shape1);
        const size_t n_final = finalists.size() + 2;
        for (size_t i = 0; i < shapes.size() && finalists.size() < n_final; ++i)
            if (std::memcmp(&shapes[i].second, &win, sizeof win) != 0 &&
                std::memcmp(&shapes[i].second, &shape1, sizeof shape1) != 0)
                finalists.push_back(shapes[i].second);
        float best_ms = 1e30f;
        for (const svo_config& cand : finalists) {
            float ms = 0.f;
            rc = time_cand(cand, ms, 30);
            if (rc == SVO_ERANGE) continue;
            if (rc) break;
            if (ms < best_ms) {
                best_ms = ms;
                win = cand;
            }
        }
    }
    cleanup();
    if (rc && rc != SVO_ERANGE) {
        S->tuned = was_tuned;
        S->cfg = was_cfg;
        return rc;
    }
    if (win_ms >= 1e30f) {
        S->tuned = was_tuned;
        S->cfg = was_cfg;
        return fail(SVO_ERANGE, "no candidate configuration fits this scene");
    }
    S->tuned = true;
    S->cfg = win;
    if (best) *best = win;
    return SVO_OK;
}

int svo_shade(svo_ctx* ctx, svo_scene scene, const uint32_t* prim_id, const uint32_t* ao_id, uint32_t width,
              uint32_t height, uint32_t samples, uint32_t tiled, uint32_t k, uint32_t ambient_permille,
              uint32_t background_rgba, uint32_t* out_rgba, void* stream) {
    if (!ctx) return fail(SVO_EINVAL, "ctx is NULL");
    Scene* S = find_scene(ctx, scene);
    if (!S) return fail(SVO_EINVAL, "unknown scene %u", scene);
    if ((uint64_t)width * height == 0) return SVO_OK;
    if (!prim_id || !out_rgba || (k && !ao_id)) return fail(SVO_EINVAL, "prim_id, out_rgba (and ao_id when k > 0) are required");
    if (samples == 0 || samples > 1024 || k > 64) return fail(SVO_ERANGE, "samples must be 1..1024 and k at most 64");
    if (ambient_permille > 1000) return fail(SVO_EINVAL, "ambient_permille must be at most 1000");
    // the kernels index pixels in 32 bits: every 8-row band must stay below 2^32
    if (width > kMaxImageSide || height > kMaxImageSide || (uint64_t)width * height * samples > 0xFF000000ull)
        return fail(SVO_ERANGE, "image too large (sides at most %u, at most 0xff000000 samples)", kMaxImageSide);
    if ((uint64_t)width * height * samples * (k ? k : 1) >= (1ull << 40)) return fail(SVO_ERANGE, "image too large");
    HIP_TRY(hipSetDevice(ctx->device));
    svo::ShadeArgs a{};
    a.nodes = S->d_nodes;
    a.n_nodes = S->n_nodes;
    a.prim_id = prim_id;
    a.ao_id = ao_id;
    a.width = width;
    a.height = height;
    a.samples = samples;
    a.tiled = tiled ? 1u : 0u;
    a.k = k;
    a.ambient = ambient_permille;
    a.background = background_rgba;
    a.out = out_rgba;
    const hipError_t e = svo::launch_shade(a, (hipStream_t)stream);
    if (e != hipSuccess) return fail(SVO_EDEVICE, "shade launch failed: %s", hipGetErrorString(e));
    return SVO_OK;
}

int svo_generate_primary_rays(svo_ctx* ctx, const svo_camera* cam, float* out_rays, void* stream) {
    if (!ctx || !cam || !out_rays) return fail(SVO_EINVAL, "ctx, cam and out_rays are required");
    if (((uintptr_t)out_rays) & 15u) return fail(SVO_EINVAL, "out_rays must be 16-byte aligned");
    svo::CameraArgs c;
    const int rc = camera_args(cam, c);
    if (rc) return rc;
    HIP_TRY(hipSetDevice(ctx->device));
    const hipError_t e = svo::launch_primary_rays(c, out_rays, (hipStream_t)stream);
    if (e != hipSuccess) return fail(SVO_EDEVICE, "ray generation launch failed: %s", hipGetErrorString(e));
    return SVO_OK;
}

int svo_generate_ao_rays(svo_ctx* ctx, const float* rays, const float* t, const float* normal, uint64_t n, uint32_t k,
                         uint32_t seed, float radius, float offset, float* out_rays, void* stream) {
    if (!ctx) return fail(SVO_EINVAL, "ctx is NULL");
    if (n == 0 || k == 0) return SVO_OK;
    if (!rays || !t || !normal || !out_rays) return fail(SVO_EINVAL, "rays, t, normal and out_rays are required");
    if ((((uintptr_t)rays) | ((uintptr_t)out_rays)) & 15u) return fail(SVO_EINVAL, "ray buffers must be 16-byte aligned");
    if (n * (uint64_t)k > 0xFF000000ull) return fail(SVO_ERANGE, "too many rays");
    if (!(radius >= 0.f) || !std::isfinite(offset)) return fail(SVO_EINVAL, "bad radius or offset");
    svo::AoArgs a{};
    a.rays = reinterpret_cast<const float4*>(rays);
    a.t = t;
    a.normal = normal;
    a.n = n;
    a.k = k;
    a.seed = seed;
    a.radius = radius;
    a.offset = offset;
    a.out = reinterpret_cast<float4*>(out_rays);
    HIP_TRY(hipSetDevice(ctx->device));
    const hipError_t e = svo::launch_ao_rays(a, (hipStream_t)stream);
    if (e != hipSuccess) return fail(SVO_EDEVICE, "AO ray launch failed: %s", hipGetErrorString(e));
    return SVO_OK;
}

}  // extern "C"
