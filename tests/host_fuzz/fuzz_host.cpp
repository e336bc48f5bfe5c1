// Host-side fuzz of the library's pool validation and frame-table builder,
// built for the CPU under AddressSanitizer and UndefinedBehaviorSanitizer
// (test infrastructure: tests/test_host_sanitize.py compiles and runs it).
//
// The library's host source is included whole, so its internal functions
// (pool analysis, FP64 compose + invert, frame records, candidate
// hierarchy) are called directly; the few device entry points it references
// are stubbed, and nothing here touches a GPU.  Seeded, so a failure
// reproduces with the same arguments.
//
//   fuzz_host <seed> <iterations>
#include "../../paper_1911_06001_amd/csrc/svo_host.cpp"

#include <cinttypes>
#include <cstdlib>
#include <random>

namespace svo {
hipError_t launch_primary_rays(const CameraArgs&, float*, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_ao_rays(const AoArgs&, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_shade(const ShadeArgs&, hipStream_t) { return hipErrorNoDevice; }
hipError_t static_scratch(int, unsigned char**) { return hipErrorNoDevice; }
hipError_t launch_zero_words(uint32_t*, uint32_t, hipStream_t) { return hipErrorNoDevice; }
size_t trace_lds_bytes(const TraceArgs&, uint32_t) { return 0; }
hipError_t prepare_trace(size_t) { return hipErrorNoDevice; }
hipError_t launch_trace(const TraceArgs&, const LaunchCfg&, hipStream_t, const unsigned char*, size_t) {
    return hipErrorNoDevice;
}
hipError_t launch_trace_counted(const TraceArgs&, const LaunchCfg&, hipStream_t, const unsigned char*, size_t) {
    return hipErrorNoDevice;
}
}  // namespace svo

namespace {

using Rng = std::mt19937_64;

uint64_t node_word(uint32_t mask, uint32_t c24, uint32_t w1) {
    return (uint64_t)(mask & 0xFFu) | ((uint64_t)(c24 & 0xFFFFFFu) << 8) | ((uint64_t)w1 << 32);
}

// A random well-formed pool: depth <= D, child groups laid out breadth
// first after their parent, some far pointers, some transformed interior
// nodes (their slot's child index in slot_child).
struct Pool {
    std::vector<uint64_t> nodes;
    std::vector<uint32_t> slot_child;
    uint32_t root = 0, depth = 0;
};

Pool random_pool(Rng& g, uint32_t D, uint32_t max_slots) {
    Pool P;
    P.depth = D;
    struct Item {
        uint32_t idx, level;
    };
    std::vector<Item> q;
    P.nodes.push_back(0);
    q.push_back({0, 0});
    std::uniform_int_distribution<int> coin(0, 99);
    for (size_t h = 0; h < q.size(); ++h) {
        const Item it = q[h];
        if (it.level == D || (it.level > 0 && coin(g) < 30)) {
            P.nodes[it.idx] = node_word(0, 0, (uint32_t)g());   // leaf with a colour
            continue;
        }
        uint32_t mask = (uint32_t)(g() & 0xFFu);
        if (!mask) mask = 1u << (g() % 8);
        const uint32_t start = (uint32_t)P.nodes.size();
        const int cnt = __builtin_popcount(mask);
        for (int c = 0; c < cnt; ++c) {
            P.nodes.push_back(0);
            q.push_back({start + (uint32_t)c, it.level + 1});
        }
        const bool can_xf = it.level > 0 && P.slot_child.size() < max_slots;
        if (can_xf && coin(g) < 12) {
            const uint32_t s = (uint32_t)P.slot_child.size();
            P.slot_child.push_back(start);
            P.nodes[it.idx] = node_word(mask, 1, 0x80000000u | s);
        } else if (coin(g) < 10) {
            P.nodes[it.idx] = node_word(mask, 0xFFFFFFu, start);
        } else {
            P.nodes[it.idx] = node_word(mask, start - it.idx, 0);
        }
    }
    return P;
}

void mutate(Rng& g, Pool& P, uint32_t& root, uint32_t& max_depth, uint32_t& n_slots) {
    const int kinds = 1 + (int)(g() % 3);
    for (int k = 0; k < kinds; ++k) {
        const size_t i = g() % P.nodes.size();
        switch (g() % 9) {
            case 0: P.nodes[i] ^= 1ull << (g() % 64); break;
            case 1: P.nodes[i] = (P.nodes[i] & ~0xFFFFFF00ull) | ((uint64_t)(g() & 0xFFFFFFu) << 8); break;
            case 2: P.nodes[i] = (P.nodes[i] & 0xFFFFFFFFull) | ((uint64_t)(uint32_t)g() << 32); break;
            case 3: P.nodes[i] = g(); break;
            case 4: if (!P.slot_child.empty()) P.slot_child[g() % P.slot_child.size()] = (uint32_t)g() % (P.nodes.size() + 4); break;
            case 5: root = (uint32_t)(g() % (P.nodes.size() + 2)); break;
            case 6: max_depth = (uint32_t)(g() % 24); break;
            case 7: n_slots = (uint32_t)(g() % (P.slot_child.size() + 2)); break;
            default: P.nodes[i] = node_word((uint32_t)g(), (uint32_t)(P.nodes.size() - i + g() % 3), 0); break;
        }
    }
}

// A random forward map: rotation, anisotropic scale (sometimes extreme or
// zero, i.e. singular), translation.
Aff random_map(Rng& g, double cell) {
    std::uniform_real_distribution<double> u(-1.0, 1.0);
    Aff A = aff_identity();
    double q[4] = {u(g), u(g), u(g), u(g)};
    double n = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    if (n < 1e-9) n = 1, q[0] = 1;
    for (double& x : q) x /= n;
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    const double R[3][3] = {{1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)},
                            {2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)},
                            {2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)}};
    double s[3];
    for (double& v : s) {
        const int pick = (int)(g() % 100);
        v = pick == 0 ? 0.0 : (pick == 1 ? 1e-30 : (pick == 2 ? 1e30 : std::exp2(2.0 * u(g))));
    }
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) A.m[r][c] = (double)(float)(R[r][c] * s[c]);
        A.m[r][3] = (double)(float)(cell * 4.0 * u(g));
    }
    return A;
}

}  // namespace

int main(int argc, char** argv) {
    const uint64_t seed = argc > 1 ? strtoull(argv[1], nullptr, 10) : 1;
    const int iters = argc > 2 ? atoi(argv[2]) : 2000;
    Rng g(seed);
    uint64_t accepted = 0, rejected = 0, tables = 0, singular = 0, cands = 0;
    for (int it = 0; it < iters; ++it) {
        const uint32_t D = 1 + (uint32_t)(g() % 6);
        Pool P = random_pool(g, D, 40);
        uint32_t root = P.root, max_depth = D, n_slots = (uint32_t)P.slot_child.size();
        const bool bad = (g() % 3) == 0;
        if (bad) mutate(g, P, root, max_depth, n_slots);
        std::vector<uint32_t> sc(P.slot_child);
        sc.resize(std::max<size_t>(sc.size(), n_slots), 0);
        svo_pool_info info;
        const int rc = svo_validate(P.nodes.data(), P.nodes.size(), root, max_depth, n_slots ? sc.data() : nullptr,
                                    n_slots, &info);
        if (rc != SVO_OK) {
            if (rc != SVO_EINVAL && rc != SVO_ERANGE) {
                fprintf(stderr, "seed %" PRIu64 " iter %d: unexpected code %d\n", seed, it, rc);
                return 2;
            }
            ++rejected;
            continue;
        }
        ++accepted;
        // the scene as svo_upload sets it up on the host, then frame tables
        // for random maps
        Scene S;
        if (analyse(P.nodes.data(), P.nodes.size(), root, max_depth, sc.data(), n_slots, S.an) != SVO_OK) {
            fprintf(stderr, "seed %" PRIu64 " iter %d: analyse disagrees with svo_validate\n", seed, it);
            return 3;
        }
        S.n_nodes = P.nodes.size();
        S.root = root;
        std::uniform_real_distribution<double> u(-1.0, 1.0);
        for (int a = 0; a < 3; ++a) S.root_min[a] = (float)(1000.0 * u(g));
        S.root_size = (float)std::exp2(1 + (int)(g() % 12));
        S.n_slots = n_slots;
        S.slot_child.assign(sc.begin(), sc.begin() + n_slots);
        S.slot_cell.resize(4 * (size_t)n_slots);
        for (uint32_t s = 0; s < n_slots; ++s) {
            const float size = S.root_size / (float)std::exp2(1 + (int)(g() % 4));
            for (int a = 0; a < 3; ++a) S.slot_cell[4 * s + a] = S.root_min[a] + size * (float)(g() % 4);
            S.slot_cell[4 * s + 3] = size;
        }
        if (root != SVO_NONE && !nd_leaf(P.nodes[root])) {
            uint64_t st;
            int cnt;
            children_of(P.nodes.data(), root, S.slot_child.data(), st, cnt);
            S.world_child = (uint32_t)st;
            S.world_mask = nd_mask(P.nodes[root]);
        }
        S.n_frames = 1 + n_slots;
        S.table_bytes = table_size(S.n_frames, n_slots);
        std::vector<unsigned char> tab(S.table_bytes);
        for (int rep = 0; rep < 3; ++rep) {
            std::vector<Aff> fwd(n_slots);
            for (uint32_t s = 0; s < n_slots; ++s) fwd[s] = random_map(g, S.slot_cell[4 * s + 3]);
            TableInfo T;
            const int rb = build_frames(S, fwd, tab.data(), T);
            if (rb == SVO_EINVAL) {
                ++singular;
                continue;
            }
            if (rb != SVO_OK && rb != SVO_ERANGE) {
                fprintf(stderr, "seed %" PRIu64 " iter %d: build_frames code %d\n", seed, it, rb);
                return 4;
            }
            if (rb == SVO_OK) {
                ++tables;
                cands += T.n_cand;
                if (T.n_cand + T.n_inline > n_slots || T.n_bvh > bvh_capacity(n_slots)) {
                    fprintf(stderr, "seed %" PRIu64 " iter %d: table counts out of range\n", seed, it);
                    return 5;
                }
            }
        }
    }
    printf("accepted %" PRIu64 " rejected %" PRIu64 " tables %" PRIu64 " singular %" PRIu64 " candidates %" PRIu64 "\n",
           accepted, rejected, tables, singular, cands);
    return 0;
}
