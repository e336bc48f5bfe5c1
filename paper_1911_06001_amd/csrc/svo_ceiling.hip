// Memory ceilings for the traversal's access pattern: random 8-byte gathers
// over a buffer of a node pool's size, and streaming reads.  They bound what
// any traversal of that pool can reach on this GPU at a given occupancy and
// serve as the denominators of its roofline, beside the HBM spec peak.
//
// Every kernel is a grid-stride loop with an exit every thread reaches; the
// loaded words are folded into one 64-bit value per thread and written to
// `sink` so that no load can be removed.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>

#include "svo_ceiling.h"

namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    // SplitMix64 finaliser (Steele, Lea, Flood 2014)
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

typedef unsigned int v4u __attribute__((ext_vector_type(4)));

template <typename T>
__device__ __forceinline__ T gload(const T* p, uint64_t i) {
    return ((const __attribute__((address_space(1))) T*)p)[i];
}

// Each thread follows `chains` random index streams, `loads` loads each;
// an index is the high half of (32-bit hash) x n_words.  The stream state
// costs a handful of integer operations per load, so the loads, not the
// index arithmetic, bound the kernel.
// dependent = 0: the next state is a xorshift32 step of the previous one,
//   so all loads of a thread can be in flight together (throughput).
// dependent = 1: the next state is hashed from the word just loaded and
//   the stream's own salt, so a stream has one load in flight at a time
//   (latency; the octree walk has this shape: the next node address comes
//   out of the last node).  The salt keeps streams apart: without it two
//   streams that load the same word would follow one path from then on, and
//   the streams would collapse onto a few cache-resident words.
__device__ __forceinline__ uint32_t xorshift32(uint32_t x) {
    x ^= x << 13;
    x ^= x >> 17;
    x ^= x << 5;
    return x;
}

template <int CHAINS>
__global__ __launch_bounds__(1024) void gather_kernel(const uint64_t* __restrict__ buf, uint32_t n_words,
                                                      uint32_t loads, uint32_t dependent, uint64_t seed,
                                                      uint64_t* __restrict__ sink) {
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t st[CHAINS], salt[CHAINS];
    uint64_t acc = 0;
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) {
        const uint64_t h = mix64(seed ^ (tid * CHAINS + c));
        st[c] = (uint32_t)h | 1u;
        salt[c] = (uint32_t)(h >> 32);
    }
    for (uint32_t k = 0; k < loads; ++k) {
        uint64_t w[CHAINS];
#pragma unroll
        for (int c = 0; c < CHAINS; ++c) w[c] = gload(buf, __umulhi(st[c], n_words));
#pragma unroll
        for (int c = 0; c < CHAINS; ++c) {
            acc ^= w[c];
            st[c] = dependent ? (((uint32_t)w[c] ^ (uint32_t)(w[c] >> 32) ^ salt[c]) * 0x9E3779B1u + k) | 1u
                              : xorshift32(st[c]);
        }
    }
    ((__attribute__((address_space(1))) uint64_t*)sink)[tid] = acc;
}

// Every thread reads 16-byte words in a grid-stride sweep over the buffer,
// `reps` times.
__global__ __launch_bounds__(1024) void stream_kernel(const v4u* __restrict__ buf, uint64_t n16, uint32_t reps,
                                                      uint64_t* __restrict__ sink) {
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint32_t a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    for (uint32_t r = 0; r < reps; ++r) {
        uint64_t i = tid;
        for (; i + 3 * stride < n16; i += 4 * stride) {
            const v4u v0 = gload(buf, i), v1 = gload(buf, i + stride), v2 = gload(buf, i + 2 * stride),
                        v3 = gload(buf, i + 3 * stride);
            a0 ^= v0.x ^ v1.x ^ v2.x ^ v3.x;
            a1 ^= v0.y ^ v1.y ^ v2.y ^ v3.y;
            a2 ^= v0.z ^ v1.z ^ v2.z ^ v3.z;
            a3 ^= v0.w ^ v1.w ^ v2.w ^ v3.w;
        }
        for (; i < n16; i += stride) {
            const v4u v = gload(buf, i);
            a0 ^= v.x;
            a1 ^= v.y;
            a2 ^= v.z;
            a3 ^= v.w;
        }
    }
    ((__attribute__((address_space(1))) uint64_t*)sink)[tid] = ((uint64_t)(a0 ^ a1) << 32) | (a2 ^ a3);
}

// Replay of a trace's recorded memory traffic with none of its arithmetic:
// each lane takes one ray (64 consecutive rays per wave, waves striding
// over the 64-ray tiles), reads the ray (32 bytes), then, in order, the
// node words its trace read -- trail[k n + g] for k below the ray's pool
// reads (counts[g] - counts[n + g]) and cap, from the LDS copy of the pool
// prefix when bit 31 is set (every work-group fills it first, as the trace
// does) -- each load's address waiting on the word before it (the walk
// decides its next step from the node it just read; dep_mask = 0 keeps the
// addresses unchanged), and writes 24 bytes of result.
__global__ __launch_bounds__(1024) void replay_kernel(const uint64_t* __restrict__ nodes, uint32_t n_nodes, uint32_t n_lds,
                                                      const uint32_t* __restrict__ trail,
                                                      const uint32_t* __restrict__ counts, uint64_t n, uint32_t cap,
                                                      const v4u* __restrict__ rays, uint32_t* __restrict__ out,
                                                      uint32_t dep_mask, uint64_t* __restrict__ sink) {
    extern __shared__ uint64_t lds[];
    for (uint32_t i = threadIdx.x; i < n_lds; i += blockDim.x) lds[i] = gload(nodes, i);
    __syncthreads();
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t waves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    const uint64_t tiles = (n + 63) >> 6;
    const uint32_t lane = threadIdx.x & 63u;
    uint64_t acc = 0;
    for (uint64_t t = tid >> 6; t < tiles; t += waves) {
        const uint64_t g = t * 64 + lane;
        if (g >= n) continue;
        const v4u r0 = gload(rays, 2 * g), r1 = gload(rays, 2 * g + 1);
        uint32_t carry = r0.x ^ r0.y ^ r0.z ^ r0.w ^ r1.x ^ r1.y ^ r1.z ^ r1.w;
        carry &= dep_mask;
        const uint32_t reads = gload(counts, g) - gload(counts, n + g);
        const uint32_t m = reads < cap ? reads : cap;
        for (uint32_t k = 0; k < m; ++k) {
            const uint32_t e = gload(trail, (uint64_t)k * n + g) ^ carry;
            const uint32_t idx = e & 0x7FFFFFFFu;
            const uint64_t w = (e >> 31) ? lds[idx < n_lds ? idx : 0] : gload(nodes, idx < n_nodes ? idx : 0);
            acc ^= w;
            carry = ((uint32_t)w ^ (uint32_t)(w >> 32)) & dep_mask;
        }
        __attribute__((address_space(1))) uint32_t* o = (__attribute__((address_space(1))) uint32_t*)out;
        o[g] = (uint32_t)acc;                 // id
        o[n + g] = (uint32_t)(acc >> 32);     // slot
        o[2 * n + g] = m;                     // t
        o[3 * n + 3 * g] = carry;             // normal
        o[3 * n + 3 * g + 1] = carry;
        o[3 * n + 3 * g + 2] = carry;
    }
    ((__attribute__((address_space(1))) uint64_t*)sink)[tid] = acc;
}

thread_local char g_err[256];

int fail(int code, const char* msg) {
    snprintf(g_err, sizeof g_err, "%s", msg);
    return code;
}

}  // namespace

extern "C" {

const char* svo_ceiling_last_error(void) { return g_err; }

int svo_ceiling_gather(const uint64_t* buf, uint64_t n_words, uint32_t blocks, uint32_t threads_per_block,
                       uint32_t chains, uint32_t loads, uint32_t dependent, uint64_t seed, uint64_t* sink,
                       void* stream) {
    if (!buf || !sink || n_words == 0) return fail(SVO_CEILING_EINVAL, "buf, sink and n_words are required");
    if (n_words > 0xFFFFFFFFull) return fail(SVO_CEILING_EINVAL, "n_words must be below 2^32");
    if (blocks == 0 || threads_per_block == 0 || threads_per_block > 1024 || (threads_per_block & 63u))
        return fail(SVO_CEILING_EINVAL, "threads_per_block must be a multiple of 64 in 64..1024");
    if (dependent > 1) return fail(SVO_CEILING_EINVAL, "dependent must be 0 or 1");
    hipStream_t st = (hipStream_t)stream;
    const dim3 g(blocks), b(threads_per_block);
    switch (chains) {
        case 1: hipLaunchKernelGGL(gather_kernel<1>, g, b, 0, st, buf, (uint32_t)n_words, loads, dependent, seed, sink); break;
        case 2: hipLaunchKernelGGL(gather_kernel<2>, g, b, 0, st, buf, (uint32_t)n_words, loads, dependent, seed, sink); break;
        case 4: hipLaunchKernelGGL(gather_kernel<4>, g, b, 0, st, buf, (uint32_t)n_words, loads, dependent, seed, sink); break;
        case 8: hipLaunchKernelGGL(gather_kernel<8>, g, b, 0, st, buf, (uint32_t)n_words, loads, dependent, seed, sink); break;
        default: return fail(SVO_CEILING_EINVAL, "chains must be 1, 2, 4 or 8");
    }
    return hipGetLastError() == hipSuccess ? 0 : fail(SVO_CEILING_EDEVICE, "gather launch failed");
}

int svo_ceiling_replay(const uint64_t* nodes, uint64_t n_nodes, uint32_t n_lds, const uint32_t* trail,
                       const uint32_t* counts, uint64_t n, uint32_t cap, const float* rays, uint32_t* out,
                       uint32_t blocks, uint32_t threads_per_block, uint64_t* sink, void* stream) {
    if (!nodes || !counts || !rays || !out || !sink || (cap && !trail) || n == 0 || n_nodes == 0)
        return fail(SVO_CEILING_EINVAL, "nodes, counts, rays, out, sink (and trail when cap > 0) and n are required");
    if (n_lds > n_nodes || n_lds > 16384) return fail(SVO_CEILING_EINVAL, "n_lds must be at most n_nodes and 16384");
    if (n_nodes > 0x7FFFFFFFull) return fail(SVO_CEILING_EINVAL, "n_nodes must be below 2^31");
    if (((uintptr_t)rays) & 15u) return fail(SVO_CEILING_EINVAL, "rays must be 16-byte aligned");
    if (blocks == 0 || threads_per_block == 0 || threads_per_block > 1024 || (threads_per_block & 63u))
        return fail(SVO_CEILING_EINVAL, "threads_per_block must be a multiple of 64 in 64..1024");
    hipLaunchKernelGGL(replay_kernel, dim3(blocks), dim3(threads_per_block), (size_t)n_lds * 8, (hipStream_t)stream,
                       nodes, (uint32_t)n_nodes, n_lds, trail, counts, n, cap, reinterpret_cast<const v4u*>(rays), out,
                       0u, sink);
    return hipGetLastError() == hipSuccess ? 0 : fail(SVO_CEILING_EDEVICE, "replay launch failed");
}

int svo_ceiling_stream(const void* buf, uint64_t bytes, uint32_t blocks, uint32_t threads_per_block, uint32_t reps,
                       uint64_t* sink, void* stream) {
    if (!buf || !sink || bytes < 16 || (bytes & 15u) || (((uintptr_t)buf) & 15u))
        return fail(SVO_CEILING_EINVAL, "buf must be 16-byte aligned and bytes a positive multiple of 16");
    if (blocks == 0 || threads_per_block == 0 || threads_per_block > 1024 || (threads_per_block & 63u))
        return fail(SVO_CEILING_EINVAL, "threads_per_block must be a multiple of 64 in 64..1024");
    hipLaunchKernelGGL(stream_kernel, dim3(blocks), dim3(threads_per_block), 0, (hipStream_t)stream,
                       reinterpret_cast<const v4u*>(buf), bytes / 16, reps, sink);
    return hipGetLastError() == hipSuccess ? 0 : fail(SVO_CEILING_EDEVICE, "stream launch failed");
}

}  // extern "C"
