/*
 * svo_ceiling.h -- memory-ceiling kernels for the roofline of the SVO trace
 * (separate library libsvo_ceiling.so; measurement only, no tracing).
 *
 * The octree walk of the trace reads 8-byte nodes whose addresses come out
 * of the previous node (the top-down traversal of the paper, Sec. 2.1 and
 * Sec. 5; its cost is dominated by these reads, Sec. 6).  These kernels
 * measure what that access pattern can reach on the device, so that the
 * trace's achieved algorithmic bandwidth can be stated as a fraction of an
 * attainable ceiling as well as of the HBM spec peak:
 *   - random 8-byte gathers over a buffer the size of a node pool, either
 *     independent (all loads of a thread in flight: throughput) or
 *     dependent (each address hashed from the word just loaded: latency),
 *     launched with the trace's own grid so the occupancy matches;
 *   - streaming 16-byte reads over a buffer (HBM-sized or cache-sized);
 *   - a replay of the trace's own recorded node loads, in its order, with
 *     its dependence and at its grid, without its arithmetic.
 * The caller times the launch (events on `stream`) and divides the bytes
 * read, 8 * blocks * threads_per_block * chains * loads for a gather and
 * bytes * reps for a stream, by the elapsed time.
 *
 * Conventions: return 0 or a negative code; svo_ceiling_last_error() gives
 * the calling thread's last message.  Pointers are device pointers owned by
 * the caller; work is ordered on `stream` (hipStream_t, NULL = null stream).
 */
#ifndef SVO_CEILING_H
#define SVO_CEILING_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { SVO_CEILING_EINVAL = -1, SVO_CEILING_EDEVICE = -3 };

const char* svo_ceiling_last_error(void);

/* Random gathers.  buf: device, 1 <= n_words < 2^32 uint64 words, any
 * content.  blocks x threads_per_block threads (threads_per_block a
 * multiple of 64, at most 1024); each thread follows `chains` (1, 2, 4 or 8)
 * index streams of `loads` loads.  A stream's 32-bit state starts from
 * SplitMix64 of (seed, thread * chains + stream), odd; the load index is
 * the high half of state * n_words; the next state is a xorshift32 step
 * (dependent = 0) or (lo ^ hi of the loaded word ^ the stream's salt, the
 * high half of its SplitMix64 value) * 0x9E3779B1 + step, odd (dependent =
 * 1).  sink: device, blocks * threads_per_block uint64,
 * written (one folded value per thread).  Errors: SVO_CEILING_EINVAL for a
 * NULL pointer, n_words = 0 or a bad shape; SVO_CEILING_EDEVICE when the
 * launch fails. */
int svo_ceiling_gather(const uint64_t* buf, uint64_t n_words, uint32_t blocks, uint32_t threads_per_block,
                       uint32_t chains, uint32_t loads, uint32_t dependent, uint64_t seed, uint64_t* sink,
                       void* stream);

/* Replay of a trace's memory traffic (the trace's own ceiling: the same
 * loads in the same per-ray order and dependence, at the same grid, with
 * none of its arithmetic).  nodes: device pool of n_nodes (< 2^31) words;
 * n_lds (<= n_nodes, <= 16384): pool prefix every work-group copies to LDS
 * first, as the trace does.  counts, trail, cap: as written by
 * svo_trace_rays_counted for the n rays (device; trail may be NULL when
 * cap = 0).  Lane g reads ray g (rays: device, n * 8 floats, 16-byte
 * aligned), then trail[k * n + g] for k < min(counts[g] - counts[n + g], cap)
 * in order, each address waiting on the word before it (entries with bit
 * 31 from LDS), then writes 24 bytes to out (device, 6 * n uint32).  Each
 * wave takes 64 consecutive rays; waves stride over the 64-ray tiles.  sink:
 * device, blocks * threads_per_block uint64.  Trail entries must be below
 * n_nodes (n_lds for LDS ones), as the trace writes them.  Errors as for
 * svo_ceiling_gather. */
int svo_ceiling_replay(const uint64_t* nodes, uint64_t n_nodes, uint32_t n_lds, const uint32_t* trail,
                       const uint32_t* counts, uint64_t n, uint32_t cap, const float* rays, uint32_t* out,
                       uint32_t blocks, uint32_t threads_per_block, uint64_t* sink, void* stream);

/* Streaming read.  buf: device, 16-byte aligned, `bytes` a positive
 * multiple of 16, read `reps` times by a grid-stride sweep of 16-byte
 * loads.  sink: device, blocks * threads_per_block uint64, written.  Errors
 * as for svo_ceiling_gather. */
int svo_ceiling_stream(const void* buf, uint64_t bytes, uint32_t blocks, uint32_t threads_per_block, uint32_t reps,
                       uint64_t* sink, void* stream);

#ifdef __cplusplus
}
#endif

#endif
