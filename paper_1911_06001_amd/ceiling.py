"""ctypes binding of libsvo_ceiling.so (include/svo_ceiling.h) and the
ceiling measurements built on it: random 8-byte gathers over a pool-sized
buffer at the trace kernel's grid, and streaming reads from HBM and from
cache-resident buffers.  Argument marshalling and event timing only; the
loads run in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsvo_ceiling.so")
EXPORTS = ("svo_ceiling_last_error", "svo_ceiling_gather", "svo_ceiling_stream", "svo_ceiling_replay")

_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libsvo_ceiling.so is not built (run paper_1911_06001_amd/build.py)")
    L = ctypes.CDLL(LIB_PATH)
    P, U32, U64, I = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    L.svo_ceiling_last_error.restype = ctypes.c_char_p
    L.svo_ceiling_last_error.argtypes = []
    L.svo_ceiling_gather.restype = I
    L.svo_ceiling_gather.argtypes = [P, U64, U32, U32, U32, U32, U32, U64, P, P]
    L.svo_ceiling_stream.restype = I
    L.svo_ceiling_stream.argtypes = [P, U64, U32, U32, U32, P, P]
    L.svo_ceiling_replay.restype = I
    L.svo_ceiling_replay.argtypes = [P, U64, U32, P, P, U64, U32, P, P, U32, U32, P, P]
    _lib = L
    return L


def _check(rc: int):
    if rc != 0:
        raise RuntimeError("svo_ceiling error %d: %s" % (rc, lib().svo_ceiling_last_error().decode()))


def gather(buf, blocks: int, threads: int, chains: int, loads: int, dependent: bool, seed: int, sink, stream=None):
    """Enqueue one gather launch (buf: int64 device tensor; sink: int64
    device tensor of at least blocks * threads elements)."""
    import torch
    assert buf.dtype == torch.int64 and sink.dtype == torch.int64 and buf.is_cuda and sink.is_cuda
    assert sink.numel() >= blocks * threads
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().svo_ceiling_gather(buf.data_ptr(), buf.numel(), blocks, threads, chains, loads, int(bool(dependent)),
                                    seed & (2**64 - 1), sink.data_ptr(), st.cuda_stream))


def stream_read(buf, blocks: int, threads: int, reps: int, sink, stream=None):
    """Enqueue one streaming-read launch over the whole of `buf`."""
    import torch
    assert buf.is_cuda and sink.is_cuda and sink.dtype == torch.int64 and sink.numel() >= blocks * threads
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().svo_ceiling_stream(buf.data_ptr(), buf.numel() * buf.element_size(), blocks, threads, reps,
                                    sink.data_ptr(), st.cuda_stream))


def replay(nodes, n_lds: int, trail, counts, rays, out, blocks: int, threads: int, sink, stream=None):
    """Enqueue one replay of a counted trace's node loads (nodes: int64
    device pool; trail [cap, n] and counts [3, n] int32 device tensors from
    svo_trace_rays_counted; rays [n, 8] float32; out: int32 device tensor of
    at least 6 n elements)."""
    import torch
    n = rays.shape[0]
    cap = trail.shape[0] if trail is not None else 0
    assert counts.shape == (3, n) and sink.numel() >= blocks * threads and out.numel() >= 6 * n
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().svo_ceiling_replay(nodes.data_ptr(), nodes.numel(), n_lds,
                                    trail.data_ptr() if trail is not None else None, counts.data_ptr(), n, cap,
                                    rays.data_ptr(), out.data_ptr(), blocks, threads, sink.data_ptr(), st.cuda_stream))


def _time(fn, reps: int) -> float:
    """Mean seconds per call of fn() over `reps` calls, after one warm-up."""
    import torch
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / reps


def measure(pool_bytes: int, blocks: int, threads: int, hbm_bytes: int = 4 << 30, reps: int = 5) -> dict:
    """Ceilings in GB/s for a pool of `pool_bytes` traced with a grid of
    `blocks` x `threads` (the trace kernel's launch shape)."""
    import torch
    dev = torch.device("cuda", torch.cuda.current_device())
    g = torch.Generator(device=dev)
    g.manual_seed(11)
    n_words = max(1, pool_bytes // 8)
    pool = torch.randint(-2**62, 2**62, (n_words,), dtype=torch.int64, device=dev, generator=g)
    sblocks, sthreads = 4096, 512
    sink = torch.empty(max(blocks * threads, sblocks * sthreads), dtype=torch.int64, device=dev)
    out = {"grid": [blocks, threads], "pool_bytes": int(n_words * 8)}

    # independent gathers: the best over loads in flight per thread (too
    # many outstanding misses thrash the memory system)
    loads_ind = 64
    per_chain = {}
    for chains in (1, 2, 4, 8):
        t = _time(lambda: gather(pool, blocks, threads, chains, loads_ind, False, 1, sink), reps)
        per_chain[chains] = round(blocks * threads * chains * loads_ind * 8 / t / 1e9, 1)
    out["gather_independent_by_chains_GBps"] = per_chain
    out["gather_independent_GBps"] = max(per_chain.values())
    loads_dep = 256
    t = _time(lambda: gather(pool, blocks, threads, 1, loads_dep, True, 2, sink), reps)
    out["gather_dependent_GBps"] = round(blocks * threads * loads_dep * 8 / t / 1e9, 1)
    out["gather_dependent_latency_ns"] = round(t / loads_dep * 1e9, 1)

    cache_reps = max(1, (1 << 30) // max(pool.numel() * 8, 1))
    t = _time(lambda: stream_read(pool, sblocks, sthreads, cache_reps, sink), reps)
    out["stream_pool_GBps"] = round(pool.numel() * 8 * cache_reps / t / 1e9, 1)
    del pool
    big = torch.empty(hbm_bytes // 8, dtype=torch.int64, device=dev).fill_(3)
    t = _time(lambda: stream_read(big, sblocks, sthreads, 1, sink), reps)
    out["stream_hbm_GBps"] = round(big.numel() * 8 / t / 1e9, 1)
    del big
    torch.cuda.empty_cache()
    return out
