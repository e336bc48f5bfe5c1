"""Ceiling kernels (libsvo_ceiling.so): the gather kernel reads exactly the
words its index streams name (checked against a host replay of the
SplitMix64 index streams, dependent streams salted per stream), and the
stream kernel folds every word."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
M64 = (1 << 64) - 1


def _say(*a):
    print("[gpu-ceiling]", *a, flush=True)
    sys.stdout.flush()


def _mix64(z):
    z &= M64
    z = ((z ^ (z >> 30)) * 0xbf58476d1ce4e5b9) & M64
    z = ((z ^ (z >> 27)) * 0x94d049bb133111eb) & M64
    return z ^ (z >> 31)


def _xorshift32(x):
    x ^= (x << 13) & 0xFFFFFFFF
    x ^= x >> 17
    x ^= (x << 5) & 0xFFFFFFFF
    return x


def _expected_gather(words, blocks, threads, chains, loads, dependent, seed):
    n = len(words)
    out = []
    for tid in range(blocks * threads):
        h = [_mix64(seed ^ (tid * chains + c)) for c in range(chains)]
        st = [(x & 0xFFFFFFFF) | 1 for x in h]
        salt = [x >> 32 for x in h]
        acc = 0
        for k in range(loads):
            w = [words[(s * n) >> 32] for s in st]
            for c in range(chains):
                acc ^= w[c]
                if dependent:
                    st[c] = ((((w[c] & 0xFFFFFFFF) ^ (w[c] >> 32) ^ salt[c]) * 0x9E3779B1 + k) & 0xFFFFFFFF) | 1
                else:
                    st[c] = _xorshift32(st[c])
        out.append(acc)
    return out


@pytest.mark.parametrize("chains,dependent", [(1, 1), (2, 0), (8, 0), (4, 1)])
def test_gather_reads_the_named_words(chains, dependent):
    import torch
    from paper_1911_06001_amd import ceiling
    rng = np.random.default_rng(5)
    n = 1000
    host = rng.integers(0, 2**63 - 1, n, dtype=np.int64)
    buf = torch.from_numpy(host).cuda()
    blocks, threads, loads, seed = 2, 64, 3, 12345
    sink = torch.zeros(blocks * threads, dtype=torch.int64, device="cuda")
    _say("gather", chains, dependent)
    ceiling.gather(buf, blocks, threads, chains, loads, bool(dependent), seed, sink)
    torch.cuda.synchronize()
    got = [int(v) & M64 for v in sink.cpu().numpy()]
    exp = _expected_gather([int(v) for v in host], blocks, threads, chains, loads, dependent, seed)
    assert got == exp


def test_stream_folds_every_word():
    import torch
    from paper_1911_06001_amd import ceiling
    rng = np.random.default_rng(6)
    words = rng.integers(0, 2**32, 4 * 1003, dtype=np.uint64).astype(np.uint32)   # 1003 x 16 B (ragged tail)
    buf = torch.from_numpy(words.view(np.int32).copy()).cuda()
    blocks, threads = 3, 128
    sink = torch.zeros(blocks * threads, dtype=torch.int64, device="cuda")
    _say("stream")
    ceiling.stream_read(buf, blocks, threads, 1, sink)
    torch.cuda.synchronize()
    s = sink.cpu().numpy().view(np.uint64)
    hi = np.bitwise_xor.reduce((s >> np.uint64(32)).astype(np.uint32))
    lo = np.bitwise_xor.reduce((s & np.uint64(0xFFFFFFFF)).astype(np.uint32))
    w = words.reshape(-1, 4)
    assert hi == np.bitwise_xor.reduce(w[:, 0] ^ w[:, 1])
    assert lo == np.bitwise_xor.reduce(w[:, 2] ^ w[:, 3])


def test_measure_small():
    import torch
    from paper_1911_06001_amd import ceiling
    r = ceiling.measure(1 << 20, 256, 256, hbm_bytes=64 << 20, reps=1)
    _say(r)
    for k in ("gather_independent_GBps", "gather_dependent_GBps", "stream_pool_GBps", "stream_hbm_GBps"):
        assert r[k] > 0
