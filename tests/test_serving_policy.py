"""The serving loop's batching policy on the host (no device): admission never
exceeds the budget and is first come first served, steps cover every ray of
every admitted request exactly once, a request larger than the budget is
rejected."""
import collections

import numpy as np
import pytest

from paper_1911_06001_amd.serve import Request, Scheduler, _Active, Result, poisson_requests


def _sim(reqs, budget, max_rays, finish_after=2, seed=0, policy="fair", max_jobs=256):
    """Drive the scheduler with a fake executor: a step completes
    `finish_after` plans after it was issued."""
    rng = np.random.default_rng(seed)
    s = Scheduler(budget, max_rays, policy=policy, min_chunk=16, max_jobs=max_jobs, max_frames=40)
    waiting = collections.deque(reqs)
    active, inflight, order, done = [], collections.deque(), [], []
    covered = {r.rid: np.zeros(r.rays, np.int32) for r in reqs}
    while waiting or active or inflight:
        def on_admit(req):
            a = _Active(req, Result(req), None, {}, None, frames=9 if req.scene == "b" else 2)
            active.append(a)
            order.append(req.rid)
            return a
        s.admit(waiting, on_admit)
        assert s.used <= budget
        chunks = s.plan(active)
        for a, lo, hi in chunks:
            assert hi - lo > 0
            covered[a.req.rid][lo:hi] += 1
        # a remainder of at most a quarter of the cap rides along
        assert sum(hi - lo for _, lo, hi in chunks) <= max_rays + max_rays // 4 * len(chunks)
        assert len(chunks) <= max_jobs and sum(a.frames for a, _, _ in chunks) <= 40
        if chunks:
            inflight.append(chunks)
        if inflight and (len(inflight) >= finish_after or not chunks or rng.random() < 0.3):
            for a, lo, hi in inflight.popleft():
                a.pending_chunks -= 1
                if a.pending_chunks == 0 and a.next_ray >= a.req.rays:
                    active.remove(a)
                    s.release(a.req)
                    done.append(a.req.rid)
    return s, order, done, covered


@pytest.mark.parametrize("policy", ["fifo", "fair", "edf"])
def test_budget_fifo_and_exact_coverage(policy):
    reqs = poisson_requests(60, 1000.0, 4, ["a", "b"], resolutions=((16, 16), (40, 30), (64, 48)), samples=(1, 3))
    budget = max(r.footprint for r in reqs) * 3
    s, order, done, covered = _sim(reqs, budget, max_rays=5000, policy=policy, max_jobs=5)
    assert order == sorted(order)                      # admitted first come first served
    assert sorted(done) == [r.rid for r in reqs]      # everything finished
    assert all((c == 1).all() for c in covered.values())   # each ray submitted exactly once
    assert s.max_used <= budget and s.used == 0


def test_small_steps_split_large_requests():
    reqs = [Request(i, 0.0, "a", 0, 100, 100, 2) for i in range(3)]
    s, order, done, covered = _sim(reqs, budget=10**9, max_rays=777)
    assert all((c == 1).all() for c in covered.values())


def test_oversized_request_is_rejected():
    big = Request(0, 0.0, "a", 0, 1000, 1000, 5)
    s = Scheduler(budget=big.footprint - 1, max_rays=1 << 20)
    with pytest.raises(ValueError):
        s.admit(collections.deque([big]), lambda r: r)


def test_poisson_trace_is_seeded():
    a = poisson_requests(50, 100.0, 7, ["x", "y"])
    b = poisson_requests(50, 100.0, 7, ["x", "y"])
    assert [(r.arrival, r.scene, r.width, r.samples) for r in a] == [(r.arrival, r.scene, r.width, r.samples) for r in b]
    gaps = np.diff([r.arrival for r in a])
    assert (gaps >= 0).all() and 0.003 < gaps.mean() < 0.03


def test_fair_share_lets_small_requests_through():
    big = Request(0, 0.0, "a", 0, 1000, 1000, 1)
    small = Request(1, 0.0, "a", 0, 8, 8, 1)
    for policy, small_first_step in (("fifo", False), ("fair", True)):
        s = Scheduler(10**12, max_rays=100000, policy=policy, min_chunk=64)
        active = []
        s.admit(collections.deque([big, small]), lambda r: active.append(_Active(r, Result(r), None, {}, None)) or active[-1])
        chunks = s.plan(active)
        got_small = any(a.req.rid == 1 for a, _, _ in chunks)
        assert got_small == small_first_step, policy


def test_edf_orders_by_deadline():
    """edf: deadline = arrival + slack * rays / ref_rate.  A small request
    that arrives shortly after a large one goes first; a large request whose
    deadline has come is not passed by small work that arrived later."""
    big = Request(0, 0.0, "a", 0, 2000, 1000, 2)          # 4e6 rays: deadline 3 ms at 4e9 rays/s, slack 3
    small = Request(1, 0.0005, "a", 0, 64, 64, 1)         # deadline 0.5 ms + 3 us
    late = Request(2, 0.004, "a", 0, 64, 64, 1)           # arrives after the big one's deadline
    s = Scheduler(10**12, max_rays=5000, policy="edf")
    active = []
    adm = lambda r: active.append(_Active(r, Result(r), None, {}, None)) or active[-1]
    s.admit(collections.deque([big, small]), adm)
    first = s.plan(active)
    assert first[0][0].req.rid == 1                       # the small request first
    s.admit(collections.deque([late]), adm)
    nxt = s.plan(active)
    assert nxt[0][0].req.rid == 0                         # the big request is not passed again


def test_request_that_cannot_fit_a_step_is_rejected():
    """A request whose chunk needs more frame records than a step allows
    would never be planned: admission refuses it instead of waiting."""
    s = Scheduler(10**12, max_rays=1 << 20, max_frames=64)
    big = Request(0, 0.0, "deep", 0, 64, 64, 1)
    with pytest.raises(ValueError):
        s.admit(collections.deque([big]), lambda r: r, frames_of=lambda r: 257)
    ok = Request(1, 0.0, "small", 0, 64, 64, 1)
    assert len(s.admit(collections.deque([ok]), lambda r: r, frames_of=lambda r: 9)) == 1


@pytest.mark.parametrize("policy", ["fifo", "fair", "edf"])
def test_a_lone_request_takes_up_to_the_solo_cap(policy):
    """With solo_rays, a request that is the only one with work left goes in
    one step (up to that cap); beside another request the step cap holds."""
    big = Request(0, 0.0, "a", 0, 2048, 1152, 4)          # 9,437,184 rays
    small = Request(1, 0.0, "a", 0, 256, 256, 1)
    s = Scheduler(1 << 40, 1 << 22, policy=policy, solo_rays=1 << 24)
    a = _Active(big, Result(big), None, {}, None)
    chunks = s.plan([a])
    assert chunks == [(a, 0, big.rays)]
    # capped at solo_rays when the lone request is larger still
    s2 = Scheduler(1 << 40, 1 << 22, policy=policy, solo_rays=1 << 23)
    a2 = _Active(big, Result(big), None, {}, None)
    assert [(lo, hi) for _, lo, hi in s2.plan([a2])] == [(0, 1 << 23)]
    # two requests with work: the step cap applies
    a3, b3 = _Active(big, Result(big), None, {}, None), _Active(small, Result(small), None, {}, None)
    chunks = s.plan([a3, b3])
    assert sum(hi - lo for _, lo, hi in chunks) <= 1 << 22
    # solo_rays = 0 (the default) keeps the step cap for a lone request too
    s4 = Scheduler(1 << 40, 1 << 22, policy=policy)
    a4 = _Active(big, Result(big), None, {}, None)
    assert [(lo, hi) for _, lo, hi in s4.plan([a4])] == [(0, 1 << 22)]


@pytest.mark.parametrize("policy", ["fifo", "edf"])
def test_small_remainder_rides_along(policy):
    """A chunk that would leave at most a quarter of the step cap takes the
    rest too (no step of its own for a small tail), within 1.25 caps; a
    larger remainder waits for the next step."""
    cap = 1 << 16
    tail = Request(0, 0.0, "a", 0, 256, 288, 1)          # 73,728 rays = cap + cap / 8
    far = Request(1, 0.0, "a", 0, 256, 384, 1)           # 98,304 rays = cap + cap / 2
    s = Scheduler(1 << 40, cap, policy=policy)
    a = _Active(tail, Result(tail), None, {}, None)
    chunks = s.plan([a])
    assert chunks == [(a, 0, tail.rays)]
    b = _Active(far, Result(far), None, {}, None)
    chunks = s.plan([b])
    assert chunks == [(b, 0, cap)]
