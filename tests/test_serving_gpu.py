"""GPU tests of the continuous-batching service (one batched launch per tick
over all live requests of all grid sizes)."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sv():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2103_14890_amd import serving
    return serving


def _alone(sv, req, split=True):
    s = sv.Server(split=split)
    alone = sv.Request(req.rid, req.N, req.kernel, req.steps, req.f0, 0.0)
    s.run([alone], realtime=False)
    out = s.results[req.rid].f
    s.close()
    return out


@pytest.mark.parametrize("split", [False, True])
def test_each_result_same_alone_and_in_mix(sv, split):
    """Unsplit, a request's result does not depend on what it ran beside,
    bitwise. With the transform split (its factor follows the group sizes) the
    FP64 gain sums of a step may run in another order: equal to FP32 rounding."""
    reqs = sv.poisson_requests(40, rate=2000.0, seed=5, steps=(5, 30))
    s = sv.Server(split=split)
    stats = s.run(reqs, realtime=True)
    assert stats["requests"] == 40 and stats["failed"] == 0
    assert stats["p99_latency_s"] >= stats["p50_latency_s"] > 0
    for r in reqs[:: 7]:
        a, b = s.results[r.rid].f, _alone(sv, r, split)
        if split:
            assert np.abs(a - b).max() <= 1e-6 * np.abs(b).max(), r.rid
        else:
            assert np.array_equal(a, b), r.rid
    # work really overlapped: fewer ticks than the sum of steps
    assert stats["ticks"] < sum(r.steps for r in reqs)
    s.close()


def test_budget_forces_queueing_and_is_never_exceeded(sv):
    """The budget bounds what the service really allocates on the device (its
    pools, their status flags and the transient of a pool growth), measured by
    the caching allocator, not only its own counter."""
    reqs = sv.poisson_requests(30, rate=1e5, seed=6, sizes=(16, 32), steps=(3, 12))
    budget = 3 * (4 * 32 * 32 + 4) + 512   # about three 32x32 slots at once
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    torch.cuda.reset_peak_memory_stats()
    s = sv.Server(budget_bytes=budget)
    stats = s.run(reqs, realtime=False)
    torch.cuda.synchronize()
    device_peak = torch.cuda.max_memory_allocated() - base
    assert stats["failed"] == 0 and stats["requests"] == 30
    assert 0 < s.peak_bytes <= budget
    assert 0 < device_peak <= budget, (device_peak, budget)
    assert stats["waited"] > 0
    waited = [r for r in s.results.values() if r.admitted > r.arrival]
    assert waited, "the small budget should have made some requests wait"
    for r in reqs[:: 10]:
        assert np.array_equal(s.results[r.rid].f, _alone(sv, r))
    s.close()


def test_nonfinite_request_is_evicted_alone(sv):
    reqs = sv.poisson_requests(12, rate=1e5, seed=7, sizes=(16, 24), steps=(4, 8))
    bad = reqs[3]
    bad.f0 = bad.f0.copy()
    bad.f0[2, 3] = np.nan
    s = sv.Server()
    s.run(reqs, realtime=False)
    assert s.results[bad.rid].failed and s.results[bad.rid].f is None
    for r in reqs:
        if r.rid != bad.rid:
            assert not s.results[r.rid].failed
            assert np.array_equal(s.results[r.rid].f, _alone(sv, r))
    s.close()


def test_request_larger_than_budget_is_refused(sv):
    s = sv.Server(budget_bytes=1000)
    with pytest.raises(ValueError):
        s.submit(sv.Request(0, 32, "maxwell", 3, np.zeros((32, 32), np.float32)))
    s.close()
