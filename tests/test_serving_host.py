"""Host logic of the serving loop (admission, chunking, continuous batching, statistics),
driven by a fake executor on the CPU.  The fake executor fills each chunk's outputs with a
simple function of its points, so the tests also check that every point is served exactly
once and lands in its own output row."""
import numpy as np
import pytest

from paper_2402_14415_amd.serving import Server, request_footprint, run_trace


class FakeGrid:
    def __init__(self, dim=3):
        self.dim = dim


class FakeClock:
    def __init__(self, step=1e-4):
        self.t = 0.0
        self.step = step

    def __call__(self):
        self.t += self.step
        return self.t


class FakeExecutor:
    """Completes a launch after `lag` polls of its token; records every launch."""

    def __init__(self, lag=2):
        self.lag = lag
        self.launches = []
        self.writes = {}

    def check_points(self, q, dim):
        assert q.ndim == 2 and q.shape[1] == dim
        return q.shape[0]

    def mark_ready(self, q):
        return None

    def alloc(self, n, dim):
        return np.full(n, np.nan), np.full((n, dim), np.nan)

    def launch(self, chunks):
        for r, a, b in chunks:
            assert 0 <= a < b <= r.n
            r.sdf[a:b] = r.q[a:b].sum(axis=1) + 10.0 * r.grid
            r.normal[a:b] = -r.q[a:b]
            self.writes[r.rid] = self.writes.get(r.rid, 0) + (b - a)
        tok = {"left": self.lag, "chunks": [(r.rid, a, b) for r, a, b in chunks]}
        self.launches.append(tok)
        return tok

    def done(self, tok):
        tok["left"] -= 1
        return tok["left"] <= 0


def _server(budget=1 << 20, lag=2, **kw):
    ex = FakeExecutor(lag)
    return Server([FakeGrid(), FakeGrid(), FakeGrid()], budget, executor=ex, clock=FakeClock(), **kw), ex


def _pts(n, seed):
    return np.random.default_rng(seed).uniform(-1, 1, size=(n, 3))


def _check_outputs(r):
    np.testing.assert_array_equal(r.sdf, r.q.sum(axis=1) + 10.0 * r.grid)
    np.testing.assert_array_equal(r.normal, -r.q)


def test_footprint():
    assert request_footprint(1000, 3) == 28000
    assert request_footprint(1000, 2) == 20000
    assert request_footprint(0, 3) == 0


def test_every_point_served_once_and_in_place():
    srv, ex = _server(chunk_points=100, max_reqs=4)
    reqs = [srv.submit(i % 3, _pts(n, i)) for i, n in enumerate([5, 250, 1000, 1, 99, 100, 101])]
    srv.drain()
    for r in reqs:
        assert r.done and ex.writes[r.rid] == r.n
        _check_outputs(r)
    for L in ex.launches:
        assert len(L["chunks"]) <= 4
        assert all(b - a <= 100 for _, a, b in L["chunks"])
    # chunks of one request are handed out in order, without gaps or overlaps
    for r in reqs:
        spans = [(a, b) for L in ex.launches for rid, a, b in L["chunks"] if rid == r.rid]
        assert spans[0][0] == 0 and spans[-1][1] == r.n
        assert all(spans[k][1] == spans[k + 1][0] for k in range(len(spans) - 1))


def test_admission_respects_budget_and_arrival_order():
    budget = request_footprint(600, 3)
    srv, _ = _server(budget=budget, chunk_points=128)
    sizes = [300, 200, 250, 50, 600, 10, 400, 5]
    reqs = [srv.submit(0, _pts(n, k)) for k, n in enumerate(sizes)]
    srv.drain()
    assert srv.peak_bytes <= budget
    assert srv.used_bytes == 0
    admits = [r.t_admit for r in reqs]
    assert admits == sorted(admits)  # first come, first admitted
    for r in reqs:
        _check_outputs(r)


def test_request_above_budget_is_rejected():
    srv, _ = _server(budget=request_footprint(100, 3))
    with pytest.raises(ValueError):
        srv.submit(0, _pts(101, 0))
    with pytest.raises(IndexError):
        srv.submit(3, _pts(1, 0))


def test_small_request_overtakes_large_one():
    """Continuous batching: a small request that arrives while a large one is being served
    joins the next launch and finishes first."""
    srv, _ = _server(budget=1 << 22, chunk_points=1000, depth=1, lag=1)
    big = srv.submit(0, _pts(50_000, 0))
    srv.poll()
    small = srv.submit(1, _pts(10, 1))
    srv.drain()
    assert small.t_done < big.t_done
    _check_outputs(big)
    _check_outputs(small)


def test_depth_bounds_launches_in_flight():
    srv, _ = _server(chunk_points=10, depth=3, lag=5)
    for k in range(20):
        srv.submit(k % 3, _pts(37, k))
        assert len(srv._inflight) <= 3
    srv.drain()
    assert srv.launches >= 20 * 4 // 32


def test_empty_request_completes():
    srv, _ = _server()
    r = srv.submit(0, _pts(0, 0))
    assert r.done and r.sdf.shape == (0,)
    srv.drain()
    assert srv.used_bytes == 0


def test_run_trace_statistics():
    srv, _ = _server(chunk_points=256, lag=3)
    rng = np.random.default_rng(0)
    arrivals = np.cumsum(rng.exponential(2e-3, size=40))
    trace = [(float(t), int(rng.integers(0, 3)), _pts(int(rng.integers(1, 3000)), k)) for k, t in enumerate(arrivals)]
    out = run_trace(srv, trace)
    assert out["requests"] == 40
    assert out["points"] == sum(len(q) for _, _, q in trace)
    assert 0 < out["p50_ms"] <= out["p99_ms"] <= out["max_ms"]
    assert out["peak_inflight_bytes"] <= srv.budget
    for r in srv.completed:
        _check_outputs(r)
