"""The serving loop: admission by slots and HBM footprint (CPU, with a
simulated clock and fake jobs), and on the GPU that every answer is the same
alone and in the mix and meets the FP64 backward-error bound."""
import numpy as np
import pytest

from paper_0707_3548_amd import serving


class FakeGpu:
    """Jobs that finish `duration` simulated seconds after launch."""

    def __init__(self, durations):
        self.t = 0.0
        self.durations = durations
        self.launched = []

    def clock(self):
        return self.t

    def idle(self, dt):
        self.t += max(dt, 1e-4)

    def launch(self, req, slot):
        self.launched.append((req.rid, slot, self.t))
        return (req.rid, self.t + self.durations[req.rid])

    def poll(self, handle):
        rid, end = handle
        return rid if self.t >= end else None


def make(reqs):
    return [serving.Request(rid=i, t_arrive=t, m=1, n=1, nrhs=1, footprint=fp) for i, (t, fp) in enumerate(reqs)]


def test_fifo_and_slot_limit():
    g = FakeGpu({i: 1.0 for i in range(5)})
    s = serving.Scheduler(2, 1 << 40, g.launch, g.poll, clock=g.clock, idle=g.idle)
    done = s.run(make([(0.0, 1)] * 5))
    assert [r for r, _, _ in g.launched] == [0, 1, 2, 3, 4]
    assert s.peak_inflight == 2
    assert len(done) == 5
    # two at a time, each taking 1 s: the last starts at about 2 s
    assert abs(g.launched[-1][2] - 2.0) < 1e-2
    lat = sorted(c.latency for c in done)
    assert abs(lat[0] - 1.0) < 1e-2 and abs(lat[-1] - 3.0) < 2e-2


def test_hbm_budget_blocks_admission():
    # budget 10: requests of 6 and 6 cannot run together
    g = FakeGpu({0: 1.0, 1: 1.0, 2: 0.5})
    s = serving.Scheduler(4, 10, g.launch, g.poll, clock=g.clock, idle=g.idle)
    done = s.run(make([(0.0, 6), (0.0, 6), (0.0, 4)]))
    starts = {r: t for r, _, t in g.launched}
    assert starts[1] >= 1.0 - 1e-9          # waited for request 0 to free memory
    assert starts[2] >= starts[1] - 1e-9    # FIFO: no overtaking
    assert s.peak_bytes <= 10
    assert len(done) == 3


def test_oversize_request_runs_alone():
    g = FakeGpu({0: 1.0, 1: 1.0})
    s = serving.Scheduler(4, 10, g.launch, g.poll, clock=g.clock, idle=g.idle)
    done = s.run(make([(0.0, 50), (0.0, 1)]))
    starts = {r: t for r, _, t in g.launched}
    assert starts[0] == 0.0 and starts[1] >= 1.0 - 1e-9
    assert len(done) == 2


def test_arrivals_are_respected():
    g = FakeGpu({0: 0.1, 1: 0.1})
    s = serving.Scheduler(4, 1 << 40, g.launch, g.poll, clock=g.clock, idle=g.idle)
    done = s.run(make([(0.0, 1), (5.0, 1)]))
    starts = {r: t for r, _, t in g.launched}
    assert starts[1] >= 5.0 - 1e-9
    by = {c.rid: c for c in done}
    assert abs(by[1].latency - 0.1) < 1e-2


def test_latency_stats():
    done = [serving.Completion(i, 0.0, 0.0, (i + 1) / 100.0) for i in range(100)]
    st = serving.latency_stats(done)
    assert abs(st["p50_ms"] - 505.0) < 1.0 and st["count"] == 100
    assert st["p99_ms"] <= st["max_ms"] == 1000.0


def test_size_rules():
    assert serving.tiling_for(8192, 8192) == (256, 16)
    assert serving.tiling_for(300, 40)[0] == 32
    assert serving.workers_for(8192, 8192, 256, 256) == 256
    assert 4 <= serving.workers_for(100, 50, 64, 256) <= 4


@pytest.mark.gpu
@pytest.mark.parametrize("solver", ["mixed", "fp64"])
def test_answers_are_the_same_alone_and_in_the_mix(solver):
    """Every answer is bitwise the same alone and in the mix (the factor does
    not depend on the schedule or the worker count, and the refinement's
    sums run in a fixed order), is accepted (info, status and, for the mixed
    solver, the refinement's convergence), and meets the FP64 backward-error
    bound against the oracle."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    from paper_0707_3548_amd import workloads
    print(f"case serving mix of 16 requests, solver {solver}", flush=True)
    arr = workloads.arrivals(rate=2000.0, count=16, seed=21, m_lo=48, m_hi=700, cond_lo=1e1, cond_hi=1e6)
    data = [workloads.ls_request(r["m"], r["n"], r["nrhs"], r["cond"], r["seed"]) for r in arr]
    ex = serving.GpuExecutor(slots=4, solver=solver)

    def requests():
        return [ex.prepare(serving.Request(i, r["t"], r["m"], r["n"], r["nrhs"]), A, b)
                for i, (r, (A, b, _)) in enumerate(zip(arr, data))]

    sch = serving.Scheduler(4, 1 << 34, ex.launch, ex.poll)
    mix = {c.rid: c for c in sch.run(requests())}
    assert len(mix) == 16 and sch.peak_inflight >= 2
    alone = {}
    for req in requests():
        one = serving.Scheduler(1, 1 << 34, ex.launch, ex.poll)
        req.t_arrive = 0.0
        alone[req.rid] = one.run([req])[0]
    for i, (A, b, _) in enumerate(data):
        Xm = mix[i].result["X"].numpy().T
        Xa = alone[i].result["X"].numpy().T
        assert mix[i].result["ok"], mix[i].result
        assert np.array_equal(Xm, Xa), f"request {i} differs between the mix and alone"
        for c in range(b.shape[1]):
            assert oracle.ls_backward_error(A, Xm[:, c], b[:, c]) < 1e-14


@pytest.mark.gpu
def test_a_request_that_does_not_converge_counts_as_failed():
    """A mixed solve whose refinement is cut off (one iteration on a cond 1e5
    problem) is reported as not ok, not as an answer."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0707_3548_amd import workloads
    print("case serving refinement cut off", flush=True)
    A, b, _ = workloads.ls_request(600, 300, 1, 1e5, seed=22)
    ex = serving.GpuExecutor(slots=1, solver="mixed", iterations=1)
    req = ex.prepare(serving.Request(0, 0.0, 600, 300, 1), A, b)
    done = serving.Scheduler(1, 1 << 34, ex.launch, ex.poll).run([req])
    res = done[0].result
    assert not res["ok"]
    assert res["refine"][0]["stop"] == 3   # the iteration limit
