"""Scheduling logic of the quotient server on the CPU, with an executor backed
by the oracle (no GPU): admission by memory budget, FIFO waiting, rejection
of jobs larger than the budget, continuous batching across ticks, and that
every finished job carries the oracle's quotient."""
import numpy as np

import seeded_inputs as si
from oracle import coracle
from paper_2509_22684_amd.serve import QuotientServer, Request, STAGES, summarize

FIELD = "bls12_381_fr"


class OracleExecutor:
    """Executor with the GpuExecutor interface that computes each finished
    job's quotient with the C oracle and records every tick."""

    def __init__(self, plan_bytes_per_elem=32):
        self.ticks = []
        self.pb = plan_bytes_per_elem

    def plan_bytes(self, log2n):
        return self.pb << log2n

    @staticmethod
    def job_bytes(log2n):
        return 9 * 32 << log2n

    def admit(self, req):
        return {"req": req}

    def run_tick(self, items):
        self.ticks.append([(h["req"].job_id, stage) for h, stage in items])
        for h, stage in items:
            if stage == STAGES - 1:
                A, B, C = h["req"].inputs
                h["H"] = coracle.quotient(FIELD, A, B, C, threads=2)

    def result(self, h):
        return h["H"]

    def release(self, h):
        h.clear()


def make_requests(sizes, gaps=None):
    reqs = []
    t = 0.0
    for k, L in enumerate(sizes):
        ins = tuple(si.uniform_field_vector(FIELD, 1 << L, si.stream_seed(50 + k, k, v)) for v in range(3))
        reqs.append(Request(k, L, t, ins))
        t += gaps[k] if gaps else 0.0
    return reqs


def check_results(results, reqs):
    for r, q in zip(results, reqs):
        assert r.status == "done"
        assert np.array_equal(r.H, coracle.quotient(FIELD, *q.inputs, threads=2))


def test_all_jobs_finish_with_oracle_results_and_share_ticks():
    reqs = make_requests([4, 6, 5, 4, 7])
    ex = OracleExecutor()
    srv = QuotientServer(ex, budget_bytes=1 << 30)
    res = srv.run(reqs, realtime=False)
    check_results(res, reqs)
    # all five admitted at once: the first tick batches stage 0 of every job
    assert len(ex.ticks[0]) == 5 and srv.max_inflight == 5
    assert len(ex.ticks) == STAGES
    s = summarize(res)
    assert s["done"] == 5 and s["rejected"] == 0


def test_tiny_budget_serialises_jobs():
    reqs = make_requests([5, 5, 5])
    ex = OracleExecutor()
    one_job = ex.job_bytes(5) + ex.plan_bytes(5)
    srv = QuotientServer(ex, budget_bytes=one_job)
    res = srv.run(reqs, realtime=False)
    check_results(res, reqs)
    assert srv.max_inflight == 1
    assert len(ex.ticks) == 3 * STAGES
    assert srv.peak_bytes <= one_job


def test_oversize_job_rejected_others_served():
    reqs = make_requests([4, 9, 4])
    ex = OracleExecutor()
    budget = ex.job_bytes(6) + ex.plan_bytes(4) + ex.plan_bytes(6)
    srv = QuotientServer(ex, budget_bytes=budget)
    res = srv.run(reqs, realtime=False)
    assert [r.status for r in res] == ["done", "rejected", "done"]
    check_results([res[0], res[2]], [reqs[0], reqs[2]])


def test_jobs_join_in_flight_batches():
    """A job that arrives while others run starts at the next tick, in the same
    launch as stages of the jobs already in flight (continuous batching)."""

    class SteppedClock:
        def __init__(self):
            self.t = 0.0

        def __call__(self):
            return self.t

    clock = SteppedClock()
    reqs = make_requests([5, 5], gaps=[1.5, 0.0])  # second job arrives at t = 1.5

    class TickingExecutor(OracleExecutor):
        def run_tick(self, items):
            super().run_tick(items)
            clock.t += 1.0  # each tick takes one time unit

    ex = TickingExecutor()
    srv = QuotientServer(ex, budget_bytes=1 << 30, clock=clock)
    res = srv.run(reqs, realtime=True)
    check_results(res, reqs)
    mixed = [t for t in ex.ticks if len({j for j, _ in t}) == 2]
    assert mixed, "the late job never shared a tick with the first"
    stages_in_mixed = {tuple(sorted(t)) for t in mixed}
    assert any(dict(t)[0] != dict(t)[1] for t in stages_in_mixed), "jobs at different stages share a launch"
    assert res[1].admit_s >= reqs[1].arrival_s
