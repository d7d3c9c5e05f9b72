"""Scheduling logic of the quotient server on the CPU, with an executor backed
by the oracle (no GPU): admission by memory budget, FIFO waiting, rejection
of jobs larger than the budget or of unsupported sizes, ticks enqueued ahead
without waiting, lanes by size, continuous batching across ticks, and that
every finished job carries the oracle's quotient."""
import numpy as np

import seeded_inputs as si
from oracle import coracle
from paper_2509_22684_amd.serve import QuotientServer, Request, STAGES, summarize

FIELD = "bls12_381_fr"


class OracleExecutor:
    """Executor with the GpuExecutor interface that computes each finished
    job's quotient with the C oracle and records every tick.  Ticks complete
    when `complete_after` polls have seen them (0: at once)."""

    def __init__(self, plan_bytes_per_elem=32, lane_bounds=(), complete_after=0):
        self.ticks = []
        self.lane_ticks = []
        self.pb = plan_bytes_per_elem
        self.lane_bounds = tuple(lane_bounds)
        self.complete_after = complete_after
        self.allocations = 0
        self.plans = set()
        self.tokens = []
        self.max_open_at_enqueue = 0  # ticks launched and not yet complete when another is launched

    @property
    def lanes(self):
        return len(self.lane_bounds) + 1

    def lane_of(self, log2n):
        return sum(log2n > b for b in self.lane_bounds)

    @staticmethod
    def supports(log2n):
        return 2 <= log2n <= 32

    def plan_bytes(self, log2n):
        return self.pb << log2n  # a formula: no plan is built to learn it

    @staticmethod
    def job_bytes(log2n):
        return 9 * 32 << log2n

    def admit(self, req):
        self.plans.add(req.log2n)
        self.allocations += 1
        return {"req": req}

    def enqueue_tick(self, lane, items):
        self.ticks.append([(h["req"].job_id, stage) for h, stage in items])
        self.lane_ticks.append(lane)
        for h, stage in items:
            assert self.lane_of(h["req"].log2n) == lane
            if stage == STAGES - 1:
                A, B, C = h["req"].inputs
                h["H"] = coracle.quotient(FIELD, A, B, C, threads=2)
        open_ticks = sum(t["polls"] <= self.complete_after for t in self.tokens)
        self.max_open_at_enqueue = max(self.max_open_at_enqueue, open_ticks)
        token = {"polls": 0}
        self.tokens.append(token)
        return token

    def tick_done(self, token):
        token["polls"] += 1
        return token["polls"] > self.complete_after

    def finish_tick(self, token):
        pass

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


def test_ticks_are_enqueued_ahead_of_completion():
    """With depth 2 the next stage is launched before the current tick has
    completed: the host never waits for a tick to build the next one."""
    reqs = make_requests([5, 5])
    ex = OracleExecutor(complete_after=3)
    srv = QuotientServer(ex, budget_bytes=1 << 30, depth=2, poll_s=0)
    res = srv.run(reqs, realtime=False)
    check_results(res, reqs)
    assert [sorted(st for _, st in t) for t in ex.ticks] == [[s, s] for s in range(STAGES)]
    assert ex.max_open_at_enqueue == 1
    # depth 1: same ticks, each enqueued only after the previous completed
    ex1 = OracleExecutor(complete_after=3)
    res1 = QuotientServer(ex1, budget_bytes=1 << 30, depth=1, poll_s=0).run(reqs, realtime=False)
    check_results(res1, reqs)
    assert ex1.ticks == ex.ticks
    assert ex1.max_open_at_enqueue == 0


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


def test_oversize_and_unsupported_jobs_rejected_others_served():
    reqs = make_requests([4, 9, 4, 4])
    reqs[3] = Request(3, 40, 0.0, reqs[0].inputs)  # beyond the field's 2-adicity
    ex = OracleExecutor()
    budget = ex.job_bytes(6) + ex.plan_bytes(4) + ex.plan_bytes(6)
    srv = QuotientServer(ex, budget_bytes=budget)
    res = srv.run(reqs, realtime=False)
    assert [r.status for r in res] == ["done", "rejected", "done", "rejected"]
    check_results([res[0], res[2]], [reqs[0], reqs[2]])
    # a rejected size never got a plan or a buffer
    assert ex.plans == {4} and ex.allocations == 2


def test_lanes_by_size_tick_independently():
    """Small and large jobs go to different lanes; each lane's ticks hold
    only its own jobs, and a lane with a slow tick does not hold the other."""
    reqs = make_requests([4, 8, 4, 8])
    ex = OracleExecutor(lane_bounds=(6,))
    srv = QuotientServer(ex, budget_bytes=1 << 30)
    res = srv.run(reqs, realtime=False)
    check_results(res, reqs)
    small = [t for t, ln in zip(ex.ticks, ex.lane_ticks) if ln == 0]
    large = [t for t, ln in zip(ex.ticks, ex.lane_ticks) if ln == 1]
    assert len(small) == STAGES and len(large) == STAGES
    assert all({j for j, _ in t} == {0, 2} for t in small)
    assert all({j for j, _ in t} == {1, 3} for t in large)


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
        def enqueue_tick(self, lane, items):
            clock.t += 1.0  # each tick takes one time unit
            return super().enqueue_tick(lane, items)

    ex = TickingExecutor()
    srv = QuotientServer(ex, budget_bytes=1 << 30, clock=clock)
    res = srv.run(reqs, realtime=True)
    check_results(res, reqs)
    mixed = [t for t in ex.ticks if len({j for j, _ in t}) == 2]
    assert mixed, "the late job never shared a tick with the first"
    stages_in_mixed = {tuple(sorted(t)) for t in mixed}
    assert any(dict(t)[0] != dict(t)[1] for t in stages_in_mixed), "jobs at different stages share a launch"
    assert res[1].admit_s >= reqs[1].arrival_s


def test_summary_slowdown_against_solo():
    reqs = make_requests([4, 5])
    ex = OracleExecutor()
    res = QuotientServer(ex, budget_bytes=1 << 30).run(reqs, realtime=False)
    s = summarize(res, solo_s={4: 1.0, 5: 1.0})
    assert s["p50_slowdown"] >= 0 and set(s["by_log2n"]) == {"4", "5"}


class WholeOracleExecutor(OracleExecutor):
    """Also offers the whole-chain path: a lone job's quotient in one tick."""

    def __init__(self, **kw):
        super().__init__(**kw)
        self.whole = []

    def enqueue_whole(self, lane, h):
        assert self.lane_of(h["req"].log2n) == lane
        self.whole.append(h["req"].job_id)
        return self.enqueue_tick(lane, [(h, STAGES - 1)])


def test_lone_job_runs_its_whole_chain_in_one_tick():
    reqs = make_requests([5])
    ex = WholeOracleExecutor()
    res = QuotientServer(ex, budget_bytes=1 << 30).run(reqs, realtime=False)
    check_results(res, reqs)
    assert ex.whole == [0] and ex.ticks == [[(0, STAGES - 1)]]


def test_overlapping_jobs_share_batched_ticks_not_whole_chains():
    """Jobs admitted together in one lane batch their stages; alone in their
    lanes they run whole."""
    reqs = make_requests([5, 5, 5])
    ex = WholeOracleExecutor()
    res = QuotientServer(ex, budget_bytes=1 << 30).run(reqs, realtime=False)
    check_results(res, reqs)
    assert ex.whole == [] and len(ex.ticks) == STAGES and all(len(t) == 3 for t in ex.ticks)
    reqs2 = make_requests([4, 8])
    ex2 = WholeOracleExecutor(lane_bounds=(6,))
    res2 = QuotientServer(ex2, budget_bytes=1 << 30).run(reqs2, realtime=False)
    check_results(res2, reqs2)
    assert sorted(ex2.whole) == [0, 1]


def test_job_arriving_during_a_whole_chain_is_batched_after_it():
    """A second job that arrives while the first runs whole finds the lane
    busy (one job in it) and starts with ordinary ticks; both finish with the
    oracle's results."""

    class SteppedClock:
        def __init__(self):
            self.t = 0.0

        def __call__(self):
            return self.t

    clock = SteppedClock()
    reqs = make_requests([5, 5], gaps=[0.5, 0.0])

    class Ticking(WholeOracleExecutor):
        def enqueue_tick(self, lane, items):
            clock.t += 1.0
            return super().enqueue_tick(lane, items)

    ex = Ticking(complete_after=2)
    res = QuotientServer(ex, budget_bytes=1 << 30, clock=clock, poll_s=0).run(reqs, realtime=True)
    check_results(res, reqs)
    assert ex.whole == [0]
    assert sorted(st for t in ex.ticks for j, st in t if j == 1) == list(range(STAGES))
