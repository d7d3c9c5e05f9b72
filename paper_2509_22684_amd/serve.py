"""Continuous-batching server for Groth16 quotient jobs.

Requests (A, B, C evaluation vectors of one size, BLS12-381 Fr by default)
arrive over time.  The server keeps admitted jobs resident on the device and
advances every job by one stage per tick, a tick being ONE batched launch of
the C library (ntt_batch_create_jobs) over the current stage of every job it
holds:

    stage 0: A -> T1, B -> T2, C -> H      inverse NTT with the coset shift fused
    stage 1: T1, T2, H in place            forward NTT (evaluations on g<w>)
    stage 2: H = (T1 T2 - H) / (g^n - 1)   pointwise quotient
    stage 3: H in place                    coset inverse NTT -> coefficients

which is the seven-transform chain of the paper's Groth16 prover (Section II,
Fig. 3; Section IV-A) with each job's three independent chains side by side.

Lanes.  Jobs are assigned by size to lanes, each with its own stream and its
own sequence of ticks, so the long stages of large jobs (which fill the chip
by themselves) do not hold back the next stage of small ones; the lanes'
launches overlap on the device.  A tick's batch runs as pass launches only
(transforms of equal plans grouped into one launch per pass, ZK_BATCH_DIRECT):
the batch's persistent kernel, whose workgroups are large, would wait for
room on CUs that the other lane's pass kernels keep filling.

A lone job runs whole.  When a lane holds a single job that has not
started, its tick is that job's whole chain as one quotient_poly call (A's
and B's chains on forked streams, the pointwise step fused): at light load
a job then costs its stand-alone time instead of four batch builds and four
dependent ticks.  As soon as two jobs overlap in a lane they share batched
ticks again.

No host wait per tick.  A lane keeps up to `depth` ticks enqueued: tick k+1
(every job's next stage, in stream order after tick k) is built and launched
while tick k runs, and completions are found by polling the ticks' events,
so the host never blocks on the device and the device never waits for the
host to build a batch.  A job finishes when the tick holding its last stage
completes; its memory is freed at once.

Admission.  A request is admitted in FIFO order when the device bytes of its
vectors fit the HBM budget next to the jobs in flight and the plans (twiddle
and coset tables, created on a size's first admission and counted once, with
their size known beforehand from ntt_plan_table_bytes); a request larger
than the whole budget, or of a size the field does not support, is rejected.
New requests join their lane's next tick, so their transforms share launches
with jobs already in flight (continuous batching).

Every tile of every job computes exactly what the stand-alone quotient_poly
computes, so a job's result does not depend on its batch-mates.

The executor is pluggable: GpuExecutor drives the HIP library; tests use an
oracle-backed executor on the CPU to check the scheduling logic alone.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable

STAGES = 4


@dataclasses.dataclass
class Request:
    job_id: int
    log2n: int
    arrival_s: float
    inputs: tuple  # (A, B, C): host arrays [n, 8] uint32, or device tensors


@dataclasses.dataclass
class Result:
    job_id: int
    log2n: int
    status: str  # "done" | "rejected"
    arrival_s: float
    admit_s: float = float("nan")
    done_s: float = float("nan")
    H: object = None

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s


class GpuExecutor:
    """Runs ticks on one GPU through the C library, one stream per lane."""

    def __init__(self, field: str = "bls12_381_fr", device=None, keep_results: bool = True,
                 lane_bounds: tuple = (19,)):
        import torch

        from ._lib import FIELD_ADICITY, _register_tuning_for_current_device

        self.torch = torch
        self.field = field
        self.device = torch.device(device or "cuda:0")
        # lane i holds jobs with lane_bounds[i-1] < log2n <= lane_bounds[i]
        self.lane_bounds = tuple(lane_bounds)
        self.streams = [torch.cuda.Stream(self.device) for _ in range(len(self.lane_bounds) + 1)]
        self.copy_stream = torch.cuda.Stream(self.device)  # uploads
        self.plans = {}
        self.keep_results = keep_results
        self.max_log2n = FIELD_ADICITY.get(field, 47)
        self.ticks = 0
        self.tick_jobs = 0
        self.whole_jobs = 0
        with torch.cuda.device(self.device):
            _register_tuning_for_current_device()  # plans and their sizes follow the tuned schedules

    @property
    def lanes(self) -> int:
        return len(self.streams)

    def lane_of(self, log2n: int) -> int:
        return sum(log2n > b for b in self.lane_bounds)

    def supports(self, log2n: int) -> bool:
        # batched jobs need n >= 4
        return 2 <= log2n <= self.max_log2n

    def plan(self, log2n: int):
        from ._lib import Plan

        if log2n not in self.plans:
            with self.torch.cuda.device(self.device):
                self.plans[log2n] = Plan(self.field, log2n)
        return self.plans[log2n]

    def plan_bytes(self, log2n: int) -> int:
        """Device bytes of the plan's tables, known without creating it."""
        from ._lib import ntt_plan_table_bytes

        return ntt_plan_table_bytes(self.field, log2n)

    @staticmethod
    def job_bytes(log2n: int) -> int:
        # A, B, C, H, T1, T2 and one workspace per chain: 9 vectors of n x 32 B
        return 9 * 32 << log2n

    def admit(self, req: Request):
        torch = self.torch
        n = 1 << req.log2n
        plan = self.plan(req.log2n)
        bufs = torch.empty(9 * n, 8, dtype=torch.int32, device=self.device)
        A, B, C, H, T1, T2, W1, W2, W3 = (bufs[k * n:(k + 1) * n] for k in range(9))
        # the uploads wait for the allocation's stream, then run on their own
        self.copy_stream.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(self.copy_stream):
            for dst, src in zip((A, B, C), req.inputs):
                if isinstance(src, torch.Tensor):
                    dst.copy_(src, non_blocking=True)
                else:
                    import numpy as np

                    host = torch.from_numpy(np.ascontiguousarray(src).view(np.int32)).pin_memory()
                    dst.copy_(host, non_blocking=True)
            ready = torch.cuda.Event()
            ready.record(self.copy_stream)
        return {"plan": plan, "bufs": bufs, "A": A, "B": B, "C": C, "H": H, "T1": T1, "T2": T2,
                "W": (W1, W2, W3), "ready": ready}

    def _stage_jobs(self, h, stage: int):
        p, W1, W2, W3 = h["plan"], *h["W"]
        if stage == 0:
            return [dict(plan=p, op="inverse_to_coset", **{"in": h["A"]}, out=h["T1"], work=W1),
                    dict(plan=p, op="inverse_to_coset", **{"in": h["B"]}, out=h["T2"], work=W2),
                    dict(plan=p, op="inverse_to_coset", **{"in": h["C"]}, out=h["H"], work=W3)]
        if stage == 1:
            return [dict(plan=p, op="forward", **{"in": h["T1"]}, out=h["T1"], work=W1),
                    dict(plan=p, op="forward", **{"in": h["T2"]}, out=h["T2"], work=W2),
                    dict(plan=p, op="forward", **{"in": h["H"]}, out=h["H"], work=W3)]
        if stage == 2:
            return [dict(plan=p, op="quotient_pointwise", **{"in": h["T1"]}, in2=h["T2"], in3=h["H"], out=h["H"])]
        return [dict(plan=p, op="coset_inverse", **{"in": h["H"]}, out=h["H"], work=W1)]

    def enqueue_tick(self, lane: int, items):
        """items: list of (handle, stage).  Builds one batch of those stages and
        launches it on the lane's stream after everything already there;
        returns a token for tick_done / finish_tick.  Does not wait."""
        from ._lib import ntt_batch_create_jobs, ntt_batch_destroy, ntt_batch_launch_eager

        stream = self.streams[lane]
        jobs = []
        for h, stage in items:
            if stage == 0:
                stream.wait_event(h["ready"])
            jobs.extend(self._stage_jobs(h, stage))
        with self.torch.cuda.device(self.device):
            # pass launches only: beside the other lanes' pass kernels the
            # persistent kernel's large workgroups wait long for room on the
            # CUs (p99 at rho = 0.5: 18 ms with it, 13-14 ms without)
            b = ntt_batch_create_jobs(jobs, direct=True)
            try:
                ntt_batch_launch_eager(b, stream)
            except Exception:
                ntt_batch_destroy(b)
                raise
            ev = self.torch.cuda.Event()
            ev.record(stream)
        self.ticks += 1
        self.tick_jobs += len(items)
        return (b, ev)

    def enqueue_whole(self, lane: int, h):
        """One job's whole quotient chain as one quotient_poly call on the
        lane's stream (after its uploads); the job's T1, T2 and workspace
        vectors, contiguous, are the chain's workspace.  Does not wait."""
        from ._lib import quotient_poly, quotient_workspace_bytes

        stream = self.streams[lane]
        stream.wait_event(h["ready"])
        p = h["plan"]
        n = h["A"].shape[0]
        work = h["bufs"][4 * n:]  # T1, T2, W1, W2, W3: 5 n elements
        if quotient_workspace_bytes(p.handle) > work.numel() * 4:
            raise RuntimeError("quotient workspace larger than a job's spare vectors")
        with self.torch.cuda.device(self.device):
            quotient_poly(p.handle, h["A"], h["B"], h["C"], h["H"], work, stream)
            ev = self.torch.cuda.Event()
            ev.record(stream)
        self.ticks += 1
        self.tick_jobs += 1
        self.whole_jobs += 1
        return (None, ev)

    @staticmethod
    def tick_done(token) -> bool:
        return token[1].query()

    def finish_tick(self, token) -> None:
        """After tick_done: check the batch's status and free it."""
        from ._lib import ntt_batch_destroy, ntt_batch_status

        b, _ = token
        if b is None:  # a whole job: quotient_poly reports errors when called
            return
        try:
            rc = ntt_batch_status(b)
        finally:
            ntt_batch_destroy(b)
        if rc != 0:
            raise RuntimeError(f"batched tick failed with status {rc}")

    def result(self, h):
        return h["H"].clone() if self.keep_results else None

    def release(self, h) -> None:
        h.clear()


@dataclasses.dataclass
class _Job:
    req: Request
    handle: object
    lane: int
    res: Result
    next_stage: int = 0  # first stage not yet enqueued


@dataclasses.dataclass
class _Tick:
    token: object
    items: list  # [(_Job, stage)]


class QuotientServer:
    """Admission by HBM budget; per lane, ticks of one batched launch each,
    up to `depth` enqueued ahead; completions found by polling."""

    def __init__(self, executor, budget_bytes: int, clock: Callable[[], float] | None = None, depth: int = 2,
                 poll_s: float = 20e-6):
        self.ex = executor
        self.budget = budget_bytes
        self.clock = clock or time.perf_counter
        self.depth = max(1, depth)
        self.poll_s = poll_s
        self.max_inflight = 0
        self.peak_bytes = 0

    def run(self, requests: list[Request], realtime: bool = True) -> list[Result]:
        ex = self.ex
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival_s, r.job_id)))
        queue: collections.deque = collections.deque()
        lanes = [{"jobs": [], "ticks": collections.deque()} for _ in range(ex.lanes)]
        results: dict[int, Result] = {}
        used = 0
        plan_sizes: set = set()
        plans_bytes = 0
        t0 = self.clock()

        def now() -> float:
            return self.clock() - t0

        def active() -> int:
            return sum(len(ln["jobs"]) for ln in lanes)

        while pending or queue or active():
            t = now()
            while pending and (not realtime or pending[0].arrival_s <= t):
                queue.append(pending.popleft())
            # FIFO admission under the budget
            while queue:
                r = queue[0]
                if not ex.supports(r.log2n):
                    queue.popleft()
                    results[r.job_id] = Result(r.job_id, r.log2n, "rejected", r.arrival_s)
                    continue
                need = ex.job_bytes(r.log2n)
                extra_plan = 0 if r.log2n in plan_sizes else ex.plan_bytes(r.log2n)
                if need + extra_plan + plans_bytes > self.budget:
                    # cannot fit even alone next to the resident plans: reject now
                    queue.popleft()
                    results[r.job_id] = Result(r.job_id, r.log2n, "rejected", r.arrival_s)
                    continue
                if used + need + extra_plan + plans_bytes > self.budget:
                    break
                queue.popleft()
                if r.log2n not in plan_sizes:
                    plan_sizes.add(r.log2n)
                    plans_bytes += extra_plan
                h = ex.admit(r)
                used += need
                lane = ex.lane_of(r.log2n)
                lanes[lane]["jobs"].append(_Job(r, h, lane, Result(r.job_id, r.log2n, "done", r.arrival_s,
                                                                  admit_s=now())))
            self.max_inflight = max(self.max_inflight, active())
            self.peak_bytes = max(self.peak_bytes, used + plans_bytes)

            progress = False
            for li, ln in enumerate(lanes):
                # retire finished ticks in launch order
                while ln["ticks"] and ex.tick_done(ln["ticks"][0].token):
                    tick = ln["ticks"].popleft()
                    ex.finish_tick(tick.token)
                    progress = True
                    done_t = now()
                    for job, stage in tick.items:
                        if stage == STAGES - 1:
                            job.res.done_s = done_t
                            job.res.H = ex.result(job.handle)
                            ex.release(job.handle)
                            used -= ex.job_bytes(job.req.log2n)
                            results[job.req.job_id] = job.res
                            ln["jobs"].remove(job)
                # a lone job that has not started runs its whole chain at once
                whole = getattr(ex, "enqueue_whole", None)
                if whole and len(ln["jobs"]) == 1 and ln["jobs"][0].next_stage == 0 and len(ln["ticks"]) < self.depth:
                    job = ln["jobs"][0]
                    ln["ticks"].append(_Tick(whole(li, job.handle), [(job, STAGES - 1)]))
                    job.next_stage = STAGES
                    progress = True
                # keep up to `depth` ticks enqueued: each advances every job
                # of the lane that has a stage left by one stage
                while len(ln["ticks"]) < self.depth:
                    items = [(job, job.next_stage) for job in ln["jobs"] if job.next_stage < STAGES]
                    if not items:
                        break
                    token = ex.enqueue_tick(li, [(job.handle, stage) for job, stage in items])
                    for job, _ in items:
                        job.next_stage += 1
                    ln["ticks"].append(_Tick(token, items))
                    progress = True
            if not progress:
                if not active() and pending and realtime:
                    time.sleep(max(0.0, min(0.01, pending[0].arrival_s - now())))
                elif active():
                    time.sleep(self.poll_s)
        return [results[r.job_id] for r in sorted(requests, key=lambda r: r.job_id)]


def summarize(results: list[Result], solo_s: dict | None = None) -> dict:
    """p50/p99 latency and throughput; with solo_s (log2n -> seconds of one
    job alone) also the slowdown of each job against its size alone."""
    import numpy as np

    done = [r for r in results if r.status == "done"]
    lat = np.array([r.latency_s for r in done]) if done else np.array([float("nan")])
    span = (max(r.done_s for r in done) - min(r.arrival_s for r in done)) if done else float("nan")
    out = {
        "jobs": len(results),
        "done": len(done),
        "rejected": sum(r.status == "rejected" for r in results),
        "p50_latency_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_latency_ms": float(np.percentile(lat, 99) * 1e3),
        "jobs_per_s": len(done) / span if done else 0.0,
        "makespan_s": span,
    }
    if solo_s and done:
        slow = np.array([r.latency_s / solo_s[r.log2n] for r in done if r.log2n in solo_s])
        out["p50_slowdown"] = float(np.percentile(slow, 50))
        out["p99_slowdown"] = float(np.percentile(slow, 99))
        by = {}
        for L in sorted({r.log2n for r in done}):
            ls = np.array([r.latency_s for r in done if r.log2n == L])
            by[str(L)] = {"p50_ms": float(np.percentile(ls, 50) * 1e3), "p99_ms": float(np.percentile(ls, 99) * 1e3),
                          "solo_ms": solo_s.get(L, float("nan")) * 1e3}
        out["by_log2n"] = by
    return out
