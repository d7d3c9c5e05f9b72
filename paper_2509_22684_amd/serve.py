"""Continuous-batching server for Groth16 quotient jobs.

Requests (A, B, C evaluation vectors of one size, BLS12-381 Fr by default)
arrive over time.  The scheduler keeps jobs resident on the device and
advances every in-flight job by one stage per tick, running the whole tick
as ONE persistent batched launch of the C library (ntt_batch_create_jobs):

    stage 0: A -> T1, B -> T2, C -> H      inverse NTT with the coset shift fused
    stage 1: T1, T2, H in place            forward NTT (evaluations on g<w>)
    stage 2: H = (T1 T2 - H) / (g^n - 1)   pointwise quotient
    stage 3: H in place                    coset inverse NTT -> coefficients

which is the seven-transform chain of the paper's Groth16 prover (Section II,
Fig. 3; Section IV-A) with each job's three independent chains side by side.
A request is admitted when the device bytes of its vectors fit the HBM budget
next to the jobs in flight (plans with their twiddle tables are cached per
size and counted once); otherwise it waits in FIFO order, and a request larger
than the whole budget is rejected.  New requests join at the next tick, so
their transforms share launches with jobs already in flight; finished jobs
free their memory at once.

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
    """Runs ticks on one GPU through the C library."""

    def __init__(self, field: str = "bls12_381_fr", device=None, keep_results: bool = True):
        import torch

        self.torch = torch
        self.field = field
        self.device = torch.device(device or "cuda:0")
        self.stream = torch.cuda.Stream(self.device)       # compute
        self.copy_stream = torch.cuda.Stream(self.device)  # uploads
        self.plans = {}
        self.keep_results = keep_results
        self.ticks = 0
        self.tick_jobs = 0

    def plan(self, log2n: int):
        from ._lib import Plan

        if log2n not in self.plans:
            with self.torch.cuda.device(self.device):
                self.plans[log2n] = Plan(self.field, log2n)
        return self.plans[log2n]

    def plan_bytes(self, log2n: int) -> int:
        return self.plan(log2n).device_bytes

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

    def run_tick(self, items) -> None:
        """items: list of (handle, stage); one batched launch, then wait."""
        from ._lib import ntt_batch_create_jobs, ntt_batch_destroy, ntt_batch_launch_eager, ntt_batch_status

        jobs = []
        for h, stage in items:
            if stage == 0:
                self.stream.wait_event(h["ready"])
            jobs.extend(self._stage_jobs(h, stage))
        with self.torch.cuda.device(self.device):
            b = ntt_batch_create_jobs(jobs)
            try:
                ntt_batch_launch_eager(b, self.stream)
                self.stream.synchronize()
                rc = ntt_batch_status(b)
            finally:
                ntt_batch_destroy(b)
        if rc != 0:
            raise RuntimeError(f"batched tick failed with status {rc}")
        self.ticks += 1
        self.tick_jobs += len(items)

    def result(self, h):
        return h["H"].clone() if self.keep_results else None

    def release(self, h) -> None:
        h.clear()


class QuotientServer:
    """Admission by HBM budget and one batched launch per tick."""

    def __init__(self, executor, budget_bytes: int, clock: Callable[[], float] | None = None):
        self.ex = executor
        self.budget = budget_bytes
        self.clock = clock or time.perf_counter
        self.max_inflight = 0
        self.peak_bytes = 0

    def _plans_bytes(self, sizes) -> int:
        return sum(self.ex.plan_bytes(s) for s in sizes)

    def run(self, requests: list[Request], realtime: bool = True) -> list[Result]:
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival_s, r.job_id)))
        queue: collections.deque = collections.deque()
        inflight = []  # [request, handle, stage, result]
        results: dict[int, Result] = {}
        used = 0
        plan_sizes: set = set()
        t0 = self.clock()

        def now() -> float:
            return self.clock() - t0

        while pending or queue or inflight:
            t = now()
            while pending and (not realtime or pending[0].arrival_s <= t):
                queue.append(pending.popleft())
            # FIFO admission under the budget
            while queue:
                r = queue[0]
                need = self.ex.job_bytes(r.log2n)
                extra_plan = 0 if r.log2n in plan_sizes else self.ex.plan_bytes(r.log2n)
                if need + extra_plan + self._plans_bytes(plan_sizes) > self.budget:
                    # cannot fit even alone next to the resident plans: reject now
                    queue.popleft()
                    results[r.job_id] = Result(r.job_id, r.log2n, "rejected", r.arrival_s)
                    continue
                if used + need + extra_plan + self._plans_bytes(plan_sizes) > self.budget:
                    break
                queue.popleft()
                plan_sizes.add(r.log2n)
                h = self.ex.admit(r)
                used += need
                res = Result(r.job_id, r.log2n, "done", r.arrival_s, admit_s=now())
                inflight.append([r, h, 0, res])
            self.max_inflight = max(self.max_inflight, len(inflight))
            self.peak_bytes = max(self.peak_bytes, used + self._plans_bytes(plan_sizes))
            if not inflight:
                if pending and realtime:
                    time.sleep(max(0.0, min(0.01, pending[0].arrival_s - now())))
                continue
            self.ex.run_tick([(h, stage) for _, h, stage, _ in inflight])
            still = []
            for entry in inflight:
                r, h, stage, res = entry
                if stage + 1 == STAGES:
                    res.done_s = now()
                    res.H = self.ex.result(h)
                    self.ex.release(h)
                    used -= self.ex.job_bytes(r.log2n)
                    results[r.job_id] = res
                else:
                    entry[2] = stage + 1
                    still.append(entry)
            inflight = still
        return [results[r.job_id] for r in sorted(requests, key=lambda r: r.job_id)]


def summarize(results: list[Result]) -> dict:
    import numpy as np

    done = [r for r in results if r.status == "done"]
    lat = np.array([r.latency_s for r in done]) if done else np.array([float("nan")])
    span = (max(r.done_s for r in done) - min(r.arrival_s for r in done)) if done else float("nan")
    return {
        "jobs": len(results),
        "done": len(done),
        "rejected": sum(r.status == "rejected" for r in results),
        "p50_latency_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_latency_ms": float(np.percentile(lat, 99) * 1e3),
        "jobs_per_s": len(done) / span if done else 0.0,
        "makespan_s": span,
    }
