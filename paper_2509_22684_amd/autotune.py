"""Autotuner for NTT plan schedules.

The paper observes that the tunable parameters of GPU ZKP kernels are picked
by hand for each application and calls for tools that adapt them to the GPU
at run time (Section V-A).  For every (field, log2 n) this module times the
candidate schedules of the C library on the current device — how many
butterfly stages one global pass fuses (log2_pass_radix), where inter-pass
twiddles come from (a precomputed table per pass, or two small tables and one
extra multiplication), the tile a workgroup holds (2^11 or 2^10 elements:
fewer, larger workgroups or more, smaller ones per CU) and the in-register
radix — and records the fastest
in a JSON database keyed by device name.  Every candidate computes the same
bytes (the GPU tests check each schedule against the oracle), so tuning only
changes speed.

    python -m paper_2509_22684_amd.autotune --field bls12_381_fr --sizes 10-24
"""
from __future__ import annotations

import argparse
import json
import os
import statistics

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_DB = os.path.join(HERE, "tuning_db.json")


def db_path() -> str:
    return os.environ.get("ZKNTT_TUNING_DB", DEFAULT_DB)


def candidates(log2n: int, batchable: bool = False) -> list[dict]:
    """Schedules to try at this size.  The batch kernel runs every tile with
    its own radix-4 body on its own tile size, so batchable candidates vary
    only the pass split and the twiddle source."""
    if log2n <= 11:
        return [dict(log2_radix=2)] if batchable else [dict(log2_radix=e) for e in (1, 2, 3)]
    if batchable:
        return [dict(log2_radix=2, log2_pass_radix=pr, twiddle_mode=tm) for pr in (6, 7, 8, 9) for tm in (1, 2)]
    out = [dict(log2_radix=2, log2_pass_radix=pr, twiddle_mode=tm, log2_tile=tile)
           for pr in (6, 7, 8, 9) for tm in (1, 2) for tile in (11, 10)]
    # radix-2 and radix-8 register rounds on the default split
    out += [dict(log2_radix=1), dict(log2_radix=3)]
    if log2n <= 16:  # small transforms: 2^8-element tiles spread a pass over more CUs
        out += [dict(log2_radix=e, log2_tile=8) for e in (1, 2)]
    return out


def _device_name() -> str:
    import torch

    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", p.name)


def time_forward(plan, x, out, reps: int) -> float:
    import torch

    stream = torch.cuda.current_stream()
    for _ in range(2):
        plan.forward(x, out)
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        plan.forward(x, out)
        e1.record(stream)
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    return statistics.median(ms)


def batch_jobs_for(log2n: int) -> int:
    """Jobs of one size in the batch a batchable schedule is timed in: about
    2^20 elements in all, 1 to 64 jobs."""
    return max(1, min(64, (1 << 20) >> log2n))


def time_batched(plan, bufs, reps: int) -> float:
    """Median time of one graph replay of an in-place forward batch over
    `bufs`, all with `plan`: the schedule as the batch runs it (its tiles,
    pass split and choice of grouped launches)."""
    import torch

    from ._lib import Batch

    batch = Batch([plan] * len(bufs), bufs)
    stream = torch.cuda.current_stream()
    for _ in range(2):
        batch.launch(stream)
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        batch.launch(stream)
        e1.record(stream)
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    if batch.status() != 0:
        raise RuntimeError(f"batch status {batch.status()} while tuning")
    batch.close()
    return statistics.median(ms)


def tune(field: str, log2n: int, reps: int = 5, batchable: bool = False) -> dict:
    """Time every candidate; return {"opts": best, "ms": t, "candidates": [...]}.
    Stand-alone schedules are timed as one forward NTT; batchable ones inside
    a batch of batch_jobs_for(log2n) equal jobs."""
    import numpy as np
    import torch

    import seeded_inputs as si

    from ._lib import Plan, ZkError

    n = 1 << log2n
    host = si.uniform_field_vector(field, n, si.stream_seed(77, log2n, 0))
    x = torch.from_numpy(host.view(np.int32)).cuda()
    out = torch.empty_like(x)
    bufs = [x.clone() for _ in range(batch_jobs_for(log2n))] if batchable else []
    rows = []
    for opts in candidates(log2n, batchable):
        try:
            plan = Plan(field, log2n, **opts)
        except ZkError:
            continue
        ms = time_batched(plan, bufs, reps) if batchable else time_forward(plan, x, out, reps)
        rows.append({"opts": opts, "ms": ms, "passes": plan.passes})
        plan.close()
    best = min(rows, key=lambda r: r["ms"])
    return {"opts": best["opts"], "ms": best["ms"], "candidates": rows}


class TuningDB:
    def __init__(self, path: str | None = None):
        self.path = path or db_path()
        self.data = {"devices": {}}
        if os.path.exists(self.path):
            with open(self.path) as f:
                self.data = json.load(f)

    @staticmethod
    def key(field: str, log2n: int, batchable: bool) -> str:
        return f"{field}:{log2n}:{'batch' if batchable else 'single'}"

    def get(self, field: str, log2n: int, batchable: bool = False, device: str | None = None):
        dev = device or _device_name()
        return self.data["devices"].get(dev, {}).get(self.key(field, log2n, batchable))

    def put(self, field: str, log2n: int, entry: dict, batchable: bool = False, device: str | None = None):
        dev = device or _device_name()
        self.data["devices"].setdefault(dev, {})[self.key(field, log2n, batchable)] = entry

    def save(self) -> None:
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.data, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def tuned_opts(field: str, log2n: int, batchable: bool = False, db: TuningDB | None = None) -> dict:
    """The database's best schedule for this size on this device, else {}."""
    db = db or TuningDB()
    e = db.get(field, log2n, batchable)
    return dict(e["opts"]) if e else {}


def tuned_plan(field: str, log2n: int, batchable: bool = False, db: TuningDB | None = None):
    from ._lib import Plan

    return Plan(field, log2n, **tuned_opts(field, log2n, batchable, db))


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--field", action="append", default=None)
    ap.add_argument("--sizes", default="10-24")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--batchable", action="store_true")
    ap.add_argument("--db", default=None)
    args = ap.parse_args()
    lo, hi = (int(v) for v in args.sizes.split("-"))
    db = TuningDB(args.db)
    for field in args.field or ["bls12_381_fr", "bn254_fr", "bls12_377_fr"]:
        for L in range(lo, hi + 1):
            e = tune(field, L, args.reps, args.batchable)
            db.put(field, L, e, args.batchable)
            print(f"{field} 2^{L} {'batch' if args.batchable else 'single'}: best {e['opts']} {e['ms']:.4f} ms "
                  f"({len(e['candidates'])} candidates)", flush=True)
            db.save()


if __name__ == "__main__":
    main()
