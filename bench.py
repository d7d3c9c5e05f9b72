"""Benchmark: Fr255 NTT throughput at n = 2^24 on one MI355X.

A step is one pass of the whole hot path on one batch of synthetic input: the
Groth16 quotient chain at n = 2^24 over BLS12-381 Fr (three inverse NTTs with
the coset shift fused, three forward NTTs, the pointwise (A B - C)/Z_H
product and the coset inverse NTT: seven transforms).  `value` counts NTT
elements per second over those seven transforms: 7 * 2^24 / step time.

Also reported: the single forward NTT at 2^24 (elements/s); the roofline of
the dominant kernel (the radix-256 pass kernel, timed per launch with HIP
events on the stream it runs on); batched versus per-launch jobs/s for 64
uneven forward NTTs over both fields; and the CPU oracle timed on a bounded
sample on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

LOG2N = 24
FIELD = "bls12_381_fr"
# MI355X: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz; v_mad_u64_u32 issues at
# the full VALU rate on gfx950 (one 32x32->64 multiply-add per lane per
# cycle), so the integer multiply-add peak equals the VALU lane rate.
PEAK_MAD_PER_S = 256 * 4 * 16 * 2.4e9
PEAK_HBM_BYTES_PER_S = 8.0e12
MADS_PER_FFMUL = 136  # 2 s^2 + s for s = 8 limbs (one CIOS/FIPS Montgomery product)
KERNEL_SOURCES = ["paper_2509_22684_amd/csrc/field.hpp", "paper_2509_22684_amd/csrc/ntt_pass_impl.hpp"]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profile(khash: str):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "ntt_pass_r256_t10_2e24_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_hash") != khash:
        return None
    return d.get("hbm_bytes_per_launch")


def valu_from_profile(khash: str):
    """VALU wave instructions per launch of the dominant kernel from the
    committed rocprofv3 counter summary, if taken on the current source."""
    path = os.path.join(ROOT, "profiles", "ntt_pass_r256_t10_2e24_valu.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_hash") != khash:
        return None
    return d.get("valu_wave_instructions_per_launch")


def cpu_baseline(x_host, runs: int = 3) -> dict:
    """The C oracle on the host cores: one forward NTT at n = 2^24, median of
    `runs` runs."""
    from oracle import coracle

    threads = coracle.default_threads()
    dts = []
    for _ in range(runs):
        t0 = time.perf_counter()
        coracle.transform(FIELD, "forward", x_host, threads=threads)
        dts.append(time.perf_counter() - t0)
    dt = statistics.median(dts)
    return {"value": (1 << LOG2N) / dt, "unit": "elements/s", "cores": threads, "kind": "oracle",
            "sample": f"one forward NTT at n=2^24 (BLS12-381 Fr) with the C oracle, median of {runs} runs: "
                      + ", ".join(f"{d:.2f}" for d in dts) + " s wall"}


def peaks_leg(dev) -> dict:
    """Measured roofline denominators (zk_microbench): the all-CU rates of
    the instructions the pass kernel is made of, Montgomery products, and a
    streaming copy's HBM bandwidth."""
    import torch

    from paper_2509_22684_amd import zk_microbench

    small = torch.empty(1 << 20, 8, dtype=torch.int32, device=dev)  # 32 MiB: per-thread results
    out = {}
    for kind, iters in (("mad_u64_u32", 2048), ("fma_f64", 2048), ("add_u32", 2048), ("addc_u32", 1024),
                        ("mad_addc", 1024), ("mad_fma", 1024), ("mad_add", 1024), ("ffmul_bls12_381", 128),
                        ("ffmul_k2", 192), ("ffmul_k4", 96), ("ffmul_f64", 96), ("ffmul_lazy", 128),
                        ("ffmul_bn254", 128)):
        rate, ms = zk_microbench(kind, small, iters=iters, reps=5)
        out[kind] = {"per_s": rate, "ms_per_launch": ms, "iters": iters}
    big = torch.empty(1 << 26, 8, dtype=torch.int32, device=dev)  # 2 GiB: 1 GiB read, 1 GiB written
    rate, ms = zk_microbench("copy", big, reps=5)
    out["copy"] = {"bytes_per_s": rate, "ms_per_launch": ms, "bytes_per_launch": big.numel() * 4}
    del big
    spec = PEAK_MAD_PER_S
    out["summary"] = {
        "mad_u64_u32_T_per_s": out["mad_u64_u32"]["per_s"] / 1e12,
        "mad_u64_u32_over_spec_issue_rate": out["mad_u64_u32"]["per_s"] / spec,
        "fma_f64_T_per_s": out["fma_f64"]["per_s"] / 1e12,
        "add_u32_T_per_s": out["add_u32"]["per_s"] / 1e12,
        "addc_u32_T_per_s": out["addc_u32"]["per_s"] / 1e12,
        "fips_column_steps_T_per_s": out["mad_addc"]["per_s"] / 1e12,
        "mad_with_fma_f64_T_instr_per_s": out["mad_fma"]["per_s"] / 1e12,
        "mad_with_add_u32_T_instr_per_s": out["mad_add"]["per_s"] / 1e12,
        "ffmul_G_per_s": {k: out[f"ffmul_{k}"]["per_s"] / 1e9 for k in ("bls12_381", "k2", "k4", "f64", "lazy", "bn254")},
        "hbm_copy_TB_per_s": out["copy"]["bytes_per_s"] / 1e12,
        "spec_issue_rate_T_per_s": spec / 1e12,
    }
    return out


def cpu_one_core(log2n: int = 20) -> dict:
    """The C oracle on one host thread, on a smaller forward NTT."""
    import seeded_inputs as si
    from oracle import coracle

    x = si.uniform_field_vector(FIELD, 1 << log2n, si.stream_seed(2, 0, 0))
    t0 = time.perf_counter()
    coracle.transform(FIELD, "forward", x, threads=1)
    dt = time.perf_counter() - t0
    return {"value": (1 << log2n) / dt, "unit": "elements/s", "cores": 1, "kind": "oracle",
            "sample": f"one forward NTT at n=2^{log2n} (BLS12-381 Fr) with the C oracle on one thread, {dt:.2f} s"}


def small_configs_leg(dev) -> dict:
    """The two smaller configurations: a radix-2 forward NTT at n = 2^12, and
    forward, inverse, coset forward and coset inverse at n = 2^20 (with both
    round trips checked on the device)."""
    import numpy as np
    import torch

    import seeded_inputs as si
    from paper_2509_22684_amd import Plan

    def med(fn, reps):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        return statistics.median(ts)

    out = {}
    x = torch.from_numpy(si.uniform_field_vector(FIELD, 1 << 12, si.stream_seed(1, 0, 0)).view(np.int32)).to(dev)
    p = Plan(FIELD, 12, log2_radix=1)
    y = torch.empty_like(x)
    ms = med(lambda: p.forward(x, y), 50)
    out["n2e12_radix2"] = {"us_per_forward": ms * 1e3, "elements_per_s": (1 << 12) / (ms * 1e-3),
                           "note": "launch-bound at this size; not a roofline claim"}
    x = torch.from_numpy(si.uniform_field_vector(FIELD, 1 << 20, si.stream_seed(2, 0, 0)).view(np.int32)).to(dev)
    p = Plan(FIELD, 20)
    y, z = torch.empty_like(x), torch.empty_like(x)
    c20 = {}
    for kind, fn in (("forward", p.forward), ("inverse", p.inverse), ("coset_forward", p.coset_forward),
                     ("coset_inverse", p.coset_inverse)):
        ms = med(lambda: fn(x, y), 20)
        c20[kind] = {"ms": ms, "elements_per_s": (1 << 20) / (ms * 1e-3)}
    p.inverse(p.forward(x, y), z)
    rt = torch.equal(z, x)
    p.coset_inverse(p.coset_forward(x, y), z)
    c20["round_trips_exact"] = rt and torch.equal(z, x)
    out["n2e20"] = c20
    return out


def batch_leg(dev, reps: int = 50, warm: int = 100) -> dict:
    """64 forward NTTs (log2 n uniform in [10, 18], 48 BLS12-381 + 16 BN254):
    jobs/s for one launch sequence per NTT (each size on its tuned stand-alone
    schedule) versus one batch (tuned batchable schedules) replayed from its
    graph or launched directly.  Each way is timed in steady state, after
    `warm` untimed repetitions: the first few dozen replays in a process run
    up to 15% slower while the GPU's clocks rise under the new load."""
    import numpy as np
    import torch

    import seeded_inputs as si
    from paper_2509_22684_amd import Batch, Plan
    from paper_2509_22684_amd.autotune import tuned_opts

    jobs = si.batch_jobs()
    plans = {}  # batch plans: the tuned batchable schedule per size
    solo = {}  # per-launch plans: the tuned stand-alone schedule per size
    bufs = []
    for jb in jobs:
        key = (jb.field, jb.log2n)
        if key not in plans:
            plans[key] = Plan(jb.field, jb.log2n, **tuned_opts(jb.field, jb.log2n, batchable=True))
            solo[key] = Plan(jb.field, jb.log2n, **tuned_opts(jb.field, jb.log2n, batchable=False))
        x = si.uniform_field_vector(jb.field, 1 << jb.log2n, jb.seed)
        bufs.append(torch.from_numpy(x.view(np.int32)).to(dev))
    job_plans = [plans[(j.field, j.log2n)] for j in jobs]
    solo_plans = [solo[(j.field, j.log2n)] for j in jobs]
    works = [p.workspace(b) for p, b in zip(solo_plans, bufs)]
    stream = torch.cuda.current_stream(dev)

    def per_launch():
        for p, b, w in zip(solo_plans, bufs, works):
            p.forward(b, out=b)

    batch = Batch(job_plans, bufs)

    def timed(fn):
        for _ in range(warm):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    t_per = timed(per_launch)
    # the same per-job launch sequence captured once in a graph: what is left
    # of the per-launch cost without host launch overhead
    torch.cuda.synchronize()
    side = torch.cuda.Stream(dev)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        for p, b, w in zip(solo_plans, bufs, works):
            p.forward(b, out=b)
    t_per_graph = timed(g.replay)
    t_graph = timed(batch.launch)
    t_eager = timed(batch.launch_eager)
    status = batch.status()
    elems = sum(1 << j.log2n for j in jobs)
    launches = sum(p.passes for p in solo_plans)
    return {
        "workload": "64 forward NTTs, log2 n uniform in [10,18], 48 BLS12-381 Fr + 16 BN254 Fr, seed 4",
        "elements": elems,
        "per_launch": {"ms": t_per, "jobs_per_s": len(jobs) / (t_per * 1e-3), "kernel_launches": launches},
        "per_launch_in_graph": {"ms": t_per_graph, "jobs_per_s": len(jobs) / (t_per_graph * 1e-3)},
        "batched_graph": {"ms": t_graph, "jobs_per_s": len(jobs) / (t_graph * 1e-3), "items": batch.items,
                          "workgroups": batch.grid},
        "batched_direct": {"ms": t_eager, "jobs_per_s": len(jobs) / (t_eager * 1e-3)},
        "batched_over_per_launch": t_per / t_graph,
        "warmup_repetitions": warm, "timed_repetitions": reps,
        "status": status,
    }


def serve_leg(dev, njobs: int = 256, rhos=(0.5, 0.8, 1.0, 1.25, 1.5)) -> dict:
    """Quotient jobs on BLS12-381 Fr (log2 n uniform in [14, 22], seed 5)
    served with continuous batching.  mu = solo throughput on the same size
    mix (one quotient_poly call at a time); then Poisson arrivals at
    lambda = rho mu for each rho under a 200 GB HBM budget (rho above 1
    offers more than one-at-a-time execution can sustain), and once more at
    rho = 1 under a 2 GB budget so that admission has to hold jobs back.
    Each job's A, B, C come from a device-resident pool of one seeded vector
    triple per size, copied into the job's own buffers on admission; latency
    runs from arrival to H ready on the device; slowdown is a job's latency
    over the time of its size alone."""
    import numpy as np
    import torch

    import seeded_inputs as si
    from paper_2509_22684_amd.serve import GpuExecutor, QuotientServer, Request, summarize

    sizes = [s.log2n for s in si.serve_jobs(master=5, njobs=njobs, rate_per_s=1.0)]
    pool = {}
    for L in sorted(set(sizes)):
        pool[L] = tuple(torch.from_numpy(si.uniform_field_vector(FIELD, 1 << L, si.stream_seed(5, 1000 + L, v))
                                         .view(np.int32)).to(dev) for v in range(3))
    ex = GpuExecutor(FIELD, dev, keep_results=False)
    for L in pool:  # plans (twiddle tables) stay resident across jobs
        ex.plan(L)

    # mu: the size mix run solo, one job after another; and each size alone
    H = {L: torch.empty_like(pool[L][0]) for L in pool}
    for L in pool:
        ex.plan(L).quotient(*pool[L], H[L])
    torch.cuda.synchronize()
    solo_s = {}
    for L in pool:
        ts = []
        for _ in range(5):
            t0 = time.perf_counter()
            ex.plan(L).quotient(*pool[L], H[L])
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        solo_s[L] = statistics.median(ts)
    t0 = time.perf_counter()
    for L in sizes:
        ex.plan(L).quotient(*pool[L], H[L])
        torch.cuda.synchronize()
    mu = len(sizes) / (time.perf_counter() - t0)
    del H

    def run(rate: float, budget: int) -> dict:
        specs = si.serve_jobs(master=5, njobs=njobs, rate_per_s=rate)
        reqs = [Request(s.job_id, s.log2n, s.arrival_s, pool[s.log2n]) for s in specs]
        ex.ticks = ex.tick_jobs = ex.whole_jobs = 0
        srv = QuotientServer(ex, budget_bytes=budget)
        res = srv.run(reqs, realtime=True)
        out = summarize(res, solo_s)
        out.update({"rate_per_s": rate, "budget_bytes": budget, "ticks": ex.ticks,
                    "mean_jobs_per_tick": ex.tick_jobs / max(1, ex.ticks), "jobs_run_whole": ex.whole_jobs,
                    "max_inflight": srv.max_inflight, "peak_bytes": srv.peak_bytes})
        return out

    run(mu, 200 << 30)  # warm-up
    runs = []
    for r in rhos:
        print(f"[bench] serving rho={r}", file=sys.stderr, flush=True)
        runs.append(dict(rho=r, **run(r * mu, 200 << 30)))
    admission = dict(rho=1.0, **run(mu, 2 << 30))
    return {"workload": f"{njobs} quotient jobs, log2 n uniform in [14,22] (seed 5), BLS12-381 Fr, Poisson arrivals "
                        "at rho x solo throughput",
            "lanes": {"bounds_log2n": list(ex.lane_bounds), "ticks_enqueued_ahead": 2,
                      "lone_job_runs_whole_chain": True, "tick_batches": "pass launches only (ZK_BATCH_DIRECT)"},
            "mu_solo_jobs_per_s": mu, "solo_ms_by_log2n": {str(L): t * 1e3 for L, t in solo_s.items()},
            "runs": runs, "admission_2GB": admission}


def msm_leg(dev, log2n: int = 20, reps: int = 10) -> dict:
    """MSM on BLS12-381 G1 (the paper's other proving kernel): n = 2^20 fixed
    bases P_i = (i + 1) G, G a point of the order-r subgroup, with their
    per-window multiples precomputed once (timed separately), and uniform
    scalars (Montgomery Fr limbs, as the NTT produces them).  The result is
    checked against the closed form (sum_i s_i (i + 1)) G from the oracle."""
    import numpy as np
    import torch

    import seeded_inputs as si
    from oracle import msm_ref as M
    from oracle import ref
    from paper_2509_22684_amd import MsmBases

    n = 1 << log2n
    G = M.subgroup_point(7)
    t0 = time.perf_counter()
    pts = M.multiples(G, n)
    gen_s = time.perf_counter() - t0
    d_pts = torch.from_numpy(M.points_to_device_layout(pts).view(np.int32)).to(dev)
    sc = si.uniform_field_vector(FIELD, n, si.stream_seed(8, 0, 0))
    d_sc = torch.from_numpy(sc.view(np.int32)).to(dev)
    stream = torch.cuda.current_stream(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bases = MsmBases(d_pts)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    res = torch.empty(64, dtype=torch.int32, device=dev)
    for _ in range(2):
        bases.msm(d_sc, res)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        bases.msm(d_sc, res)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    words = res.cpu().numpy().view(np.uint32)[:48]
    X, Y, ZZ, ZZZ = (M.fq_from_limbs(words[12 * k:12 * (k + 1)].reshape(1, 12))[0] for k in range(4))
    FR = ref.BLS12_381_FR
    s_plain = FR.from_mont(si.limbs_to_ints(sc))
    want = M.mul(sum(v * (i + 1) for i, v in enumerate(s_plain)) % FR.p, G)
    c = bases.window_bits
    windows = (255 + c - 1) // c
    return {"workload": f"MSM over BLS12-381 G1, n=2^{log2n} fixed bases (i+1)G, uniform scalars (seed 8)",
            "ms": ms, "points_per_s": n / (ms * 1e-3), "window_bits": c, "windows": windows,
            "mixed_additions": n * windows, "precompute_s": setup_s, "table_bytes": bases.device_bytes,
            "host_point_generation_s": gen_s, "matches_closed_form": M.xyzz_to_affine(X, Y, ZZ, ZZZ) == want}


def host_pipeline_leg(dev, log2n: int = 22, njobs: int = 8) -> dict:
    """Quotient jobs whose A, B, C start in pinned host memory and whose H
    returns there: one job at a time with nothing overlapped, against the
    three-stream pipeline that overlaps uploads, compute and downloads."""
    import numpy as np
    import torch

    import seeded_inputs as si
    from paper_2509_22684_amd.pipeline import HostQuotientPipeline

    n = 1 << log2n
    triples = [[torch.from_numpy(si.uniform_field_vector(FIELD, n, si.stream_seed(6, t, v)).view(np.int32))
                .pin_memory() for v in range(3)] for t in range(2)]
    outs = [torch.empty((n, 8), dtype=torch.int32).pin_memory() for _ in range(2)]
    pipe = HostQuotientPipeline(FIELD, dev, depth=2)
    pipe.run_serial(*triples[0], outs[0])  # warm-up: plan and slots
    pipe.submit(*triples[1], outs[1]).synchronize()

    t0 = time.perf_counter()
    for k in range(njobs):
        pipe.run_serial(*triples[k % 2], outs[k % 2])
    serial = (time.perf_counter() - t0) / njobs
    t0 = time.perf_counter()
    evs = [pipe.submit(*triples[k % 2], outs[k % 2]) for k in range(njobs)]
    for e in evs:
        e.synchronize()
    piped = (time.perf_counter() - t0) / njobs

    # the parts alone: PCIe (three uploads, one download) and device compute
    d = [torch.empty((n, 8), dtype=torch.int32, device=dev) for _ in range(4)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(njobs):
        for dst, src in zip(d[:3], triples[k % 2]):
            dst.copy_(src, non_blocking=True)
        torch.cuda.synchronize()
        outs[k % 2].copy_(d[3], non_blocking=True)
        torch.cuda.synchronize()
    pcie = (time.perf_counter() - t0) / njobs
    # the same bytes with the upload (DMA) and the download (copy kernel) on
    # two streams at once: the floor the pipeline can reach
    from paper_2509_22684_amd import zk_copy_to_host

    up, down = torch.cuda.Stream(dev), torch.cuda.Stream(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(njobs):
        with torch.cuda.stream(up):
            for dst, src in zip(d[:3], triples[k % 2]):
                dst.copy_(src, non_blocking=True)
        zk_copy_to_host(outs[k % 2], d[3], n * 32, down)
        torch.cuda.synchronize()
    duplex = (time.perf_counter() - t0) / njobs
    plan = pipe.plan(log2n)
    for _ in range(2):
        plan.quotient(d[0], d[1], d[2], d[3])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(njobs):
        plan.quotient(d[0], d[1], d[2], d[3])
    torch.cuda.synchronize()
    compute = (time.perf_counter() - t0) / njobs
    gb = 4 * n * 32 / 1e9
    return {"workload": f"{njobs} quotient jobs at n=2^{log2n}, BLS12-381 Fr, A, B, C and H in pinned host memory",
            "serial_ms_per_job": serial * 1e3, "pipelined_ms_per_job": piped * 1e3,
            "pipelined_over_serial": serial / piped, "pcie_only_ms_per_job": pcie * 1e3,
            "pcie_gb_per_job": gb, "pcie_gbs": gb / pcie, "pcie_both_directions_ms_per_job": duplex * 1e3,
            "compute_only_ms_per_job": compute * 1e3}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-launch leg")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-pipeline", action="store_true", help="skip the host-resident pipeline leg")
    ap.add_argument("--no-msm", action="store_true", help="skip the MSM leg")
    ap.add_argument("--only", choices=["forward", "copy", "batch", "quotient", "peaks", "serve", "msm"],
                    default=None,
                    help="for profiler runs: only run --steps forward NTTs at 2^24, --steps plain device "
                         "copies of one 512 MiB vector (the traffic calibration kernel), --warmup + --steps "
                         "graph replays of the 64-job batch, or --warmup + --steps quotient chains at 2^24 "
                         "(the metric step), or the micro-benchmarks of the roofline denominators "
                         "(peaks), then exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this library has no multi-GPU path "
              "(independent jobs shard across GPUs without communication).", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import seeded_inputs as si
    from paper_2509_22684_amd import Plan, ntt_profile_passes

    dev = torch.device("cuda:0")
    n = 1 << LOG2N

    def to_dev(a):
        return torch.from_numpy(np.ascontiguousarray(a).view(np.int32).copy()).to(dev)

    if args.only == "msm":
        print(json.dumps(msm_leg(dev, reps=max(1, args.steps))), flush=True)
        print("[bench] msm leg done", file=sys.stderr, flush=True)
        return 0
    if args.only == "serve":
        print(json.dumps(serve_leg(dev)), flush=True)
        print("[bench] serving leg done", file=sys.stderr, flush=True)
        return 0
    if args.only == "peaks":
        res = peaks_leg(dev)
        print(json.dumps(res), flush=True)
        print("[bench] micro-benchmarks done", file=sys.stderr, flush=True)
        return 0
    if args.only == "copy":
        src = torch.randint(-(1 << 31), (1 << 31) - 1, (n, 8), dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] {args.steps} copies of {n * 32} bytes done", file=sys.stderr, flush=True)
        return 0
    if args.only == "batch":
        # the 64-job batch as batch_leg builds it, replayed from its graph
        from paper_2509_22684_amd import Batch
        from paper_2509_22684_amd.autotune import tuned_opts

        jobs = si.batch_jobs()
        plans = {}
        for jb in jobs:
            if (jb.field, jb.log2n) not in plans:
                plans[(jb.field, jb.log2n)] = Plan(jb.field, jb.log2n,
                                                   **tuned_opts(jb.field, jb.log2n, batchable=True))
        bufs = [to_dev(si.uniform_field_vector(jb.field, 1 << jb.log2n, jb.seed)) for jb in jobs]
        batch = Batch([plans[(j.field, j.log2n)] for j in jobs], bufs)
        stream = torch.cuda.current_stream(dev)
        for _ in range(args.warmup):
            batch.launch(stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            batch.launch(stream)
        e1.record(stream)
        torch.cuda.synchronize()
        print(json.dumps({"batch_ms_mean": e0.elapsed_time(e1) / max(1, args.steps), "items": batch.items,
                          "workgroups": batch.grid, "status": batch.status(), "warmup": args.warmup,
                          "steps": args.steps}), flush=True)
        print(f"[bench] {args.warmup}+{args.steps} batch replays done", file=sys.stderr, flush=True)
        return 0
    if args.only == "quotient":
        A, B, C = (to_dev(si.uniform_field_vector(FIELD, n, si.stream_seed(3, 0, v))) for v in range(3))
        H = torch.empty_like(A)
        plan = Plan(FIELD, LOG2N)
        stream = torch.cuda.current_stream(dev)
        for _ in range(args.warmup):
            plan.quotient(A, B, C, H)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            plan.quotient(A, B, C, H)
        e1.record(stream)
        torch.cuda.synchronize()
        print(json.dumps({"quotient_ms_mean": e0.elapsed_time(e1) / max(1, args.steps), "warmup": args.warmup,
                          "steps": args.steps}), flush=True)
        print(f"[bench] {args.warmup}+{args.steps} quotient chains at 2^{LOG2N} done", file=sys.stderr, flush=True)
        return 0
    if args.only == "forward":
        # --warmup untimed forwards (clocks settle), then --steps forwards
        # whose passes are timed with HIP events on the launch stream, the
        # same measurement as the roofline below; prints the per-pass means.
        x = to_dev(si.uniform_field_vector(FIELD, n, si.stream_seed(3, 0, 0)))
        plan = Plan(FIELD, LOG2N)
        out = torch.empty_like(x)
        work = plan.workspace(x)
        stream = torch.cuda.current_stream(dev)
        for _ in range(args.warmup):
            plan.forward(x, out)
        torch.cuda.synchronize()
        per = [ntt_profile_passes(plan.handle, 0, x, out, work, stream) for _ in range(args.steps)]
        pass_ms = [sum(p[k] for p in per) / len(per) for k in range(len(per[0]))]
        print(json.dumps({"forward_passes_ms_mean": pass_ms, "avg_launch_ms": sum(pass_ms) / len(pass_ms),
                          "warmup": args.warmup, "steps": args.steps}), flush=True)
        print(f"[bench] {args.warmup}+{args.steps} forward NTTs at 2^{LOG2N} done", file=sys.stderr, flush=True)
        return 0

    print(f"[bench] generating inputs n=2^{LOG2N}", file=sys.stderr, flush=True)
    host = [si.uniform_field_vector(FIELD, n, si.stream_seed(3, 0, v)) for v in range(3)]
    A, B, C = (to_dev(h) for h in host)
    H = torch.empty_like(A)
    plan = Plan(FIELD, LOG2N)
    stream = torch.cuda.current_stream(dev)

    # --- the step: quotient chain (7 transforms) ---
    print("[bench] warmup", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        plan.quotient(A, B, C, H)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        plan.quotient(A, B, C, H)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = ev0.elapsed_time(ev1) / args.steps
    value = 7 * n / (ms_per_step * 1e-3)

    # --- single forward NTT at 2^24 (median of 10 after 3 warm-ups) ---
    out = torch.empty_like(A)
    for _ in range(3):
        plan.forward(A, out)
    fwd_ms = []
    for _ in range(10):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        plan.forward(A, out)
        e1.record(stream)
        torch.cuda.synchronize()
        fwd_ms.append(e0.elapsed_time(e1))
    fwd_med = statistics.median(fwd_ms)

    # --- dominant kernel: per-pass HIP events on the launch stream ---
    work = plan.workspace(A)
    per_pass = [ntt_profile_passes(plan.handle, 0, A, out, work, stream) for _ in range(5)]
    npass = len(per_pass[0])
    pass_ms = [statistics.median(p[k] for p in per_pass) for k in range(npass)]
    avg_pass_ms = sum(pass_ms) / npass
    log_r = LOG2N // npass
    mads_per_launch = (n // 2) * log_r * MADS_PER_FFMUL  # butterflies in one pass x MADs per FF_mul
    achieved = mads_per_launch / (avg_pass_ms * 1e-3)
    khash = kernel_hash()
    traffic = traffic_from_profile(khash)
    valu = valu_from_profile(khash)
    print("[bench] micro-benchmarks (measured peaks)", file=sys.stderr, flush=True)
    peaks = peaks_leg(dev)
    mad_measured = peaks["mad_u64_u32"]["per_s"]
    roofline = {
        "bound": "alu",
        "kernel": f"ntt_pass_kernel<Bls12_381Fr, LOG_R={log_r}, LOG_TILE={plan.opts['log2_tile'] or 10}, "
                  f"LOG_E={plan.opts['log2_radix'] or 2}>",
        "achieved": achieved / 1e12,
        "peak": PEAK_MAD_PER_S / 1e12,
        "unit": "T MAD/s",
        "frac": achieved / PEAK_MAD_PER_S,
        "peak_derivation": "256 CU x 4 SIMD x 16 lanes x 2.4 GHz: one v_mad_u64_u32 per lane per cycle",
        "measured_peak": mad_measured / 1e12,
        "frac_of_measured_peak": achieved / mad_measured,
        "traffic": traffic,
        "avg_launch_ms": avg_pass_ms,
        "pass_ms": pass_ms,
        "algorithmic_mads_per_launch": mads_per_launch,
        "hbm_gbs_min_traffic": (2 * n * 32 + (n * 32 if npass > 1 else 0)) / (avg_pass_ms * 1e-3) / 1e9,
        # the same kernel against the VALU issue peak (every wave64 VALU
        # instruction is 64 lane operations): how busy the kernel keeps the
        # units the MAD roofline is drawn on, counted instructions / time
        "valu_issue_frac": (valu * 64 / (avg_pass_ms * 1e-3) / PEAK_MAD_PER_S) if valu else None,
        "kernel_source_hash": khash,
    }

    result = {
        "metric": "Fr255 NTT elements/s at n=2^24",
        "value": value,
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "wall_s_timed": wall,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "groth16 quotient chain, n=2^24, BLS12-381 Fr (7 NTTs + pointwise), "
                               "uniform random A, B, C from seed 3",
                   "field": FIELD, "log2n": LOG2N, "transforms_per_step": 7},
        "forward_ntt_2e24": {"ms_median": fwd_med, "elements_per_s": n / (fwd_med * 1e-3), "passes": npass},
        "roofline": roofline,
        "measured_peaks": peaks["summary"],
    }
    if not args.no_batch:
        print("[bench] batched vs per-launch (64 jobs)", file=sys.stderr, flush=True)
        result["batched"] = batch_leg(dev)
    if not args.no_serve:
        print("[bench] serving (Poisson quotient jobs)", file=sys.stderr, flush=True)
        result["serving"] = serve_leg(dev)
    result["small_configs"] = small_configs_leg(dev)
    if not args.no_pipeline:
        print("[bench] host-resident quotient pipeline", file=sys.stderr, flush=True)
        result["host_pipeline"] = host_pipeline_leg(dev)
    if not args.no_msm:
        print("[bench] MSM (BLS12-381 G1, n = 2^20)", file=sys.stderr, flush=True)
        result["msm"] = msm_leg(dev)
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        cb = cpu_baseline(host[0])
        result["cpu_baseline"] = cb
        result["gpu_over_cpu_forward"] = result["forward_ntt_2e24"]["elements_per_s"] / cb["value"]
        result["cpu_one_core"] = cpu_one_core()
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
