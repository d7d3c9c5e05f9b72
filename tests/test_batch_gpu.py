"""GPU parity of the persistent batched launch.

Workload: 64 independent forward NTTs, log2 n uniform in [10, 18], 48 on
BLS12-381 Fr and 16 on BN254 Fr (seeded_inputs.batch_jobs).  Every job's
output must equal the oracle and its stand-alone ntt_forward result byte for
byte, for the graph replay (several replays with other GPU work between
them), the direct launch and the one-shot call.  The error path of the
bounded dependency wait is forced from the host.
"""
import numpy as np
import pytest

import seeded_inputs as si
from oracle import coracle
from tests.gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c4(cuda):
    from paper_2509_22684_amd import Plan

    jobs = si.batch_jobs()
    plans = {}
    inputs, want = [], []
    for jb in jobs:
        key = (jb.field, jb.log2n)
        if key not in plans:
            plans[key] = Plan(jb.field, jb.log2n)
        x = si.uniform_field_vector(jb.field, 1 << jb.log2n, jb.seed)
        inputs.append(x)
        want.append(coracle.transform(jb.field, "forward", x))
    return jobs, plans, inputs, want


def _fresh_bufs(inputs, cuda):
    return [to_dev(x, cuda) for x in inputs]


def _reset(bufs, inputs):
    import torch

    for b, x in zip(bufs, inputs):
        b.copy_(torch.from_numpy(x.view(np.int32)))


def _check_all(bufs, want, what):
    for k, (b, w) in enumerate(zip(bufs, want)):
        got = to_host(b)
        assert np.array_equal(got, w), f"{what}: job {k} differs"


def test_workload_shape(c4):
    jobs = c4[0]
    assert len(jobs) == 64
    assert sum(j.field == "bn254_fr" for j in jobs) == 16
    assert all(10 <= j.log2n <= 18 for j in jobs)


def test_batch_graph_matches_oracle_and_per_launch(c4, cuda):
    import torch

    from paper_2509_22684_amd import Batch

    jobs, plans, inputs, want = c4
    job_plans = [plans[(j.field, j.log2n)] for j in jobs]
    bufs = _fresh_bufs(inputs, cuda)
    batch = Batch(job_plans, bufs)
    assert batch.items > 64 and batch.grid > 0
    batch.launch()
    torch.cuda.synchronize()
    assert batch.status() == 0
    _check_all(bufs, want, "graph launch")
    # per-launch reference path, byte-identical
    per = _fresh_bufs(inputs, cuda)
    for p, b in zip(job_plans, per):
        p.forward(b, out=b)
    torch.cuda.synchronize()
    for k, (a, b) in enumerate(zip(bufs, per)):
        assert torch.equal(a, b), f"job {k}: batch and per-launch differ"
    # replays with unrelated GPU work in between
    for rep in range(3):
        _reset(bufs, inputs)
        junk = torch.randint(0, 1 << 30, (1 << 20, 8), dtype=torch.int32, device=cuda)
        job_plans[0].forward(junk[: job_plans[0].n].contiguous())
        torch.cuda.synchronize()
        batch.launch()
        torch.cuda.synchronize()
        assert batch.status() == 0
        _check_all(bufs, want, f"graph replay {rep}")
    # direct launch without the graph
    _reset(bufs, inputs)
    batch.launch_eager()
    torch.cuda.synchronize()
    assert batch.status() == 0
    _check_all(bufs, want, "eager launch")
    batch.close()


def test_bench_batch_schedule_matches_oracle(c4, cuda):
    """The 64-job batch exactly as the benchmark builds and times it: plans
    on the tuned batchable schedules (pass depth and twiddle source from the
    tuning database), replayed from the graph several times, every job
    against the oracle; then the same jobs on the tuned stand-alone
    schedules, one launch sequence per job, byte-identical."""
    import torch

    from paper_2509_22684_amd import Batch, Plan
    from paper_2509_22684_amd.autotune import tuned_opts

    jobs, _, inputs, want = c4
    plans, solo = {}, {}
    for jb in jobs:
        key = (jb.field, jb.log2n)
        if key not in plans:
            plans[key] = Plan(jb.field, jb.log2n, **tuned_opts(jb.field, jb.log2n, batchable=True))
            solo[key] = Plan(jb.field, jb.log2n, **tuned_opts(jb.field, jb.log2n, batchable=False))
    bufs = _fresh_bufs(inputs, cuda)
    batch = Batch([plans[(j.field, j.log2n)] for j in jobs], bufs)
    for rep in range(3):
        _reset(bufs, inputs)
        batch.launch()
        torch.cuda.synchronize()
        assert batch.status() == 0
        _check_all(bufs, want, f"tuned batch replay {rep}")
    per = _fresh_bufs(inputs, cuda)
    for j, b in zip(jobs, per):
        solo[(j.field, j.log2n)].forward(b, out=b)
    torch.cuda.synchronize()
    _check_all(per, want, "tuned per-launch")
    batch.close()


def test_batch_one_shot(c4, cuda):
    import torch

    from paper_2509_22684_amd import ntt_batch_forward, ntt_batch_workspace_bytes

    jobs, plans, inputs, want = c4
    job_plans = [plans[(j.field, j.log2n)] for j in jobs[:20]]
    bufs = _fresh_bufs(inputs[:20], cuda)
    nb = ntt_batch_workspace_bytes(job_plans)
    work = torch.empty((nb + 31) // 32, 8, dtype=torch.int32, device=cuda)
    ntt_batch_forward(job_plans, bufs, work)
    _check_all(bufs, want[:20], "one-shot")


def test_forced_dependency_timeout_reports_error_and_recovers(c4, cuda):
    """Spin limit 0 makes every dependency wait fail at once: the kernel exits
    early and the status says so; with the limit restored the same batch
    computes correct results again."""
    import torch

    from paper_2509_22684_amd import Batch

    jobs, plans, inputs, want = c4
    sel = [k for k, j in enumerate(jobs) if j.log2n >= 14][:8]
    job_plans = [plans[(jobs[k].field, jobs[k].log2n)] for k in sel]
    ins = [inputs[k] for k in sel]
    bufs = _fresh_bufs(ins, cuda)
    batch = Batch(job_plans, bufs)
    batch.set_spin_limit(0)
    batch.launch()
    torch.cuda.synchronize()
    assert batch.status() == -4
    batch.set_spin_limit(1 << 22)
    _reset(bufs, ins)
    batch.launch()
    torch.cuda.synchronize()
    assert batch.status() == 0
    _check_all(bufs, [want[k] for k in sel], "after recovery")


def test_eager_batch_status_from_host_and_recovery(c4, cuda):
    """A batch without a graph uploads its work list on its first launch's
    stream and copies its error word back on the launch stream: a spin limit
    set before the first launch (still in the host image) makes the launch
    fail and the status, read from host memory, says so; the limit restored
    on the device, the next launch is correct.  A batch destroyed before any
    launch frees its pending upload."""
    import torch

    from paper_2509_22684_amd._lib import (ntt_batch_create_jobs, ntt_batch_destroy, ntt_batch_launch_eager,
                                           ntt_batch_set_spin_limit, ntt_batch_status, ntt_workspace_bytes)

    jobs, plans, inputs, want = c4
    sel = [k for k, j in enumerate(jobs) if j.log2n >= 14][:8]
    job_plans = [plans[(jobs[k].field, jobs[k].log2n)] for k in sel]
    ins = [inputs[k] for k in sel]
    bufs = _fresh_bufs(ins, cuda)
    # every job its own workspace (jobs of one batch run concurrently)
    works = [torch.empty(max(1, ntt_workspace_bytes(p.handle) // 4), dtype=torch.int32, device=b.device)
             for p, b in zip(job_plans, bufs)]
    specs = [dict(plan=p, op="forward", out=b, work=w, **{"in": b}) for p, b, w in zip(job_plans, bufs, works)]
    ntt_batch_destroy(ntt_batch_create_jobs(specs))  # never launched
    h = ntt_batch_create_jobs(specs)
    try:
        ntt_batch_set_spin_limit(h, 0)
        ntt_batch_launch_eager(h)
        torch.cuda.synchronize()
        assert ntt_batch_status(h) == -4
        ntt_batch_set_spin_limit(h, 1 << 22)
        _reset(bufs, ins)
        ntt_batch_launch_eager(h)
        torch.cuda.synchronize()
        assert ntt_batch_status(h) == 0
    finally:
        ntt_batch_destroy(h)
    _check_all(bufs, [want[k] for k in sel], "eager after recovery")


def test_direct_batch_matches_oracle(c4, cuda):
    """ZK_BATCH_DIRECT: every job of the 64-job workload as pass launches
    (equal plans grouped, every other job a group of its own), no persistent
    kernel: byte-identical to the oracle."""
    import torch

    from paper_2509_22684_amd._lib import (lib, ntt_batch_create_jobs, ntt_batch_destroy, ntt_batch_launch_eager,
                                           ntt_batch_status, ntt_workspace_bytes)

    jobs, plans, inputs, want = c4
    job_plans = [plans[(j.field, j.log2n)] for j in jobs]
    bufs = _fresh_bufs(inputs, cuda)
    works = [torch.empty(max(1, ntt_workspace_bytes(p.handle) // 4), dtype=torch.int32, device=b.device)
             for p, b in zip(job_plans, bufs)]
    specs = [dict(plan=p, op="forward", out=b, work=w, **{"in": b}) for p, b, w in zip(job_plans, bufs, works)]
    h = ntt_batch_create_jobs(specs, direct=True)
    try:
        assert lib().ntt_batch_items(h) == 0
        ntt_batch_launch_eager(h)
        torch.cuda.synchronize()
        assert ntt_batch_status(h) == 0
    finally:
        ntt_batch_destroy(h)
    _check_all(bufs, want, "direct")


def test_batch_rejects_unsupported_jobs(cuda):
    from paper_2509_22684_amd import Batch, Plan, ZkError

    # a 2-point transform has no radix-4 round
    tiny = Plan("bls12_381_fr", 1)
    buf = to_dev(si.uniform_field_vector("bls12_381_fr", 2, 1), cuda)
    with pytest.raises(ZkError) as e:
        Batch([tiny], [buf])
    assert e.value.code == -2
    # six global passes of 2^4 points exceed the batch's four
    deep = Plan("bls12_381_fr", 24, log2_pass_radix=4)
    assert deep.passes == 6
    big = torch_empty_fe(1 << 24, cuda)
    with pytest.raises(ZkError) as e:
        Batch([deep], [big])
    assert e.value.code == -2


def torch_empty_fe(n, cuda):
    import torch

    return torch.empty(n, 8, dtype=torch.int32, device=cuda)


@pytest.mark.parametrize("log2n", [2, 3, 5, 8, 9, 11])
def test_batch_small_jobs(cuda, log2n):
    """Jobs below one 2^11 tile run as single-pass tiles with fewer threads
    than the workgroup; mixed with a multi-pass job they all equal the
    oracle."""
    import torch

    from paper_2509_22684_amd import Batch, Plan

    cases = [("bls12_381_fr", log2n), ("bn254_fr", log2n), ("bls12_381_fr", 13)]
    ins = [si.uniform_field_vector(f, 1 << L, si.stream_seed(41, L, k)) for k, (f, L) in enumerate(cases)]
    want = [coracle.transform(f, "forward", x) for (f, _), x in zip(cases, ins)]
    plans = [Plan(f, L) for f, L in cases]
    bufs = _fresh_bufs(ins, cuda)
    batch = Batch(plans, bufs)
    batch.launch()
    torch.cuda.synchronize()
    assert batch.status() == 0
    _check_all(bufs, want, f"small jobs 2^{log2n}")
    batch.close()


@pytest.mark.parametrize("opts", [dict(log2_radix=1), dict(log2_radix=3), dict(log2_pass_radix=6, twiddle_mode=2),
                                  dict(log2_pass_radix=7, twiddle_mode=1), dict(log2_tile=8, log2_radix=1)])
def test_batch_other_schedules(cuda, opts):
    """Plans built with other schedules batch too: the batch kernel runs each
    plan's own pass split and twiddle source, so every job still equals the
    oracle."""
    import torch

    from paper_2509_22684_amd import Batch, Plan

    cases = [("bls12_381_fr", 10), ("bn254_fr", 12), ("bls12_381_fr", 16), ("bls12_381_fr", 18), ("bn254_fr", 18)]
    ins = [si.uniform_field_vector(f, 1 << L, si.stream_seed(31, L, k)) for k, (f, L) in enumerate(cases)]
    want = [coracle.transform(f, "forward", x) for (f, _), x in zip(cases, ins)]
    job_plans = [Plan(f, L, **opts) for f, L in cases]
    bufs = _fresh_bufs(ins, cuda)
    batch = Batch(job_plans, bufs)
    batch.launch()
    torch.cuda.synchronize()
    assert batch.status() == 0
    _check_all(bufs, want, f"batch {opts}")
    batch.close()
    for p in job_plans:
        p.close()


@pytest.mark.parametrize("queues", [1, 3, 8])
def test_batch_queue_counts(c4, cuda, queues):
    """Any number of work queues per field gives the same bytes (one queue:
    every job of a field on one XCD; more: spread over the XCDs)."""
    import torch

    from paper_2509_22684_amd import Batch

    jobs, plans, inputs, want = c4
    job_plans = [plans[(j.field, j.log2n)] for j in jobs]
    bufs = _fresh_bufs(inputs, cuda)
    batch = Batch(job_plans, bufs, queues=queues)
    batch.launch()
    torch.cuda.synchronize()
    assert batch.status() == 0
    _check_all(bufs, want, f"{queues} queues per field")
    batch.close()


@pytest.mark.parametrize("cases", [
    [("bls12_381_fr", 20)],
    [("bls12_381_fr", 20), ("bls12_381_fr", 12), ("bls12_381_fr", 11), ("bn254_fr", 19), ("bn254_fr", 14)],
    [("bn254_fr", 18), ("bn254_fr", 18), ("bls12_381_fr", 10)],
])
def test_batch_large_jobs_run_direct(cuda, cases):
    """Jobs that would be the critical path on one XCD run as grouped pass
    launches on side streams, beside the persistent kernel's XCD-local jobs;
    all equal the oracle, on two graph replays."""
    import torch

    from paper_2509_22684_amd import Batch, Plan

    ins = [si.uniform_field_vector(f, 1 << L, si.stream_seed(51, L, k)) for k, (f, L) in enumerate(cases)]
    want = [coracle.transform(f, "forward", x) for (f, _), x in zip(cases, ins)]
    plans = [Plan(f, L) for f, L in cases]
    bufs = _fresh_bufs(ins, cuda)
    batch = Batch(plans, bufs)
    for rep in range(2):
        if rep:
            _reset(bufs, ins)
        batch.launch()
        torch.cuda.synchronize()
        assert batch.status() == 0
        _check_all(bufs, want, f"large jobs {cases} launch {rep}")
    batch.close()


def test_batch_three_fields(cuda):
    """BLS12-381, BN254 and BLS12-377 jobs of several sizes in one batch, each
    field drained by its own loop of the persistent kernel, plus a pointwise
    quotient job: all equal the oracle."""
    import torch

    from paper_2509_22684_amd import Plan, ntt_batch_create_jobs, ntt_batch_destroy, ntt_batch_launch_eager, \
        ntt_batch_status

    cases = [("bls12_377_fr", 12), ("bn254_fr", 13), ("bls12_381_fr", 11), ("bls12_377_fr", 16),
             ("bls12_377_fr", 10), ("bn254_fr", 15), ("bls12_381_fr", 14), ("bls12_377_fr", 5)]
    ins = [si.uniform_field_vector(f, 1 << L, si.stream_seed(61, L, k)) for k, (f, L) in enumerate(cases)]
    plans = [Plan(f, L) for f, L in cases]
    bufs = _fresh_bufs(ins, cuda)
    works = [p.workspace(b) for p, b in zip(plans, bufs)]
    # and a pointwise job on BLS12-377 Fr
    pw_in = [si.uniform_field_vector("bls12_377_fr", 1 << 12, si.stream_seed(62, 12, v)) for v in range(3)]
    pw_dev = _fresh_bufs(pw_in, cuda)
    pw_out = torch.empty_like(pw_dev[0])
    jobs = [dict(plan=p, op="forward", out=b, work=w, **{"in": b}) for p, b, w in zip(plans, bufs, works)]
    jobs.append(dict(plan=plans[0], op="quotient_pointwise", in2=pw_dev[1], in3=pw_dev[2], out=pw_out,
                     **{"in": pw_dev[0]}))
    h = ntt_batch_create_jobs(jobs)
    ntt_batch_launch_eager(h)
    torch.cuda.synchronize()
    assert ntt_batch_status(h) == 0
    ntt_batch_destroy(h)
    _check_all(bufs, [coracle.transform(f, "forward", x) for (f, _), x in zip(cases, ins)], "three fields")
    from oracle import ref

    F = ref.FIELDS["bls12_377_fr"]
    n = 1 << 12
    a, b_, c = (F.from_mont(si.limbs_to_ints(v)) for v in pw_in)
    zinv = pow(pow(F.generator, n, F.p) - 1, -1, F.p)
    want = F.to_mont([(x * y - z) * zinv % F.p for x, y, z in zip(a, b_, c)])
    assert si.limbs_to_ints(to_host(pw_out)) == want


def test_empty_batch(cuda):
    """A batch of no jobs launches (only the counter reset runs) and reports
    success."""
    import torch

    from paper_2509_22684_amd import ntt_batch_create_jobs, ntt_batch_destroy, ntt_batch_launch, ntt_batch_status

    h = ntt_batch_create_jobs([], graph=True)
    ntt_batch_launch(h)
    torch.cuda.synchronize()
    assert ntt_batch_status(h) == 0
    ntt_batch_destroy(h)


@pytest.mark.parametrize("log2n", [17, 19])
def test_batch_grouped_launches_every_kind(cuda, log2n):
    """Transforms of equal plans and kind form groups; a group that fills the
    chip runs as one grouped launch per pass (workgroup b of a launch takes a
    tile of job b / tiles-per-job).  Every kind, in place and
    out of place, with two plans built separately for the same size, next to
    small jobs in the persistent kernel: all equal the oracle on two graph
    replays, and the grouped jobs leave the persistent kernel's queues."""
    import torch

    from oracle import ref
    from paper_2509_22684_amd import Plan, ntt_batch_create_jobs, ntt_batch_destroy, ntt_batch_launch, \
        ntt_batch_status, lib

    field = "bls12_381_fr"
    n = 1 << log2n
    plan_a, plan_b = Plan(field, log2n), Plan(field, log2n)  # equal schedules, separate tables
    kinds = ["forward", "inverse", "coset_forward", "coset_inverse", "inverse_to_coset"]
    jobs, checks = [], []
    for k, kind in enumerate(kinds):
        for m in range(8):  # eight jobs of 2^17 fill one round of pass tiles over the chip
            x = si.uniform_field_vector(field, n, si.stream_seed(81, log2n, 8 * k + m))
            plan = plan_a if m != 1 else plan_b
            src = to_dev(x, cuda)
            dst = src if m == 0 else torch.empty_like(src)  # job 0 of each kind in place
            work = torch.empty_like(src)
            jobs.append(dict(plan=plan, op=kind, out=dst, work=work, **{"in": src}))
            checks.append((kind, x, dst))
    small = [("bn254_fr", 10), ("bls12_381_fr", 12), ("bls12_377_fr", 11)]
    small_plans = [Plan(f, L) for f, L in small]
    small_in = [si.uniform_field_vector(f, 1 << L, si.stream_seed(82, L, i)) for i, (f, L) in enumerate(small)]
    small_bufs = [to_dev(x, cuda) for x in small_in]
    for p, b in zip(small_plans, small_bufs):
        jobs.append(dict(plan=p, op="forward", out=b, work=p.workspace(b), **{"in": b}))
    h = ntt_batch_create_jobs(jobs, graph=True)
    # only the small jobs' tiles stay in the persistent kernel's queues (the
    # batch tile holds min(n, 2^11) elements)
    from paper_2509_22684_amd import ntt_plan_passes

    small_items = sum(ntt_plan_passes(p.handle) * max(1, (1 << L) >> 11) for p, (_, L) in zip(small_plans, small))
    assert lib().ntt_batch_items(h) == small_items
    F = ref.FIELDS[field]
    gpow = [pow(F.generator, j, F.p) for j in range(n)]
    want = []
    for kind, x, _ in checks:
        if kind == "inverse_to_coset":
            inv = si.limbs_to_ints(coracle.transform(field, "inverse", x))
            want.append(si.ints_to_limbs([v * g % F.p for v, g in zip(inv, gpow)]))
        else:
            want.append(coracle.transform(field, kind, x))
    small_want = [coracle.transform(f, "forward", x) for (f, _), x in zip(small, small_in)]
    for rep in range(2):
        for (kind, x, dst), job in zip(checks, jobs):
            job["in"].copy_(torch.from_numpy(x.view(np.int32)))
        for b, x in zip(small_bufs, small_in):
            b.copy_(torch.from_numpy(x.view(np.int32)))
        ntt_batch_launch(h)
        torch.cuda.synchronize()
        assert ntt_batch_status(h) == 0
        for (kind, _, dst), w in zip(checks, want):
            assert np.array_equal(to_host(dst), w), f"grouped {kind} 2^{log2n} launch {rep}"
        _check_all(small_bufs, small_want, f"small jobs beside groups, launch {rep}")
    ntt_batch_destroy(h)


@pytest.mark.parametrize("opts", [dict(twiddle_mode=2), dict(log2_pass_radix=6), dict(log2_radix=3),
                                  dict(log2_radix=1), dict(log2_pass_radix=7, twiddle_mode=2),
                                  dict(log2_tile=8, log2_radix=1)])
def test_batch_grouped_launches_other_schedules(cuda, opts):
    """Grouped launches run the plans' pass split, tile and twiddle source
    with radix-4 register rounds whatever the plans' register radix; eight
    2^17 jobs of one schedule form a group that fills the chip, and every job
    equals the oracle."""
    import torch

    from paper_2509_22684_amd import Batch, Plan, lib

    field, log2n = "bn254_fr", 17
    plan = Plan(field, log2n, **opts)
    ins = [si.uniform_field_vector(field, 1 << log2n, si.stream_seed(83, log2n, k)) for k in range(8)]
    want = [coracle.transform(field, "forward", x) for x in ins]
    bufs = _fresh_bufs(ins, cuda)
    batch = Batch([plan] * len(bufs), bufs)
    assert lib().ntt_batch_items(batch.handle) == 0  # the whole group runs as grouped launches
    batch.launch()
    torch.cuda.synchronize()
    assert batch.status() == 0
    _check_all(bufs, want, f"grouped {opts}")
    batch.close()
