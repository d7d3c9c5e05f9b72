"""GPU parity: every transform of the HIP library against the CPU oracle,
bit for bit, through the C ABI.

Inputs are seeded uniform field vectors (seeded_inputs); expected values come
from the C oracle (Barrett arithmetic, radix-2 textbook NTT), which the CPU
suite pins to the mathematics.
"""
import numpy as np
import pytest

import seeded_inputs as si
from oracle import coracle
from tests.gpu_util import first_mismatch, to_dev, to_host

pytestmark = pytest.mark.gpu

FIELDS = ["bls12_381_fr", "bn254_fr", "bls12_377_fr"]
KINDS = ["forward", "inverse", "coset_forward", "coset_inverse"]


def _plan(field, log2n, **kw):
    from paper_2509_22684_amd import Plan

    return Plan(field, log2n, **kw)


def _run(plan, kind, x, out=None):
    return getattr(plan, kind)(x, out=out)


def _check(got, want, what):
    nbad, first = first_mismatch(got, want)
    assert nbad == 0, f"{what}: {nbad} mismatching elements, first at {first}"


@pytest.mark.parametrize("field", FIELDS)
@pytest.mark.parametrize("log2n", list(range(0, 13)) + [13, 14, 16, 17, 19])
def test_all_kinds_small_and_medium(cuda, field, log2n):
    n = 1 << log2n
    x = si.uniform_field_vector(field, n, si.stream_seed(100 + log2n, 0, 0))
    plan = _plan(field, log2n)
    dx = to_dev(x, cuda)
    for kind in KINDS:
        got = to_host(_run(plan, kind, dx))
        want = coracle.transform(field, kind, x)
        _check(got, want, f"{field} 2^{log2n} {kind}")
    assert np.array_equal(to_host(dx), x), "input was modified"


@pytest.mark.parametrize("field", FIELDS)
def test_size_2_20_all_kinds_and_round_trips(cuda, field):
    """Forward, inverse and coset transforms at n = 2^20 on one seeded vector;
    INTT(NTT(x)) = x and cosetINTT(cosetNTT(x)) = x on the GPU alone."""
    import torch

    log2n = 20
    x = si.uniform_field_vector(field, 1 << log2n, si.stream_seed(2, 0, 0))
    plan = _plan(field, log2n)
    dx = to_dev(x, cuda)
    outs = {}
    for kind in KINDS:
        outs[kind] = _run(plan, kind, dx)
        _check(to_host(outs[kind]), coracle.transform(field, kind, x), f"{field} 2^20 {kind}")
    assert torch.equal(plan.inverse(outs["forward"]), dx)
    assert torch.equal(plan.forward(outs["inverse"]), dx)
    assert torch.equal(plan.coset_inverse(outs["coset_forward"]), dx)
    assert torch.equal(plan.coset_forward(outs["coset_inverse"]), dx)


@pytest.mark.parametrize("radix", [1, 2])
@pytest.mark.parametrize("log2n", [1, 2, 3, 10, 12, 16, 19])
def test_register_radix_schedules_are_byte_identical(cuda, log2n, radix):
    """The radix-2 and radix-4 register schedules (log2_radix = 1, 2) give the
    same bytes as the default radix-8 schedule and the oracle."""
    field = "bls12_381_fr"
    x = si.uniform_field_vector(field, 1 << log2n, si.stream_seed(1, 0, 0))
    dx = to_dev(x, cuda)
    p8 = _plan(field, log2n)
    p2 = _plan(field, log2n, log2_radix=radix)
    want = coracle.transform(field, "forward", x)
    for kind in KINDS:
        a = to_host(_run(p8, kind, dx))
        b = to_host(_run(p2, kind, dx))
        assert np.array_equal(a, b), f"radix-2 and radix-8 differ for {kind}"
    _check(to_host(p2.forward(dx)), want, "radix-2 forward")


@pytest.mark.parametrize("log2n", [5, 11, 12, 18])
def test_in_place(cuda, log2n):
    field = "bls12_381_fr"
    x = si.uniform_field_vector(field, 1 << log2n, si.stream_seed(7, log2n, 0))
    plan = _plan(field, log2n)
    for kind in KINDS:
        d = to_dev(x, cuda)
        _run(plan, kind, d, out=d)
        _check(to_host(d), coracle.transform(field, kind, x), f"in-place {kind} 2^{log2n}")


def test_poisoned_outputs_are_fully_overwritten(cuda):
    import torch

    field, log2n = "bn254_fr", 15
    x = si.uniform_field_vector(field, 1 << log2n, 31)
    plan = _plan(field, log2n)
    dx = to_dev(x, cuda)
    out = torch.full_like(dx, -1)
    plan.forward(dx, out=out)
    _check(to_host(out), coracle.transform(field, "forward", x), "poisoned output")


@pytest.mark.parametrize("field", FIELDS)
@pytest.mark.parametrize("log2n", [0, 1, 2, 5, 9, 12, 15])
def test_quotient_small(cuda, field, log2n):
    n = 1 << log2n
    A, B, C = (si.uniform_field_vector(field, n, si.stream_seed(3, log2n, v)) for v in range(3))
    plan = _plan(field, log2n)
    got = to_host(plan.quotient(to_dev(A, cuda), to_dev(B, cuda), to_dev(C, cuda)))
    _check(got, coracle.quotient(field, A, B, C), f"quotient {field} 2^{log2n}")


@pytest.mark.parametrize("log2n", [19, pytest.param(22, marks=pytest.mark.slow)])
def test_quotient_forked_chains_three_passes(cuda, log2n):
    """Up to 2^22 quotient_poly runs A's and B's chains on forked streams;
    from 2^19 each transform takes three passes.  The forked three-pass
    path, which the serving baseline and the host pipeline time, against the
    oracle element by element."""
    from paper_2509_22684_amd import ntt_plan_passes

    field = "bls12_381_fr"
    n = 1 << log2n
    A, B, C = (si.uniform_field_vector(field, n, si.stream_seed(23, log2n, v)) for v in range(3))
    plan = _plan(field, log2n)
    assert ntt_plan_passes(plan.handle) == 3
    got = to_host(plan.quotient(to_dev(A, cuda), to_dev(B, cuda), to_dev(C, cuda)))
    _check(got, coracle.quotient(field, A, B, C), f"forked quotient 2^{log2n}")


@pytest.mark.parametrize("field,log2n", [("bls12_381_fr", 3), ("bn254_fr", 12), ("bls12_381_fr", 17)])
def test_quotient_stages_compose(cuda, field, log2n):
    """quotient_coset_evals x3, quotient_pointwise and the coset inverse give
    quotient_poly's bytes; each stage also matches its oracle definition."""
    import torch

    n = 1 << log2n
    A, B, C = (si.uniform_field_vector(field, n, si.stream_seed(13, log2n, v)) for v in range(3))
    plan = _plan(field, log2n)
    dA, dB, dC = (to_dev(v, cuda) for v in (A, B, C))
    ea = plan.coset_evals(dA)
    _check(to_host(ea), coracle.transform(field, "coset_forward", coracle.transform(field, "inverse", A)),
           "coset_evals(A)")
    eb = plan.coset_evals(dB)
    ec = dC.clone()
    plan.coset_evals(ec, out=ec)  # in place
    h = plan.pointwise(ea, eb, ec, out=ec)
    plan.coset_inverse(h, out=h)
    whole = plan.quotient(dA, dB, dC)
    torch.cuda.synchronize()
    assert torch.equal(h, whole)
    _check(to_host(h), coracle.quotient(field, A, B, C), "staged quotient")


def test_error_codes(cuda):
    import torch

    from paper_2509_22684_amd import ZkError, ntt_forward, ntt_plan_create

    with pytest.raises(ZkError) as e:
        ntt_plan_create("bls12_381_fr", 33)
    assert e.value.code == -2
    with pytest.raises(ZkError) as e:
        ntt_plan_create("bn254_fr", 29)
    assert e.value.code == -2
    with pytest.raises(ZkError) as e:
        ntt_plan_create("bls12_377_fr", 48)
    assert e.value.code == -2
    with pytest.raises(ZkError) as e:
        ntt_plan_create(4, 10)  # no such field
    assert e.value.code == -2
    for bad in (3, 10):  # pass depths without a kernel
        with pytest.raises(ZkError) as e:
            ntt_plan_create("bls12_381_fr", 20, log2_pass_radix=bad)
        assert e.value.code == -2
    plan = _plan("bls12_381_fr", 14)
    buf = torch.zeros(2 * plan.n + 8, 8, dtype=torch.int32, device=cuda)
    work = torch.zeros(plan.n, 8, dtype=torch.int32, device=cuda)
    with pytest.raises(ZkError) as e:  # misaligned input (32 bytes past an aligned base)
        ntt_forward(plan.handle, buf[1:], buf[plan.n + 8:], work)
    assert e.value.code == -1
    with pytest.raises(ZkError) as e:  # missing workspace
        ntt_forward(plan.handle, buf[:plan.n], buf[plan.n + 8:], None)
    assert e.value.code == -1


def test_overlapping_buffers_are_refused(cuda):
    """Aliasing is checked on byte ranges, not only base pointers."""
    import torch

    from paper_2509_22684_amd import ZkError, ntt_forward, quotient_poly, quotient_workspace_bytes

    plan = _plan("bls12_381_fr", 14)
    n = plan.n
    big = torch.zeros(4 * n + 64, 8, dtype=torch.int32, device=cuda)
    x, out = big[:n], big[n + 8:2 * n + 8]
    with pytest.raises(ZkError) as e:  # workspace starts inside the output
        ntt_forward(plan.handle, x, out, big[n + 16:])
    assert e.value.code == -1
    with pytest.raises(ZkError) as e:  # out overlaps in without being the same buffer
        ntt_forward(plan.handle, x, big[8:], big[2 * n + 16:])
    assert e.value.code == -1
    qw = torch.zeros(quotient_workspace_bytes(plan.handle) // 32 + 8, 8, dtype=torch.int32, device=cuda)
    A = big[:n]
    with pytest.raises(ZkError) as e:  # H overlaps A's tail
        quotient_poly(plan.handle, A, A, A, big[n - 8:], qw)
    assert e.value.code == -1


def test_validate_refused_under_capture(cuda):
    """ZK_FLAG_VALIDATE reads its count back to the host, so a call on a
    stream being captured is refused instead of breaking the capture."""
    import torch

    from paper_2509_22684_amd import Plan, ZkError

    plan = Plan("bls12_381_fr", 10, flags=1)
    x = to_dev(si.uniform_field_vector("bls12_381_fr", 1 << 10, 6), cuda)
    y = torch.empty_like(x)
    s = torch.cuda.Stream(cuda)
    g = torch.cuda.CUDAGraph()
    raised = None
    with torch.cuda.graph(g, stream=s):
        try:
            plan.forward(x, y, stream=s)
        except ZkError as e:
            raised = e
    assert raised is not None and raised.code == -1 and "capture" in str(raised)


@pytest.mark.parametrize("log2n,opts", [(10, {}), (16, {}), (20, {}), (24, {}), (20, dict(twiddle_mode=2)),
                                        (18, dict(log2_pass_radix=6)), (21, dict(log2_tile=11))])
def test_plan_table_bytes_matches_the_plan(cuda, log2n, opts):
    """The host-side size query equals what the created plan holds."""
    from paper_2509_22684_amd import ntt_plan_device_bytes, ntt_plan_table_bytes

    plan = _plan("bls12_381_fr", log2n, **opts)
    assert ntt_plan_table_bytes("bls12_381_fr", log2n, **opts) == ntt_plan_device_bytes(plan.handle) > 0


def test_default_plan_runs_the_registered_tuned_schedule(cuda):
    """Plan() with zero options registers the tuning database for this device
    and resolves its schedule through it."""
    from paper_2509_22684_amd import _lib, ntt_plan_resolve_opts

    for log2n in (16, 20, 24):
        plan = _plan("bls12_381_fr", log2n)
        assert plan.opts == ntt_plan_resolve_opts("bls12_381_fr", log2n)
    assert _lib._tuning_loaded


def test_validate_flag_rejects_noncanonical(cuda):
    from paper_2509_22684_amd import Plan, ZkError

    field, log2n = "bls12_381_fr", 12
    x = si.uniform_field_vector(field, 1 << log2n, 5)
    bad = x.copy()
    bad[77] = np.frombuffer(si.MODULI[field].to_bytes(32, "little"), dtype="<u4")  # exactly p
    plan = Plan(field, log2n, flags=1)
    plan.forward(to_dev(x, cuda))  # canonical input passes
    with pytest.raises(ZkError) as e:
        plan.forward(to_dev(bad, cuda))
    assert e.value.code == -1


@pytest.mark.parametrize("opts", [dict(twiddle_mode=2), dict(log2_pass_radix=6), dict(log2_pass_radix=4),
                                  dict(log2_pass_radix=7, twiddle_mode=2), dict(log2_pass_radix=5),
                                  dict(log2_pass_radix=4, twiddle_mode=2), dict(log2_tile=10),
                                  dict(log2_tile=10, log2_pass_radix=7, twiddle_mode=2),
                                  dict(log2_tile=10, log2_radix=3), dict(log2_tile=10, log2_radix=1),
                                  dict(log2_pass_radix=8), dict(log2_pass_radix=9), dict(log2_pass_radix=9, log2_tile=11),
                                  dict(log2_pass_radix=9, twiddle_mode=2), dict(log2_pass_radix=9, log2_radix=3),
                                  dict(log2_pass_radix=9, log2_radix=1), dict(log2_tile=8, log2_radix=1),
                                  dict(log2_tile=8, log2_radix=2), dict(log2_tile=8, log2_radix=1, twiddle_mode=2),
                                  dict(log2_tile=8, log2_radix=2, log2_pass_radix=5)])
@pytest.mark.parametrize("log2n", [8, 9, 11, 12, 17, 18, 20])
def test_schedules_are_byte_identical(cuda, opts, log2n):
    """Every schedule the autotuner may pick (pass fusion depth, twiddle
    source) gives the oracle's bytes for all four transforms."""
    field = "bn254_fr" if log2n == 17 else "bls12_381_fr"
    x = si.uniform_field_vector(field, 1 << log2n, si.stream_seed(9, log2n, 0))
    dx = to_dev(x, cuda)
    plan = _plan(field, log2n, **opts)
    for kind in KINDS:
        _check(to_host(_run(plan, kind, dx)), coracle.transform(field, kind, x), f"{opts} {kind} 2^{log2n}")


@pytest.mark.parametrize("log2n", [10, 16, 22, 23])
def test_quotient_workspace_size(cuda, log2n):
    """Up to 2^22 the quotient runs A's and B's transforms on forked streams,
    each with its own transform workspace: the quotient workspace is two
    vectors plus three transform workspaces there, plus one above."""
    from paper_2509_22684_amd import ntt_workspace_bytes, quotient_workspace_bytes

    plan = _plan("bls12_381_fr", log2n)
    n = 1 << log2n
    ws = ntt_workspace_bytes(plan.handle)
    assert quotient_workspace_bytes(plan.handle) == 2 * n * 32 + (3 if log2n <= 22 else 1) * ws


def test_quotient_forked_chains_keep_stream_order(cuda):
    """The forked chains start only after earlier work on the caller's stream
    and finish before later work on it: two quotients on a side stream, with
    A overwritten in between and H copied out after each, both equal the
    oracle."""
    import torch

    field, log2n = "bn254_fr", 16
    n = 1 << log2n
    A1, A2, B, C = (si.uniform_field_vector(field, n, si.stream_seed(91, log2n, v)) for v in range(4))
    plan = _plan(field, log2n)
    dA, dB, dC = to_dev(A1, cuda), to_dev(B, cuda), to_dev(C, cuda)
    a2 = to_dev(A2, cuda)
    H = torch.empty_like(dA)
    s = torch.cuda.Stream(cuda)
    s.wait_stream(torch.cuda.current_stream(cuda))
    with torch.cuda.stream(s):
        plan.quotient(dA, dB, dC, H, stream=s)
        H1 = H.clone()
        dA.copy_(a2)
        plan.quotient(dA, dB, dC, H, stream=s)
        H2 = H.clone()
    s.synchronize()
    _check(to_host(H1), coracle.quotient(field, A1, B, C), "first quotient on a side stream")
    _check(to_host(H2), coracle.quotient(field, A2, B, C), "second quotient after A changed")


def test_quotient_one_plan_two_streams(cuda):
    """One plan, two quotients enqueued back to back on two streams with
    their own workspaces (the forked chains share the plan's side streams):
    both equal the oracle."""
    import torch

    from paper_2509_22684_amd import quotient_poly, quotient_workspace_bytes

    field, log2n = "bls12_381_fr", 14
    n = 1 << log2n
    plan = _plan(field, log2n)
    host = [[si.uniform_field_vector(field, n, si.stream_seed(93, j, v)) for v in range(3)] for j in range(2)]
    dev = [[to_dev(v, cuda) for v in h] for h in host]
    Hs = [torch.empty_like(dev[0][0]) for _ in range(2)]
    nb = quotient_workspace_bytes(plan.handle)
    works = [torch.empty((nb + 31) // 32, 8, dtype=torch.int32, device=cuda) for _ in range(2)]
    streams = [torch.cuda.Stream(cuda) for _ in range(2)]
    for s in streams:
        s.wait_stream(torch.cuda.current_stream(cuda))
    for j in range(2):
        quotient_poly(plan.handle, *dev[j], Hs[j], works[j], streams[j])
    for s in streams:
        s.synchronize()
    for j in range(2):
        _check(to_host(Hs[j]), coracle.quotient(field, *host[j]), f"quotient on stream {j}")
