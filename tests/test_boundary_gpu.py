"""GPU parity on inputs at the edges of the field: values 0, 1, p - 1, p - 2,
(p +- 1) / 2, 2^256 mod p, values within 2^64 of p or of 0, mixed with
uniform elements (seeded_inputs.boundary_field_vector).  Uniform inputs almost
never make a modular add, subtract or product land exactly on 0 or p, or
carry out of the top limb; these do.

Expected values come from the C oracle, and for constant and one-point
vectors also from closed forms that need no oracle: the transforms are
linear, so on raw Montgomery limbs the forward NTT of the constant vector c
is (n c mod p, 0, ..., 0), of c at index 0 it is c everywhere, and the inverse
of the constant c is (c, 0, ..., 0) (Section II-B, the NTT and its inverse).
"""
import numpy as np
import pytest

import seeded_inputs as si
from oracle import coracle
from tests.gpu_util import first_mismatch, to_dev, to_host

pytestmark = pytest.mark.gpu

FIELDS = ["bls12_381_fr", "bn254_fr", "bls12_377_fr"]
KINDS = ["forward", "inverse", "coset_forward", "coset_inverse"]


def _check(got, want, what):
    nbad, first = first_mismatch(got, want)
    assert nbad == 0, f"{what}: {nbad} mismatching elements, first at {first}"


def _const(c, n):
    return si.ints_to_limbs([c] * n)


def _delta0(c, n):
    return si.ints_to_limbs([c] + [0] * (n - 1))


@pytest.mark.parametrize("field", FIELDS)
@pytest.mark.parametrize("log2n", [1, 2, 4, 7, 10, 11, 12, 13, 16, 17, 18])
def test_boundary_inputs_all_kinds(cuda, field, log2n):
    from paper_2509_22684_amd import Plan

    x = si.boundary_field_vector(field, 1 << log2n, si.stream_seed(71, log2n, 0))
    plan = Plan(field, log2n)
    dx = to_dev(x, cuda)
    for kind in KINDS:
        got = to_host(getattr(plan, kind)(dx))
        _check(got, coracle.transform(field, kind, x), f"{field} 2^{log2n} {kind} boundary inputs")


@pytest.mark.parametrize("field", FIELDS)
@pytest.mark.parametrize("log2n", [3, 10, 13, 16])
def test_constant_and_one_point_vectors(cuda, field, log2n):
    from paper_2509_22684_amd import Plan

    p = si.MODULI[field]
    n = 1 << log2n
    n_inv = pow(n, -1, p)
    plan = Plan(field, log2n)
    for c in (p - 1, p - 2, 1, (p + 1) // 2, (1 << 256) % p):
        const = to_dev(_const(c, n), cuda)
        delta = to_dev(_delta0(c, n), cuda)
        zero_tail = [0] * (n - 1)
        assert si.limbs_to_ints(to_host(plan.forward(const))) == [n * c % p] + zero_tail, f"forward(const {c})"
        assert si.limbs_to_ints(to_host(plan.inverse(const))) == [c] + zero_tail, f"inverse(const {c})"
        assert si.limbs_to_ints(to_host(plan.coset_inverse(const))) == [c] + zero_tail, f"coset_inverse(const {c})"
        assert si.limbs_to_ints(to_host(plan.forward(delta))) == [c] * n, f"forward(delta {c})"
        assert si.limbs_to_ints(to_host(plan.coset_forward(delta))) == [c] * n, f"coset_forward(delta {c})"
        assert si.limbs_to_ints(to_host(plan.inverse(delta))) == [c * n_inv % p] * n, f"inverse(delta {c})"


@pytest.mark.parametrize("opts", [dict(log2_radix=1), dict(log2_radix=3), dict(log2_tile=11),
                                  dict(log2_pass_radix=4), dict(log2_pass_radix=6, twiddle_mode=2),
                                  dict(log2_pass_radix=7, twiddle_mode=1), dict(twiddle_mode=2),
                                  dict(log2_pass_radix=9, twiddle_mode=2)])
@pytest.mark.parametrize("log2n", [13, 16, 18])
def test_boundary_inputs_other_schedules(cuda, opts, log2n):
    from paper_2509_22684_amd import Plan

    field = "bls12_381_fr"
    x = si.boundary_field_vector(field, 1 << log2n, si.stream_seed(72, log2n, 1))
    plan = Plan(field, log2n, **opts)
    dx = to_dev(x, cuda)
    for kind in KINDS:
        got = to_host(getattr(plan, kind)(dx))
        _check(got, coracle.transform(field, kind, x), f"{opts} 2^{log2n} {kind} boundary inputs")


@pytest.mark.parametrize("field", FIELDS)
@pytest.mark.parametrize("log2n", [4, 10, 13])
def test_boundary_quotient(cuda, field, log2n):
    """The fused quotient chain and its split form (coset evaluations,
    pointwise step, coset inverse) on boundary inputs, against the oracle."""
    import torch

    from paper_2509_22684_amd import Plan, ntt_coset_inverse, quotient_coset_evals, quotient_pointwise

    n = 1 << log2n
    A, B, C = (si.boundary_field_vector(field, n, si.stream_seed(73, log2n, v)) for v in range(3))
    want = coracle.quotient(field, A, B, C)
    plan = Plan(field, log2n)
    dA, dB, dC = (to_dev(v, cuda) for v in (A, B, C))
    _check(to_host(plan.quotient(dA, dB, dC)), want, f"{field} 2^{log2n} quotient boundary inputs")
    work = plan.workspace(dA)
    s = torch.cuda.current_stream()
    for buf in (dA, dB, dC):
        quotient_coset_evals(plan.handle, buf, buf, work, s)
    quotient_pointwise(plan.handle, dA, dB, dC, dC, s)
    ntt_coset_inverse(plan.handle, dC, dC, work, s)
    torch.cuda.synchronize()
    _check(to_host(dC), want, f"{field} 2^{log2n} split quotient boundary inputs")


def test_boundary_batch(cuda):
    """One persistent batch holding every transform kind on boundary inputs,
    three fields, plus a pointwise job whose inputs include 0 and p - 1."""
    import torch

    from oracle import ref
    from paper_2509_22684_amd import Plan, ntt_batch_create_jobs, ntt_batch_destroy, ntt_batch_launch_eager, \
        ntt_batch_status

    cases = [("bls12_381_fr", 12, "forward"), ("bls12_381_fr", 14, "inverse"), ("bn254_fr", 13, "coset_forward"),
             ("bn254_fr", 11, "coset_inverse"), ("bls12_377_fr", 15, "forward"), ("bls12_377_fr", 9, "inverse"),
             ("bls12_381_fr", 5, "coset_forward"), ("bls12_381_fr", 17, "coset_inverse"), ("bn254_fr", 18, "forward")]
    ins = [si.boundary_field_vector(f, 1 << L, si.stream_seed(74, L, k)) for k, (f, L, _) in enumerate(cases)]
    plans = [Plan(f, L) for f, L, _ in cases]
    bufs = [to_dev(x, cuda) for x in ins]
    outs = [torch.empty_like(b) for b in bufs]
    works = [p.workspace(b) for p, b in zip(plans, bufs)]
    jobs = [dict(plan=p, op=k, out=o, work=w, **{"in": b})
            for p, (_, _, k), b, o, w in zip(plans, cases, bufs, outs, works)]
    field, log2n = "bls12_381_fr", 12
    pw_in = [si.boundary_field_vector(field, 1 << log2n, si.stream_seed(75, log2n, v)) for v in range(3)]
    pw_dev = [to_dev(v, cuda) for v in pw_in]
    pw_out = torch.empty_like(pw_dev[0])
    jobs.append(dict(plan=plans[0], op="quotient_pointwise", in2=pw_dev[1], in3=pw_dev[2], out=pw_out,
                     **{"in": pw_dev[0]}))
    h = ntt_batch_create_jobs(jobs)
    ntt_batch_launch_eager(h)
    torch.cuda.synchronize()
    assert ntt_batch_status(h) == 0
    ntt_batch_destroy(h)
    for (f, L, k), x, o in zip(cases, ins, outs):
        _check(to_host(o), coracle.transform(f, k, x), f"batch {f} 2^{L} {k} boundary inputs")
    F = ref.FIELDS[field]
    n = 1 << log2n
    a, b_, c = (F.from_mont(si.limbs_to_ints(v)) for v in pw_in)
    zinv = pow(pow(F.generator, n, F.p) - 1, -1, F.p)
    want = F.to_mont([(x * y - z) * zinv % F.p for x, y, z in zip(a, b_, c)])
    assert si.limbs_to_ints(to_host(pw_out)) == want
