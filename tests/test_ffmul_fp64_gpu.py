"""The FP64 multiplier (ZK_FLAG_FFMUL_FP64): the element-wise products of
both multipliers against the Montgomery product's definition on uniform and
boundary-valued inputs, and every transform kind of plans that run all their
products on it against the oracle, byte for byte."""
import numpy as np
import pytest

import seeded_inputs as si
from oracle import coracle, ref
from tests.gpu_util import first_mismatch, to_dev, to_host

pytestmark = pytest.mark.gpu

FIELDS = ["bls12_381_fr", "bn254_fr", "bls12_377_fr"]
KINDS = ["forward", "inverse", "coset_forward", "coset_inverse"]


@pytest.mark.parametrize("field", FIELDS)
@pytest.mark.parametrize("inputs", ["uniform", "boundary"])
def test_field_mul_both_variants_match_definition(cuda, field, inputs):
    import torch

    from paper_2509_22684_amd import zk_field_mul

    F = ref.FIELDS[field]
    n = 4096 + 37  # several workgroups and a ragged tail
    gen = si.uniform_field_vector if inputs == "uniform" else si.boundary_field_vector
    a = gen(field, n, si.stream_seed(61, n, 0))
    b = gen(field, n, si.stream_seed(61, n, 1))
    xs, ys = si.limbs_to_ints(a), si.limbs_to_ints(b)
    da, db = to_dev(a, cuda), to_dev(b, cuda)
    out = torch.empty_like(da)
    for variant, bits in ((0, 256), (1, 288)):
        zk_field_mul(field, variant, da, db, out)
        torch.cuda.synchronize()
        want = si.ints_to_limbs(ref.montgomery_product(F, xs, ys, bits))
        nbad, first = first_mismatch(to_host(out), want)
        assert nbad == 0, f"{field} variant {variant}: {nbad} mismatches, first at {first}"


@pytest.mark.parametrize("log2n", [0, 1, 2, 5, 8, 10, 11, 12, 16, 17, 20])
def test_fp64_plan_transforms_match_oracle(cuda, log2n):
    from paper_2509_22684_amd import Plan, ZK_FLAG_FFMUL_FP64

    field = "bls12_381_fr"
    x = si.uniform_field_vector(field, 1 << log2n, si.stream_seed(62, log2n, 0))
    plan = Plan(field, log2n, flags=ZK_FLAG_FFMUL_FP64)
    assert plan.opts["log2_radix"] == 2
    dx = to_dev(x, cuda)
    for kind in KINDS:
        got = to_host(getattr(plan, kind)(dx))
        nbad, first = first_mismatch(got, coracle.transform(field, kind, x))
        assert nbad == 0, f"fp64 {kind} 2^{log2n}: {nbad} mismatches, first at {first}"


@pytest.mark.parametrize("opts", [dict(twiddle_mode=2), dict(log2_tile=8), dict(log2_pass_radix=6),
                                  dict(log2_tile=11)])
def test_fp64_plan_other_schedules_and_boundary_inputs(cuda, opts):
    from paper_2509_22684_amd import Plan, ZK_FLAG_FFMUL_FP64

    field, log2n = "bls12_381_fr", 14
    x = si.boundary_field_vector(field, 1 << log2n, si.stream_seed(63, log2n, 0))
    plan = Plan(field, log2n, flags=ZK_FLAG_FFMUL_FP64, **opts)
    dx = to_dev(x, cuda)
    for kind in KINDS:
        assert np.array_equal(to_host(getattr(plan, kind)(dx)), coracle.transform(field, kind, x)), (opts, kind)


def test_fp64_plan_refusals(cuda):
    import torch

    from paper_2509_22684_amd import Plan, ZK_FLAG_FFMUL_FP64, ZkError, ntt_plan_create

    with pytest.raises(ZkError) as e:
        ntt_plan_create("bn254_fr", 10, flags=ZK_FLAG_FFMUL_FP64)
    assert e.value.code == -2
    with pytest.raises(ZkError) as e:
        ntt_plan_create("bls12_381_fr", 10, log2_radix=1, flags=ZK_FLAG_FFMUL_FP64)
    assert e.value.code == -2
    plan = Plan("bls12_381_fr", 10, flags=ZK_FLAG_FFMUL_FP64)
    x = torch.zeros(1 << 10, 8, dtype=torch.int32, device=cuda)
    with pytest.raises(ZkError) as e:
        plan.quotient(x, x, x)
    assert e.value.code == -2
