"""ntt_forward_noalloc (the entry point that allocates nothing: its
workspace is a fixed device array of the library) against ntt_forward,
through the C ABI, on two calls in a row, the second with a smaller input."""
import numpy as np
import pytest

import seeded_inputs as si
from tests.gpu_util import first_mismatch, to_dev, to_host

pytestmark = pytest.mark.gpu


def _fwd_both(plan, x, cuda):
    import torch

    from paper_2509_22684_amd import _lib

    dx = to_dev(x, cuda)
    want = torch.empty_like(dx)
    _lib.ntt_forward(plan.handle, dx, want, plan.workspace(dx))
    got = torch.empty_like(dx)
    _lib.ntt_forward_noalloc(plan.handle, dx, got)
    inplace = dx.clone()
    _lib.ntt_forward_noalloc(plan.handle, inplace, inplace)
    torch.cuda.synchronize()
    return to_host(got), to_host(inplace), to_host(want)


@pytest.mark.parametrize("field", ["bls12_381_fr", "bn254_fr"])
def test_noalloc_forward_equals_forward_two_calls(cuda, field):
    from paper_2509_22684_amd import Plan

    print(f"\n[no_alloc] {field}: 2^20 then 2^14", flush=True)
    for log2n, seed in ((20, 31), (14, 32)):  # the full workspace, then a smaller one
        plan = Plan(field, log2n)
        assert plan.passes >= 2  # the workspace is in use
        x = si.uniform_field_vector(field, 1 << log2n, si.stream_seed(seed, 0, 0))
        got, inplace, want = _fwd_both(plan, x, cuda)
        for g in (got, inplace):
            nbad, first = first_mismatch(g, want)
            assert nbad == 0, f"{field} 2^{log2n}: {nbad} mismatches, first at {first}"


def test_noalloc_single_pass_and_oversize(cuda):
    """A single-pass plan needs no workspace; a plan whose workspace exceeds
    the fixed one is refused before anything is launched."""
    from paper_2509_22684_amd import Plan, ZkError, _lib

    plan = Plan("bls12_381_fr", 10)
    x = si.uniform_field_vector("bls12_381_fr", 1 << 10, si.stream_seed(33, 0, 0))
    got, inplace, want = _fwd_both(plan, x, cuda)
    assert np.array_equal(got, want) and np.array_equal(inplace, want)
    big = Plan("bls12_381_fr", 21)
    dx = to_dev(np.zeros((1 << 21, 8), dtype=np.uint32), cuda)
    with pytest.raises(ZkError) as e:
        _lib.ntt_forward_noalloc(big.handle, dx, dx)
    assert e.value.code == -2 and "2^20" in str(e.value)
