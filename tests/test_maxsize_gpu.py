"""Maximum-size parity (opt-in: set ZKNTT_MAXSIZE=1; about three minutes,
most of it generating and checking 2^28-element inputs on the host).

n = 2^28 is the largest transform BN254 Fr has (2-adicity 28) and, for
BLS12-381 Fr, the largest size tested: a 2^32-point BLS12-381 transform would
need 128 GiB per vector, more than its input, output, workspace and tables
leave room for in one GPU's 288 GB.  At these sizes the oracle checks
sampled outputs one by one (Horner's rule, A_i = a(w^i), no NTT code), and
two properties that hold at any size are checked in full on the device:
INTT(NTT(x)) = x, and the coset round trip.
"""
import os

import numpy as np
import pytest

import seeded_inputs as si
from oracle import coracle
from tests.gpu_util import to_dev, to_host

pytestmark = [pytest.mark.gpu, pytest.mark.slow,
              pytest.mark.skipif(os.environ.get("ZKNTT_MAXSIZE") != "1",
                                 reason="2^28 transforms: set ZKNTT_MAXSIZE=1 to run")]

LOG2N = 28


@pytest.mark.parametrize("field", ["bn254_fr", "bls12_381_fr"])
def test_forward_2_28(cuda, field):
    import torch

    from paper_2509_22684_amd import Plan

    n = 1 << LOG2N
    print(f"[maxsize] {field} 2^{LOG2N}: generating input", flush=True)
    x = si.uniform_field_vector(field, n, si.stream_seed(28, 0, 0))
    dx = to_dev(x, cuda)
    plan = Plan(field, LOG2N)
    print(f"[maxsize] {field}: forward ({plan.passes} passes)", flush=True)
    out = plan.forward(dx)
    back = plan.inverse(out)
    assert torch.equal(back, dx), "INTT(NTT(x)) != x"
    del back
    cos = plan.coset_inverse(plan.coset_forward(dx))
    assert torch.equal(cos, dx), "coset round trip"
    del cos
    rng = np.random.Generator(np.random.PCG64(28))
    idx = np.concatenate([[0, 1, n // 2, n - 1], rng.integers(0, n, size=12)]).astype(np.uint64)
    got = to_host(out[torch.from_numpy(idx.astype(np.int64)).to(cuda)])
    print(f"[maxsize] {field}: Horner at {len(idx)} points", flush=True)
    want = coracle.eval_at_roots(field, x, idx)
    assert np.array_equal(got, want)
