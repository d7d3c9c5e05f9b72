"""Full-size GPU parity in the configuration the benchmark times.

* n = 2^24 forward NTT on BLS12-381 Fr (the headline workload), compared
  element by element with the threaded C oracle, plus Horner spot checks
  A_i = a(w^i) that use no NTT code at all.
* The Groth16 quotient chain at n = 2^24 (A, B, C of 512 MiB each), compared
  element by element with the oracle's seven-transform pipeline.
"""
import numpy as np
import pytest

import seeded_inputs as si
from oracle import coracle
from tests.gpu_util import first_mismatch, to_dev, to_host

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

FIELD = "bls12_381_fr"
LOG2N = 24


def test_forward_2_24_full_compare_and_horner(cuda):
    from paper_2509_22684_amd import Plan

    x = si.uniform_field_vector(FIELD, 1 << LOG2N, si.stream_seed(3, 0, 0))
    plan = Plan(FIELD, LOG2N)
    got = to_host(plan.forward(to_dev(x, cuda)))
    want = coracle.transform(FIELD, "forward", x)
    nbad, first = first_mismatch(got, want)
    assert nbad == 0, f"{nbad} mismatches, first at {first}"
    rng = np.random.Generator(np.random.PCG64(24))
    idx = np.concatenate([[0, 1, (1 << LOG2N) - 1], rng.integers(0, 1 << LOG2N, size=5)]).astype(np.uint64)
    spot = coracle.eval_at_roots(FIELD, x, idx)
    assert np.array_equal(got[idx.astype(np.int64)], spot)


def test_quotient_2_24_full_compare(cuda):
    from paper_2509_22684_amd import Plan

    A, B, C = (si.uniform_field_vector(FIELD, 1 << LOG2N, si.stream_seed(3, 0, v)) for v in range(3))
    plan = Plan(FIELD, LOG2N)
    got = to_host(plan.quotient(to_dev(A, cuda), to_dev(B, cuda), to_dev(C, cuda)))
    want = coracle.quotient(FIELD, A, B, C)
    nbad, first = first_mismatch(got, want)
    assert nbad == 0, f"{nbad} mismatches, first at {first}"
