"""Continuous-batching server on the GPU: every job's H in the mix equals the
same job run alone through quotient_poly and the oracle, byte for byte, with
jobs of different sizes at different stages sharing launches."""
import numpy as np
import pytest

import seeded_inputs as si
from oracle import coracle
from tests.gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu

FIELD = "bls12_381_fr"


def _requests(sizes, gap_s=0.0):
    from paper_2509_22684_amd.serve import Request

    reqs = []
    for k, L in enumerate(sizes):
        ins = tuple(si.uniform_field_vector(FIELD, 1 << L, si.stream_seed(5, k, v)) for v in range(3))
        reqs.append(Request(k, L, k * gap_s, ins))
    return reqs


def _check(results, reqs, cuda):
    from paper_2509_22684_amd import Plan

    plans = {}
    for r, q in zip(results, reqs):
        assert r.status == "done"
        got = to_host(r.H)
        assert np.array_equal(got, coracle.quotient(FIELD, *q.inputs)), f"job {q.job_id} vs oracle"
        if q.log2n not in plans:
            plans[q.log2n] = Plan(FIELD, q.log2n)
        alone = to_host(plans[q.log2n].quotient(*(to_dev(v, cuda) for v in q.inputs)))
        assert np.array_equal(got, alone), f"job {q.job_id}: mix and alone differ"


def test_mix_equals_alone(cuda):
    from paper_2509_22684_amd.serve import GpuExecutor, QuotientServer

    reqs = _requests([14, 10, 12, 16, 11, 14, 13, 10])
    ex = GpuExecutor(FIELD)
    srv = QuotientServer(ex, budget_bytes=200 << 30)
    res = srv.run(reqs, realtime=False)
    assert srv.max_inflight == len(reqs)  # all in one mix
    _check(res, reqs, cuda)


def test_staggered_arrivals_and_tight_budget(cuda):
    """Jobs arrive while others run and join at the next tick; a budget of
    about two jobs forces admission to wait."""
    from paper_2509_22684_amd.serve import GpuExecutor, QuotientServer

    reqs = _requests([12, 13, 12, 14, 12, 13], gap_s=0.002)
    ex = GpuExecutor(FIELD)
    budget = 2 * ex.job_bytes(14) + sum(ex.plan_bytes(L) for L in (12, 13, 14))
    srv = QuotientServer(ex, budget_bytes=budget)
    res = srv.run(reqs, realtime=True)
    assert srv.peak_bytes <= budget
    assert 1 <= srv.max_inflight < len(reqs)
    _check(res, reqs, cuda)


@pytest.mark.slow
def test_serving_sizes_up_to_2_22(cuda):
    """The serving size range at its ends: a 2^22 job (its stages run as
    grouped pass launches) beside small ones; every H equals the oracle's
    quotient in full."""
    from paper_2509_22684_amd.serve import GpuExecutor, QuotientServer

    reqs = _requests([22, 14, 18, 14])
    ex = GpuExecutor(FIELD)
    res = QuotientServer(ex, budget_bytes=200 << 30).run(reqs, realtime=False)
    for r, q in zip(res, reqs):
        assert r.status == "done"
        assert np.array_equal(to_host(r.H), coracle.quotient(FIELD, *q.inputs)), f"job {q.job_id} (2^{q.log2n})"


def test_lone_jobs_run_whole_and_match(cuda):
    """A job alone in its lane runs its whole chain as one quotient_poly call
    on the job's own buffers; its H equals the oracle's and the stand-alone
    call's.  Jobs sharing a lane still go through batched ticks."""
    from paper_2509_22684_amd.serve import GpuExecutor, QuotientServer

    reqs = _requests([12, 20, 13, 13])  # lanes by 2^19: {12, 13, 13} and {20}
    ex = GpuExecutor(FIELD)
    res = QuotientServer(ex, budget_bytes=200 << 30).run(reqs, realtime=False)
    assert ex.whole_jobs == 1  # the 2^20 job; the three small ones share ticks
    _check(res, reqs, cuda)
    reqs1 = _requests([15])
    ex1 = GpuExecutor(FIELD)
    res1 = QuotientServer(ex1, budget_bytes=200 << 30).run(reqs1, realtime=False)
    assert ex1.whole_jobs == 1 and ex1.ticks == 1
    _check(res1, reqs1, cuda)
