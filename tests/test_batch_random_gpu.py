"""Seeded random batches: every transform kind and the pointwise step, all
three fields, sizes 2^2..2^17, random queue counts, graph and direct
launches, each job against the oracle.  Covers mixes the fixed workloads do
not (many kinds and fields in one batch, jobs that run as direct pass
launches next to queued ones)."""
import numpy as np
import pytest

import seeded_inputs as si
from oracle import coracle, ref
from tests.gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu

FIELDS = ["bls12_381_fr", "bn254_fr", "bls12_377_fr"]
OPS = ["forward", "inverse", "coset_forward", "coset_inverse", "inverse_to_coset", "quotient_pointwise"]


def _oracle(field, op, ins):
    if op == "inverse_to_coset":
        # INTT, then coefficient j times g^j: the input of a coset NTT
        F = ref.FIELDS[field]
        coeffs = F.from_mont(si.limbs_to_ints(coracle.transform(field, "inverse", ins[0])))
        g = F.generator
        return si.ints_to_limbs(F.to_mont([c * pow(g, j, F.p) % F.p for j, c in enumerate(coeffs)]))
    if op == "quotient_pointwise":
        F = ref.FIELDS[field]
        a, b, c = (F.from_mont(si.limbs_to_ints(v)) for v in ins)
        zinv = pow(pow(F.generator, len(a), F.p) - 1, -1, F.p)
        return si.ints_to_limbs(F.to_mont([(x * y - z) * zinv % F.p for x, y, z in zip(a, b, c)]))
    return coracle.transform(field, op, ins[0])


@pytest.mark.parametrize("seed", range(6))
def test_random_batch(cuda, seed):
    import torch

    from paper_2509_22684_amd import Plan, ntt_batch_create_jobs, ntt_batch_destroy, ntt_batch_launch, \
        ntt_batch_launch_eager, ntt_batch_status

    rng = np.random.Generator(np.random.PCG64(1000 + seed))
    njobs = int(rng.integers(1, 40))
    plans, jobs, want, outs = {}, [], [], []
    keep = []  # device buffers stay alive until the batch has run
    for k in range(njobs):
        field = FIELDS[int(rng.integers(0, 3))]
        op = OPS[int(rng.integers(0, len(OPS)))]
        log2n = int(rng.integers(2, 18)) if op != "quotient_pointwise" else int(rng.integers(2, 15))
        if (field, log2n) not in plans:
            plans[(field, log2n)] = Plan(field, log2n)
        p = plans[(field, log2n)]
        nin = 3 if op == "quotient_pointwise" else 1
        ins = [si.uniform_field_vector(field, 1 << log2n, si.stream_seed(70 + seed, k, v)) for v in range(nin)]
        dins = [to_dev(x, cuda) for x in ins]
        out = dins[0] if (op != "quotient_pointwise" and rng.integers(0, 2)) else torch.empty_like(dins[0])
        wb = p.workspace(dins[0])
        work = None if wb is None else torch.empty_like(wb)  # a workspace of its own per job
        job = dict(plan=p, op=op, out=out, work=work, **{"in": dins[0]})
        if nin == 3:
            job.update(in2=dins[1], in3=dins[2])
        jobs.append(job)
        want.append(_oracle(field, op, ins))
        outs.append(out)
        keep.append((dins, work))
    queues = int(rng.integers(0, 9))
    graph = bool(seed % 2)
    h = ntt_batch_create_jobs(jobs, graph=graph, queues=queues)
    if graph:
        ntt_batch_launch(h)
    else:
        ntt_batch_launch_eager(h)
    torch.cuda.synchronize()
    assert ntt_batch_status(h) == 0
    ntt_batch_destroy(h)
    for k, (o, w) in enumerate(zip(outs, want)):
        assert np.array_equal(to_host(o), w), f"seed {seed} job {k} {jobs[k]['op']} graph={graph} queues={queues}"
