"""GPU parity of the MSM (BLS12-381 G1) against the MSM oracle: small sizes
against the definition and the bucket method in Python integers, edge cases
of the point additions (repeated points, opposite points, zero scalars, the
largest scalar), every window size class, and sizes up to 2^20 on structured
bases P_i = (i + 1) G, whose sum has the closed form (sum_i s_i (i + 1)) G."""
import random

import pytest

import seeded_inputs as si
from oracle import msm_ref as M
from oracle import ref
from tests.gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu

FR = ref.BLS12_381_FR


def _scalars_dev(scal, cuda):
    return to_dev(si.ints_to_limbs(FR.to_mont(scal)), cuda)


def _result_point(res):
    words = to_host(res)[:48]
    X, Y, ZZ, ZZZ = (M.fq_from_limbs(words[12 * k:12 * (k + 1)].reshape(1, 12))[0] for k in range(4))
    return M.xyzz_to_affine(X, Y, ZZ, ZZZ)


def _run(points, scal, cuda, window_bits=0):
    from paper_2509_22684_amd import MsmBases

    pts = to_dev(M.points_to_device_layout(points), cuda)
    bases = MsmBases(pts, window_bits)
    res = bases.msm(_scalars_dev(scal, cuda))
    return _result_point(res), bases


@pytest.fixture(scope="module")
def small_points():
    return [M.subgroup_point(300 + k) for k in range(24)]


@pytest.mark.parametrize("n", [1, 2, 5, 24])
def test_msm_small_equals_definition(cuda, small_points, n):
    rng = random.Random(n)
    pts = small_points[:n]
    scal = [rng.randrange(FR.p) for _ in pts]
    got, _ = _run(pts, scal, cuda)
    assert got == M.msm_naive(scal, pts)


def test_msm_edge_cases(cuda, small_points):
    """Equal points with equal scalars meet in every bucket (the doubling
    case of the mixed addition), opposite points cancel (infinity), zero
    scalars add nothing, r - 1 is the largest scalar."""
    P, Q2 = small_points[0], small_points[1]
    rng = random.Random(77)
    s = rng.randrange(FR.p)
    pts = [P, P, Q2, M.neg(Q2), P, Q2, small_points[2]]
    scal = [s, s, s, s, 0, FR.p - 1, 1]
    got, _ = _run(pts, scal, cuda)
    assert got == M.msm_naive(scal, pts)
    # everything cancels: the point at infinity
    got, _ = _run([P, M.neg(P)], [s, s], cuda)
    assert got is None
    got, _ = _run([P, Q2], [0, 0], cuda)
    assert got is None


@pytest.mark.parametrize("window_bits", [1, 4, 7, 13, 16])
def test_msm_window_sizes(cuda, small_points, window_bits):
    rng = random.Random(window_bits)
    pts = small_points[:12]
    scal = [rng.randrange(FR.p) for _ in pts]
    got, bases = _run(pts, scal, cuda, window_bits)
    assert bases.window_bits == window_bits
    assert got == M.msm_naive(scal, pts)


@pytest.fixture(scope="module")
def multiples_g():
    G = M.subgroup_point(7)
    return G, M.multiples(G, 1 << 16)


@pytest.mark.parametrize("n", [1000, 1 << 12, 1 << 16])
def test_msm_structured_bases_closed_form(cuda, multiples_g, n):
    G, mults = multiples_g
    rng = random.Random(n)
    scal = [rng.randrange(FR.p) for _ in range(n)]
    got, _ = _run(mults[:n], scal, cuda)
    want = M.mul(sum(s * (i + 1) for i, s in enumerate(scal)) % FR.p, G)
    assert got == want
    if n == 1000:
        assert got == M.msm_buckets(scal, mults[:n], 8)


def _repeated_digit_scalar(c, d):
    """The scalar whose c-bit windows all hold d (below 2^255), reduced mod r."""
    v = 0
    for w in range((255 + c - 1) // c):
        v |= d << (c * w)
    return (v & ((1 << 255) - 1)) % FR.p


@pytest.mark.parametrize("window_bits", [0, 16])
@pytest.mark.parametrize("mix", ["all_equal", "half_equal", "mostly_zero", "zero_one"])
def test_msm_skewed_buckets_closed_form(cuda, multiples_g, mix, window_bits):
    """Bucket sizes far from uniform: one bucket holding most entries (its
    sum spans thousands of accumulation lanes and goes to the workgroup
    combine), many buckets inside one lane's run, mostly empty buckets, and
    witness-like scalars that are mostly 0 or 1 (bucket 1 of window 0)."""
    G, mults = multiples_g
    n = 1 << 14
    rng = random.Random(f"{mix}-{window_bits}")
    c = window_bits or 12
    rep = _repeated_digit_scalar(c, 5)
    if mix == "all_equal":
        scal = [rep] * n
    elif mix == "half_equal":
        scal = [rep if k % 2 else rng.randrange(FR.p) for k in range(n)]
    elif mix == "mostly_zero":
        scal = [rng.randrange(FR.p) if k % 10 == 0 else 0 for k in range(n)]
    else:
        scal = [rng.randrange(FR.p) if k % 50 == 0 else k % 2 for k in range(n)]
    got, bases = _run(mults[:n], scal, cuda, window_bits)
    assert bases.window_bits == c
    assert got == M.mul(sum(s * (i + 1) for i, s in enumerate(scal)) % FR.p, G)


def test_msm_scalars_from_the_quotient(cuda, multiples_g):
    """The quotient chain's output H (Montgomery Fr limbs) feeds the MSM
    directly, as in a Groth16 prover's H-query."""
    from paper_2509_22684_amd import MsmBases, Plan

    G, mults = multiples_g
    log2n = 10
    n = 1 << log2n
    A, B, C = (si.uniform_field_vector("bls12_381_fr", n, si.stream_seed(91, 0, v)) for v in range(3))
    H = Plan("bls12_381_fr", log2n).quotient(to_dev(A, cuda), to_dev(B, cuda), to_dev(C, cuda))
    h = FR.from_mont(si.limbs_to_ints(to_host(H)))
    bases = MsmBases(to_dev(M.points_to_device_layout(mults[:n]), cuda))
    got = _result_point(bases.msm(H))
    assert got == M.mul(sum(v * (i + 1) for i, v in enumerate(h)) % FR.p, G)


def test_msm_one_bucket_2_16(cuda, multiples_g):
    """2^16 equal scalars with every window digit equal: one bucket of about
    1.2 M entries, summed by the workgroup combine over its runs' heads."""
    G, mults = multiples_g
    n = 1 << 16
    rep = _repeated_digit_scalar(14, 9)
    got, bases = _run(mults, [rep] * n, cuda)
    assert bases.window_bits == 14
    assert got == M.mul(rep * (n * (n + 1) // 2) % FR.p, G)


@pytest.mark.slow
def test_msm_2_20_closed_form(cuda, multiples_g):
    G, _ = multiples_g
    n = 1 << 20
    mults = M.multiples(G, n)
    rng = random.Random(20)
    scal = [rng.randrange(FR.p) for _ in range(n)]
    got, _ = _run(mults, scal, cuda)
    assert got == M.mul(sum(s * (i + 1) for i, s in enumerate(scal)) % FR.p, G)


def test_msm_argument_checks(cuda, small_points):
    """Overlapping result, workspace and scalars, and misaligned pointers, are
    refused before anything runs."""
    import torch

    from paper_2509_22684_amd import ZkError

    pts = small_points[:4]
    _, bases = _run(pts, [1, 2, 3, 4], cuda)
    scal = _scalars_dev([5, 6, 7, 8], cuda)
    work = bases.workspace()
    for out, w in ((work.view(-1)[:64], None), (scal.view(-1)[:64], None), (None, scal.view(-1, 8))):
        with pytest.raises(ZkError) as e:
            bases.msm(scal, out=out, work=w)
        assert e.value.code == -1
    big = torch.zeros(4 * 8 + 64, dtype=torch.int32, device=cuda)
    with pytest.raises(ZkError) as e:  # scalars 4 bytes past a 256-byte boundary
        bases.msm(big[1:33].view(4, 8))
    assert e.value.code == -1
