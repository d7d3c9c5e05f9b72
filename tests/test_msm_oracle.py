"""Pins of the MSM oracle (oracle/msm_ref.py) to mathematics, on the CPU."""
import random

import pytest

from oracle import msm_ref as M
from oracle import ref


def test_curve_parameters_follow_from_the_seed():
    """r from the family seed is the BLS12-381 scalar field the NTT uses; q is
    a 381-bit prime = 3 mod 4; the curve order q + 1 - t (t = x0 + 1) is h r."""
    import sympy

    assert M.R == ref.BLS12_381_FR.p
    assert sympy.isprime(M.Q) and M.Q.bit_length() == 381 and M.Q % 4 == 3
    assert (M.X0 - 1) ** 2 % 3 == 0 and ((M.X0 - 1) ** 2 * M.R) % 3 == 0
    assert M.Q + 1 - (M.X0 + 1) == M.H * M.R


def test_subgroup_points_and_group_law():
    G = M.subgroup_point(11)
    P = M.subgroup_point(12)
    Q2 = M.subgroup_point(13)
    for X in (G, P, Q2):
        assert X is not None and M.on_curve(X)
        assert M.mul(M.R, X) is None  # order r
    assert M.add(G, P) == M.add(P, G)
    assert M.add(M.add(G, P), Q2) == M.add(G, M.add(P, Q2))
    assert M.add(G, M.neg(G)) is None and M.add(G, None) == G
    assert M.dbl(G) == M.add(G, G) and M.on_curve(M.dbl(G))
    rng = random.Random(5)
    a, b = rng.randrange(M.R), rng.randrange(M.R)
    assert M.mul(a + b, G) == M.add(M.mul(a, G), M.mul(b, G))
    assert M.mul(a * b % M.R, G) == M.mul(a, M.mul(b, G))
    assert M.mul(M.R - 1, G) == M.neg(G)


def test_points_off_the_subgroup_need_the_cofactor():
    """A raw curve point (before scaling by h) is generally not of order r."""
    x = 1
    while M.sqrt_q(x ** 3 + 4) is None:
        x += 1
    P = (x, M.sqrt_q(x ** 3 + 4))
    assert M.on_curve(P) and M.mul(M.R, P) is not None
    assert M.mul(M.R, M.mul(M.H, P)) is None


@pytest.mark.parametrize("c", [1, 3, 4, 7])
def test_bucket_method_equals_definition(c):
    rng = random.Random(20 + c)
    pts = [M.subgroup_point(100 + k) for k in range(6)]
    pts += [pts[0], M.neg(pts[1]), pts[2]]  # repeats and negatives land in shared buckets
    scal = [rng.randrange(M.R) for _ in pts]
    scal[3] = 0
    scal[4] = M.R - 1
    scal[5] = 1
    assert M.msm_buckets(scal, pts, c) == M.msm_naive(scal, pts)


def test_msm_structured_inputs_closed_form():
    """With P_i = (i + 1) G, sum s_i P_i = (sum s_i (i + 1) mod r) G; the
    batched multiples equal repeated addition."""
    G = M.subgroup_point(7)
    mults = M.multiples(G, 2100, block=256)
    acc = None
    for i in range(40):
        acc = M.add(acc, G)
        assert mults[i] == acc
    assert mults[2099] == M.mul(2100, G)
    rng = random.Random(9)
    scal = [rng.randrange(M.R) for _ in range(50)]
    want = M.mul(sum(s * (i + 1) for i, s in enumerate(scal)) % M.R, G)
    assert M.msm_naive(scal, mults[:50]) == want


def test_device_layout_round_trip():
    G = M.subgroup_point(8)
    a = M.points_to_device_layout([G, M.dbl(G)])
    assert a.shape == (2, 24)
    assert M.fq_from_limbs(a[:, :12]) == [G[0], M.dbl(G)[0]]
    assert M.fq_from_limbs(a[:, 12:]) == [G[1], M.dbl(G)[1]]
    X, Y, ZZ, ZZZ = G[0] * 9 % M.Q, G[1] * 27 % M.Q, 9, 27  # Z = 3
    assert M.xyzz_to_affine(X, Y, ZZ, ZZZ) == G and M.xyzz_to_affine(1, 1, 0, 0) is None
