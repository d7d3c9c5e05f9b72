"""Pins of the CPU oracle to mathematics (no GPU).

The oracle (oracle/ref.py in Python integers, oracle/ntt_oracle.c in C with
Barrett arithmetic) is checked here against things other than itself:

* number theory: p prime, g a generator of F_p^* (sympy factorisation of
  p - 1), g the smallest generator, w^n = 1 and w^(n/2) = -1 at every n;
* the definition: the radix-2 NTT equals the O(n^2) DFT at n <= 256;
* closed forms and special inputs: deltas, constants, n = 4 worked example,
  linearity, the halving identity A_2i = NTT_{n/2}(a_j + a_{j+n/2})_i;
* inverses and cosets: round trips, cosetNTT(delta_1) = (g w^i);
* the convolution theorem against schoolbook polynomial products;
* the quotient against its closed form ((a b - c) mod (X^n - g^n)) /
  (g^n - 1) and, for satisfied inputs (C = A.B on H), against
  h(z)(z^n - 1) = a(z) b(z) - c(z) at random z;
* the C oracle against the Python oracle, Python integers and Horner's rule.

The planted-mistake tests at the end check that the pins are sharp: each
plants a plausible error in a copy of the oracle and expects a pin to fail.
"""
import random

import numpy as np
import pytest
import sympy

import seeded_inputs as si
from oracle import coracle, ref

FIELDS = [ref.BLS12_381_FR, ref.BN254_FR, ref.BLS12_377_FR]
IDS = [F.name for F in FIELDS]


def rand_vec(F, n, seed):
    rng = random.Random(seed)
    return [rng.randrange(F.p) for _ in range(n)]


# ---------------------------------------------------------------------------
# number theory

@pytest.mark.parametrize("F", FIELDS, ids=IDS)
def test_modulus_prime_and_matches_input_recipe(F):
    assert sympy.isprime(F.p)
    assert si.MODULI[F.name] == F.p
    assert coracle.constant(F.name, "modulus") == F.p


@pytest.mark.parametrize("F", FIELDS, ids=IDS)
def test_two_adicity(F):
    s = F.two_adicity
    assert (F.p - 1) % (1 << s) == 0 and ((F.p - 1) >> s) % 2 == 1


@pytest.mark.parametrize("F", FIELDS, ids=IDS)
def test_generator_is_smallest_primitive_root(F):
    factors = sympy.factorint(F.p - 1)
    prod = 1
    for q, e in factors.items():
        assert sympy.isprime(q)
        prod *= q ** e

    assert prod == F.p - 1

    def is_generator(x):
        return all(pow(x, (F.p - 1) // q, F.p) != 1 for q in factors)

    assert is_generator(F.generator)
    assert not any(is_generator(x) for x in range(2, F.generator))


@pytest.mark.parametrize("F", FIELDS, ids=IDS)
def test_roots_of_unity_every_size(F):
    for k in range(1, F.two_adicity + 1):
        n = 1 << k
        w = F.root(n)
        assert pow(w, n, F.p) == 1
        assert pow(w, n // 2, F.p) == F.p - 1  # primitive: w^(n/2) = -1
        if k < F.two_adicity:
            assert pow(F.root(2 * n), 2, F.p) == w  # one chain of roots
    assert F.root(1) == 1


@pytest.mark.parametrize("F", FIELDS, ids=IDS)
def test_c_oracle_constants(F):
    assert coracle.constant(F.name, "mu") == (1 << 512) // F.p  # Barrett constant
    assert coracle.constant(F.name, "r_mod") == (1 << 256) % F.p
    for k in (0, 1, 2, 5, 17, F.two_adicity):
        assert coracle.constant(F.name, "root", k) == F.root(1 << k)


# ---------------------------------------------------------------------------
# C oracle field arithmetic against Python integers

def edge_values(F):
    p = F.p
    vals = [0, 1, 2, p - 1, p - 2, (p - 1) // 2, (p + 1) // 2, (1 << 256) % p, (1 << 255) % p,
            (1 << 32) - 1, (1 << 64) - 1, (1 << 192) + 5]
    # limbs of p with the lowest limb lowered: differs from p only at the bottom
    vals.append(p - 1 - (p & 0xFFFFFFFF) if (p & 0xFFFFFFFF) else p - 3)
    # all-ones limbs below p
    vals.append(int("ffffffff" * 7, 16))
    return [v % p for v in vals]


@pytest.mark.parametrize("F", FIELDS, ids=IDS)
def test_c_field_ops_match_python(F):
    p = F.p
    vals = edge_values(F) + rand_vec(F, 40, 9)
    pairs = [(a, b) for a in vals for b in vals[:20]]
    A = si.ints_to_limbs([a for a, _ in pairs])
    B = si.ints_to_limbs([b for _, b in pairs])
    for op, fn in [("add", lambda a, b: (a + b) % p), ("sub", lambda a, b: (a - b) % p),
                   ("mul", lambda a, b: a * b % p), ("pow", lambda a, b: pow(a, b, p))]:
        got = si.limbs_to_ints(coracle.field_op(F.name, op, A, B))
        assert got == [fn(a, b) for a, b in pairs], op
    nz = [v for v in vals if v]
    got = si.limbs_to_ints(coracle.field_op(F.name, "inv", si.ints_to_limbs(nz), si.ints_to_limbs(nz)))
    assert all(g * v % p == 1 for g, v in zip(got, nz))


@pytest.mark.parametrize("F", FIELDS, ids=IDS)
def test_montgomery_boundary(F):
    """A stored value y represents y 2^-256: the n = 1 transform is the
    identity, and NTT of the stored form of delta_0 is the stored form of 1
    everywhere."""
    ys = rand_vec(F, 1, 3)
    assert coracle.transform(F.name, "forward", si.ints_to_limbs(ys)).tolist() == si.ints_to_limbs(ys).tolist()
    one_stored = (1 << 256) % F.p
    n = 16
    delta0 = si.ints_to_limbs([one_stored] + [0] * (n - 1))
    out = si.limbs_to_ints(coracle.transform(F.name, "forward", delta0))
    assert out == [one_stored] * n
    x = rand_vec(F, 8, 4)
    assert F.from_mont(F.to_mont(x)) == x
    assert F.to_mont([1]) == [one_stored]


# ---------------------------------------------------------------------------
# forward transform

def pin_dft(F, ntt_fn, sizes=(1, 2, 4, 8, 16, 64, 256), seed=0):
    for n in sizes:
        a = rand_vec(F, n, seed + n)
        assert ntt_fn(F, a) == ref.dft(F, a), f"n={n}"


def pin_special_inputs(F, ntt_fn, n=32):
    p, w = F.p, F.root(n)
    delta0 = [1] + [0] * (n - 1)
    assert ntt_fn(F, delta0) == [1] * n
    assert ntt_fn(F, [1] * n) == [n] + [0] * (n - 1)
    for k in (1, 3, n - 1):
        dk = [0] * n
        dk[k] = 1
        assert ntt_fn(F, dk) == [pow(w, i * k, p) for i in range(n)]
    c = 123456789
    assert ntt_fn(F, [c] * n) == [c * n % p] + [0] * (n - 1)


def pin_n4_worked_example(F, ntt_fn):
    """[1, 2, 3, 4] -> [10, -2 - 2w, -2, -2 + 2w] with w = w_4, w^2 = -1."""
    p, w = F.p, F.root(4)
    assert w * w % p == p - 1
    assert ntt_fn(F, [1, 2, 3, 4]) == [10, (-2 - 2 * w) % p, p - 2, (-2 + 2 * w) % p]


@pytest.mark.parametrize("F", FIELDS, ids=IDS)
def test_ntt_equals_dft(F):
    pin_dft(F, ref.ntt)


@pytest.mark.parametrize("F", FIELDS, ids=IDS)
def test_special_inputs(F):
    pin_special_inputs(F, ref.ntt)


@pytest.mark.parametrize("F", FIELDS, ids=IDS)
def test_n4_worked_example(F):
    pin_n4_worked_example(F, ref.ntt)


@pytest.mark.parametrize("F", FIELDS, ids=IDS)
def test_linearity_and_halving(F):
    p, n = F.p, 64
    x, y = rand_vec(F, n, 1), rand_vec(F, n, 2)
    al, be = 987654321, F.p - 5
    lhs = ref.ntt(F, [(al * u + be * v) % p for u, v in zip(x, y)])
    X, Y = ref.ntt(F, x), ref.ntt(F, y)
    assert lhs == [(al * u + be * v) % p for u, v in zip(X, Y)]
    half = ref.ntt(F, [(x[j] + x[j + n // 2]) % p for j in range(n // 2)])
    assert X[0::2] == half


# ---------------------------------------------------------------------------
# inverse and coset transforms

def pin_inverse(F, ntt_fn, intt_fn, n=64):
    x = rand_vec(F, n, 11)
    assert intt_fn(F, ntt_fn(F, x)) == x
    assert ntt_fn(F, intt_fn(F, x)) == x
    assert intt_fn(F, x) == ref.idft(F, x)


def pin_coset(F, coset_fn, coset_inv_fn, n=32):
    p, w, g = F.p, F.root(n), F.generator
    d1 = [0, 1] + [0] * (n - 2)
    assert coset_fn(F, d1) == [g * pow(w, i, p) % p for i in range(n)]
    x = rand_vec(F, n, 12)
    assert coset_inv_fn(F, coset_fn(F, x)) == x
    # evaluations on the coset: out_i = x(g w^i) by Horner
    ev = coset_fn(F, x)
    for i in (0, 1, 7, n - 1):
        assert ev[i] == ref.horner(F, x, g * pow(w, i, p) % p)


@pytest.mark.parametrize("F", FIELDS, ids=IDS)
def test_inverse(F):
    pin_inverse(F, ref.ntt, ref.intt)


@pytest.mark.parametrize("F", FIELDS, ids=IDS)
def test_coset(F):
    pin_coset(F, ref.coset_ntt, ref.coset_intt)


# ---------------------------------------------------------------------------
# convolution theorem

def schoolbook(F, a, b):
    out = [0] * (len(a) + len(b) - 1)
    for i, u in enumerate(a):
        for j, v in enumerate(b):
            out[i + j] = (out[i + j] + u * v) % F.p
    return out


@pytest.mark.parametrize("F", FIELDS, ids=IDS)
def test_convolution_theorem(F):
    p, n = F.p, 16
    x, y = rand_vec(F, n, 21), rand_vec(F, n, 22)
    X = ref.ntt(F, x + [0] * n)
    Y = ref.ntt(F, y + [0] * n)
    prod = ref.intt(F, [u * v % p for u, v in zip(X, Y)])
    assert prod == schoolbook(F, x, y) + [0]
    # cyclic: product mod X^n - 1
    cyc = ref.intt(F, [u * v % p for u, v in zip(ref.ntt(F, x), ref.ntt(F, y))])
    full = schoolbook(F, x, y)
    want = [(full[k] + (full[k + n] if k + n < len(full) else 0)) % p for k in range(n)]
    assert cyc == want


# ---------------------------------------------------------------------------
# quotient

def quotient_closed_form(F, A, B, C):
    """((a b - c) mod (X^n - g^n)) / (g^n - 1), interpolants by the inverse
    DFT definition and products by schoolbook."""
    p, n = F.p, len(A)
    a, b, c = ref.idft(F, A), ref.idft(F, B), ref.idft(F, C)
    ab = schoolbook(F, a, b)
    num = [(ab[k] - (c[k] if k < n else 0)) % p for k in range(len(ab))]
    gn = pow(F.generator, n, p)
    red = num[:n] + [0] * (n - len(num[:n]))
    for k in range(n, len(num)):  # X^k = g^n X^(k - n) modulo X^n - g^n
        red[k - n] = (red[k - n] + gn * num[k]) % p
    zinv = pow(gn - 1, -1, p)
    return [v * zinv % p for v in red]


@pytest.mark.parametrize("F", FIELDS, ids=IDS)
@pytest.mark.parametrize("n", [1, 2, 4, 8, 32])
def test_quotient_closed_form(F, n):
    A, B, C = (rand_vec(F, n, 30 + v) for v in range(3))
    assert ref.quotient(F, A, B, C) == quotient_closed_form(F, A, B, C)


@pytest.mark.parametrize("F", FIELDS, ids=IDS)
def test_quotient_satisfied_r1cs_invariant(F):
    """With C = A . B on H, a b - c vanishes on H, so h = (a b - c) / Z_H
    exactly: deg h <= n - 2 and h(z) (z^n - 1) = a(z) b(z) - c(z)."""
    p, n = F.p, 64
    A, B = rand_vec(F, n, 41), rand_vec(F, n, 42)
    C = [u * v % p for u, v in zip(A, B)]
    h = ref.quotient(F, A, B, C)
    assert h[n - 1] == 0
    a, b, c = ref.intt(F, A), ref.intt(F, B), ref.intt(F, C)
    rng = random.Random(43)
    for _ in range(3):
        z = rng.randrange(p)
        lhs = ref.horner(F, h, z) * (pow(z, n, p) - 1) % p
        rhs = (ref.horner(F, a, z) * ref.horner(F, b, z) - ref.horner(F, c, z)) % p
        assert lhs == rhs


# ---------------------------------------------------------------------------
# C oracle against the Python oracle and Horner

@pytest.mark.parametrize("field", ["bls12_381_fr", "bn254_fr", "bls12_377_fr"])
@pytest.mark.parametrize("log2n", [0, 1, 2, 3, 4, 7, 10, 12])
def test_c_oracle_equals_python_oracle(field, log2n):
    F = ref.FIELDS[field]
    n = 1 << log2n
    x = si.uniform_field_vector(field, n, 500 + log2n)
    ys = si.limbs_to_ints(x)
    for kind in ("forward", "inverse", "coset_forward", "coset_inverse"):
        assert si.limbs_to_ints(coracle.transform(field, kind, x)) == ref.transform_mont(F, kind, ys), kind
    if log2n <= 10:
        A, B, C = (si.uniform_field_vector(field, n, 600 + log2n + v) for v in range(3))
        want = ref.quotient_mont(F, *(si.limbs_to_ints(v) for v in (A, B, C)))
        assert si.limbs_to_ints(coracle.quotient(field, A, B, C)) == want


@pytest.mark.parametrize("field", ["bls12_381_fr", "bn254_fr", "bls12_377_fr"])
@pytest.mark.parametrize("log2n", [13, 14])
@pytest.mark.parametrize("threads", [1, 3, 8])
def test_c_oracle_threaded_stages_equal_python_oracle(field, log2n, threads):
    """From n = 2^13 the C oracle splits every butterfly stage over threads
    (a stage has n/2 >= 4096 butterflies); with 1, 3 (uneven ranges) and 8
    threads each kind equals the Python-integer oracle element by element."""
    F = ref.FIELDS[field]
    n = 1 << log2n
    x = si.uniform_field_vector(field, n, 700 + log2n)
    ys = si.limbs_to_ints(x)
    for kind in ("forward", "inverse", "coset_forward", "coset_inverse"):
        got = coracle.transform(field, kind, x, threads=threads)
        assert si.limbs_to_ints(got) == ref.transform_mont(F, kind, ys), kind


@pytest.mark.parametrize("field", ["bls12_381_fr", "bn254_fr", "bls12_377_fr"])
@pytest.mark.parametrize("log2n", [11, 12, 13])
@pytest.mark.parametrize("threads", [3, 8])
def test_c_oracle_threaded_quotient_equals_python_oracle(field, log2n, threads):
    """The quotient chain with threaded conversions, scalings, stages and
    pointwise step (threaded from n = 2^12 for the elementwise work and from
    2^13 for the stages) equals the Python oracle."""
    F = ref.FIELDS[field]
    n = 1 << log2n
    A, B, C = (si.uniform_field_vector(field, n, 800 + log2n + v) for v in range(3))
    want = ref.quotient_mont(F, *(si.limbs_to_ints(v) for v in (A, B, C)))
    assert si.limbs_to_ints(coracle.quotient(field, A, B, C, threads=threads)) == want


@pytest.mark.parametrize("field", ["bls12_381_fr", "bn254_fr", "bls12_377_fr"])
def test_c_oracle_large_n_horner(field):
    """At n = 2^16 the C oracle's outputs equal a(w^i) evaluated by Horner in
    Python integers, and its own Horner routine agrees."""
    F = ref.FIELDS[field]
    log2n = 16
    n = 1 << log2n
    x = si.uniform_field_vector(field, n, 77)
    out = si.limbs_to_ints(coracle.transform(field, "forward", x))
    coeffs = F.from_mont(si.limbs_to_ints(x))
    w = F.root(n)
    idx = [0, 1, 2, n // 2, n - 1, 12345]
    for i in idx:
        assert F.from_mont([out[i]])[0] == ref.horner(F, coeffs, pow(w, i, F.p))
    spot = si.limbs_to_ints(coracle.eval_at_roots(field, x, np.array(idx, dtype=np.uint64)))
    assert spot == [out[i] for i in idx]
    # coset forward: a(g w^i) by Horner; inverse and coset inverse undo
    # their forward transforms (threaded at this size)
    cos = si.limbs_to_ints(coracle.transform(field, "coset_forward", x, threads=6))
    for i in idx:
        assert F.from_mont([cos[i]])[0] == ref.horner(F, coeffs, F.generator * pow(w, i, F.p) % F.p)
    fwd = coracle.transform(field, "forward", x, threads=5)
    assert np.array_equal(coracle.transform(field, "inverse", fwd, threads=7), x)
    cf = coracle.transform(field, "coset_forward", x, threads=4)
    assert np.array_equal(coracle.transform(field, "coset_inverse", cf, threads=3), x)


def test_c_oracle_rejects_bad_sizes():
    x = si.uniform_field_vector("bn254_fr", 4, 1)
    lib = coracle.lib()
    assert lib.orc_transform(2, 29, 0, coracle._u32(x), coracle._u32(x), 1) == -1
    assert lib.orc_transform(4, 2, 0, coracle._u32(x), coracle._u32(x), 1) == -1  # unknown field id
    assert lib.orc_transform(1, 2, 9, coracle._u32(x), coracle._u32(x), 1) == -1


# ---------------------------------------------------------------------------
# planted mistakes: each must be caught by a pin

def _mutant_ntt(mistake):
    """Radix-2 NTT of ref.ntt_radix2 with one planted mistake."""

    def ntt_fn(F, a):
        n, p = len(a), F.p
        w = F.root(n)
        if mistake == "inverse_root":
            w = pow(w, -1, p)
        x = [v % p for v in a] if mistake == "no_bitrev" else ref.bit_reverse([v % p for v in a])
        m = 2
        while m <= n:
            wm = pow(w, n // m, p)
            half = m // 2
            tw = [pow(wm, j + (1 if mistake == "twiddle_index" else 0), p) for j in range(half)]
            for b in range(0, n, m):
                for j in range(half):
                    u, t = x[b + j], tw[j] * x[b + j + half] % p
                    if mistake == "butterfly_sign":
                        x[b + j], x[b + j + half] = (u - t) % p, (u + t) % p
                    elif mistake == "dropped_twiddle":
                        x[b + j], x[b + j + half] = (u + x[b + j + half]) % p, (u - x[b + j + half]) % p
                    else:
                        x[b + j], x[b + j + half] = (u + t) % p, (u - t) % p
            m *= 2
        return x

    return ntt_fn


@pytest.mark.parametrize("mistake", ["inverse_root", "no_bitrev", "twiddle_index", "butterfly_sign",
                                     "dropped_twiddle"])
def test_planted_ntt_mistakes_are_caught(mistake):
    F = ref.BLS12_381_FR
    fn = _mutant_ntt(mistake)
    caught = 0
    for pin in (lambda: pin_dft(F, fn), lambda: pin_special_inputs(F, fn), lambda: pin_n4_worked_example(F, fn)):
        try:
            pin()
        except AssertionError:
            caught += 1
    assert caught >= 1


def test_planted_inverse_and_coset_mistakes_are_caught():
    F = ref.BLS12_381_FR

    def intt_no_scale(F_, A):
        return ref.ntt_radix2(F_, A, pow(F_.root(len(A)), -1, F_.p))

    with pytest.raises(AssertionError):
        pin_inverse(F, ref.ntt, intt_no_scale)

    def coset_wrong_dir(F_, a):
        ginv = pow(F_.generator, -1, F_.p)
        return ref.ntt(F_, [v * pow(ginv, j, F_.p) % F_.p for j, v in enumerate(a)])

    with pytest.raises(AssertionError):
        pin_coset(F, coset_wrong_dir, ref.coset_intt)


def test_planted_quotient_mistake_is_caught():
    """Using Z_H = g^n + 1 instead of g^n - 1 breaks the closed form."""
    F = ref.BN254_FR
    n = 8
    A, B, C = (rand_vec(F, n, 90 + v) for v in range(3))
    good = ref.quotient(F, A, B, C)
    gn = pow(F.generator, n, F.p)
    fix = (gn - 1) * pow(gn + 1, -1, F.p) % F.p  # rescale: wrong zinv
    bad = [v * fix % F.p for v in good]
    assert good == quotient_closed_form(F, A, B, C)
    assert bad != quotient_closed_form(F, A, B, C)


@pytest.mark.parametrize("F", FIELDS, ids=IDS)
def test_montgomery_product_definition(F):
    """The Montgomery product of stored elements is the stored form of the
    plain product (to_mont(x) * to_mont(y) * 2^-256 = to_mont(x y)), and
    with radix 2^288 a second operand held as y 2^288 gives the same."""
    rng = random.Random(3)
    xs = [rng.randrange(F.p) for _ in range(20)] + [0, 1, F.p - 1]
    ys = [rng.randrange(F.p) for _ in range(20)] + [F.p - 1, 0, F.p - 1]
    got = ref.montgomery_product(F, F.to_mont(xs), F.to_mont(ys))
    assert got == F.to_mont([x * y % F.p for x, y in zip(xs, ys)])
    y288 = [(y << 288) % F.p for y in ys]
    assert ref.montgomery_product(F, F.to_mont(xs), y288, 288) == got
    # a planted mistake (radix 2^255) breaks the identity
    assert ref.montgomery_product(F, F.to_mont(xs), F.to_mont(ys), 255) != got
