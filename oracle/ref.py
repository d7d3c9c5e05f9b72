"""Definitional oracle in Python integers (slow; small n only).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Notation follows the paper's background on the NTT (Section II-B): a vector
a = [a_0 .. a_{n-1}] of field elements maps to A with
A_i = sum_j a_j * w^(i*j), w a primitive n-th root of unity; the fast
algorithm is radix-2 Cooley-Tukey with n/2 butterflies per stage over
log2(n) stages (Fig. 4(b)).  The Groth16 prover computes the quotient h with
forward and inverse NTTs and elementwise products (Section II, Fig. 3;
seven NTTs, Section IV-A).

Readings where the paper is silent:
* w_n = g^((p-1)/n) with g the smallest multiplicative generator
  (7 for BLS12-381 Fr, 5 for BN254 Fr, 22 for BLS12-377 Fr).
* natural order in and out; inverse = transform with w^-1, scaled by n^-1.
* coset NTT evaluates on g*<w>: coefficient j is multiplied by g^j first.
* quotient: H = cosetINTT((cosetNTT(INTT A) . cosetNTT(INTT B)
  - cosetNTT(INTT C)) * (g^n - 1)^-1); Z_H(x) = x^n - 1 equals g^n - 1 at
  every coset point.
"""
from __future__ import annotations

import dataclasses

R_BITS = 256


@dataclasses.dataclass(frozen=True)
class Field:
    name: str
    p: int
    generator: int
    two_adicity: int

    @property
    def R(self) -> int:
        """Montgomery radix 2^256 reduced mod p."""
        return pow(2, R_BITS, self.p)

    @property
    def R_inv(self) -> int:
        return pow(2, -R_BITS, self.p)

    def root(self, n: int) -> int:
        """Primitive n-th root of unity g^((p-1)/n), n a power of two."""
        if n <= 0 or n & (n - 1) or n > (1 << self.two_adicity):
            raise ValueError(f"no power-of-two root of order {n}")
        return pow(self.generator, (self.p - 1) // n, self.p)

    # Montgomery boundary: stored value y represents y * 2^-256 mod p.
    def from_mont(self, ys):
        return [(y * self.R_inv) % self.p for y in ys]

    def to_mont(self, xs):
        return [(x << R_BITS) % self.p for x in xs]


BLS12_381_FR = Field(
    "bls12_381_fr",
    0x73EDA753299D7D483339D80809A1D80553BDA402FFFE5BFEFFFFFFFF00000001,
    7,
    32,
)
BN254_FR = Field(
    "bn254_fr",
    0x30644E72E131A029B85045B68181585D2833E84879B9709143E1F593F0000001,
    5,
    28,
)
BLS12_377_FR = Field(
    "bls12_377_fr",
    0x12AB655E9A2CA55660B44D1E5C37B00159AA76FED00000010A11800000000001,
    22,
    47,
)
FIELDS = {f.name: f for f in (BLS12_381_FR, BN254_FR, BLS12_377_FR)}


def _log2(n: int) -> int:
    if n <= 0 or n & (n - 1):
        raise ValueError("length must be a power of two")
    return n.bit_length() - 1


# --------------------------------------------------------------------------
# Plain definitions (quadratic).

def dft(F: Field, a, w=None):
    """A_i = sum_j a_j w^(i j) (Section II-B), straight from the definition."""
    n = len(a)
    p = F.p
    if w is None:
        w = F.root(n)
    out = []
    for i in range(n):
        wi = pow(w, i, p)
        acc = 0
        x = 1
        for j in range(n):
            acc = (acc + a[j] * x) % p
            x = x * wi % p
        out.append(acc)
    return out


def idft(F: Field, A):
    """a_j = n^-1 sum_i A_i w^(-i j): the definition of the inverse transform."""
    n = len(A)
    winv = pow(F.root(n), -1, F.p)
    ninv = pow(n, -1, F.p)
    return [x * ninv % F.p for x in dft(F, A, winv)]


def horner(F: Field, coeffs, x: int) -> int:
    """Evaluate sum_j coeffs_j x^j."""
    acc = 0
    for c in reversed(coeffs):
        acc = (acc * x + c) % F.p
    return acc


# --------------------------------------------------------------------------
# Radix-2 Cooley-Tukey (Section II-B, Fig. 4(b)).

def bit_reverse(a):
    n = len(a)
    k = _log2(n)
    out = list(a)
    for i in range(n):
        j = int(format(i, f"0{k}b")[::-1], 2) if k else 0
        if j > i:
            out[i], out[j] = out[j], out[i]
    return out


def ntt_radix2(F: Field, a, w=None):
    """Iterative decimation-in-time radix-2 NTT, natural order in and out.

    Bit-reverse the input, then for each stage with span m = 2, 4, ..., n
    apply the butterfly (x, y) -> (x + w_m^j y, x - w_m^j y) to every pair
    (b + j, b + j + m/2), w_m = w^(n/m).
    """
    n = len(a)
    p = F.p
    if w is None:
        w = F.root(n)
    x = bit_reverse([v % p for v in a])
    m = 2
    while m <= n:
        wm = pow(w, n // m, p)
        half = m // 2
        tw = [1] * half
        for j in range(1, half):
            tw[j] = tw[j - 1] * wm % p
        for b in range(0, n, m):
            for j in range(half):
                u = x[b + j]
                t = tw[j] * x[b + j + half] % p
                x[b + j] = (u + t) % p
                x[b + j + half] = (u - t) % p
        m *= 2
    return x


def ntt(F: Field, a):
    """Forward NTT of plain values (Section II-B)."""
    return ntt_radix2(F, a)


def intt(F: Field, A):
    """Inverse NTT: transform with w^-1, then scale by n^-1."""
    n = len(A)
    winv = pow(F.root(n), -1, F.p)
    ninv = pow(n, -1, F.p)
    return [v * ninv % F.p for v in ntt_radix2(F, A, winv)]


def coset_ntt(F: Field, a):
    """Evaluations on the coset g<w>: NTT(a_j g^j)."""
    p = F.p
    scaled = []
    gj = 1
    for v in a:
        scaled.append(v * gj % p)
        gj = gj * F.generator % p
    return ntt(F, scaled)


def coset_intt(F: Field, A):
    """Coefficients from coset evaluations: INTT(A)_j g^-j."""
    p = F.p
    ginv = pow(F.generator, -1, p)
    out = []
    gj = 1
    for v in intt(F, A):
        out.append(v * gj % p)
        gj = gj * ginv % p
    return out


def quotient(F: Field, A, B, C):
    """Groth16 quotient chain (Section II, Fig. 3; seven NTTs, Section IV-A).

    Inputs are evaluations on <w>; the output is the coefficient vector of
    h = (a b - c) / Z_H computed on the coset, where Z_H = g^n - 1.
    """
    n = len(A)
    p = F.p
    ah = coset_ntt(F, intt(F, A))
    bh = coset_ntt(F, intt(F, B))
    ch = coset_ntt(F, intt(F, C))
    zinv = pow(pow(F.generator, n, p) - 1, -1, p)
    e = [((x * y - z) * zinv) % p for x, y, z in zip(ah, bh, ch)]
    return coset_intt(F, e)


# --------------------------------------------------------------------------
# Montgomery-boundary wrappers: the library's inputs and outputs are
# Montgomery representations; the transforms are linear, so the wrapped
# result is to_mont(f(from_mont(y))).

_KINDS = {"forward": ntt, "inverse": intt, "coset_forward": coset_ntt, "coset_inverse": coset_intt}


def transform_mont(F: Field, kind: str, ys):
    return F.to_mont(_KINDS[kind](F, F.from_mont(ys)))


def quotient_mont(F: Field, As, Bs, Cs):
    return F.to_mont(quotient(F, F.from_mont(As), F.from_mont(Bs), F.from_mont(Cs)))


def montgomery_product(F: Field, xs, ys, radix_bits: int = R_BITS):
    """Montgomery product with radix 2^radix_bits, by its definition:
    x y 2^-radix_bits mod p for each pair (the FF_mul of the paper's
    finite-field layer, Section IV-B, in Montgomery form).  With radix 2^256
    it multiplies two stored elements; the FP64 multiplier uses 2^288."""
    k = pow(2, -radix_bits, F.p)
    return [x * y % F.p * k % F.p for x, y in zip(xs, ys)]
