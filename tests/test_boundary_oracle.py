"""The boundary-value input generator, and the C oracle on such inputs pinned
to closed forms and to the Python reference (CPU only).

The closed forms follow from linearity of the transforms (Section II-B): on
raw Montgomery limbs the forward NTT of the constant vector c is
(n c mod p, 0, ..., 0), of c at index 0 it is c everywhere, and the inverse of
the constant c is (c, 0, ..., 0).  NTT(x + y) = NTT(x) + NTT(y) holds for any
x, y, which catches a modular add or subtract that mishandles sums at p.
"""
import pytest

import seeded_inputs as si
from oracle import coracle, ref

FIELDS = ["bls12_381_fr", "bn254_fr", "bls12_377_fr"]


@pytest.mark.parametrize("field", FIELDS)
def test_boundary_vector_is_canonical_seeded_and_covers_the_edges(field):
    p = si.MODULI[field]
    x = si.boundary_field_vector(field, 4096, 11)
    assert x.shape == (4096, 8)
    vals = si.limbs_to_ints(x)
    assert all(0 <= v < p for v in vals)
    assert set(si.boundary_values(field)) <= set(vals)
    assert sum(v >= p - (1 << 64) for v in vals) > 1000  # the near-p class
    assert sum(v < (1 << 64) for v in vals) > 1000  # the small class
    assert (si.boundary_field_vector(field, 4096, 11) == x).all()
    assert not (si.boundary_field_vector(field, 4096, 12) == x).all()


@pytest.mark.parametrize("field", FIELDS)
@pytest.mark.parametrize("log2n", [0, 3, 10])
def test_oracle_closed_forms_at_boundary_values(field, log2n):
    p = si.MODULI[field]
    n = 1 << log2n
    n_inv = pow(n, -1, p)
    for c in si.boundary_values(field):
        const = si.ints_to_limbs([c] * n)
        delta = si.ints_to_limbs([c] + [0] * (n - 1))
        tail = [0] * (n - 1)
        assert si.limbs_to_ints(coracle.transform(field, "forward", const)) == [n * c % p] + tail
        assert si.limbs_to_ints(coracle.transform(field, "inverse", const)) == [c] + tail
        assert si.limbs_to_ints(coracle.transform(field, "coset_inverse", const)) == [c] + tail
        assert si.limbs_to_ints(coracle.transform(field, "forward", delta)) == [c] * n
        assert si.limbs_to_ints(coracle.transform(field, "coset_forward", delta)) == [c] * n
        assert si.limbs_to_ints(coracle.transform(field, "inverse", delta)) == [c * n_inv % p] * n


@pytest.mark.parametrize("field", FIELDS)
def test_oracle_is_linear_on_boundary_inputs(field):
    p = si.MODULI[field]
    n = 1 << 9
    x = si.boundary_field_vector(field, n, 21)
    y = si.boundary_field_vector(field, n, 22)
    s = si.ints_to_limbs([(a + b) % p for a, b in zip(si.limbs_to_ints(x), si.limbs_to_ints(y))])
    for kind in ("forward", "inverse", "coset_forward", "coset_inverse"):
        fx, fy, fs = (si.limbs_to_ints(coracle.transform(field, kind, v)) for v in (x, y, s))
        assert fs == [(a + b) % p for a, b in zip(fx, fy)], kind


@pytest.mark.parametrize("field", FIELDS)
def test_oracle_matches_python_reference_on_boundary_inputs(field):
    """The C oracle (Barrett arithmetic in C) against the Python reference
    (Python big integers) on boundary inputs: the O(n^2) DFT for the forward
    kind, the reference's transforms for all four kinds, and the quotient."""
    F = ref.FIELDS[field]
    n = 1 << 6
    x = si.boundary_field_vector(field, n, 31)
    ys = si.limbs_to_ints(x)
    assert si.limbs_to_ints(coracle.transform(field, "forward", x)) == F.to_mont(ref.dft(F, F.from_mont(ys)))
    for kind in ("forward", "inverse", "coset_forward", "coset_inverse"):
        assert si.limbs_to_ints(coracle.transform(field, kind, x)) == ref.transform_mont(F, kind, ys), kind
    A, B, C = (si.boundary_field_vector(field, n, 40 + v) for v in range(3))
    want = ref.quotient_mont(F, *(si.limbs_to_ints(v) for v in (A, B, C)))
    assert si.limbs_to_ints(coracle.quotient(field, A, B, C)) == want
