"""The butterflies' Montgomery product without its final subtraction (lazy
reduction): for any eight-limb a and canonical b the result is congruent to
a b 2^-256 mod p and below 2p, on every field, uniform, boundary and
above-p first operands.  The canonical product (variant 0) on the same
inputs is the definition itself."""
import numpy as np
import pytest

import seeded_inputs as si
from oracle import ref
from tests.gpu_util import first_mismatch, to_dev, to_host

pytestmark = pytest.mark.gpu

FIELDS = ["bls12_381_fr", "bn254_fr", "bls12_377_fr"]


def any_limbs(n: int, seed: int) -> np.ndarray:
    """n uniform 256-bit values (not reduced) as [n, 8] uint32 limbs."""
    return si.splitmix_outputs(seed, 0, 4 * n).view(np.uint32).reshape(n, 8).copy()


@pytest.mark.parametrize("field", FIELDS)
@pytest.mark.parametrize("inputs", ["uniform", "boundary", "any_a", "near_2p"])
def test_lazy_product_congruent_and_below_2p(cuda, field, inputs):
    import torch

    from paper_2509_22684_amd import zk_field_mul

    F = ref.FIELDS[field]
    p = F.p
    n = 4096 + 29
    b = si.boundary_field_vector(field, n, si.stream_seed(64, n, 1)) if inputs == "boundary" else \
        si.uniform_field_vector(field, n, si.stream_seed(64, n, 1))
    if inputs == "uniform":
        a = si.uniform_field_vector(field, n, si.stream_seed(64, n, 0))
    elif inputs == "boundary":
        a = si.boundary_field_vector(field, n, si.stream_seed(64, n, 0))
    elif inputs == "any_a":
        a = any_limbs(n, si.stream_seed(64, n, 2))
        a[:4] = np.uint32(0xFFFFFFFF)  # 2^256 - 1
    else:  # a in [p, 2p): what a butterfly may hand to the next product
        base = si.limbs_to_ints(si.uniform_field_vector(field, n, si.stream_seed(64, n, 3)))
        a = si.ints_to_limbs([p + (v % p) for v in base[:-2]] + [2 * p - 1, p])
    xs, ys = si.limbs_to_ints(a), si.limbs_to_ints(b)
    da, db = to_dev(a, cuda), to_dev(b, cuda)
    out = torch.empty_like(da)
    zk_field_mul(field, 2, da, db, out)
    torch.cuda.synchronize()
    got = si.limbs_to_ints(to_host(out))
    want = ref.montgomery_product(F, [x % p for x in xs], ys, 256)
    above = [i for i, g in enumerate(got) if g >= 2 * p]
    assert not above, f"{field} {inputs}: {len(above)} results >= 2p, first at {above[0]}"
    bad = [i for i, (g, w) in enumerate(zip(got, want)) if g % p != w]
    assert not bad, f"{field} {inputs}: {len(bad)} results not congruent, first at {bad[0]}"
    if inputs in ("uniform", "boundary"):  # canonical product: the definition, byte for byte
        zk_field_mul(field, 0, da, db, out)
        torch.cuda.synchronize()
        nbad, first = first_mismatch(to_host(out), si.ints_to_limbs(want))
        assert nbad == 0, f"{field} variant 0: {nbad} mismatches, first at {first}"


def test_field_mul_rejects_unknown_variant(cuda):
    import torch

    from paper_2509_22684_amd import ZkError, zk_field_mul

    x = torch.zeros(8, 8, dtype=torch.int32, device=cuda)
    with pytest.raises(ZkError) as e:
        zk_field_mul("bls12_381_fr", 3, x, x, x)
    assert e.value.code == -2
