"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module draws random numbers and nothing else: it holds none of the
transform's arithmetic.  Both sides of every parity check (the CPU oracle and
the HIP library) receive the same arrays from here.

Random source: SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), used in its counter form:
output k of a stream with seed s is mix64(s + (k + 1) * GOLDEN).

Field vectors: a vector of n elements is an array of shape [n, 8] of uint32,
limb 0 least significant.  Each element is drawn uniformly from [0, p) by
rejection: four 64-bit outputs form a candidate, the top word is masked to
the bit length of p, and candidates >= p are discarded.  The accepted value is
stored as the element's limbs as they are, i.e. it is the element's Montgomery
representation.  Montgomery conversion is a bijection of [0, p), so this is
the same distribution as drawing a plain value uniformly and converting it.
"""
from __future__ import annotations

import dataclasses

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# The moduli are needed here only as the upper end of the sampling range.
MODULI = {
    "bls12_381_fr": 0x73EDA753299D7D483339D80809A1D80553BDA402FFFE5BFEFFFFFFFF00000001,
    "bn254_fr": 0x30644E72E131A029B85045B68181585D2833E84879B9709143E1F593F0000001,
    "bls12_377_fr": 0x12AB655E9A2CA55660B44D1E5C37B00159AA76FED00000010A11800000000001,
}


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function applied elementwise to uint64 states."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream_seed(master: int, job: int = 0, vector: int = 0) -> int:
    """Seed of the stream that feeds vector `vector` of job `job`."""
    s = (int(master) ^ (int(job) << 20) ^ int(vector)) & 0xFFFFFFFFFFFFFFFF
    return int(mix64(np.array([s], dtype=np.uint64))[0])


def splitmix_outputs(seed: int, start: int, count: int) -> np.ndarray:
    """Outputs start .. start+count-1 of the counter-form SplitMix64 stream."""
    k = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        states = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * GOLDEN
    return mix64(states)


def _modulus_words(p: int) -> np.ndarray:
    return np.array([(p >> (64 * i)) & 0xFFFFFFFFFFFFFFFF for i in range(4)], dtype=np.uint64)


def uniform_field_vector(field: str, n: int, seed: int) -> np.ndarray:
    """n elements uniform in [0, p) as a C-contiguous [n, 8] uint32 array."""
    p = MODULI[field]
    pw = _modulus_words(p)
    top_mask = np.uint64((1 << (p.bit_length() - 192)) - 1)
    out = np.empty((n, 4), dtype=np.uint64)
    filled = 0
    drawn = 0  # candidates consumed so far
    while filled < n:
        want = n - filled
        batch = max(1024, int(want * 1.35) + 64)
        raw = splitmix_outputs(seed, 4 * drawn, 4 * batch).reshape(batch, 4)
        raw[:, 3] &= top_mask
        # candidate < p, compared from the top word down
        lt = np.zeros(batch, dtype=bool)
        eq = np.ones(batch, dtype=bool)
        for w in (3, 2, 1, 0):
            lt |= eq & (raw[:, w] < pw[w])
            eq &= raw[:, w] == pw[w]
        acc = raw[lt]
        take = min(want, acc.shape[0])
        out[filled:filled + take] = acc[:take]
        filled += take
        if take < acc.shape[0]:
            break
        drawn += batch
    return np.ascontiguousarray(out).view(np.uint32).reshape(n, 8)


def boundary_values(field: str) -> list[int]:
    """Values at the edges of [0, p) and of the 32-bit limbs: 0..3, p - 1 ..
    p - 3, (p -+ 1) / 2, the largest values of 1, 2, 4 and 6 limbs, 2^32 and
    2^64, the largest power of two below p, 2^256 mod p, and p minus 2^32,
    2^64 and 2^128.  All are canonical (< p)."""
    p = MODULI[field]
    top = 1 << (p.bit_length() - 1)
    vals = [0, 1, 2, 3, p - 1, p - 2, p - 3, (p - 1) // 2, (p + 1) // 2,
            (1 << 32) - 1, 1 << 32, (1 << 64) - 1, 1 << 64, (1 << 128) - 1, (1 << 192) - 1,
            top, (1 << 256) % p, p - (1 << 32), p - (1 << 64), p - (1 << 128)]
    assert all(0 <= v < p for v in vals)
    return vals


def boundary_field_vector(field: str, n: int, seed: int) -> np.ndarray:
    """n canonical elements concentrated at the edges of the range, as an
    [n, 8] uint32 array: per element, one stream output picks the class --
    a value from boundary_values, p - 1 - s or s with s a random number of
    random bit length below 64, or a uniform element -- and a second one
    picks the value within the class."""
    p = MODULI[field]
    vals = boundary_values(field)
    uni = limbs_to_ints(uniform_field_vector(field, n, seed ^ 0x5EED))
    u = splitmix_outputs(seed, 0, 2 * n).reshape(n, 2)
    out = []
    for i in range(n):
        a, b = int(u[i, 0]), int(u[i, 1])
        cls = a & 3
        if cls == 0:
            out.append(vals[(a >> 8) % len(vals)])
        elif cls == 1:
            out.append(p - 1 - (b >> ((a >> 8) & 63)))
        elif cls == 2:
            out.append(b >> ((a >> 8) & 63))
        else:
            out.append(uni[i])
    return ints_to_limbs(out)


def limbs_to_ints(a: np.ndarray) -> list[int]:
    """[n, 8] uint32 limbs to Python ints (no reduction, no conversion)."""
    a = np.ascontiguousarray(a, dtype=np.uint32)
    b = a.astype("<u4").tobytes()
    return [int.from_bytes(b[32 * i:32 * i + 32], "little") for i in range(a.shape[0])]


def ints_to_limbs(xs) -> np.ndarray:
    """Python ints in [0, 2^256) to an [n, 8] uint32 limb array."""
    xs = list(xs)
    buf = b"".join(int(x).to_bytes(32, "little") for x in xs)
    return np.frombuffer(buf, dtype="<u4").reshape(len(xs), 8).astype(np.uint32)


# ---------------------------------------------------------------------------
# Workload recipes.  Master seeds 1..5 label the five workloads below.

@dataclasses.dataclass(frozen=True)
class BatchJob:
    field: str
    log2n: int
    seed: int


def batch_jobs(master: int = 4, njobs: int = 64, n_bn: int = 16, lo: int = 10, hi: int = 18) -> list[BatchJob]:
    """64 independent forward NTTs: log2 n uniform on [lo, hi] inclusive; the
    n_bn BN254 slots are picked by a seeded shuffle, the rest are BLS12-381."""
    rng = np.random.Generator(np.random.PCG64(master))
    sizes = rng.integers(lo, hi + 1, size=njobs)
    slots = rng.permutation(njobs)
    is_bn = np.zeros(njobs, dtype=bool)
    is_bn[slots[:n_bn]] = True
    return [
        BatchJob("bn254_fr" if is_bn[j] else "bls12_381_fr", int(sizes[j]), stream_seed(master, j, 0))
        for j in range(njobs)
    ]


@dataclasses.dataclass(frozen=True)
class ServeJob:
    job_id: int
    log2n: int
    arrival_s: float
    seeds: tuple  # seeds of A, B, C


def serve_jobs(master: int = 5, njobs: int = 256, rate_per_s: float = 100.0,
               lo: int = 14, hi: int = 22) -> list[ServeJob]:
    """Quotient jobs with Poisson arrivals at `rate_per_s` and log2 n uniform
    on [lo, hi] inclusive, all on BLS12-381 Fr."""
    rng = np.random.Generator(np.random.PCG64(master))
    gaps = rng.exponential(1.0 / rate_per_s, size=njobs)
    sizes = rng.integers(lo, hi + 1, size=njobs)
    t = np.cumsum(gaps) - gaps[0]
    return [
        ServeJob(j, int(sizes[j]), float(t[j]),
                 tuple(stream_seed(master, j, v) for v in range(3)))
        for j in range(njobs)
    ]
