"""Definitional oracle for multi-scalar multiplication on BLS12-381 G1, in
Python integers (slow; small n, or structured inputs at large n).

TEST INFRASTRUCTURE ONLY (see the package docstring).

What it computes.  The paper's other dominant kernel, MSM, is the sum
Q = s_1 P_1 + ... + s_n P_n of points P_i on an elliptic curve scaled by
scalars s_i of the scalar field (Section II-A, Fig. 4(a)); GPU libraries
compute it with Pippenger's bucket method and count its cost in point
additions and doublings (Table V).  This module holds the definition (the
group law written out in affine coordinates, scalar multiplication by
double-and-add, the naive sum) and a textbook bucket method that the tests
check against the definition.

The curve is BLS12-381 G1: y^2 = x^3 + 4 over F_q.  Its parameters all follow
from the family's seed x0 = -0xd201000000010000: the group order
r = x0^4 - x0^2 + 1 (the scalar field the NTT works over, whose modulus the
tests compare), the base field q = (x0 - 1)^2 r / 3 + x0 and the cofactor
h = (x0 - 1)^2 / 3 of the r-torsion subgroup in E(F_q), whose order is
q + 1 - (x0 + 1) = h r.

Points are tuples (x, y) of integers mod q, or None for the point at
infinity.  Device layout (the library's): a point is 24 32-bit limbs, x then
y, each 12 little-endian limbs of the Montgomery form v 2^384 mod q.
"""
from __future__ import annotations

import numpy as np

X0 = -0xD201000000010000
R = X0 ** 4 - X0 ** 2 + 1
Q = (X0 - 1) ** 2 * R // 3 + X0
H = (X0 - 1) ** 2 // 3
B = 4
Q_LIMBS = 12
Q_RBITS = 32 * Q_LIMBS


def on_curve(P) -> bool:
    if P is None:
        return True
    x, y = P
    return 0 <= x < Q and 0 <= y < Q and (y * y - x * x * x - B) % Q == 0


def neg(P):
    return None if P is None else (P[0], (-P[1]) % Q)


def add(P1, P2):
    """Chord-and-tangent addition in affine coordinates."""
    if P1 is None:
        return P2
    if P2 is None:
        return P1
    x1, y1 = P1
    x2, y2 = P2
    if x1 == x2:
        if (y1 + y2) % Q == 0:
            return None
        return dbl(P1)
    lam = (y2 - y1) * pow(x2 - x1, -1, Q) % Q
    x3 = (lam * lam - x1 - x2) % Q
    return (x3, (lam * (x1 - x3) - y1) % Q)


def dbl(P):
    if P is None or P[1] == 0:
        return None
    x, y = P
    lam = 3 * x * x * pow(2 * y, -1, Q) % Q
    x3 = (lam * lam - 2 * x) % Q
    return (x3, (lam * (x - x3) - y) % Q)


def mul(k: int, P):
    """k P by double-and-add from the top bit (k >= 0)."""
    acc = None
    for bit in bin(k)[2:] if k > 0 else "":
        acc = dbl(acc)
        if bit == "1":
            acc = add(acc, P)
    return acc


def msm_naive(scalars, points):
    """The definition: sum of s_i P_i."""
    acc = None
    for s, P in zip(scalars, points):
        acc = add(acc, mul(s, P))
    return acc


def msm_buckets(scalars, points, c: int):
    """Pippenger's bucket method with c-bit windows: for each window w, bucket
    k collects the points whose scalar has digit k there; the window's sum
    sum_k k B_k comes from running sums taken from the top bucket down; the
    windows combine by Horner's rule, c doublings per window."""
    nbits = max([s.bit_length() for s in scalars] + [1])
    windows = (nbits + c - 1) // c
    total = None
    for w in reversed(range(windows)):
        for _ in range(c):
            total = dbl(total)
        buckets = [None] * (1 << c)
        for s, P in zip(scalars, points):
            d = (s >> (c * w)) & ((1 << c) - 1)
            if d:
                buckets[d] = add(buckets[d], P)
        running, window_sum = None, None
        for k in range((1 << c) - 1, 0, -1):
            running = add(running, buckets[k])
            window_sum = add(window_sum, running)
        total = add(total, window_sum)
    return total


def sqrt_q(a: int):
    """A square root mod q (q = 3 mod 4), or None if a is not a square."""
    y = pow(a, (Q + 1) // 4, Q)
    return y if y * y % Q == a % Q else None


def point_from_candidates(cands) -> tuple:
    """The first candidate x (an integer, reduced mod q) with x^3 + 4 a
    square gives (x, y) with the even root y; scaled by the cofactor h it
    lies in the order-r subgroup.  Try-and-increment over given candidates."""
    for x in cands:
        x %= Q
        y = sqrt_q(x * x * x + B)
        if y is not None:
            if y & 1:
                y = Q - y
            P = mul(H, (x, y))
            if P is not None:
                return P
    raise ValueError("no candidate gave a point")


def subgroup_point(seed: int):
    """A point of the order-r subgroup from seeded 384-bit candidates."""
    import seeded_inputs as si

    words = si.splitmix_outputs(seed, 0, 6 * 16).reshape(16, 6)
    cands = [int.from_bytes(w.astype("<u8").tobytes(), "little") for w in words]
    return point_from_candidates(cands)


def batch_inverse(vals):
    """Inverses of nonzero field elements with one modular inversion
    (prefix products, then back-substitution)."""
    pre = [1] * (len(vals) + 1)
    for i, v in enumerate(vals):
        pre[i + 1] = pre[i] * v % Q
    inv = pow(pre[-1], -1, Q)
    out = [0] * len(vals)
    for i in range(len(vals) - 1, -1, -1):
        out[i] = pre[i] * inv % Q
        inv = inv * vals[i] % Q
    return out


def multiples(G, n: int, block: int = 1024):
    """[G, 2G, ..., nG] by affine additions, a block at a time: the block's
    additions kG + jG (j < block) share one batched inversion."""
    if n <= 0:
        return []
    base = [None]
    for j in range(1, block + 1):
        base.append(add(base[-1], G))  # base[j] = jG
    out = base[1:min(n, block) + 1]
    start = block  # out holds G .. start G
    step = base[block]  # block G
    cur = base[block]
    while len(out) < n:
        m = min(block, n - len(out))
        # (start + j) G = cur + jG for j = 1..m, cur = start G
        dens = [(base[j][0] - cur[0]) % Q for j in range(1, m + 1)]
        if any(d == 0 for d in dens):  # cur = +-jG: fall back to the plain law
            pts = [add(cur, base[j]) for j in range(1, m + 1)]
        else:
            invs = batch_inverse(dens)
            pts = []
            for j in range(1, m + 1):
                x2, y2 = base[j]
                lam = (y2 - cur[1]) * invs[j - 1] % Q
                x3 = (lam * lam - cur[0] - x2) % Q
                pts.append((x3, (lam * (cur[0] - x3) - cur[1]) % Q))
        out.extend(pts)
        cur = add(cur, step)
        start += block
    return out[:n]


# ---------------------------------------------------------------------------
# Device layout: Montgomery limbs over F_q

def fq_to_limbs(vals) -> np.ndarray:
    """[len, 12] uint32: Montgomery form v 2^384 mod q, little-endian limbs."""
    out = np.zeros((len(vals), Q_LIMBS), dtype=np.uint32)
    for i, v in enumerate(vals):
        m = (v << Q_RBITS) % Q
        out[i] = np.frombuffer(m.to_bytes(4 * Q_LIMBS, "little"), dtype="<u4")
    return out


def fq_from_limbs(a: np.ndarray) -> list:
    rinv = pow(2, -Q_RBITS, Q)
    return [int.from_bytes(np.ascontiguousarray(row, dtype="<u4").tobytes(), "little") * rinv % Q
            for row in np.asarray(a)]


def points_to_device_layout(points) -> np.ndarray:
    """[n, 24] uint32: x then y in Montgomery limbs (no point at infinity)."""
    xs = fq_to_limbs([P[0] for P in points])
    ys = fq_to_limbs([P[1] for P in points])
    return np.ascontiguousarray(np.concatenate([xs, ys], axis=1))


def xyzz_to_affine(X: int, Y: int, ZZ: int, ZZZ: int):
    """(X, Y, ZZ, ZZZ) with x = X / ZZ, y = Y / ZZZ; ZZ = 0 is infinity."""
    if ZZ % Q == 0:
        return None
    return (X * pow(ZZ, -1, Q) % Q, Y * pow(ZZZ, -1, Q) % Q)
