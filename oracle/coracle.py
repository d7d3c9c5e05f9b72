"""ctypes wrapper of the C oracle (ntt_oracle.c).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Inputs and outputs are
[n, 8] uint32 arrays of Montgomery-form limbs, like the library's; the C code
converts to plain residues with its own arithmetic (Barrett, never
Montgomery multiplication) and back.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ntt_oracle.c")
LIB = os.path.join(HERE, "libntt_oracle.so")

FIELD_IDS = {"bls12_381_fr": 1, "bn254_fr": 2, "bls12_377_fr": 3}
KINDS = {"forward": 0, "inverse": 1, "coset_forward": 2, "coset_inverse": 3}


def build(force: bool = True) -> str:
    """Compile ntt_oracle.c into libntt_oracle.so with gcc."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared", "-pthread",
                               SRC, "-o", tmp])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        L = ctypes.CDLL(LIB)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        L.orc_transform.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, u32p, u32p, ctypes.c_int]
        L.orc_quotient.argtypes = [ctypes.c_int, ctypes.c_int, u32p, u32p, u32p, u32p, ctypes.c_int]
        L.orc_eval_at_roots.argtypes = [ctypes.c_int, ctypes.c_int, u32p, u64p, ctypes.c_int, u32p, ctypes.c_int]
        L.orc_field_op.argtypes = [ctypes.c_int, ctypes.c_int, u32p, u32p, u32p, ctypes.c_int]
        L.orc_constant.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, u32p]
        for f in (L.orc_transform, L.orc_quotient, L.orc_eval_at_roots, L.orc_field_op, L.orc_constant):
            f.restype = ctypes.c_int
        _lib = L
    return _lib


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        return os.cpu_count() or 1


def _u32(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def _vec(a) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint32)
    if a.ndim != 2 or a.shape[1] != 8:
        raise ValueError("expected an [n, 8] uint32 array")
    return a


def _log2(n: int) -> int:
    if n <= 0 or n & (n - 1):
        raise ValueError("length must be a power of two")
    return n.bit_length() - 1


def transform(field: str, kind: str, a, threads: int | None = None) -> np.ndarray:
    a = _vec(a)
    out = np.empty_like(a)
    rc = lib().orc_transform(FIELD_IDS[field], _log2(a.shape[0]), KINDS[kind], _u32(a), _u32(out),
                             threads or default_threads())
    if rc:
        raise RuntimeError(f"orc_transform failed: {rc}")
    return out


def quotient(field: str, A, B, C, threads: int | None = None) -> np.ndarray:
    A, B, C = _vec(A), _vec(B), _vec(C)
    if not (A.shape == B.shape == C.shape):
        raise ValueError("A, B, C must have the same shape")
    H = np.empty_like(A)
    rc = lib().orc_quotient(FIELD_IDS[field], _log2(A.shape[0]), _u32(A), _u32(B), _u32(C), _u32(H),
                            threads or default_threads())
    if rc:
        raise RuntimeError(f"orc_quotient failed: {rc}")
    return H


def eval_at_roots(field: str, coeffs, idx, threads: int | None = None) -> np.ndarray:
    """sum_j coeffs_j w^(i j) for each i in idx, by Horner's rule."""
    c = _vec(coeffs)
    idx = np.ascontiguousarray(idx, dtype=np.uint64)
    out = np.empty((idx.shape[0], 8), dtype=np.uint32)
    rc = lib().orc_eval_at_roots(FIELD_IDS[field], _log2(c.shape[0]), _u32(c),
                                 idx.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), idx.shape[0], _u32(out),
                                 threads or default_threads())
    if rc:
        raise RuntimeError(f"orc_eval_at_roots failed: {rc}")
    return out


def field_op(field: str, op: str, a, b) -> np.ndarray:
    ops = {"add": 0, "sub": 1, "mul": 2, "inv": 3, "pow": 4}
    a, b = _vec(a), _vec(b)
    out = np.empty_like(a)
    rc = lib().orc_field_op(FIELD_IDS[field], ops[op], _u32(a), _u32(b), _u32(out), a.shape[0])
    if rc:
        raise RuntimeError(f"orc_field_op failed: {rc}")
    return out


def constant(field: str, which: str, log2n: int = 0) -> int:
    w = {"modulus": 0, "mu": 1, "r_mod": 2, "root": 3}[which]
    out = np.zeros(10, dtype=np.uint32)
    rc = lib().orc_constant(FIELD_IDS[field], w, log2n, _u32(out))
    if rc:
        raise RuntimeError(f"orc_constant failed: {rc}")
    return int.from_bytes(out.astype("<u4").tobytes(), "little")
