"""ctypes binding of libzkntt.so: same names as the C ABI, marshalling only.

Vectors are torch tensors on a HIP device, dtype int32 (the limbs' bit
patterns), shape [n, 8], contiguous; a vector's storage is handed to the
library as a raw device pointer.  Streams are torch streams (default: the
current stream of the tensor's device).
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libzkntt.so")

FIELDS = {"bls12_381_fr": 1, "bn254_fr": 2}
FIELD_ADICITY = {"bls12_381_fr": 32, "bn254_fr": 28}

ZK_FLAG_VALIDATE = 1


class ZkError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where} failed with status {code}: {msg}")
        self.code = code


class _Opts(ctypes.Structure):
    _fields_ = [("twiddle_mode", ctypes.c_uint32), ("log2_radix", ctypes.c_uint32),
                ("log2_tile", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2509_22684_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, sz = ctypes.c_void_p, ctypes.c_size_t
        L.ntt_plan_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_uint32, ctypes.POINTER(_Opts)]
        L.ntt_plan_create.restype = ctypes.c_int
        L.ntt_plan_destroy.argtypes = [vp]
        L.ntt_plan_destroy.restype = None
        for name in ("ntt_workspace_bytes", "ntt_plan_device_bytes", "quotient_workspace_bytes"):
            getattr(L, name).argtypes = [vp]
            getattr(L, name).restype = sz
        L.ntt_plan_passes.argtypes = [vp]
        L.ntt_plan_passes.restype = ctypes.c_int
        for name in ("ntt_forward", "ntt_inverse", "ntt_coset_forward", "ntt_coset_inverse"):
            getattr(L, name).argtypes = [vp, vp, vp, vp, vp]
            getattr(L, name).restype = ctypes.c_int
        L.quotient_poly.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.quotient_poly.restype = ctypes.c_int
        L.ntt_profile_passes.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp, ctypes.POINTER(ctypes.c_float),
                                         ctypes.c_int]
        L.ntt_profile_passes.restype = ctypes.c_int
        L.zk_last_error.argtypes = []
        L.zk_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def zk_last_error() -> str:
    return lib().zk_last_error().decode()


def _check(rc: int, where: str) -> None:
    if rc != 0:
        raise ZkError(rc, where, zk_last_error())


def _ptr(t) -> int | None:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream, like=None) -> int | None:
    import torch

    if stream is None:
        dev = like.device if like is not None and hasattr(like, "device") else None
        stream = torch.cuda.current_stream(dev)
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _field_id(field) -> int:
    return FIELDS[field] if isinstance(field, str) else int(field)


# ---------------------------------------------------------------------------
# C ABI, one function per entry point

def ntt_plan_create(field, log2n: int, twiddle_mode: int = 0, log2_radix: int = 0, log2_tile: int = 0,
                    flags: int = 0) -> int:
    h = ctypes.c_void_p()
    opts = _Opts(twiddle_mode, log2_radix, log2_tile, flags)
    _check(lib().ntt_plan_create(ctypes.byref(h), _field_id(field), log2n, ctypes.byref(opts)), "ntt_plan_create")
    return h.value


def ntt_plan_destroy(plan: int) -> None:
    lib().ntt_plan_destroy(plan)


def ntt_workspace_bytes(plan: int) -> int:
    return lib().ntt_workspace_bytes(plan)


def ntt_plan_device_bytes(plan: int) -> int:
    return lib().ntt_plan_device_bytes(plan)


def ntt_plan_passes(plan: int) -> int:
    return lib().ntt_plan_passes(plan)


def quotient_workspace_bytes(plan: int) -> int:
    return lib().quotient_workspace_bytes(plan)


def _transform(name: str, plan: int, d_in, d_out, d_work=None, stream=None) -> None:
    fn = getattr(lib(), name)
    _check(fn(plan, _ptr(d_in), _ptr(d_out), _ptr(d_work), _stream(stream, d_in)), name)


def ntt_forward(plan, d_in, d_out, d_work=None, stream=None) -> None:
    _transform("ntt_forward", plan, d_in, d_out, d_work, stream)


def ntt_inverse(plan, d_in, d_out, d_work=None, stream=None) -> None:
    _transform("ntt_inverse", plan, d_in, d_out, d_work, stream)


def ntt_coset_forward(plan, d_in, d_out, d_work=None, stream=None) -> None:
    _transform("ntt_coset_forward", plan, d_in, d_out, d_work, stream)


def ntt_coset_inverse(plan, d_in, d_out, d_work=None, stream=None) -> None:
    _transform("ntt_coset_inverse", plan, d_in, d_out, d_work, stream)


def quotient_poly(plan, d_A, d_B, d_C, d_H, d_work, stream=None) -> None:
    _check(lib().quotient_poly(plan, _ptr(d_A), _ptr(d_B), _ptr(d_C), _ptr(d_H), _ptr(d_work),
                               _stream(stream, d_A)), "quotient_poly")


def ntt_profile_passes(plan, kind: int, d_in, d_out, d_work=None, stream=None) -> list:
    """Per-pass durations (ms) of one transform, from HIP events on `stream`."""
    buf = (ctypes.c_float * 64)()
    rc = lib().ntt_profile_passes(plan, kind, _ptr(d_in), _ptr(d_out), _ptr(d_work), _stream(stream, d_in), buf, 64)
    if rc < 0:
        _check(rc, "ntt_profile_passes")
    return [buf[k] for k in range(rc)]


# ---------------------------------------------------------------------------
# Convenience wrapper owning a plan and its workspaces (torch tensors)

class Plan:
    """A plan for n = 2^log2n transforms over `field` on the current device."""

    def __init__(self, field: str, log2n: int, twiddle_mode: int = 0, log2_radix: int = 0, log2_tile: int = 0,
                 flags: int = 0):
        self.field = field
        self.log2n = log2n
        self.n = 1 << log2n
        self.handle = ntt_plan_create(field, log2n, twiddle_mode, log2_radix, log2_tile, flags)
        self._work = None
        self._qwork = None

    def close(self) -> None:
        if self.handle:
            ntt_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def passes(self) -> int:
        return ntt_plan_passes(self.handle)

    @property
    def device_bytes(self) -> int:
        return ntt_plan_device_bytes(self.handle)

    def _buf(self, nbytes: int, like):
        import torch

        return torch.empty((max(nbytes, 32) + 31) // 32, 8, dtype=torch.int32, device=like.device)

    def workspace(self, like):
        nb = ntt_workspace_bytes(self.handle)
        if nb == 0:
            return None
        if self._work is None or self._work.device != like.device:
            self._work = self._buf(nb, like)
        return self._work

    def _run(self, fn, x, out, stream):
        import torch

        if out is None:
            out = torch.empty_like(x)
        fn(self.handle, x, out, self.workspace(x), stream)
        return out

    def forward(self, x, out=None, stream=None):
        return self._run(ntt_forward, x, out, stream)

    def inverse(self, x, out=None, stream=None):
        return self._run(ntt_inverse, x, out, stream)

    def coset_forward(self, x, out=None, stream=None):
        return self._run(ntt_coset_forward, x, out, stream)

    def coset_inverse(self, x, out=None, stream=None):
        return self._run(ntt_coset_inverse, x, out, stream)

    def quotient(self, A, B, C, H=None, stream=None):
        import torch

        if H is None:
            H = torch.empty_like(A)
        nb = quotient_workspace_bytes(self.handle)
        if self._qwork is None or self._qwork.device != A.device:
            self._qwork = self._buf(nb, A)
        quotient_poly(self.handle, A, B, C, H, self._qwork, stream)
        return H
