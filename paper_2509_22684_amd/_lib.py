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

FIELDS = {"bls12_381_fr": 1, "bn254_fr": 2, "bls12_377_fr": 3}
FIELD_ADICITY = {"bls12_381_fr": 32, "bn254_fr": 28, "bls12_377_fr": 47}

ZK_FLAG_VALIDATE = 1
ZK_FLAG_FFMUL_FP64 = 2


class ZkError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where} failed with status {code}: {msg}")
        self.code = code


class _Opts(ctypes.Structure):
    _fields_ = [("twiddle_mode", ctypes.c_uint32), ("log2_radix", ctypes.c_uint32),
                ("log2_tile", ctypes.c_uint32), ("flags", ctypes.c_uint32), ("log2_pass_radix", ctypes.c_uint32)]


class _BatchJob(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("op", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("in_", ctypes.c_void_p), ("in2", ctypes.c_void_p), ("in3", ctypes.c_void_p),
                ("out", ctypes.c_void_p), ("work", ctypes.c_void_p)]


OPS = {"forward": 0, "inverse": 1, "coset_forward": 2, "coset_inverse": 3, "inverse_to_coset": 4,
       "quotient_pointwise": 5}
ZK_BATCH_GRAPH = 1
ZK_BATCH_DIRECT = 2
ZK_BATCH_QUEUES_SHIFT = 8

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
        L.ntt_tuning_register.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.POINTER(_Opts)]
        L.ntt_tuning_register.restype = ctypes.c_int
        L.ntt_tuning_clear.argtypes = []
        L.ntt_tuning_clear.restype = None
        L.ntt_plan_resolve_opts.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.POINTER(_Opts),
                                            ctypes.POINTER(_Opts)]
        L.ntt_plan_resolve_opts.restype = ctypes.c_int
        L.ntt_plan_table_bytes.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.POINTER(_Opts)]
        L.ntt_plan_table_bytes.restype = sz
        L.ntt_plan_get_opts.argtypes = [vp, ctypes.POINTER(_Opts)]
        L.ntt_plan_get_opts.restype = ctypes.c_int
        for name in ("ntt_workspace_bytes", "ntt_plan_device_bytes", "quotient_workspace_bytes"):
            getattr(L, name).argtypes = [vp]
            getattr(L, name).restype = sz
        L.ntt_plan_passes.argtypes = [vp]
        L.ntt_plan_passes.restype = ctypes.c_int
        for name in ("ntt_forward", "ntt_inverse", "ntt_coset_forward", "ntt_coset_inverse"):
            getattr(L, name).argtypes = [vp, vp, vp, vp, vp]
            getattr(L, name).restype = ctypes.c_int
        L.ntt_forward_noalloc.argtypes = [vp, vp, vp, vp]
        L.ntt_forward_noalloc.restype = ctypes.c_int
        L.quotient_poly.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.quotient_poly.restype = ctypes.c_int
        L.quotient_coset_evals.argtypes = [vp, vp, vp, vp, vp]
        L.quotient_coset_evals.restype = ctypes.c_int
        L.quotient_pointwise.argtypes = [vp, vp, vp, vp, vp, vp]
        L.quotient_pointwise.restype = ctypes.c_int
        L.zk_copy_to_host.argtypes = [vp, vp, sz, vp]
        L.zk_copy_to_host.restype = ctypes.c_int
        L.ntt_profile_passes.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp, ctypes.POINTER(ctypes.c_float),
                                         ctypes.c_int]
        L.ntt_profile_passes.restype = ctypes.c_int
        pp = ctypes.POINTER(vp)
        L.ntt_batch_workspace_bytes.argtypes = [pp, ctypes.c_int]
        L.ntt_batch_workspace_bytes.restype = sz
        L.ntt_batch_create.argtypes = [pp, pp, pp, ctypes.c_int, vp]
        L.ntt_batch_create.restype = ctypes.c_int
        for name in ("ntt_batch_launch", "ntt_batch_launch_eager"):
            getattr(L, name).argtypes = [vp, vp]
            getattr(L, name).restype = ctypes.c_int
        for name in ("ntt_batch_status", "ntt_batch_items", "ntt_batch_grid"):
            getattr(L, name).argtypes = [vp]
            getattr(L, name).restype = ctypes.c_int
        L.ntt_batch_set_spin_limit.argtypes = [vp, ctypes.c_uint32]
        L.ntt_batch_set_spin_limit.restype = ctypes.c_int
        L.ntt_batch_destroy.argtypes = [vp]
        L.ntt_batch_destroy.restype = None
        L.ntt_batch_create_jobs.argtypes = [pp, ctypes.POINTER(_BatchJob), ctypes.c_int, ctypes.c_int]
        L.ntt_batch_create_jobs.restype = ctypes.c_int
        L.ntt_batch_forward.argtypes = [pp, pp, ctypes.c_int, vp, vp]
        L.ntt_batch_forward.restype = ctypes.c_int
        L.zk_microbench.argtypes = [ctypes.c_int, ctypes.c_uint32, vp, sz, vp, ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_float)]
        L.zk_microbench.restype = ctypes.c_int
        L.zk_field_mul.argtypes = [ctypes.c_int, ctypes.c_int, vp, vp, vp, ctypes.c_uint64, vp]
        L.zk_field_mul.restype = ctypes.c_int
        L.msm_bases_create.argtypes = [ctypes.POINTER(vp), vp, ctypes.c_uint64, ctypes.c_uint32, vp]
        L.msm_bases_create.restype = ctypes.c_int
        L.msm_bases_destroy.argtypes = [vp]
        L.msm_bases_destroy.restype = None
        L.msm_bases_count.argtypes = [vp]
        L.msm_bases_count.restype = ctypes.c_uint64
        L.msm_bases_window_bits.argtypes = [vp]
        L.msm_bases_window_bits.restype = ctypes.c_int
        for name in ("msm_bases_device_bytes", "msm_workspace_bytes"):
            getattr(L, name).argtypes = [vp]
            getattr(L, name).restype = sz
        L.msm_compute.argtypes = [vp, vp, vp, vp, vp]
        L.msm_compute.restype = ctypes.c_int
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
                    flags: int = 0, log2_pass_radix: int = 0) -> int:
    h = ctypes.c_void_p()
    opts = _Opts(twiddle_mode, log2_radix, log2_tile, flags, log2_pass_radix)
    _check(lib().ntt_plan_create(ctypes.byref(h), _field_id(field), log2n, ctypes.byref(opts)), "ntt_plan_create")
    return h.value


def ntt_plan_destroy(plan: int) -> None:
    lib().ntt_plan_destroy(plan)


_OPT_KEYS = ("twiddle_mode", "log2_radix", "log2_tile", "flags", "log2_pass_radix")


def _opts_dict(o: _Opts) -> dict:
    return {k: int(getattr(o, k)) for k in _OPT_KEYS}


def ntt_tuning_register(field, log2n: int, twiddle_mode: int = 0, log2_radix: int = 0, log2_tile: int = 0,
                        log2_pass_radix: int = 0) -> None:
    opts = _Opts(twiddle_mode, log2_radix, log2_tile, 0, log2_pass_radix)
    _check(lib().ntt_tuning_register(_field_id(field), log2n, ctypes.byref(opts)), "ntt_tuning_register")


def ntt_tuning_clear() -> None:
    lib().ntt_tuning_clear()


def ntt_plan_resolve_opts(field, log2n: int, twiddle_mode: int = 0, log2_radix: int = 0, log2_tile: int = 0,
                          flags: int = 0, log2_pass_radix: int = 0) -> dict:
    """The schedule ntt_plan_create would pick (host only; no device needed)."""
    opts = _Opts(twiddle_mode, log2_radix, log2_tile, flags, log2_pass_radix)
    out = _Opts()
    _check(lib().ntt_plan_resolve_opts(_field_id(field), log2n, ctypes.byref(opts), ctypes.byref(out)),
           "ntt_plan_resolve_opts")
    return _opts_dict(out)


def ntt_plan_table_bytes(field, log2n: int, twiddle_mode: int = 0, log2_radix: int = 0, log2_tile: int = 0,
                         flags: int = 0, log2_pass_radix: int = 0) -> int:
    """Device bytes of the tables a plan would hold (host only; 0 if the
    arguments are unsupported)."""
    opts = _Opts(twiddle_mode, log2_radix, log2_tile, flags, log2_pass_radix)
    return lib().ntt_plan_table_bytes(_field_id(field), log2n, ctypes.byref(opts))


def ntt_plan_get_opts(plan: int) -> dict:
    out = _Opts()
    _check(lib().ntt_plan_get_opts(plan, ctypes.byref(out)), "ntt_plan_get_opts")
    return _opts_dict(out)


_tuning_loaded = set()


def register_tuning_db(device: str, path: str | None = None, force: bool = False) -> int:
    """Register the stand-alone ("single") schedules that the autotuner's
    database holds for `device` (a gcnArchName such as
    "gfx950:sramecc+:xnack-"), so that plans created afterwards with zero
    options run them.  Once per (device, path) unless force.  Returns the
    number of schedules registered."""
    import json

    from .autotune import db_path

    path = path or db_path()
    key = (device, os.path.abspath(path))
    if key in _tuning_loaded and not force:
        return 0
    _tuning_loaded.add(key)
    if not os.path.exists(path):
        return 0
    with open(path) as f:
        entries = json.load(f).get("devices", {}).get(device, {})
    count = 0
    for k, e in entries.items():
        field, log2n, mode = k.split(":")
        if mode != "single" or field not in FIELDS:
            continue
        o = {kk: int(v) for kk, v in e["opts"].items() if kk in _OPT_KEYS and kk != "flags"}
        ntt_tuning_register(field, int(log2n), **o)
        count += 1
    return count


def _register_tuning_for_current_device() -> None:
    import torch

    dev = torch.cuda.current_device()
    props = torch.cuda.get_device_properties(dev)
    register_tuning_db(getattr(props, "gcnArchName", props.name))


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


def ntt_forward_noalloc(plan, d_in, d_out, stream=None) -> None:
    _check(lib().ntt_forward_noalloc(plan, _ptr(d_in), _ptr(d_out), _stream(stream, d_in)), "ntt_forward_noalloc")


def ntt_inverse(plan, d_in, d_out, d_work=None, stream=None) -> None:
    _transform("ntt_inverse", plan, d_in, d_out, d_work, stream)


def ntt_coset_forward(plan, d_in, d_out, d_work=None, stream=None) -> None:
    _transform("ntt_coset_forward", plan, d_in, d_out, d_work, stream)


def ntt_coset_inverse(plan, d_in, d_out, d_work=None, stream=None) -> None:
    _transform("ntt_coset_inverse", plan, d_in, d_out, d_work, stream)


def quotient_poly(plan, d_A, d_B, d_C, d_H, d_work, stream=None) -> None:
    _check(lib().quotient_poly(plan, _ptr(d_A), _ptr(d_B), _ptr(d_C), _ptr(d_H), _ptr(d_work),
                               _stream(stream, d_A)), "quotient_poly")


def quotient_coset_evals(plan, d_in, d_out, d_work=None, stream=None) -> None:
    _check(lib().quotient_coset_evals(plan, _ptr(d_in), _ptr(d_out), _ptr(d_work), _stream(stream, d_in)),
           "quotient_coset_evals")


def quotient_pointwise(plan, d_A, d_B, d_C, d_out, stream=None) -> None:
    _check(lib().quotient_pointwise(plan, _ptr(d_A), _ptr(d_B), _ptr(d_C), _ptr(d_out), _stream(stream, d_A)),
           "quotient_pointwise")


def zk_copy_to_host(host_dst, dev_src, nbytes: int | None = None, stream=None) -> None:
    """Device -> pinned host copy run by a kernel (overlaps DMA uploads)."""
    if nbytes is None:
        nbytes = dev_src.numel() * dev_src.element_size()
    _check(lib().zk_copy_to_host(_ptr(host_dst), _ptr(dev_src), nbytes, _stream(stream, dev_src)),
           "zk_copy_to_host")


def ntt_profile_passes(plan, kind: int, d_in, d_out, d_work=None, stream=None) -> list:
    """Per-pass durations (ms) of one transform, from HIP events on `stream`."""
    buf = (ctypes.c_float * 64)()
    rc = lib().ntt_profile_passes(plan, kind, _ptr(d_in), _ptr(d_out), _ptr(d_work), _stream(stream, d_in), buf, 64)
    if rc < 0:
        _check(rc, "ntt_profile_passes")
    return [buf[k] for k in range(rc)]


def zk_field_mul(field, variant: int, d_a, d_b, d_out, n: int | None = None, stream=None) -> None:
    """out = a b 2^-256 (variant 0, integer) or a b 2^-288 (variant 1, FP64) mod p, element-wise;
    variant 2: the integer product without its final subtraction (congruent, in [0, 2p))."""
    if n is None:
        n = d_a.shape[0]
    _check(lib().zk_field_mul(_field_id(field), variant, _ptr(d_a), _ptr(d_b), _ptr(d_out), n,
                              _stream(stream, d_a)), "zk_field_mul")


MICROBENCH = {"mad_u64_u32": 0, "fma_f64": 1, "add_u32": 2, "addc_u32": 3, "mad_addc": 4,
              "ffmul_bls12_381": 5, "copy": 6, "ffmul_k2": 7, "ffmul_k4": 8, "mad_fma": 9, "mad_add": 10,
              "ffmul_f64": 11, "ffmul_lazy": 12, "ffmul_bn254": 13}


def zk_microbench(kind: str, d_buf, iters: int = 256, reps: int = 5, stream=None, buf_bytes: int | None = None):
    """(rate per second, ms per launch) of one micro-benchmark kernel."""
    ops, ms = ctypes.c_double(), ctypes.c_float()
    if buf_bytes is None:
        buf_bytes = d_buf.numel() * d_buf.element_size()
    rc = lib().zk_microbench(MICROBENCH[kind], iters, _ptr(d_buf), buf_bytes, _stream(stream, d_buf), reps,
                             ctypes.byref(ops), ctypes.byref(ms))
    if rc != 0:
        raise ZkError(rc, "zk_microbench", zk_last_error())
    return ops.value, ms.value


# ---------------------------------------------------------------------------
# Convenience wrapper owning a plan and its workspaces (torch tensors)

class Plan:
    """A plan for n = 2^log2n transforms over `field` on the current device."""

    def __init__(self, field: str, log2n: int, twiddle_mode: int = 0, log2_radix: int = 0, log2_tile: int = 0,
                 flags: int = 0, log2_pass_radix: int = 0):
        self.field = field
        self.log2n = log2n
        self.n = 1 << log2n
        # zero options resolve through the tuning database's schedule for
        # this device (registered once per process), then the defaults
        _register_tuning_for_current_device()
        self.handle = ntt_plan_create(field, log2n, twiddle_mode, log2_radix, log2_tile, flags, log2_pass_radix)
        self.opts = ntt_plan_get_opts(self.handle)
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

    def coset_evals(self, x, out=None, stream=None, work=None):
        """cosetNTT(INTT(x)): the first two transforms of the quotient chain."""
        import torch

        if out is None:
            out = torch.empty_like(x)
        quotient_coset_evals(self.handle, x, out, work if work is not None else self.workspace(x), stream)
        return out

    def pointwise(self, A, B, C, out=None, stream=None):
        """(A B - C) / (g^n - 1) elementwise: the quotient chain's pointwise step."""
        import torch

        if out is None:
            out = torch.empty_like(A)
        quotient_pointwise(self.handle, A, B, C, out, stream)
        return out

    def quotient(self, A, B, C, H=None, stream=None):
        import torch

        if H is None:
            H = torch.empty_like(A)
        nb = quotient_workspace_bytes(self.handle)
        if self._qwork is None or self._qwork.device != A.device:
            self._qwork = self._buf(nb, A)
        quotient_poly(self.handle, A, B, C, H, self._qwork, stream)
        return H


# ---------------------------------------------------------------------------
# Batches

def _ptr_array(xs):
    arr = (ctypes.c_void_p * max(1, len(xs)))()
    for i, x in enumerate(xs):
        arr[i] = _ptr(x)
    return arr


def _handles(plans):
    return [p.handle if isinstance(p, Plan) else p for p in plans]


def ntt_batch_workspace_bytes(plans) -> int:
    hs = _handles(plans)
    return lib().ntt_batch_workspace_bytes(_ptr_array(hs), len(hs))


def ntt_batch_create(plans, d_bufs, d_work=None) -> int:
    hs = _handles(plans)
    if len(hs) != len(d_bufs):
        raise ValueError("one buffer per plan")
    h = ctypes.c_void_p()
    _check(lib().ntt_batch_create(ctypes.byref(h), _ptr_array(hs), _ptr_array(d_bufs), len(hs), _ptr(d_work)),
           "ntt_batch_create")
    return h.value


def ntt_batch_create_jobs(jobs, graph: bool = False, queues: int = 0, direct: bool = False) -> int:
    """jobs: dicts with keys plan, op (name or zk_op), in, out and optionally
    in2, in3 (pointwise) and work.  queues: work queues per field (0: default);
    direct: every job as pass launches, no persistent kernel."""
    arr = (_BatchJob * max(1, len(jobs)))()
    for k, j in enumerate(jobs):
        plan = j["plan"]
        arr[k].plan = plan.handle if isinstance(plan, Plan) else plan
        op = j["op"]
        arr[k].op = OPS[op] if isinstance(op, str) else int(op)
        arr[k].in_ = _ptr(j.get("in"))
        arr[k].in2 = _ptr(j.get("in2"))
        arr[k].in3 = _ptr(j.get("in3"))
        arr[k].out = _ptr(j.get("out"))
        arr[k].work = _ptr(j.get("work"))
    h = ctypes.c_void_p()
    flags = (ZK_BATCH_GRAPH if graph else 0) | (ZK_BATCH_DIRECT if direct else 0) | (int(queues) << ZK_BATCH_QUEUES_SHIFT)
    _check(lib().ntt_batch_create_jobs(ctypes.byref(h), arr, len(jobs), flags), "ntt_batch_create_jobs")
    return h.value


def ntt_batch_launch(batch: int, stream=None) -> None:
    _check(lib().ntt_batch_launch(batch, _stream(stream)), "ntt_batch_launch")


def ntt_batch_launch_eager(batch: int, stream=None) -> None:
    _check(lib().ntt_batch_launch_eager(batch, _stream(stream)), "ntt_batch_launch_eager")


def ntt_batch_status(batch: int) -> int:
    return lib().ntt_batch_status(batch)


def ntt_batch_set_spin_limit(batch: int, polls: int) -> None:
    _check(lib().ntt_batch_set_spin_limit(batch, polls), "ntt_batch_set_spin_limit")


def ntt_batch_destroy(batch: int) -> None:
    lib().ntt_batch_destroy(batch)


def ntt_batch_forward(plans, d_bufs, d_work=None, stream=None) -> None:
    hs = _handles(plans)
    _check(lib().ntt_batch_forward(_ptr_array(hs), _ptr_array(d_bufs), len(hs), _ptr(d_work),
                                   _stream(stream, d_bufs[0] if d_bufs else None)), "ntt_batch_forward")


class Batch:
    """In-place forward NTTs of `bufs[k]` with `plans[k]`, one persistent launch
    replayed from a HIP graph.  Keeps plans, buffers and workspace alive."""

    def __init__(self, plans, bufs, work=None, queues: int = 0):
        import torch

        self.plans = list(plans)
        self.bufs = list(bufs)
        nb = ntt_batch_workspace_bytes(self.plans)
        if work is None and nb:
            work = torch.empty((nb + 31) // 32, 8, dtype=torch.int32, device=self.bufs[0].device)
        self.work = work
        if not queues:
            self.handle = ntt_batch_create(self.plans, self.bufs, work)
            return
        # the same in-place forward jobs through the general entry point, which
        # takes the queue count; each job gets its own slice of the workspace
        jobs, off = [], 0
        for p, b in zip(self.plans, self.bufs):
            wb = lib().ntt_workspace_bytes(p.handle)
            jobs.append(dict(plan=p, op="forward", out=b, work=work[off // 32:] if wb else None, **{"in": b}))
            off += wb
        self.handle = ntt_batch_create_jobs(jobs, graph=True, queues=queues)

    @property
    def items(self) -> int:
        return lib().ntt_batch_items(self.handle)

    @property
    def grid(self) -> int:
        return lib().ntt_batch_grid(self.handle)

    def launch(self, stream=None) -> None:
        ntt_batch_launch(self.handle, stream)

    def launch_eager(self, stream=None) -> None:
        ntt_batch_launch_eager(self.handle, stream)

    def status(self) -> int:
        return ntt_batch_status(self.handle)

    def set_spin_limit(self, polls: int) -> None:
        ntt_batch_set_spin_limit(self.handle, polls)

    def close(self) -> None:
        if self.handle:
            ntt_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Multi-scalar multiplication (BLS12-381 G1)

class MsmBases:
    """Fixed MSM bases: `points` is a device int32 tensor [n, 24] (affine x, y
    as Montgomery limbs over F_q); the per-window multiples are precomputed
    here, once."""

    def __init__(self, points, window_bits: int = 0, stream=None):
        import torch

        self.n = points.shape[0]
        h = ctypes.c_void_p()
        _check(lib().msm_bases_create(ctypes.byref(h), _ptr(points), self.n, window_bits, _stream(stream, points)),
               "msm_bases_create")
        self.handle = h.value
        self.device = points.device
        self.window_bits = lib().msm_bases_window_bits(self.handle)
        self._work = None
        self.torch = torch

    @property
    def device_bytes(self) -> int:
        return lib().msm_bases_device_bytes(self.handle)

    def workspace(self):
        if self._work is None:
            nb = lib().msm_workspace_bytes(self.handle)
            self._work = self.torch.empty((nb + 31) // 32, 8, dtype=self.torch.int32, device=self.device)
        return self._work

    def msm(self, scalars, out=None, work=None, stream=None):
        """XYZZ result [48] int32 of sum s_i P_i; scalars [n, 8] Montgomery Fr."""
        if scalars.shape[0] != self.n:
            raise ValueError("one scalar per base point")
        if out is None:
            out = self.torch.empty(64, dtype=self.torch.int32, device=self.device)
        _check(lib().msm_compute(self.handle, _ptr(scalars), _ptr(out), _ptr(work if work is not None else
                                                                             self.workspace()),
                                 _stream(stream, scalars)), "msm_compute")
        return out

    def close(self) -> None:
        if self.handle:
            lib().msm_bases_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
