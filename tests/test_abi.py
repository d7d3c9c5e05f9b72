"""The C-ABI library loads and exports every entry point include/zkntt.h
declares (no GPU needed: nothing is called)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "zkntt.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|void|size_t|char)\s*\**\s*(\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("ntt_plan_create", "ntt_plan_destroy", "ntt_forward", "ntt_inverse", "ntt_coset_forward",
                     "ntt_coset_inverse", "quotient_poly", "ntt_workspace_bytes", "quotient_workspace_bytes",
                     "zk_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2509_22684_amd import _lib

    L = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, f"not exported: {missing}"


def test_null_plan_calls_fail_cleanly():
    """Argument checks run before any device work: a null plan is ZK_EINVAL."""
    from paper_2509_22684_amd import _lib

    L = _lib.lib()
    assert L.ntt_forward(None, None, None, None, None) == -1
    assert L.quotient_poly(None, None, None, None, None, None, None) == -1
    assert L.ntt_workspace_bytes(None) == 0
    assert b"null" in L.zk_last_error()
    assert L.quotient_coset_evals(None, None, None, None, None) == -1
    assert L.quotient_pointwise(None, None, None, None, None, None) == -1
    assert L.ntt_batch_create_jobs(None, None, 0, 0) == -1
    assert L.ntt_batch_status(None) == -1


def test_copy_to_host_checks_before_launch():
    """Null, misaligned or odd-sized copies are refused before any HIP call."""
    from paper_2509_22684_amd import _lib

    L = _lib.lib()
    assert L.zk_copy_to_host(None, None, 16, None) == -1
    assert L.zk_copy_to_host(ctypes.c_void_p(256), ctypes.c_void_p(512), 24, None) == -1
    assert L.zk_copy_to_host(ctypes.c_void_p(8), ctypes.c_void_p(512), 32, None) == -1
