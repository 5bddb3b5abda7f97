"""Host-side checks of the C-ABI library (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pss.h")
LIB = os.path.join(ROOT, "paper_1606_04669_amd", "libpss.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pss_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1606_04669_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    fns = declared_functions()
    for f in ["pss_ctx_create", "pss_ctx_destroy", "pss_create", "pss_destroy", "pss_update", "pss_merge",
              "pss_query", "pss_run", "pss_strerror", "pss_last_device_error", "pss_device_error_name", "pss_block_summaries", "pss_plan_chunks", "pss_max_k",
              "pss_batch_create", "pss_batch_run", "pss_batch_destroy", "pss_run_batched"]:
        assert f in fns


def test_library_exports_every_declared_symbol(lib):
    for f in declared_functions():
        assert hasattr(lib, f), f
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (pss_\w+)", out))
    assert set(declared_functions()) <= exported


def test_strerror_and_null_handling_without_gpu(lib):
    lib.pss_strerror.restype = ctypes.c_char_p
    assert lib.pss_strerror(0) == b"ok"
    assert lib.pss_strerror(-5) == b"output buffer too small"
    assert lib.pss_strerror(12345) == b"unknown error"
    assert lib.pss_last_device_error() == 0  # nothing failed on this thread
    # null handles are rejected before any device call
    lib.pss_ctx_create.argtypes = [ctypes.c_int, ctypes.c_void_p]
    assert lib.pss_ctx_create(0, None) == -1
    lib.pss_create.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p]
    assert lib.pss_create(None, 10, None) == -1
    lib.pss_update.argtypes = [ctypes.c_void_p] * 2 + [ctypes.c_uint64, ctypes.c_uint32] + [ctypes.c_void_p] * 2
    assert lib.pss_update(None, None, 10, 0, None, None) == -1
    lib.pss_merge.argtypes = [ctypes.c_void_p] * 3
    assert lib.pss_merge(None, None, None) == -1
    lib.pss_destroy.argtypes = [ctypes.c_void_p]
    lib.pss_destroy(None)
    lib.pss_ctx_destroy.argtypes = [ctypes.c_void_p]
    lib.pss_ctx_destroy(None)
    lib.pss_batch_create.argtypes = [ctypes.c_void_p, ctypes.c_uint32] + [ctypes.c_void_p] * 4 + [ctypes.c_int,
                                                                                                  ctypes.c_void_p]
    assert lib.pss_batch_create(None, 1, None, None, None, None, 0, None) == -1
    lib.pss_batch_run.argtypes = [ctypes.c_void_p, ctypes.c_int] + [ctypes.c_void_p] * 3
    assert lib.pss_batch_run(None, 0, None, None, None) == -1
    lib.pss_batch_destroy.argtypes = [ctypes.c_void_p]
    lib.pss_batch_destroy(None)
    for f in (lib.pss_plan_chunks, lib.pss_frequent_plan_chunks):
        f.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32]
        f.restype = ctypes.c_uint32
        assert f(None, 1 << 30, 2000) == 1


def test_binding_names_match_the_abi():
    from paper_1606_04669_amd import binding
    for f in ["pss_ctx_create", "pss_ctx_destroy", "pss_create", "pss_destroy", "pss_update", "pss_merge",
              "pss_query", "pss_run", "pss_block_summaries", "strerror", "pss_batch_create", "pss_batch_run",
              "pss_batch_destroy", "pss_run_batched"]:
        assert callable(getattr(binding, f))
    assert binding.ENTRY_DTYPE.itemsize == 24


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_1606_04669_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src and "pss_oracle" not in src, f


def test_kernels_take_all_lds_dynamically():
    # the host sizes every launch's LDS from the dynamic byte counts it passes,
    # so no kernel may add static shared arrays on top of them
    import glob
    csrc = os.path.join(ROOT, "paper_1606_04669_amd", "csrc")
    for f in sorted(glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.h"))):
        for line in open(f).read().splitlines():
            if "__shared__" in line and not line.lstrip().startswith("//"):
                assert re.search(r"extern\s+__shared__", line), (f, line)
