"""The C-ABI library loads on the CPU, exports every symbol include/imin.h declares, and
rejects invalid graphs before touching a device (host logic only; no compute calls)."""
import ctypes
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

from paper_2302_13529_amd import binding

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "include", "imin.h")


def declared_functions():
    text = open(HEADER).read()
    return re.findall(r"IMIN_API\s+[\w\s\*]+?\b(imin_\w+)\s*\(", text)


def test_header_declares_the_api():
    names = set(declared_functions())
    assert {"imin_graph_create", "imin_graph_destroy", "imin_decrease", "imin_greedy",
            "imin_greedy_batch", "imin_set_launch", "imin_set_small", "imin_strerror"} <= names


def test_library_exports_every_declared_symbol():
    lib = binding.load()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_strerror():
    assert binding.imin_strerror(binding.IMIN_OK) == "ok"
    assert binding.imin_strerror(binding.IMIN_EINVAL) == "invalid argument"
    assert binding.imin_strerror(12345) == "unknown status"


@pytest.mark.parametrize("case", ["rowptr0", "nonmono", "colrange", "nan", "pneg", "pbig",
                                  "mmismatch", "n0"])
def test_graph_create_rejects_invalid(case):
    n = 4
    row_ptr = np.array([0, 1, 2, 3, 3], np.int32)
    col = np.array([1, 2, 3], np.int32)
    prob = np.array([0.5, 0.5, 0.5], np.float32)
    m = 3
    if case == "rowptr0":
        row_ptr = np.array([1, 1, 2, 3, 3], np.int32)
    elif case == "nonmono":
        row_ptr = np.array([0, 2, 1, 3, 3], np.int32)
    elif case == "colrange":
        col = np.array([1, 2, 4], np.int32)
    elif case == "nan":
        prob = np.array([0.5, np.nan, 0.5], np.float32)
    elif case == "pneg":
        prob = np.array([0.5, -0.1, 0.5], np.float32)
    elif case == "pbig":
        prob = np.array([0.5, 1.5, 0.5], np.float32)
    elif case == "mmismatch":
        m = 2
    elif case == "n0":
        n = 0
    lib = binding.load()
    h = ctypes.c_void_p()
    rc = lib.imin_graph_create(n, m, row_ptr.ctypes.data_as(ctypes.c_void_p),
                               col.ctypes.data_as(ctypes.c_void_p),
                               prob.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h))
    assert rc == binding.IMIN_EINVAL
    assert h.value is None


def test_graph_create_range_and_model_checks_come_first():
    """n = 2^31 - 1 (row_ptr would need 2^31 entries) is rejected with IMIN_ERANGE before
    row_ptr is read, and an unknown model with IMIN_EINVAL, both before any device call."""
    lib = binding.load()
    row_ptr = np.zeros(2, np.int32)
    h = ctypes.c_void_p()
    rc = lib.imin_graph_create(2**31 - 1, 0, row_ptr.ctypes.data_as(ctypes.c_void_p), None,
                               None, ctypes.byref(h))
    assert rc == binding.IMIN_ERANGE and h.value is None
    row_ptr = np.array([0, 0], np.int32)
    for model in (-1, 2, 7):
        rc = lib.imin_graph_create_model(1, 0, row_ptr.ctypes.data_as(ctypes.c_void_p), None,
                                         None, model, ctypes.byref(h))
        assert rc == binding.IMIN_EINVAL and h.value is None


def test_null_handle_is_rejected():
    lib = binding.load()
    D = np.zeros(4, np.uint64)
    S = np.array([0], np.int32)
    assert lib.imin_decrease(None, S.ctypes.data_as(ctypes.c_void_p), 1, None, 10, 0,
                             D.ctypes.data_as(ctypes.c_void_p), None) == binding.IMIN_EINVAL
    assert lib.imin_set_launch(None, 1, 1) == binding.IMIN_EINVAL
    assert lib.imin_set_small(None, 1, None) == binding.IMIN_EINVAL
    assert lib.imin_greedy_batch(None, 1, 0, None) == binding.IMIN_EINVAL
    lib.imin_graph_destroy(None)


def test_batch_rejects_null_graph_before_touching_a_device():
    lib = binding.load()
    arr = (binding.imin_instance * 1)()
    S = np.array([0], np.int32)
    arr[0].g = None
    arr[0].S = S.ctypes.data_as(ctypes.c_void_p)
    arr[0].nS = 1
    arr[0].b = 1
    arr[0].theta = 10
    assert lib.imin_greedy_batch(arr, 1, 0, None) == binding.IMIN_EINVAL
    assert lib.imin_greedy_batch(arr, 0, 0, None) == binding.IMIN_EINVAL
    for bad in (binding.imin_launch(-1, 0, 0, 0), binding.imin_launch(0, 0, 0, 2)):
        assert lib.imin_greedy_batch(arr, 1, 0, ctypes.byref(bad)) == binding.IMIN_EINVAL


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_c_program_links_and_checks_arguments(tmp_path):
    """The C ABI from C: tests/abi_check.c built as strict C99 against the header and the
    library, then run."""
    here = os.path.dirname(os.path.abspath(__file__))
    root = os.path.dirname(here)
    libdir = os.path.dirname(binding.LIB_PATH)
    exe = tmp_path / "abi_check"
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Wextra", "-Wpedantic", "-Werror",
                           "-I", os.path.join(root, "include"),
                           os.path.join(here, "abi_check.c"), "-L", libdir, "-limin",
                           f"-Wl,-rpath,{libdir}", "-Wl,-rpath-link,/opt/rocm/lib",
                           "-o", str(exe)])
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert res.returncode == 0 and "c abi ok" in res.stdout, (res.returncode, res.stdout,
                                                              res.stderr)
