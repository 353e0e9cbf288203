"""CPU-side checks of the C ABI: the library loads, exports every function
declared in include/cprrtc.h, and rejects malformed arguments before any
device work (no compute call is made here)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cprrtc.h")
LIB = os.path.join(ROOT, "paper_2505_06791_amd", "libcprrtc.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([a-z_][a-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import __graft_entry__
        __graft_entry__.build_hip()
    return C.CDLL(LIB)


def test_header_declares_the_hot_path():
    names = declared_functions()
    for n in ("fk_cc_batch", "project_validate_motions", "project_configs", "cp_robot_create",
              "cp_robot_destroy", "cp_env_create", "cp_env_destroy", "cp_last_error",
              "cp_proj_params_default"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for n in declared_functions():
        assert hasattr(lib, n), n


def test_null_arguments_are_rejected_without_device_work(lib):
    lib.cp_last_error.restype = C.c_char_p
    out = C.c_void_p()
    assert lib.cp_robot_create(None, C.byref(out)) == -1
    assert b"NULL" in lib.cp_last_error()
    assert lib.cp_env_create(None, C.byref(out)) == -1
    assert lib.fk_cc_batch(None, None, 10, None, None, None, None, 0, None) == -1
    assert lib.project_validate_motions(None, None, None, None, 1, None, None, None, None, None,
                                        None, 0, None) == -1
    assert lib.project_configs(None, None, 1, None, None, None, C.c_double(1e-5), 10,
                               C.c_double(1.0), C.c_double(1e-2), None) == -1


def test_default_parameters(lib):
    from paper_2505_06791_amd import cprrtc
    p = cprrtc.ProjParams()
    lib.cp_proj_params_default(C.byref(p))
    assert (p.W, p.max_iters, p.tau, p.tau_sm, p.tau_task, p.alpha, p.lam, p.sphere_batch) == (
        64, 32, 0.05, 0.025, 1e-3, 1.0, 1e-2, 8)


def test_oracle_is_not_linked_into_the_library():
    data = open(LIB, "rb").read()
    assert b"or_parallel_project" not in data and b"liboracle" not in data
