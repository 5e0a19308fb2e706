"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol declared in include/pdhg.h, and rejects invalid problems before
touching the device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "pdhg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pdhg_[a-z_]+)\s*\(", src)))


def _lib():
    from paper_2207_07234_amd import _binding
    if not os.path.exists(_binding.LIB_PATH):
        pytest.fail("libpdhg.so not built (run __graft_entry__.build())")
    return _binding, _binding.load()


def test_header_declares_the_core_entry_points():
    syms = _declared_symbols()
    for name in ("pdhg_setup", "pdhg_solve", "pdhg_residual", "pdhg_adjoint", "pdhg_destroy"):
        assert name in syms


def test_binding_enum_values_match_header():
    """Every enumerator the binding mirrors has the value the header gives it."""
    B, _ = _lib()
    src = open(os.path.join(ROOT, "include", "pdhg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    vals = {}
    for body in re.findall(r"typedef enum\s*\{(.*?)\}", src, flags=re.S):
        for name, val in re.findall(r"(PDHG_[A-Z0-9_]+)\s*=\s*(-?\d+)", body):
            vals[name] = int(val)
    assert vals["PDHG_DG_P1_UPWIND"] == 3
    for name, val in vals.items():
        if hasattr(B, name):
            assert getattr(B, name) == val, name


def test_library_exports_every_declared_symbol():
    _, lib = _lib()
    for name in _declared_symbols():
        assert hasattr(lib, name), name


def test_binding_struct_sizes_match_header_layout():
    B, _ = _lib()
    # field order/size mirrors include/pdhg.h; natural alignment on x86-64
    assert C.sizeof(B.pdhg_problem) == 4 * 2 + 8 * 5 + 4 * 4 + 8 * 3
    assert C.sizeof(B.pdhg_params) == 8 * 3 + 8 + 4 * 2 + 8 + 4 * 2 + 8 + 8 + 4 * 2 + 8 * 2
    assert C.sizeof(B.pdhg_stats) == 8 * 10 + 4 * 2


@pytest.mark.parametrize("bad", [dict(nx=100), dict(nx=4), dict(nx=8192), dict(nt=0), dict(time=7),
                                 dict(space=9), dict(dtype=5), dict(t_final=0.0), dict(gamma=-1.0)])
def test_setup_rejects_invalid_problems(bad):
    B, lib = _lib()
    p = B.pdhg_problem()
    p.nx, p.nt, p.length, p.t_final, p.alpha, p.beta = 64, 16, 1.0, 0.5, 0.5, 0.0
    p.time, p.space, p.dtype = B.PDHG_BDF2, B.PDHG_FD_LF, B.PDHG_F64
    for k, v in bad.items():
        setattr(p, k, v)
    h = C.c_void_p()
    assert lib.pdhg_setup(C.byref(p), C.byref(h)) == B.PDHG_EINVAL
    assert not h.value


def test_status_strings():
    B, lib = _lib()
    assert lib.pdhg_status_string(B.PDHG_OK) == b"converged"
    assert lib.pdhg_status_string(B.PDHG_DIVERGED) == b"diverged"
    assert lib.pdhg_status_string(12345) == b"unknown status"


def test_refine_params_struct_size():
    B, _ = _lib()
    assert C.sizeof(B.pdhg_refine_params) == 4 * 2 + 8 * 2


def test_batch_params_struct_size():
    B, _ = _lib()
    assert C.sizeof(B.pdhg_batch_params) == 8 * 3 + 8 + 4 * 2 + 8


def _batch_problem(B, **kw):
    p = B.pdhg_problem()
    p.nx, p.nt, p.length, p.t_final, p.alpha, p.beta = 512, 64, 1.0, 0.5, 0.5, 0.0
    p.time, p.space, p.dtype = B.PDHG_BDF2, B.PDHG_FD_LF, B.PDHG_F32
    p.lf_speed = p.precond_c = -1.0
    for k, v in kw.items():
        setattr(p, k, v)
    return p


@pytest.mark.parametrize("bad,code", [
    (dict(nx=128), "PDHG_EUNSUPPORTED"), (dict(nx=8192), "PDHG_EUNSUPPORTED"), (dict(nt=1024), "PDHG_EUNSUPPORTED"),
    (dict(nx=1000), "PDHG_EINVAL"), (dict(nt=0), "PDHG_EINVAL"), (dict(dtype=1), "PDHG_EINVAL"),
    (dict(time=5), "PDHG_EINVAL")])
def test_batch_setup_rejects_before_touching_the_device(bad, code):
    """The second problem of the batch is invalid (or of another dtype); setup fails on the host."""
    B, lib = _lib()
    arr = (B.pdhg_problem * 2)(_batch_problem(B), _batch_problem(B, **bad))
    h = C.c_void_p()
    assert lib.pdhg_batch_setup(arr, 2, C.byref(h)) == getattr(B, code)
    assert not h.value
    assert lib.pdhg_batch_setup(arr, 0, C.byref(h)) == B.PDHG_EINVAL


@pytest.mark.parametrize("space", ["PDHG_DG_P2_LLF", "PDHG_DG_P1_UPWIND"])
@pytest.mark.parametrize("bad", [dict(nx=8), dict(nt=1024), dict(gamma=1e-3)])
def test_dg_setup_limits(bad, space):
    B, lib = _lib()
    p = B.pdhg_problem()
    p.nx, p.nt, p.length, p.t_final, p.alpha, p.beta = 64, 16, 1.0, 0.5, 0.5, 0.0
    p.time, p.space, p.dtype = B.PDHG_BE, getattr(B, space), B.PDHG_F32
    for k, v in bad.items():
        setattr(p, k, v)
    h = C.c_void_p()
    assert lib.pdhg_setup(C.byref(p), C.byref(h)) == B.PDHG_EUNSUPPORTED
    assert not h.value


@pytest.mark.parametrize("kind,space,nt,code", [(7, "PDHG_FD_LF", 16, "PDHG_EINVAL"),
                                                (1, "PDHG_DG_P2_LLF", 16, "PDHG_EUNSUPPORTED"),
                                                (1, "PDHG_DG_P1_UPWIND", 16, "PDHG_EUNSUPPORTED"),
                                                (1, "PDHG_FD_LF", 2048, "PDHG_EUNSUPPORTED")])
def test_precond_kind_limits(kind, space, nt, code):
    B, lib = _lib()
    p = B.pdhg_problem()
    p.nx, p.nt, p.length, p.t_final, p.alpha, p.beta = 64, nt, 1.0, 0.5, 0.5, 0.0
    p.time, p.space, p.dtype, p.precond_kind = B.PDHG_BE, getattr(B, space), B.PDHG_F64, kind
    h = C.c_void_p()
    assert lib.pdhg_setup(C.byref(p), C.byref(h)) == getattr(B, code)
    assert not h.value


def test_batch_rejects_the_full_symbol():
    B, lib = _lib()
    arr = (B.pdhg_problem * 1)()
    p = arr[0]
    p.nx, p.nt, p.length, p.t_final, p.alpha, p.beta = 256, 16, 1.0, 0.5, 0.5, 0.0
    p.time, p.space, p.dtype, p.precond_kind = B.PDHG_BE, B.PDHG_FD_LF, B.PDHG_F64, B.PDHG_PRECOND_FULL
    h = C.c_void_p()
    assert lib.pdhg_batch_setup(arr, 1, C.byref(h)) == B.PDHG_EUNSUPPORTED
    assert not h.value


@pytest.mark.parametrize("dtype,space,nt,code", [("PDHG_F32", "PDHG_FD_LF", 16, "PDHG_EUNSUPPORTED"),
                                                 ("PDHG_F64", "PDHG_DG_P2_LLF", 16, "PDHG_EUNSUPPORTED"),
                                                 ("PDHG_F64", "PDHG_DG_P1_UPWIND", 16, "PDHG_EUNSUPPORTED")])
def test_single_precision_preconditioner_limits(dtype, space, nt, code):
    """PDHG_PRECOND_GRAM_F32: FP64 finite-difference problems only; rejected before the device is touched."""
    B, lib = _lib()
    p = B.pdhg_problem()
    p.nx, p.nt, p.length, p.t_final, p.alpha, p.beta = 64, nt, 1.0, 0.5, 0.5, 0.0
    p.time, p.space, p.dtype, p.precond_kind = B.PDHG_BE, getattr(B, space), getattr(B, dtype), \
        B.PDHG_PRECOND_GRAM_F32
    h = C.c_void_p()
    assert lib.pdhg_setup(C.byref(p), C.byref(h)) == getattr(B, code)
    assert not h.value


def test_time_axis_limit():
    """N_t above 8192 (8 wavefronts of 64 lanes x 16 levels per spectrum column) is unsupported."""
    B, lib = _lib()
    p = B.pdhg_problem()
    p.nx, p.nt, p.length, p.t_final, p.alpha, p.beta = 64, 8193, 1.0, 0.5, 0.5, 0.0
    p.time, p.space, p.dtype = B.PDHG_BE, B.PDHG_FD_LF, B.PDHG_F64
    h = C.c_void_p()
    assert lib.pdhg_setup(C.byref(p), C.byref(h)) == B.PDHG_EUNSUPPORTED
    assert not h.value


def test_batch_rejects_the_single_precision_preconditioner():
    B, lib = _lib()
    arr = (B.pdhg_problem * 1)()
    p = arr[0]
    p.nx, p.nt, p.length, p.t_final, p.alpha, p.beta = 256, 16, 1.0, 0.5, 0.5, 0.0
    p.time, p.space, p.dtype, p.precond_kind = B.PDHG_BE, B.PDHG_FD_LF, B.PDHG_F64, B.PDHG_PRECOND_GRAM_F32
    h = C.c_void_p()
    assert lib.pdhg_batch_setup(arr, 1, C.byref(h)) == B.PDHG_EUNSUPPORTED
    assert not h.value
