"""Host-side checks of the C ABI: the library loads, exports every function
include/rbt.h declares, its host-only entry points match the oracle
bit-exactly, and argument errors are reported as -i without touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import coeffs, structure
from paper_2312_09376_amd import _lib

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "rbt.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rbt_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, f"{name} missing from the binding's signature table"


def test_version(lib):
    assert lib.rbt_version() >= 100


def test_option_constants_match_header():
    """The binding's option and stage constants are the header's #defines."""
    text = open(HEADER).read()
    defs = dict(re.findall(r"#define\s+(RBT_(?:OPT|STAGE)_[A-Z0-9_]+)\s+(\d+)", text))
    assert len(defs) >= 14
    for name, value in defs.items():
        assert getattr(_lib, name) == int(value), name


def test_panel_options(lib):
    """Panel width and panel order: defaults, accepted values, rejected
    values (-2), host-only (no GPU call)."""
    lib.rbt_get_option.restype = ctypes.c_int64
    lib.rbt_set_option.argtypes = [ctypes.c_int, ctypes.c_int64]
    get = lambda o: lib.rbt_get_option(o)
    w0, s0 = get(_lib.RBT_OPT_OUTER_NB), get(_lib.RBT_OPT_PANEL_SPLIT)
    assert (w0, s0) == (2048, 2)
    try:
        for v in (0, 1, 2):
            assert lib.rbt_set_option(_lib.RBT_OPT_PANEL_SPLIT, v) == 0
            assert get(_lib.RBT_OPT_PANEL_SPLIT) == v
        assert lib.rbt_set_option(_lib.RBT_OPT_PANEL_SPLIT, 3) == -2
        assert lib.rbt_set_option(_lib.RBT_OPT_PANEL_SPLIT, -1) == -2
        for v in (128, 1152, 2048):
            assert lib.rbt_set_option(_lib.RBT_OPT_OUTER_NB, v) == 0
        for v in (0, 100, 2176):
            assert lib.rbt_set_option(_lib.RBT_OPT_OUTER_NB, v) == -2
    finally:
        lib.rbt_set_option(_lib.RBT_OPT_OUTER_NB, w0)
        lib.rbt_set_option(_lib.RBT_OPT_PANEL_SPLIT, s0)


@pytest.mark.parametrize("d", [0, 1, 2, 3, 4, 6])
def test_structure_bit_exact(lib, d):
    for n in list(range(0, 70)) + [127, 128, 129, 1000, 1001, 1003, 4099]:
        out = np.full(max(1, n * d), -7, dtype=np.int64)
        assert lib.rbt_structure(n, d, out.ctypes.data_as(ctypes.c_void_p)) == 0
        if n == 0 or d == 0:
            continue
        expect = np.array(structure.partners(n, d), dtype=np.int64).reshape(-1)
        assert np.array_equal(out[: n * d], expect), (n, d)


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("granule", [1, 3, 8, 512])
def test_tiled_structure_bit_exact(lib, d, granule):
    """The tiled / Eq. 8 reference sizes: the closed form of the library
    pairs exactly the indices the oracle's Algorithm 1 loops pair."""
    for n in list(range(0, 40)) + [129, 1000, 1003, 4099]:
        assert lib.rbt_reference_size(n, d, granule) == structure.reference_size(n, d, granule)
        out = np.full(max(1, n * d), -7, dtype=np.int64)
        assert lib.rbt_structure_ex(n, d, granule, out.ctypes.data_as(ctypes.c_void_p)) == 0
        if n == 0:
            continue
        expect = np.array(structure.partners(n, d, granule), dtype=np.int64).reshape(-1)
        assert np.array_equal(out[: n * d], expect), (n, d, granule)
    for nb, p, q in [(512, 4, 4), (512, 2, 3), (64, 4, 6), (1, 1, 7)]:
        assert lib.rbt_comm_free_granule(nb, p, q) == structure.comm_free_granule(nb, p, q)
    assert lib.rbt_reference_size(5, 2, 0) == -1
    assert lib.rbt_structure_ex(5, 2, 0, None) == -3


@pytest.mark.parametrize("n,d,granule", [(1, 1, 1), (17, 2, 1), (1003, 2, 1), (300, 5, 4),
                                         (129, 3, 8)])
def test_generate_rotations_bit_exact(lib, n, d, granule):
    U = np.zeros(n * d)
    V = np.zeros(n * d)
    assert lib.rbt_generate_rotations(n, d, 2023, granule, U.ctypes.data_as(ctypes.c_void_p),
                                      V.ctypes.data_as(ctypes.c_void_p)) == 0
    Uo, Vo = coeffs.generate_rotations(n, d, 2023, granule)
    assert np.array_equal(U.reshape(d, n).T, Uo)
    assert np.array_equal(V.reshape(d, n).T, Vo)


@pytest.mark.parametrize("n,d,seed", [(1, 1, 0), (17, 2, 2023), (1003, 2, 42), (300, 5, 2 ** 64 - 1)])
def test_generate_bit_exact(lib, n, d, seed):
    U = np.zeros(n * d)
    V = np.zeros(n * d)
    assert lib.rbt_generate(n, d, seed, U.ctypes.data_as(ctypes.c_void_p),
                            V.ctypes.data_as(ctypes.c_void_p)) == 0
    Uo, Vo = coeffs.generate(n, d, seed)
    assert np.array_equal(U.reshape(d, n).T, Uo)
    assert np.array_equal(V.reshape(d, n).T, Vo)


def test_argument_errors(lib):
    vp = ctypes.c_void_p
    buf = np.zeros(64, dtype=np.int64)
    assert lib.rbt_structure(-1, 2, buf.ctypes.data_as(vp)) == -1
    assert lib.rbt_structure(4, -1, buf.ctypes.data_as(vp)) == -2
    assert lib.rbt_structure(4, 17, buf.ctypes.data_as(vp)) == -2
    assert lib.rbt_structure(4, 2, None) == -3
    assert lib.rbt_generate(-3, 2, 1, None, None) == -1
    assert lib.rbt_generate(3, 2, 1, None, None) == -4
    dummy = vp(0x1000)   # never dereferenced: every call below fails validation first
    assert lib.rbt_solve_ex(-1, 1, dummy, 1, dummy, 1, 2, 0, None, dummy, 1 << 20, None) == -1
    assert lib.rbt_solve_ex(4, -1, dummy, 4, dummy, 4, 2, 0, None, dummy, 1 << 20, None) == -2
    assert lib.rbt_solve_ex(4, 1, dummy, 3, dummy, 4, 2, 0, None, dummy, 1 << 20, None) == -4
    assert lib.rbt_solve_ex(4, 1, dummy, 4, dummy, 3, 2, 0, None, dummy, 1 << 20, None) == -6
    assert lib.rbt_solve_ex(4, 1, dummy, 4, dummy, 4, 99, 0, None, dummy, 1 << 20, None) == -7
    assert lib.rbt_solve_ex(4, 1, dummy, 4, dummy, 4, 2, 0, None, dummy, 16, None) == _lib.RBT_ERR_WORKSPACE
    assert lib.rbt_genp(5, dummy, 4, None, None) == -3
    assert lib.rbt_getrs(5, 1, dummy, 5, dummy, 5, 2, dummy, 1 << 20, None) == -7
    assert lib.rbt_getrs(5, 1, dummy, 5, dummy, 5, 0, dummy, 8, None) == _lib.RBT_ERR_WORKSPACE
    assert lib.rbt_transform2(5, dummy, 5, dummy, 5, 7, dummy, dummy, 2, None) == -6
    assert lib.rbt_transform_vec(5, 1, dummy, 5, dummy, 2, 9, None) == -7
    assert lib.rbt_solve_refine(5, 1, dummy, 5, dummy, 5, dummy, 5, dummy, 5, 2, 0, -1.0, 3,
                                None, None, None, dummy, 1 << 30, None) == -13

    def mixed(prec=_lib.RBT_FP32, solver=_lib.RBT_IR_CLASSIC, tol=1e-10, depth=2, ldlu=5):
        return lib.rbt_solve_mixed(5, 1, dummy, 5, dummy, ldlu, dummy, 5, dummy, 5, depth, 0, prec,
                                   solver, tol, 3, None, None, None, dummy, 1 << 30, None)
    assert mixed(prec=_lib.RBT_FP64) == -13
    assert mixed(solver=7) == -14
    assert mixed(tol=-1.0) == -15
    assert mixed(ldlu=4) == -6
    assert mixed(depth=17) == -11  # beyond RBT_MAX_DEPTH
    assert lib.rbt_workspace_size(1000, 1, 2, _lib.RBT_BF16) > 0
    assert lib.rbt_workspace_size(1000, 1, 2, 9) == 0
    def guarded(prec=_lib.RBT_FP32, tol=1e-10, ldlu64=5, lu64=dummy, max_iter64=3, ldx=5):
        return lib.rbt_solve_mixed_guarded(5, 1, dummy, 5, dummy, 5, lu64, ldlu64, dummy, 5,
                                           dummy, ldx, 2, 0, prec, _lib.RBT_IR_GMRES, tol, 3,
                                           max_iter64, None, None, None, None, dummy, 1 << 30,
                                           None)
    assert guarded(lu64=None) == -7
    assert guarded(ldlu64=4) == -8
    assert guarded(ldx=4) == -12
    assert guarded(prec=_lib.RBT_FP64) == -15
    assert guarded(tol=-1.0) == -17
    assert guarded(max_iter64=-1) == -19
    # adjoint of the mixed solve
    assert lib.rbt_solve_backward_mixed(5, 1, dummy, 5, dummy, 4, dummy, 5, dummy, 5, None, 5,
                                        dummy, 5, 2, 0, 1e-10, 3, None, None, dummy, 1 << 30,
                                        None) == -6
    assert lib.rbt_solve_backward_mixed(5, 1, dummy, 5, dummy, 5, dummy, 5, dummy, 5, None, 5,
                                        dummy, 5, 2, 0, -1.0, 3, None, None, dummy, 1 << 30,
                                        None) == -17


def test_batched_argument_errors(lib):
    vp = ctypes.c_void_p
    ns = np.array([10, 20], dtype=np.int64)
    ks = np.array([1, 17], dtype=np.int64)
    assert lib.rbt_batched_workspace_size(2, ns.ctypes.data_as(vp), ks.ctypes.data_as(vp), 2,
                                          _lib.RBT_FP32) == 0  # nrhs > 16
    ks[1] = 16
    a = lib.rbt_batched_workspace_size(2, ns.ctypes.data_as(vp), ks.ctypes.data_as(vp), 2,
                                       _lib.RBT_FP32)
    b = lib.rbt_batched_workspace_size(2, ns.ctypes.data_as(vp), ks.ctypes.data_as(vp), 3,
                                       _lib.RBT_FP32)
    assert 0 < a <= b
    c = lib.rbt_batched_workspace_size(2, ns.ctypes.data_as(vp), ks.ctypes.data_as(vp), 11,
                                       _lib.RBT_FP32)
    assert b <= c  # any depth up to RBT_MAX_DEPTH: more coefficient storage
    assert lib.rbt_batched_workspace_size(2, ns.ctypes.data_as(vp), ks.ctypes.data_as(vp), 17,
                                          _lib.RBT_FP32) == 0
    ks[1] = 17
    assert lib.rbt_batched_plan(2, ns.ctypes.data_as(vp), ks.ctypes.data_as(vp), 2, _lib.RBT_FP32,
                                vp(0x1000), 1 << 20, None) == _lib.RBT_ERR_UNSUPPORTED
    ks[1] = 2
    assert lib.rbt_batched_plan(2, ns.ctypes.data_as(vp), ks.ctypes.data_as(vp), 2, 7,
                                vp(0x1000), 1 << 20, None) == -5
    assert lib.rbt_batched_plan(2, ns.ctypes.data_as(vp), ks.ctypes.data_as(vp), 2, _lib.RBT_FP32,
                                vp(0x1000), 16, None) == _lib.RBT_ERR_WORKSPACE
    d = vp(0x1000)
    assert lib.rbt_solve_batched(-1, d, d, d, d, d, d, 2, 0, _lib.RBT_FP32, 1e-10, 3, None,
                                 None, None, None, d, 1 << 20, None) == -1
    assert lib.rbt_solve_batched(2, d, d, d, d, d, d, 2, 0, 5, 1e-10, 3, None, None, None, None,
                                 d, 1 << 20, None) == -10
    assert lib.rbt_solve_batched(2, d, d, d, d, d, d, 2, 0, _lib.RBT_FP32, float("nan"), 3, None,
                                 None, None, None, d, 1 << 20, None) == -11
    assert lib.rbt_solve_batched(2, d, d, d, d, d, d, 2, 0, _lib.RBT_FP32, 1e-10, 3, None,
                                 None, None, None, d, 100, None) == _lib.RBT_ERR_WORKSPACE
    assert lib.rbt_solve_batched(0, None, None, None, None, None, None, 2, 0, _lib.RBT_FP32,
                                 1e-10, 3, None, None, None, None, None, 0, None) == 0


def test_workspace_size_monotone(lib):
    a = lib.rbt_workspace_size(1000, 1, 2, 0)
    b = lib.rbt_workspace_size(1000, 64, 2, 0)
    c = lib.rbt_workspace_size(2000, 1, 2, 0)
    assert 0 < a < b and a < c
    assert lib.rbt_workspace_size(-1, 1, 2, 0) == 0
