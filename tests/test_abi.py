"""The C ABI library loads without a GPU and exports every function that
include/fmm.h declares; host-only entry points behave as documented."""
import ctypes as C
import os

import pytest

import paper_1311_1006_amd as F


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(F.LIB_PATH):
        from paper_1311_1006_amd import build
        build.build()
    return F.lib()


def test_every_declared_symbol_is_exported(L):
    names = F.header_functions()
    assert "fmm_build_tree" in names and "fmm_evaluate_adjoint" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_p_rule_matches_table_4_1(L):
    path = os.path.join(os.path.dirname(__file__), "golden", "table_4_1_p.txt")
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        tol, theta, p = line.split()
        assert F.p_from_tol(float(tol), float(theta)) == int(p)
    assert L.fmm_p_from_tol(0.0, 0.5) == -1
    assert L.fmm_p_from_tol(1e-6, 1.0) == -1


def test_invalid_tree_arguments_are_rejected_on_the_host(L):
    h = C.c_void_p()
    off = (C.c_int64 * 2)(0, 10)
    lv = (C.c_int * 1)(3)       # 16 leaves > 10 points
    rc = L.fmm_build_tree(C.c_void_p(1), off, 1, lv, None, C.byref(h))
    assert rc == -1 and not h.value
    assert b"4^(n_levels-1)" in L.fmm_last_error()
    lv0 = (C.c_int * 1)(0)
    assert L.fmm_build_tree(C.c_void_p(1), off, 1, lv0, None, C.byref(h)) == -1
    assert L.fmm_build_tree(C.c_void_p(1), off, 0, lv, None, C.byref(h)) == -1
    bad = (C.c_int64 * 2)(1, 10)
    assert L.fmm_build_tree(C.c_void_p(1), bad, 1, lv, None, C.byref(h)) == -1
    empty = (C.c_int64 * 3)(0, 5, 5)
    lv2 = (C.c_int * 2)(1, 1)
    assert L.fmm_build_tree(C.c_void_p(1), empty, 2, lv2, None, C.byref(h)) == -1


def test_null_handles_are_rejected(L):
    h = C.c_void_p()
    assert L.fmm_plan(None, 10, 0.5, 0, None, None, C.byref(h)) == -1
    assert L.fmm_evaluate(None, None, None, None) == -1
    assert L.fmm_evaluate_adjoint(None, None, None, None, None, None) == -1
    L.fmm_plan_destroy(None)
    L.fmm_tree_destroy(None)
