"""C-ABI surface of libkfmm.so on the host (no GPU is touched).

Every function that include/kfmm.h declares must be exported by the in-tree library, and the argument
checks that precede any device call must report their errors through the return code (KFMM_E_ARG) and
kfmm_last_error.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kfmm.h")
KFMM_E_ARG = -1


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)  # comments (argument notes sit inside them)
    text = re.sub(r"//[^\n]*", " ", text)
    text = "\n".join(l for l in text.splitlines() if not l.lstrip().startswith("#"))
    # a declaration: return type (optionally const / pointer), name, "(" ... ");" at file scope
    decl = re.compile(r"^\s*(?:const\s+)?(?:unsigned\s+)?[A-Za-z_]\w*\s*\**\s+\**\s*([A-Za-z_]\w*)\s*\(", re.M)
    return sorted({m.group(1) for m in decl.finditer(text)} - {"struct", "typedef", "enum"})


@pytest.fixture(scope="module")
def lib():
    from paper_1612_04082_amd import build, kfmm
    if not os.path.exists(kfmm.LIB_PATH):
        build.build()
    L = kfmm.load_library()
    L.kfmm_last_error.restype = ctypes.c_char_p
    return L


def last_error(L):
    return L.kfmm_last_error().decode()


def test_header_declarations_found():
    names = declared_functions()
    for must in ("fmm_plan", "fmm_eval", "fmm_plan_destroy", "bem_solve", "bem_stress", "ws_train",
                 "kfmm_topological_derivative", "kfmm_selftest_gemm", "kfmm_last_error"):
        assert must in names, (must, names)
    assert len(names) >= 20, names


def test_every_declared_function_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"declared in include/kfmm.h but not exported: {missing}"


def test_plan_argument_errors(lib):
    from paper_1612_04082_amd import kfmm
    plan = ctypes.c_void_p()
    xyz = (ctypes.c_double * 3)(0.0, 0.0, 0.0)

    def call(out, opts, n=1):
        return lib.fmm_plan(out, xyz, xyz, xyz, n, None, n, None, None, 0, opts, None)

    good = dict(K=1.0, G=1.0, p=6, leaf_max=64, precision=kfmm.FP64, svd_eps=0.0, max_depth=0, mem_limit=0,
                m2l_tol=0.0)
    assert call(None, ctypes.byref(kfmm.FmmOpts(**good))) == KFMM_E_ARG
    assert last_error(lib) == "out is NULL"
    assert call(ctypes.byref(plan), None) == KFMM_E_ARG
    assert last_error(lib) == "opts is NULL"
    for change, msg in ((dict(K=-1.0), "moduli"), (dict(G=float("nan")), "moduli"),
                        (dict(precision=9), "unknown precision"), (dict(precision=2), "M2L_BF16 is withdrawn"),
                        (dict(p=2), "p must be in"),
                        (dict(m2l_tol=1.5), "m2l_tol"), (dict(m2l_tol=-1e-8), "m2l_tol"),
                        (dict(m2l_tol=float("nan")), "m2l_tol"), (dict(leaf_max=-4), "negative leaf_max")):
        opts = kfmm.FmmOpts(**{**good, **change})
        assert call(ctypes.byref(plan), ctypes.byref(opts)) == KFMM_E_ARG, change
        assert msg in last_error(lib), (change, last_error(lib))
        assert not plan.value  # *out cleared before the checks
    assert call(ctypes.byref(plan), ctypes.byref(kfmm.FmmOpts(**good)), n=-1) == KFMM_E_ARG
    assert "negative size" in last_error(lib)


def test_periodic_plan_argument_errors(lib):
    """fmm_plan_periodic: a NULL cell array is refused before any device call."""
    from paper_1612_04082_amd import kfmm
    plan = ctypes.c_void_p()
    xyz = (ctypes.c_double * 3)(0.5, 0.5, 0.5)
    cells = (ctypes.c_double * 4)(0.0, 0.0, 0.0, 1.0)
    good = dict(K=1.0, G=1.0, p=6, leaf_max=64, precision=kfmm.FP64, svd_eps=0.0, max_depth=0, mem_limit=0,
                m2l_tol=0.0)

    def call(c, opts):
        return lib.fmm_plan_periodic(ctypes.byref(plan), xyz, None, None, 1, None, 1, None, None, 0, c,
                                     ctypes.byref(opts), None)

    for prec in (kfmm.FP64, kfmm.FP32, kfmm.FP32_M2L_SPLIT16):
        assert call(None, kfmm.FmmOpts(**{**good, "precision": prec})) == KFMM_E_ARG
        assert last_error(lib) == "cells is NULL" and not plan.value
    assert call(cells, kfmm.FmmOpts(**{**good, "precision": 2})) == KFMM_E_ARG  # the withdrawn BF16 mode
    assert "M2L_BF16 is withdrawn" in last_error(lib)


def test_selftest_gemm_selector_errors(lib):
    idx = (ctypes.c_int * 1)(0)

    def call(precision, mode=0, NC=96):
        return lib.kfmm_selftest_gemm(precision, None, NC, None, None, idx, idx, idx, None, 0, mode, None)

    assert call(7) == KFMM_E_ARG and last_error(lib) == "bad arguments"
    assert call(1, mode=3) == KFMM_E_ARG and last_error(lib) == "bad arguments"
    # precision 2 (the withdrawn BF16 kernel) is refused
    assert call(2) == KFMM_E_ARG and last_error(lib) == "bad arguments"
    # kernel selectors: FP64 / FP32 take 0..4, split FP16 only 0 and 1 (64-column tiles)
    assert call(3 + 16 * 2) == KFMM_E_ARG and last_error(lib) == "bad kernel selector"
    assert call(1 + 16 * 5) == KFMM_E_ARG and last_error(lib) == "bad kernel selector"
    assert call(3, NC=100) == KFMM_E_ARG and "multiple of 96 or 128" in last_error(lib)


def test_moduli_round_trip():
    """K from (G, nu) inverts the relation nu = (3K - 2G) / (2 (3K + G)) stated with the ABI."""
    from paper_1612_04082_amd import kfmm
    for G, nu in ((1.0, 0.3), (2.5, 0.0), (0.7, 0.45), (3.0, -0.2)):
        K = kfmm.moduli(G, nu)
        assert abs((3 * K - 2 * G) / (2 * (3 * K + G)) - nu) < 1e-14


def test_binding_rejects_host_and_misshaped_tensors(lib):
    """The binding hands the library device pointers only: host tensors and misshaped inputs are refused
    before any library call."""
    import torch
    from paper_1612_04082_amd import kfmm
    x = torch.zeros((8, 3), dtype=torch.float64)
    with pytest.raises(TypeError):
        kfmm._dptr(x, "src", 3)                      # host memory
    with pytest.raises(TypeError):
        kfmm.FmmPlan(x)                              # host memory, before the plan call
    with pytest.raises(ValueError):
        kfmm.FmmPlan(x, w=torch.ones(5, dtype=torch.float64))  # weights of the wrong length
    with pytest.raises(TypeError):
        kfmm.selftest_gemm(1, torch.zeros((1, 96, 96)), torch.zeros((2, 96)), torch.zeros((2, 96)), [0], [0], [0])
    assert kfmm._dptr(None, "b") is None


def test_error_code_and_message_reach_python(lib):
    """A failing ABI call surfaces as KfmmError carrying the status and the library's message."""
    from paper_1612_04082_amd import kfmm
    opts = kfmm.FmmOpts(1.0, 1.0, 6, 64, kfmm.FP64, 0.0, 0, 0, 0.0)
    with pytest.raises(kfmm.KfmmError) as e:
        kfmm.check(lib.fmm_plan(None, None, None, None, 0, None, 0, None, None, 0, ctypes.byref(opts), None))
    assert "out is NULL" in str(e.value) and e.value.code == KFMM_E_ARG


def test_other_entry_points_check_arguments_first(lib):
    """NULL handles and out-of-range selectors are reported before any device work; destroying a NULL
    handle is a no-op; an empty topological-derivative request succeeds without touching the device."""
    from paper_1612_04082_amd import kfmm
    raw = ctypes.CDLL(kfmm.LIB_PATH)  # own function objects: the binding's argtypes stay untouched
    assert raw.fmm_eval(None, 0, None, None, None, None) == KFMM_E_ARG and last_error(lib) == "plan is NULL"
    assert raw.fmm_plan_info(None, None) == KFMM_E_ARG and last_error(lib) == "NULL argument"
    assert raw.fmm_plan_target_lists(None, None) == KFMM_E_ARG and last_error(lib) == "NULL argument"
    assert raw.fmm_profile(None, 1) == KFMM_E_ARG and last_error(lib) == "plan is NULL"
    assert raw.fmm_plan_destroy(None) == 0
    assert raw.ws_destroy(None) == 0
    n = ctypes.c_int64(-1)
    assert raw.ws_num_params(None, ctypes.byref(n)) != 0 and n.value == -1
    assert last_error(lib) == "network is NULL"
    td = raw.kfmm_topological_derivative
    td.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]
    assert td(None, 0, 1.0, 1.0, None, None) == 0
    assert td(None, 0, -1.0, 1.0, None, None) == KFMM_E_ARG and "moduli" in last_error(lib)
    assert td(None, 5, 1.0, 1.0, None, None) == KFMM_E_ARG and last_error(lib) == "bad arguments"


def test_bem_entry_points_check_problem_and_options_first(lib):
    """BEM calls validate the problem (near-singular quadrature settings included) and their options before
    any device work: device pointers that are never dereferenced stand in for the arrays."""
    from paper_1612_04082_amd import kfmm
    fake = 0x1000  # a non-NULL address that no check dereferences
    prob = kfmm.BemProblem(10, fake, fake, fake, 2.0, 1.0, 0, 0.0)
    fo = kfmm.FmmOpts(2.0, 1.0, 6, 64, kfmm.FP64, 0.0, 0, 0, 0.0)
    for change, msg in ((dict(near_levels=6), "near_levels"), (dict(near_levels=-1), "near_levels"),
                        (dict(near_radius=-1.0), "near_radius"), (dict(near_radius=float("nan")), "near_radius"),
                        (dict(n_tri=0), "n_tri"), (dict(K=-1.0), "moduli")):
        p = kfmm.BemProblem(10, fake, fake, fake, 2.0, 1.0, 0, 0.0)
        for k, v in change.items():
            setattr(p, k, v)
        rc = lib.bem_matvec(ctypes.byref(p), ctypes.byref(fo), 0, ctypes.c_void_p(fake), ctypes.c_void_p(fake), None)
        assert rc == KFMM_E_ARG and msg in last_error(lib), (change, last_error(lib))
    assert lib.bem_near_pairs(ctypes.byref(prob), None, None, 0, None) == KFMM_E_ARG
    assert last_error(lib) == "count is NULL"
    opts = kfmm.BemOpts(1e-6, 50, 10, fo, None, kfmm.PC_NONE, 0, 0)
    assert lib.bem_precond_apply(ctypes.byref(prob), ctypes.byref(opts), ctypes.c_void_p(fake),
                                 ctypes.c_void_p(fake + 64), None, None) == KFMM_E_ARG
    assert "KFMM_PC_TWO_LEVEL" in last_error(lib)
    opts.precond = 7
    assert lib.bem_solve(ctypes.byref(prob), ctypes.byref(opts), None, ctypes.c_void_p(fake), None, None, None,
                         None) == KFMM_E_ARG and "preconditioner" in last_error(lib)
    # periodic cells: the side must be finite and positive; the preconditioner and bem_near_pairs are free-space
    for bad in ((0.0, 0.0, 0.0, 0.0), (0.0, 0.0, 0.0, -1.0), (float("nan"), 0.0, 0.0, 1.0),
                (0.0, 0.0, 0.0, float("inf"))):
        p = kfmm.BemProblem(10, fake, fake, fake, 2.0, 1.0, 0, 0.0, (ctypes.c_double * 4)(*bad))
        rc = lib.bem_matvec(ctypes.byref(p), ctypes.byref(fo), 0, ctypes.c_void_p(fake), ctypes.c_void_p(fake), None)
        assert rc == KFMM_E_ARG and "side > 0" in last_error(lib), (bad, last_error(lib))
    cell = (ctypes.c_double * 4)(0.0, 0.0, 0.0, 1.0)
    pc = kfmm.BemProblem(10, fake, fake, fake, 2.0, 1.0, 0, 0.0, cell)
    count = ctypes.c_int64(0)
    assert lib.bem_near_pairs(ctypes.byref(pc), ctypes.byref(count), None, 0, None) == KFMM_E_ARG
    assert "free-space surfaces only" in last_error(lib)
    opts.precond = kfmm.PC_TWO_LEVEL
    assert lib.bem_solve(ctypes.byref(pc), ctypes.byref(opts), None, ctypes.c_void_p(fake), None, None, None,
                         None) == KFMM_E_ARG and "cell must be NULL" in last_error(lib)
    assert lib.bem_precond_apply(ctypes.byref(pc), ctypes.byref(opts), ctypes.c_void_p(fake),
                                 ctypes.c_void_p(fake + 64), None, None) == KFMM_E_ARG
    assert "cell must be NULL" in last_error(lib)


def test_binding_refuses_to_run_without_the_library(monkeypatch, tmp_path):
    """No fallback path: with the built library absent the binding raises instead of computing anything."""
    from paper_1612_04082_amd import kfmm
    monkeypatch.setattr(kfmm, "_lib", None)
    monkeypatch.setattr(kfmm, "LIB_PATH", str(tmp_path / "libkfmm.so"))
    with pytest.raises(ImportError, match="not built"):
        kfmm.load_library()
