"""ctypes front end of the FP64 direct-summation oracle (oracle/direct.c).

Test infrastructure only.  Semantics (eq. fmm_summation; kernels eqs. disp_1, disp_2,
stress_2, stress_3 with the readings stated in direct.c):

  DISP   : v_t   = sum_{s: y_s != x_t} U(x_t, y_s) w_s a_s + P(x_t, y_s, n_s) w_s b_s
  STRESS : sig_t = sum_{s: y_s != x_t} D(x_t, y_s) : w_s a_s + S(x_t, y_s, n_s) : w_s b_s
           (stress components xx, yy, zz, yz, xz, xy)
"""
import ctypes
import os

import numpy as np

from . import build as _build

DISP, STRESS = 0, 1
_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            raise ImportError(f"{path} not built: run __graft_entry__.build() or python -m oracle.build")
        for f in _build.SOURCES:
            if os.path.getmtime(path) < os.path.getmtime(os.path.join(_build.HERE, f)):
                raise ImportError(f"{path} is older than oracle/{f}: rebuild it (python -m oracle.build)")
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        L.oracle_direct.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, i64, dp, dp, dp, dp, dp,
                                    i64, dp, ctypes.c_int]
        L.oracle_direct.restype = ctypes.c_int
        L.oracle_quad_blocks.argtypes = [ctypes.c_double, ctypes.c_double, dp, i64, dp, dp, dp,
                                         ctypes.POINTER(ctypes.c_int64), i64, i64, dp, dp, ctypes.c_int]
        L.oracle_quad_blocks.restype = ctypes.c_int
        L.oracle_pair_kernels.argtypes = [ctypes.c_double, ctypes.c_double, dp, dp, dp, i64, dp, dp, dp, dp]
        L.oracle_pair_kernels.restype = ctypes.c_int
        L.oracle_near_blocks.argtypes = [ctypes.c_double, ctypes.c_double, dp, dp, ctypes.POINTER(ctypes.c_int64), i64,
                                         ctypes.c_int, dp, dp, ctypes.c_int]
        L.oracle_near_blocks.restype = ctypes.c_int
        L.oracle_periodic.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, i64, dp, dp,
                                      dp, dp, dp, i64, ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                      ctypes.c_int, dp, ctypes.c_int]
        L.oracle_periodic.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(x):
    if x is None:
        return None
    return x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(x, shape_last=None):
    if x is None:
        return None
    x = np.ascontiguousarray(x, dtype=np.float64)
    return x


def moduli(G=1.0, nu=0.3):
    """Bulk modulus K from (G, nu): K = 2G(1+nu) / (3(1-2nu))."""
    return 2.0 * G * (1.0 + nu) / (3.0 * (1.0 - 2.0 * nu))


def direct(kind, trg, src, w, a=None, b=None, nrm=None, K=None, G=1.0, nthreads=0):
    """FP64 direct sum.  Returns (M,3) for DISP or (M,6) for STRESS."""
    if K is None:
        K = moduli(G, 0.3)
    trg = _f64(trg).reshape(-1, 3)
    src = _f64(src).reshape(-1, 3)
    w = _f64(w).reshape(-1)
    a = None if a is None else _f64(a).reshape(-1, 3)
    b = None if b is None else _f64(b).reshape(-1, 3)
    nrm = None if nrm is None else _f64(nrm).reshape(-1, 3)
    M, N = trg.shape[0], src.shape[0]
    out = np.zeros((M, 3 if kind == DISP else 6), dtype=np.float64)
    rc = lib().oracle_direct(kind, K, G, _p(trg), M, _p(src), _p(nrm), _p(w), _p(a), _p(b), N, _p(out), nthreads)
    if rc != 0:
        raise ValueError("oracle_direct: bad arguments")
    return out


def quad_blocks(trg, src, nrm, w, elem, n_elem, K, G, nthreads=0):
    """Dense (3M x 3E) quadrature matrices Umat, Pmat (eq. coef), coincident pairs skipped."""
    trg = _f64(trg).reshape(-1, 3)
    src = _f64(src).reshape(-1, 3)
    nrm = _f64(nrm).reshape(-1, 3)
    w = _f64(w).reshape(-1)
    elem = np.ascontiguousarray(elem, dtype=np.int64)
    M, N = trg.shape[0], src.shape[0]
    Um = np.empty((3 * M, 3 * n_elem))
    Pm = np.empty((3 * M, 3 * n_elem))
    rc = lib().oracle_quad_blocks(K, G, _p(trg), M, _p(src), _p(nrm), _p(w),
                                  elem.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), N, n_elem, _p(Um), _p(Pm),
                                  nthreads)
    if rc != 0:
        raise ValueError("oracle_quad_blocks: bad arguments")
    return Um, Pm


def pair_kernels(trg, src, nrm, K, G):
    """Kernel tensors of single pairs: U[n,3,3], P[n,3,3], D[n,3,3,3], S[n,3,3,3] ([k,i,j])."""
    trg = _f64(trg).reshape(-1, 3)
    src = _f64(src).reshape(-1, 3)
    nrm = _f64(nrm).reshape(-1, 3)
    n = trg.shape[0]
    U = np.empty((n, 3, 3)); P = np.empty((n, 3, 3)); D = np.empty((n, 3, 3, 3)); S = np.empty((n, 3, 3, 3))
    rc = lib().oracle_pair_kernels(K, G, _p(trg), _p(src), _p(nrm), n, _p(U), _p(P), _p(D), _p(S))
    if rc != 0:
        raise ValueError("oracle_pair_kernels: coincident pair or bad moduli")
    return U, P, D, S


def near_blocks(colloc, tri, pairs, levels, K, G, nthreads=0):
    """Upsampled quadrature blocks (see oracle_near_blocks in direct.c): for each pair (t, e) the 3x3 blocks
    U, P of triangle e at collocation point t with the rule of `levels` extra midpoint splits.  Returns
    U, P of shape (n, 3, 3)."""
    colloc = _f64(colloc).reshape(-1, 3)
    tri = _f64(tri).reshape(-1, 3, 3)
    pairs = np.ascontiguousarray(pairs, dtype=np.int64).reshape(-1, 2)
    n = pairs.shape[0]
    U = np.zeros((n, 3, 3))
    P = np.zeros((n, 3, 3))
    rc = lib().oracle_near_blocks(K, G, _p(colloc), _p(tri), pairs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                  n, int(levels), _p(U), _p(P), nthreads)
    if rc != 0:
        raise ValueError("oracle_near_blocks: bad arguments")
    return U, P
