"""ctypes binding of libkfmm.so (C ABI: include/kfmm.h).

Argument marshalling only: tensors must already live on the GPU in FP64; every step of the
computation runs in the library's HIP kernels.  The library must have been built
(``python -m paper_1612_04082_amd.build`` or ``__graft_entry__.build()``); nothing falls back to
another implementation when it is missing.
"""
import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkfmm.so")

DISP, STRESS = 0, 1
FP64, FP32, FP32_M2L_BF16 = 0, 1, 2
PHASES = ("permute", "s2m", "uc2ue", "m2m", "m2l_prep", "m2l", "s2l", "down", "leaf")
_STATUS = {0: "OK", -1: "E_ARG", -2: "E_OOM", -3: "E_HIP", -4: "E_NOCONV", -5: "E_STATE"}


class KfmmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"kfmm {_STATUS.get(code, code)}: {msg}")
        self.code = code


class FmmOpts(ctypes.Structure):
    _fields_ = [("K", ctypes.c_double), ("G", ctypes.c_double), ("p", ctypes.c_int), ("leaf_max", ctypes.c_int),
                ("precision", ctypes.c_int), ("svd_eps", ctypes.c_double), ("max_depth", ctypes.c_int),
                ("mem_limit", ctypes.c_size_t)]


class FmmInfo(ctypes.Structure):
    _fields_ = [("n_src", ctypes.c_int64), ("n_trg", ctypes.c_int64), ("n_box", ctypes.c_int64),
                ("n_leaf", ctypes.c_int64), ("depth", ctypes.c_int32), ("n_eq", ctypes.c_int32),
                ("n_u_pairs", ctypes.c_int64), ("n_v_pairs", ctypes.c_int64), ("n_w_pairs", ctypes.c_int64),
                ("n_x_pairs", ctypes.c_int64), ("plan_seconds", ctypes.c_double), ("device_bytes", ctypes.c_size_t)]


_lib = None


def load_library():
    """Load libkfmm.so; raises if it has not been built (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not built: run __graft_entry__.build() or python -m paper_1612_04082_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    L.fmm_plan.argtypes = [ctypes.POINTER(vp), vp, vp, vp, i64, vp, i64, ctypes.POINTER(i64), ctypes.POINTER(i64),
                           i32, ctypes.POINTER(FmmOpts), vp]
    L.fmm_plan.restype = ctypes.c_int
    L.fmm_eval.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp]
    L.fmm_eval.restype = ctypes.c_int
    L.fmm_plan_info.argtypes = [vp, ctypes.POINTER(FmmInfo)]
    L.fmm_plan_info.restype = ctypes.c_int
    L.fmm_plan_destroy.argtypes = [vp]
    L.fmm_plan_destroy.restype = ctypes.c_int
    L.fmm_profile.argtypes = [vp, ctypes.c_int]
    L.fmm_profile.restype = ctypes.c_int
    L.fmm_phase_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    L.fmm_phase_times.restype = ctypes.c_int
    ip = ctypes.POINTER(ctypes.c_int)
    L.kfmm_selftest_gemm.argtypes = [ctypes.c_int, vp, ctypes.c_int, vp, vp, ip, ip, ip,
                                     ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_int, vp]
    L.kfmm_selftest_gemm.restype = ctypes.c_int
    L.kfmm_last_error.argtypes = []
    L.kfmm_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def check(rc):
    if rc != 0:
        raise KfmmError(rc, load_library().kfmm_last_error().decode())


def moduli(G=1.0, nu=0.3):
    """Bulk modulus K from (G, nu)."""
    return 2.0 * G * (1.0 + nu) / (3.0 * (1.0 - 2.0 * nu))


def _dptr(t, name, shape_last=None):
    if t is None:
        return None
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")
    if shape_last is not None and t.shape[-1] != shape_last:
        raise ValueError(f"{name} must have last dimension {shape_last}")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class FmmPlan:
    """fmm_plan / fmm_eval / fmm_plan_destroy on torch tensors (FP64, on the current CUDA device)."""

    def __init__(self, src, nrm=None, w=None, trg=None, K=None, G=1.0, p=6, leaf_max=64, precision=FP32,
                 svd_eps=0.0, max_depth=0, mem_limit=0, batch_src=None, batch_trg=None):
        L = load_library()
        self._h = ctypes.c_void_p()
        if K is None:
            K = moduli(G, 0.3)
        self.opts = FmmOpts(K, G, p, leaf_max, precision, svd_eps, max_depth, mem_limit)
        self.n_src = int(src.shape[0])
        self.n_trg = int(trg.shape[0]) if trg is not None else self.n_src
        self._keep = (src, nrm, w, trg)
        nb = 0
        bs = bt = None
        if batch_src is not None:
            nb = len(batch_src) - 1
            bs = (ctypes.c_int64 * len(batch_src))(*[int(v) for v in batch_src])
            bt_list = batch_trg if batch_trg is not None else batch_src
            bt = (ctypes.c_int64 * len(bt_list))(*[int(v) for v in bt_list])
        check(L.fmm_plan(ctypes.byref(self._h), _dptr(src, "src", 3), _dptr(nrm, "nrm", 3), _dptr(w, "w"),
                         self.n_src, _dptr(trg, "trg", 3), self.n_trg, bs, bt, nb, ctypes.byref(self.opts),
                         _stream()))

    def eval(self, kind, a=None, b=None, out=None):
        no = 3 if kind == DISP else 6
        if out is None:
            dev = self._keep[0].device
            out = torch.empty((self.n_trg, no), dtype=torch.float64, device=dev)
        check(load_library().fmm_eval(self._h, kind, _dptr(a, "a", 3), _dptr(b, "b", 3), _dptr(out, "out", no),
                                      _stream()))
        return out

    def info(self):
        inf = FmmInfo()
        check(load_library().fmm_plan_info(self._h, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in FmmInfo._fields_}

    def profile(self, enable=True):
        check(load_library().fmm_profile(self._h, 1 if enable else 0))

    def phase_times(self):
        """Summed milliseconds per phase over the profiled evals, and the number of evals."""
        ms = (ctypes.c_double * len(PHASES))()
        calls = ctypes.c_int64()
        check(load_library().fmm_phase_times(self._h, ms, ctypes.byref(calls)))
        return dict(zip(PHASES, list(ms))), calls.value

    def close(self):
        if self._h:
            check(load_library().fmm_plan_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def selftest_gemm(precision, A, X, Y, op, cols_in, cols_out, scale=None, mode=0):
    """Test hook around kfmm_selftest_gemm (see include/kfmm.h)."""
    import numpy as np
    L = load_library()
    n = len(op)
    ia = lambda v: (ctypes.c_int * max(n, 1))(*[int(x) for x in v])
    sc = None if scale is None else (ctypes.c_double * max(n, 1))(*[float(x) for x in scale])
    NC = int(A.shape[-1])
    check(L.kfmm_selftest_gemm(precision, ctypes.c_void_p(A.data_ptr()), NC, ctypes.c_void_p(X.data_ptr()),
                               ctypes.c_void_p(Y.data_ptr()), ia(op), ia(cols_in), ia(cols_out), sc, n, mode,
                               _stream()))
