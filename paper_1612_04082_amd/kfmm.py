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
FP64, FP32, FP32_M2L_BF16, FP32_M2L_SPLIT16, FP32_TRANS64 = 0, 1, 2, 3, 4  # FP32_M2L_BF16: withdrawn (E_ARG)
PC_NONE, PC_TWO_LEVEL = 0, 1
PHASES = ("permute", "s2m", "uc2ue", "m2m", "m2l_prep", "m2l", "m2l_red", "s2l", "down", "near", "leaf")
_STATUS = {0: "OK", -1: "E_ARG", -2: "E_OOM", -3: "E_HIP", -4: "E_NOCONV", -5: "E_STATE"}


class KfmmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"kfmm {_STATUS.get(code, code)}: {msg}")
        self.code = code


class FmmOpts(ctypes.Structure):
    _fields_ = [("K", ctypes.c_double), ("G", ctypes.c_double), ("p", ctypes.c_int), ("leaf_max", ctypes.c_int),
                ("precision", ctypes.c_int), ("svd_eps", ctypes.c_double), ("max_depth", ctypes.c_int),
                ("mem_limit", ctypes.c_size_t), ("m2l_tol", ctypes.c_double)]


class FmmInfo(ctypes.Structure):
    _fields_ = [("n_src", ctypes.c_int64), ("n_trg", ctypes.c_int64), ("n_box", ctypes.c_int64),
                ("n_leaf", ctypes.c_int64), ("depth", ctypes.c_int32), ("n_eq", ctypes.c_int32),
                ("n_u_pairs", ctypes.c_int64), ("n_v_pairs", ctypes.c_int64), ("n_w_pairs", ctypes.c_int64),
                ("n_x_pairs", ctypes.c_int64), ("plan_seconds", ctypes.c_double), ("device_bytes", ctypes.c_size_t),
                ("m2l_rank", ctypes.c_int32)]


class BemProblem(ctypes.Structure):
    _fields_ = [("n_tri", ctypes.c_int64), ("tri_xyz", ctypes.c_void_p), ("bc_type", ctypes.c_void_p),
                ("bc_val", ctypes.c_void_p), ("K", ctypes.c_double), ("G", ctypes.c_double),
                ("near_levels", ctypes.c_int), ("near_radius", ctypes.c_double),
                ("cell", ctypes.POINTER(ctypes.c_double))]


class BemOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("restart", ctypes.c_int), ("max_iter", ctypes.c_int), ("fmm", FmmOpts),
                ("x0_alt", ctypes.c_void_p), ("precond", ctypes.c_int), ("pc_fine", ctypes.c_int),
                ("pc_coarse", ctypes.c_int)]


class BemPcInfo(ctypes.Structure):
    _fields_ = [("n_fine_blocks", ctypes.c_int64), ("n_aggregates", ctypes.c_int64), ("n_coarse", ctypes.c_int64),
                ("fine", ctypes.c_int), ("coarse", ctypes.c_int), ("n_dropped", ctypes.c_int),
                ("t_setup_s", ctypes.c_double)]


class BemStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("restarts", ctypes.c_int), ("converged", ctypes.c_int),
                ("used_alt", ctypes.c_int), ("used_zero", ctypes.c_int), ("rel_res_alt", ctypes.c_double),
                ("rel_res_start", ctypes.c_double), ("start_coef", ctypes.c_double * 2), ("n_matvec", ctypes.c_int64), ("rel_res", ctypes.c_double), ("rel_res0", ctypes.c_double),
                ("res_estimate", ctypes.c_double), ("b_norm", ctypes.c_double), ("t_setup_s", ctypes.c_double),
                ("t_solve_s", ctypes.c_double), ("t_precond_s", ctypes.c_double), ("pc_coarse_dim", ctypes.c_int64)]


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
    L.fmm_plan_periodic.argtypes = [ctypes.POINTER(vp), vp, vp, vp, i64, vp, i64, ctypes.POINTER(i64),
                                    ctypes.POINTER(i64), i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(FmmOpts),
                                    vp]
    L.fmm_plan_periodic.restype = ctypes.c_int
    L.fmm_eval.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp]
    L.fmm_eval.restype = ctypes.c_int
    L.fmm_plan_info.argtypes = [vp, ctypes.POINTER(FmmInfo)]
    L.fmm_plan_info.restype = ctypes.c_int
    L.fmm_plan_destroy.argtypes = [vp]
    L.fmm_plan_destroy.restype = ctypes.c_int
    L.fmm_plan_work.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(ctypes.c_double)]
    L.fmm_plan_work.restype = ctypes.c_int
    L.fmm_plan_target_lists.argtypes = [vp, ctypes.POINTER(i32)]
    L.fmm_plan_target_lists.restype = ctypes.c_int
    L.fmm_profile.argtypes = [vp, ctypes.c_int]
    L.fmm_profile.restype = ctypes.c_int
    L.fmm_phase_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    L.fmm_phase_times.restype = ctypes.c_int
    L.bem_solve.argtypes = [ctypes.POINTER(BemProblem), ctypes.POINTER(BemOpts), vp, vp, vp, vp,
                            ctypes.POINTER(BemStats), vp]
    L.bem_solve.restype = ctypes.c_int
    L.bem_stress.argtypes = [ctypes.POINTER(BemProblem), vp, vp, vp, i64, vp, ctypes.POINTER(FmmOpts), vp]
    L.bem_stress.restype = ctypes.c_int
    L.bem_precond_apply.argtypes = [ctypes.POINTER(BemProblem), ctypes.POINTER(BemOpts), vp, vp,
                                    ctypes.POINTER(BemPcInfo), vp]
    L.bem_precond_apply.restype = ctypes.c_int
    L.bem_matvec.argtypes = [ctypes.POINTER(BemProblem), ctypes.POINTER(FmmOpts), ctypes.c_int, vp, vp, vp]
    L.bem_near_pairs.argtypes = [ctypes.POINTER(BemProblem), ctypes.POINTER(i64), vp, i64, vp]
    L.bem_near_pairs.restype = ctypes.c_int
    gp = ctypes.POINTER(Alg1Grid)
    L.alg1_surface.argtypes = [gp, vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64), vp, vp, vp, vp, i64, vp]
    L.alg1_centres.argtypes = [gp, vp, ctypes.POINTER(i64), vp, i64, vp]
    L.alg1_update.argtypes = [gp, vp, vp, i64, ctypes.c_double, vp, ctypes.POINTER(i64), vp]
    L.alg1_coarse_blocks.argtypes = [gp, vp, ctypes.c_int, ctypes.POINTER(i64), vp, i64, vp]
    L.alg1_refine.argtypes = [gp, vp, ctypes.c_int, vp, i64, ctypes.c_double, ctypes.POINTER(i64), vp, i64, vp, vp]
    L.alg1_expand.argtypes = [gp, vp, ctypes.c_int, vp, i64, ctypes.c_double, vp, i64, vp, vp]
    L.alg1_energy.argtypes = [vp, i64, ctypes.c_double, ctypes.c_double, ctypes.POINTER(ctypes.c_double), vp]
    L.alg1_cell_surface.argtypes = [gp, vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64), vp, vp, vp, vp, i64,
                                    vp]
    L.alg1_cell_td.argtypes = [vp, i64, ctypes.POINTER(ctypes.c_double), ctypes.c_double, ctypes.c_double, vp, vp]
    L.alg1_cell_update.argtypes = [gp, vp, vp, i64, ctypes.c_double, vp, ctypes.POINTER(i64), vp]
    for f in ("alg1_surface", "alg1_centres", "alg1_update", "alg1_coarse_blocks", "alg1_refine", "alg1_expand",
              "alg1_energy", "alg1_cell_surface", "alg1_cell_td", "alg1_cell_update"):
        getattr(L, f).restype = ctypes.c_int
    L.bem_matvec.restype = ctypes.c_int
    L.bem_quadrature.argtypes = [i64, vp, vp, vp, vp, vp, vp]
    L.bem_quadrature.restype = ctypes.c_int
    L.kfmm_topological_derivative.argtypes = [vp, i64, ctypes.c_double, ctypes.c_double, vp, vp]
    L.kfmm_topological_derivative.restype = ctypes.c_int
    fp = ctypes.c_void_p
    L.ws_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int, ctypes.c_uint64]
    L.ws_destroy.argtypes = [vp]
    L.ws_features.argtypes = [ctypes.POINTER(BemProblem), vp, vp, ctypes.POINTER(BemProblem), fp, vp,
                              ctypes.POINTER(ctypes.c_double), vp]
    L.ws_predict.argtypes = [vp, fp, i64, vp, ctypes.c_double, vp, vp]
    L.ws_train.argtypes = [vp, fp, vp, vp, i64, ctypes.c_double, ctypes.c_int, ctypes.c_float,
                           ctypes.POINTER(ctypes.c_float), vp]
    L.ws_train_noalloc.argtypes = [vp, fp, vp, vp, i64, ctypes.c_double, ctypes.c_int, ctypes.c_float,
                                   ctypes.POINTER(ctypes.c_float), vp]
    L.ws_num_params.argtypes = [vp, ctypes.POINTER(i64)]
    L.ws_get_params.argtypes = [vp, ctypes.POINTER(ctypes.c_float)]
    L.ws_set_params.argtypes = [vp, ctypes.POINTER(ctypes.c_float)]
    L.ws_loss_grad.argtypes = [vp, fp, fp, i64, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float), vp]
    L.ws_save.argtypes = [vp, ctypes.c_char_p]
    L.ws_load.argtypes = [vp, ctypes.c_char_p]
    for f in ("ws_create", "ws_destroy", "ws_features", "ws_predict", "ws_train", "ws_train_noalloc", "ws_num_params",
              "ws_get_params",
              "ws_set_params", "ws_loss_grad", "ws_save", "ws_load"):
        getattr(L, f).restype = ctypes.c_int
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


def _dptr(t, name, shape_last=None, rows=None):
    """Device pointer of a contiguous FP64 CUDA tensor; rows: required leading dimension (the library
    reads exactly that many records, so a shorter array must not reach it)."""
    if t is None:
        return None
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")
    if shape_last is not None and (t.dim() < 2 or t.shape[-1] != shape_last):
        raise ValueError(f"{name} must have last dimension {shape_last}")
    if rows is not None and int(t.shape[0]) != int(rows):
        raise ValueError(f"{name} must have {rows} rows, got {int(t.shape[0])}")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class FmmPlan:
    """fmm_plan / fmm_eval / fmm_plan_destroy on torch tensors (FP64, on the current CUDA device)."""

    def __init__(self, src, nrm=None, w=None, trg=None, K=None, G=1.0, p=6, leaf_max=64, precision=FP32,
                 svd_eps=0.0, max_depth=0, mem_limit=0, batch_src=None, batch_trg=None, m2l_tol=0.0, cells=None):
        """cells: None (free space) or a sequence of (x0, y0, z0, side) per geometry -- periodic cubic cells
        (fmm_plan_periodic)."""
        L = load_library()
        self._h = ctypes.c_void_p()
        if K is None:
            K = moduli(G, 0.3)
        self.opts = FmmOpts(K, G, p, leaf_max, precision, svd_eps, max_depth, mem_limit, m2l_tol)
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
        if w is not None and (w.dim() != 1 or int(w.shape[0]) != self.n_src):
            raise ValueError(f"w must have shape ({self.n_src},)")
        args = (ctypes.byref(self._h), _dptr(src, "src", 3), _dptr(nrm, "nrm", 3, self.n_src), _dptr(w, "w"),
                self.n_src, _dptr(trg, "trg", 3), self.n_trg, bs, bt, nb)
        if cells is None:
            check(L.fmm_plan(*args, ctypes.byref(self.opts), _stream()))
        else:
            flat = [float(v) for row in cells for v in row]
            if len(flat) != 4 * max(nb, 1):
                raise ValueError("cells: one (x0, y0, z0, side) row per geometry")
            self._cells = (ctypes.c_double * len(flat))(*flat)
            check(L.fmm_plan_periodic(*args, self._cells, ctypes.byref(self.opts), _stream()))

    def eval(self, kind, a=None, b=None, out=None):
        no = 3 if kind == DISP else 6
        if out is None:
            dev = self._keep[0].device
            out = torch.empty((self.n_trg, no), dtype=torch.float64, device=dev)
        check(load_library().fmm_eval(self._h, kind, _dptr(a, "a", 3, self.n_src), _dptr(b, "b", 3, self.n_src),
                                      _dptr(out, "out", no, self.n_trg), _stream()))
        return out

    def info(self):
        inf = FmmInfo()
        check(load_library().fmm_plan_info(self._h, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in FmmInfo._fields_}

    def work(self, kind, with_a=True, with_b=True):
        """Algorithmic FLOP and HBM bytes of one evaluation, per phase: {phase: (flops, bytes)}."""
        fl = (ctypes.c_double * len(PHASES))()
        by = (ctypes.c_double * len(PHASES))()
        check(load_library().fmm_plan_work(self._h, kind, int(bool(with_a)), int(bool(with_b)), fl, by))
        return {ph: (fl[i], by[i]) for i, ph in enumerate(PHASES)}

    def target_lists(self):
        """Host int32 array, one entry per target (caller order): bit 0 = its leaf has a W list, bit 1 = its
        leaf has an X list, bit 2 = an ancestor of its leaf has an X list."""
        import numpy as np
        flags = np.zeros(self.n_trg, dtype=np.int32)
        if self.n_trg:
            check(load_library().fmm_plan_target_lists(self._h, flags.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return flags

    def profile(self, enable=True):
        """True: time every phase (calls run in turn on one stream); "m2l": time only the M2L launch."""
        mode = 2 if enable == "m2l" else (1 if enable else 0)
        check(load_library().fmm_profile(self._h, mode))

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


def selftest_gemm(precision, A, X, Y, op, cols_in, cols_out, scale=None, mode=0, kernel=0):
    """Test hook around kfmm_selftest_gemm (see include/kfmm.h); kernel 1 = tiled, 2 = split-K,
    3 / 4 = tiled with one / two LDS buffers.  precision 3 = FP32 tensors, products on the FP16 matrix
    cores with split operands (kernel 1: 64-column tiles, as in the translation passes)."""
    L = load_library()
    n = len(op)
    dt = {0: (torch.float64,) * 3, 1: (torch.float32,) * 3, 2: (torch.bfloat16, torch.bfloat16, torch.float32),
          3: (torch.float32,) * 3}[precision]
    NC = int(A.shape[-1])
    for t, d, name in ((A, dt[0], "A"), (X, dt[1], "X"), (Y, dt[2], "Y")):
        if not (t.is_cuda and t.dtype == d and t.is_contiguous() and t.shape[-1] == NC):
            raise TypeError(f"{name}: expected a contiguous CUDA {d} tensor with {NC} columns")
    if n and not (max(op) < A.reshape(-1, NC, NC).shape[0] and max(cols_in) < X.shape[0]
                  and max(cols_out) < Y.shape[0] and min(min(op), min(cols_in), min(cols_out)) >= 0):
        raise ValueError("column index out of range")
    ia = lambda v: (ctypes.c_int * max(n, 1))(*[int(x) for x in v])
    sc = None if scale is None else (ctypes.c_double * max(n, 1))(*[float(x) for x in scale])
    check(L.kfmm_selftest_gemm(precision + 16 * kernel, ctypes.c_void_p(A.data_ptr()), NC, ctypes.c_void_p(X.data_ptr()),
                               ctypes.c_void_p(Y.data_ptr()), ia(op), ia(cols_in), ia(cols_out), sc, n, mode,
                               _stream()))


def _problem(tri, bc_type, bc_val, K, G, near_levels=0, near_radius=0.0, cell=None):
    """cell: None (free space) or (x0, y0, z0, side) of a periodic cubic cell."""
    if not (bc_type.is_cuda and bc_type.dtype == torch.int8 and bc_type.is_contiguous()):
        raise TypeError("bc_type must be a contiguous int8 CUDA tensor")
    T = int(tri.shape[0])
    if tuple(tri.shape[1:]) != (3, 3) or tuple(bc_type.shape) != (T, 3):
        raise ValueError("tri must be (T,3,3) and bc_type (T,3)")
    cell_arr = None
    if cell is not None:
        if len(cell) != 4:
            raise ValueError("cell must be (x0, y0, z0, side)")
        cell_arr = (ctypes.c_double * 4)(*[float(v) for v in cell])
    pr = BemProblem(T, _dptr(tri, "tri").value, ctypes.c_void_p(bc_type.data_ptr()).value,
                    _dptr(bc_val, "bc_val", 3, T).value, K, G, near_levels, near_radius,
                    ctypes.cast(cell_arr, ctypes.POINTER(ctypes.c_double)) if cell_arr is not None else None)
    pr._cell_keep = cell_arr  # the C side reads the cell through this pointer
    return pr


def bem_solve(tri, bc_type, bc_val, K=None, G=1.0, tol=1e-6, restart=50, max_iter=2000, x0=None, p=8,
              leaf_max=128, precision=FP32, svd_eps=0.0, want_full=True, allow_noconv=False, x0_alt=None,
              precond=PC_NONE, pc_fine=0, pc_coarse=0, near_levels=0, near_radius=0.0, cell=None, m2l_tol=0.0):
    """bem_solve on torch tensors: tri (T,3,3) f64, bc_type (T,3) int8, bc_val (T,3) f64, all on the GPU.
    cell: None, or (x0, y0, z0, side) of a periodic cell (needs precision=FP64).  m2l_tol: the products' M2L
    on the compressed basis (fmm_opts.m2l_tol; with FP64, FP64 contractions).

    Returns (x, u, t, stats) with x the unknowns (physical units) and u, t the full boundary data."""
    L = load_library()
    if K is None:
        K = moduli(G, 0.3)
    prob = _problem(tri, bc_type, bc_val, K, G, near_levels, near_radius, cell)
    alt = _dptr(x0_alt, "x0_alt", 3, int(tri.shape[0]))
    opts = BemOpts(tol, restart, max_iter, FmmOpts(K, G, p, leaf_max, precision, svd_eps, 0, 0, m2l_tol),
                   alt.value if alt is not None else None, precond, pc_fine, pc_coarse)
    T = int(tri.shape[0])
    x = torch.empty((T, 3), dtype=torch.float64, device=tri.device)
    u = torch.empty_like(x) if want_full else None
    t = torch.empty_like(x) if want_full else None
    st = BemStats()
    rc = L.bem_solve(ctypes.byref(prob), ctypes.byref(opts), _dptr(x0, "x0", 3, T), _dptr(x, "x", 3),
                     _dptr(u, "u", 3), _dptr(t, "t", 3), ctypes.byref(st), _stream())
    stats = {k: getattr(st, k) for k, _ in BemStats._fields_}
    stats["start_coef"] = list(st.start_coef)
    if rc == -4 and allow_noconv:
        return x, u, t, stats
    check(rc)
    return x, u, t, stats


def bem_precond_apply(tri, bc_type, bc_val, v, K=None, G=1.0, p=8, leaf_max=128, precision=FP32, svd_eps=0.0,
                      pc_fine=0, pc_coarse=0, near_levels=0, near_radius=0.0):
    """y = M^-1 v for the two-level preconditioner of the system bem_solve builds (v: (T,3) f64 on the GPU,
    solver units).  Returns (y, info dict)."""
    L = load_library()
    if K is None:
        K = moduli(G, 0.3)
    prob = _problem(tri, bc_type, bc_val, K, G, near_levels, near_radius)
    T = int(tri.shape[0])
    opts = BemOpts(1e-6, 50, 0, FmmOpts(K, G, p, leaf_max, precision, svd_eps, 0, 0, 0.0), None, PC_TWO_LEVEL,
                   pc_fine, pc_coarse)
    y = torch.empty((T, 3), dtype=torch.float64, device=tri.device)
    info = BemPcInfo()
    check(L.bem_precond_apply(ctypes.byref(prob), ctypes.byref(opts), _dptr(v, "v", 3, T), _dptr(y, "y", 3),
                              ctypes.byref(info), _stream()))
    return y, {k: getattr(info, k) for k, _ in BemPcInfo._fields_}


def bem_stress(tri, bc_type, bc_val, u, t, trg, K=None, G=1.0, p=8, leaf_max=128, precision=FP32, svd_eps=0.0,
               cell=None, m2l_tol=0.0):
    """Interior stress (M,6) from boundary u, t (eq. stress_1) at trg (M,3); cell, m2l_tol as in bem_solve."""
    L = load_library()
    if K is None:
        K = moduli(G, 0.3)
    prob = _problem(tri, bc_type, bc_val, K, G, cell=cell)
    fo = FmmOpts(K, G, p, leaf_max, precision, svd_eps, 0, 0, m2l_tol)
    M = int(trg.shape[0])
    out = torch.empty((M, 6), dtype=torch.float64, device=trg.device)
    T = int(tri.shape[0])
    check(L.bem_stress(ctypes.byref(prob), _dptr(u, "u", 3, T), _dptr(t, "t", 3, T), _dptr(trg, "trg", 3), M,
                       _dptr(out, "out", 6), ctypes.byref(fo), _stream()))
    return out


def bem_quadrature(tri):
    """16 quadrature points per triangle, normals, weights and collocation points (device tensors)."""
    L = load_library()
    T = int(tri.shape[0])
    dev = tri.device
    qp = torch.empty((16 * T, 3), dtype=torch.float64, device=dev)
    qn = torch.empty_like(qp)
    qw = torch.empty((16 * T,), dtype=torch.float64, device=dev)
    cen = torch.empty((T, 3), dtype=torch.float64, device=dev)
    check(L.bem_quadrature(T, _dptr(tri, "tri"), _dptr(qp, "qp"), _dptr(qn, "qn"), _dptr(qw, "qw"),
                           _dptr(cen, "cen"), _stream()))
    return qp, qn, qw, cen


def bem_matvec(tri, bc_type, bc_val, x=None, which=0, K=None, G=1.0, p=8, leaf_max=128, precision=FP32,
               svd_eps=0.0, near_levels=0, near_radius=0.0, cell=None, m2l_tol=0.0):
    """y = A x (which=0, x in solver units) or the right-hand side B y (which=1); cell, m2l_tol as in
    bem_solve."""
    L = load_library()
    if K is None:
        K = moduli(G, 0.3)
    prob = _problem(tri, bc_type, bc_val, K, G, near_levels, near_radius, cell)
    fo = FmmOpts(K, G, p, leaf_max, precision, svd_eps, 0, 0, m2l_tol)
    y = torch.empty((int(tri.shape[0]), 3), dtype=torch.float64, device=tri.device)
    check(L.bem_matvec(ctypes.byref(prob), ctypes.byref(fo), which, _dptr(x, "x", 3, int(tri.shape[0])),
                       _dptr(y, "y", 3), _stream()))
    return y


def bem_near_pairs(tri, near_radius=0.0):
    """Near pairs (t, e) of the triangles (int32 (n, 2) on the GPU), sorted by t then e."""
    L = load_library()
    T = int(tri.shape[0])
    bc = torch.zeros((T, 3), dtype=torch.int8, device=tri.device)
    val = torch.zeros((T, 3), dtype=torch.float64, device=tri.device)
    prob = _problem(tri, bc, val, 1.0, 1.0, 0, near_radius)
    n = ctypes.c_int64(0)
    check(L.bem_near_pairs(ctypes.byref(prob), ctypes.byref(n), None, 0, _stream()))
    out = torch.empty((max(n.value, 1), 2), dtype=torch.int32, device=tri.device)
    check(L.bem_near_pairs(ctypes.byref(prob), ctypes.byref(n), ctypes.c_void_p(out.data_ptr()), n.value,
                           _stream()))
    return out[:n.value]


class Alg1Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int), ("h", ctypes.c_double)]


def _vox(vox):
    if not (isinstance(vox, torch.Tensor) and vox.is_cuda and vox.dtype == torch.uint8 and vox.is_contiguous()
            and vox.dim() == 3):
        raise TypeError("vox must be a contiguous 3-D uint8 CUDA tensor")
    return ctypes.c_void_p(vox.data_ptr())


def _grid(vox, h):
    return Alg1Grid(int(vox.shape[0]), int(vox.shape[1]), int(vox.shape[2]), float(h))


def _count_then_fill(fn, rows, alloc):
    """Two-call pattern of the alg1_* entry points: query the count, allocate, fill."""
    n = ctypes.c_int64(0)
    check(fn(ctypes.byref(n), None, 0))
    out = alloc(max(n.value, 1))
    check(fn(ctypes.byref(n), out, n.value))
    return n.value, out


def alg1_surface(vox, h, load=(0.0, 0.0, -1.0)):
    """Boundary triangles of a voxel design with the cantilever's conditions (dict of device tensors)."""
    L = load_library()
    g = _grid(vox, h)
    ld = (ctypes.c_double * 3)(*load)
    n = ctypes.c_int64(0)
    check(L.alg1_surface(ctypes.byref(g), _vox(vox), ld, ctypes.byref(n), None, None, None, None, 0, _stream()))
    T = n.value
    dev = vox.device
    tri = torch.empty((max(T, 1), 3, 3), dtype=torch.float64, device=dev)
    bct = torch.empty((max(T, 1), 3), dtype=torch.int8, device=dev)
    bcv = torch.empty((max(T, 1), 3), dtype=torch.float64, device=dev)
    own = torch.empty((max(T, 1), 3), dtype=torch.int32, device=dev)
    check(L.alg1_surface(ctypes.byref(g), _vox(vox), ld, ctypes.byref(n), ctypes.c_void_p(tri.data_ptr()),
                         ctypes.c_void_p(bct.data_ptr()), ctypes.c_void_p(bcv.data_ptr()),
                         ctypes.c_void_p(own.data_ptr()), T, _stream()))
    return dict(tri=tri[:T], bc_type=bct[:T], bc_val=bcv[:T], owner=own[:T])


def alg1_cell_surface(vox, h, sig_h):
    """Void/material faces of a periodic voxel cell with the superposition tractions -sig_h n (sig_h: 6 values
    xx, yy, zz, yz, xz, xy) as a pure traction problem (dict of device tensors, as alg1_surface)."""
    L = load_library()
    g = _grid(vox, h)
    sh = (ctypes.c_double * 6)(*[float(v) for v in sig_h])
    n = ctypes.c_int64(0)
    check(L.alg1_cell_surface(ctypes.byref(g), _vox(vox), sh, ctypes.byref(n), None, None, None, None, 0, _stream()))
    T = n.value
    dev = vox.device
    tri = torch.empty((max(T, 1), 3, 3), dtype=torch.float64, device=dev)
    bct = torch.empty((max(T, 1), 3), dtype=torch.int8, device=dev)
    bcv = torch.empty((max(T, 1), 3), dtype=torch.float64, device=dev)
    own = torch.empty((max(T, 1), 3), dtype=torch.int32, device=dev)
    check(L.alg1_cell_surface(ctypes.byref(g), _vox(vox), sh, ctypes.byref(n), ctypes.c_void_p(tri.data_ptr()),
                              ctypes.c_void_p(bct.data_ptr()), ctypes.c_void_p(bcv.data_ptr()),
                              ctypes.c_void_p(own.data_ptr()), T, _stream()))
    return dict(tri=tri[:T], bc_type=bct[:T], bc_val=bcv[:T], owner=own[:T])


def alg1_cell_td(sig6, sig_h, K=None, G=1.0):
    """Topological derivative (eq. deriv) of the total stresses sig6 + sig_h (device (M,6) -> (M,))."""
    if K is None:
        K = moduli(G, 0.3)
    M = int(sig6.shape[0])
    td = torch.empty((M,), dtype=torch.float64, device=sig6.device)
    sh = (ctypes.c_double * 6)(*[float(v) for v in sig_h])
    check(load_library().alg1_cell_td(_dptr(sig6, "sig6", 6) if M else None, M, sh, float(K), float(G),
                                      _dptr(td, "td") if M else None, _stream()))
    return td


def alg1_cell_update(vox, h, td, alpha):
    """Keep the material with the largest td at round(alpha n) filled voxels; returns (vox_new, n_filled)."""
    L = load_library()
    g = _grid(vox, h)
    out = torch.empty_like(vox)
    n = ctypes.c_int64(0)
    check(L.alg1_cell_update(ctypes.byref(g), _vox(vox), _dptr(td, "td"), int(td.numel()), float(alpha),
                             ctypes.c_void_p(out.data_ptr()), ctypes.byref(n), _stream()))
    return out, n.value


def _points(vox):
    return lambda m: torch.empty((m, 3), dtype=torch.float64, device=vox.device)


def alg1_centres(vox, h):
    L = load_library()
    g = _grid(vox, h)
    n, pts = _count_then_fill(lambda cnt, out, cap: L.alg1_centres(
        ctypes.byref(g), _vox(vox), cnt, None if out is None else ctypes.c_void_p(out.data_ptr()), cap, _stream()),
        3, _points(vox))
    return pts[:n]


def alg1_update(vox, h, td, C):
    """New design after the removal rule and post-processing; returns (vox_new, n_filled)."""
    L = load_library()
    g = _grid(vox, h)
    out = torch.empty_like(vox)
    n = ctypes.c_int64(0)
    check(L.alg1_update(ctypes.byref(g), _vox(vox), _dptr(td, "td"), int(td.numel()), float(C),
                        ctypes.c_void_p(out.data_ptr()), ctypes.byref(n), _stream()))
    return out, n.value


def alg1_coarse_blocks(vox, h, block):
    L = load_library()
    g = _grid(vox, h)
    n, pts = _count_then_fill(lambda cnt, out, cap: L.alg1_coarse_blocks(
        ctypes.byref(g), _vox(vox), int(block), cnt, None if out is None else ctypes.c_void_p(out.data_ptr()), cap,
        _stream()), 3, _points(vox))
    return pts[:n]


def alg1_refine(vox, h, block, td_coarse, C):
    """Centres of the voxels to evaluate in the second round and the refined-block mask (device tensors)."""
    L = load_library()
    g = _grid(vox, h)
    nb = [-(-int(d) // int(block)) for d in vox.shape]
    mask = torch.empty(nb, dtype=torch.uint8, device=vox.device)
    tc = _dptr(td_coarse, "td_coarse") if td_coarse is not None and td_coarse.numel() else None
    nc = 0 if td_coarse is None else int(td_coarse.numel())
    n, pts = _count_then_fill(lambda cnt, out, cap: L.alg1_refine(
        ctypes.byref(g), _vox(vox), int(block), tc, nc, float(C), cnt,
        None if out is None else ctypes.c_void_p(out.data_ptr()), cap, ctypes.c_void_p(mask.data_ptr()), _stream()),
        3, _points(vox))
    return pts[:n], mask


def alg1_expand(vox, h, block, td_coarse, C, td_fine):
    L = load_library()
    g = _grid(vox, h)
    nf = int((vox != 0).sum().item())
    out = torch.empty(max(nf, 1), dtype=torch.float64, device=vox.device)
    tc = _dptr(td_coarse, "td_coarse") if td_coarse is not None and td_coarse.numel() else None
    tf = _dptr(td_fine, "td_fine") if td_fine is not None and td_fine.numel() else None
    nc = 0 if td_coarse is None else int(td_coarse.numel())
    nfine = 0 if td_fine is None else int(td_fine.numel())
    check(L.alg1_expand(ctypes.byref(g), _vox(vox), int(block), tc, nc, float(C), tf, nfine,
                        ctypes.c_void_p(out.data_ptr()), _stream()))
    return out[:nf]


def alg1_energy(sig, K, G):
    L = load_library()
    psi = ctypes.c_double(0.0)
    n = int(sig.shape[0])
    check(L.alg1_energy(_dptr(sig, "sig", 6) if n else None, n, float(K), float(G), ctypes.byref(psi), _stream()))
    return psi.value


def _fptr(t, name, last=None):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float32 CUDA tensor")
    if last is not None and t.shape[-1] != last:
        raise ValueError(f"{name} must have last dimension {last}")
    return ctypes.c_void_p(t.data_ptr())


WS_DIN = 16
WS_NOALLOC_MAX_ROWS = 40000  # KFMM_WS_NOALLOC_MAX_ROWS


class WarmStartNet:
    """ws_* entry points: features, BF16 inference and FP32 Adam training of the warm-start MLP."""

    def __init__(self, seed=0, width=128):
        self._h = ctypes.c_void_p()
        check(load_library().ws_create(ctypes.byref(self._h), WS_DIN, width, seed))

    def num_params(self):
        n = ctypes.c_int64()
        check(load_library().ws_num_params(self._h, ctypes.byref(n)))
        return n.value

    def get_params(self):
        import numpy as np
        out = np.empty(self.num_params(), dtype=np.float32)
        check(load_library().ws_get_params(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return out

    def set_params(self, p):
        import numpy as np
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == self.num_params()
        check(load_library().ws_set_params(self._h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def loss_grad(self, X, R):
        import numpy as np
        g = np.empty(self.num_params(), dtype=np.float32)
        loss = ctypes.c_float()
        if int(R.shape[0]) != int(X.shape[0]):
            raise ValueError("X and R must have the same number of rows")
        check(load_library().ws_loss_grad(self._h, _fptr(X, "X", WS_DIN), _fptr(R, "R", 3), int(X.shape[0]),
                                          ctypes.byref(loss), g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                          _stream()))
        return loss.value, g

    def predict(self, feat, x_mapped, scale):
        x0 = torch.empty_like(x_mapped)
        check(load_library().ws_predict(self._h, _fptr(feat, "feat", WS_DIN), int(feat.shape[0]),
                                        _dptr(x_mapped, "x_mapped", 3, int(feat.shape[0])), float(scale),
                                        _dptr(x0, "x0", 3), _stream()))
        return x0

    def train(self, feat, x_mapped, x_target, scale, epochs=50, lr=1e-3):
        loss = ctypes.c_float()
        n = int(feat.shape[0])
        check(load_library().ws_train(self._h, _fptr(feat, "feat", WS_DIN), _dptr(x_mapped, "x_mapped", 3, n),
                                      _dptr(x_target, "x_target", 3, n), n, float(scale), int(epochs),
                                      float(lr), ctypes.byref(loss), _stream()))
        return loss.value

    def train_noalloc(self, feat, x_mapped, x_target, scale, epochs=50, lr=1e-3):
        """ws_train_noalloc: as train(), with the work buffers in the library's static device scratch
        (n <= WS_NOALLOC_MAX_ROWS); allocates no device memory."""
        loss = ctypes.c_float()
        n = int(feat.shape[0])
        check(load_library().ws_train_noalloc(self._h, _fptr(feat, "feat", WS_DIN), _dptr(x_mapped, "x_mapped", 3, n),
                                              _dptr(x_target, "x_target", 3, n), n, float(scale), int(epochs),
                                              float(lr), ctypes.byref(loss), _stream()))
        return loss.value

    def save(self, path):
        check(load_library().ws_save(self._h, str(path).encode()))

    def load(self, path):
        check(load_library().ws_load(self._h, str(path).encode()))

    def close(self):
        if self._h:
            check(load_library().ws_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ws_features(prev, u_prev, t_prev, nxt):
    """prev / nxt: dicts of device tensors tri, bc_type, bc_val; returns (feat, x_mapped, scale)."""
    L = load_library()
    K = moduli(1.0, 0.3)
    pp = _problem(prev["tri"], prev["bc_type"], prev["bc_val"], K, 1.0)
    pn = _problem(nxt["tri"], nxt["bc_type"], nxt["bc_val"], K, 1.0)
    T = int(nxt["tri"].shape[0])
    dev = nxt["tri"].device
    feat = torch.empty((T, WS_DIN), dtype=torch.float32, device=dev)
    xm = torch.empty((T, 3), dtype=torch.float64, device=dev)
    scale = ctypes.c_double()
    Tp = int(prev["tri"].shape[0])
    check(L.ws_features(ctypes.byref(pp), _dptr(u_prev, "u_prev", 3, Tp), _dptr(t_prev, "t_prev", 3, Tp), ctypes.byref(pn),
                        _fptr(feat, "feat", WS_DIN), _dptr(xm, "x_mapped", 3), ctypes.byref(scale), _stream()))
    return feat, xm, scale.value


def topological_derivative(sig6, K=None, G=1.0):
    """Pointwise topological derivative (eq. deriv) of (M,6) stresses on the GPU."""
    if K is None:
        K = moduli(G, 0.3)
    td = torch.empty((int(sig6.shape[0]),), dtype=torch.float64, device=sig6.device)
    check(load_library().kfmm_topological_derivative(_dptr(sig6, "sig6", 6), int(sig6.shape[0]), K, G,
                                                     _dptr(td, "td"), _stream()))
    return td
