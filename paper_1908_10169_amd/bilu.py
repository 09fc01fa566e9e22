"""Thin ctypes binding of libbilu.so (include/bilu.h).

Argument marshalling only: every step of analyze/factor/apply/solve runs in
the library.  PyTorch provides device buffers and the current HIP stream.
Importing this module never falls back to anything: a missing library raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbilu.so")

BILU_OK = 0
BILU_WARN_PERTURBED = 1
BILU_WARN_NOT_CONVERGED = 2
BILU_ERR_INVALID = -1
BILU_ERR_NO_MEMORY = -2
BILU_ERR_STATE = -3
BILU_ERR_SINGULAR = -4
BILU_ERR_DEVICE = -5
BILU_ERR_INTERNAL = -6

ORDER_ND, ORDER_NATURAL, ORDER_ND_MULTILEVEL = 0, 1, 2
PREC_F64, PREC_F32, PREC_BF16 = 0, 1, 2


class Options(C.Structure):
    _fields_ = [
        ("use_cosine", C.c_int), ("use_ilu1t", C.c_int), ("use_aggregation", C.c_int),
        ("max_block", C.c_int), ("cos_eps", C.c_double), ("ordering", C.c_int),
        ("pre_perm", C.c_void_p), ("drop_norm", C.c_int), ("perturb_tau", C.c_double),
        ("perturb_rho", C.c_double), ("pivot_eps", C.c_double), ("beta_one", C.c_int),
        ("update_precision", C.c_int), ("heap_bytes", C.c_size_t),
        ("collect_timing", C.c_int), ("factor_path", C.c_int), ("apply_path", C.c_int),
        ("use_mwm", C.c_int), ("analyze_path", C.c_int), ("apply_precision", C.c_int),
        ("update_mfma", C.c_int), ("deterministic", C.c_int),
        ("drop_log_margin", C.c_double), ("workers_per_cu", C.c_int), ("use_tuning", C.c_int),
    ]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int64), ("restarts", C.c_int64),
                ("rel_residual", C.c_double), ("seconds", C.c_double), ("converged", C.c_int)]


class Stats(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("nnz_a", C.c_int64), ("ngroups", C.c_int64),
        ("nblocks_initial", C.c_int64), ("nblocks", C.c_int64), ("max_width", C.c_int64),
        ("avg_width", C.c_double), ("std_width", C.c_double),
        ("nnz_l", C.c_int64), ("nnz_w", C.c_int64), ("nnz_d", C.c_int64),
        ("merges", C.c_int64), ("perturbed_blocks", C.c_int64), ("factor_levels", C.c_int64),
        ("apply_levels_fwd", C.c_int64), ("apply_levels_bwd", C.c_int64),
        ("flops_update", C.c_double), ("bytes_apply", C.c_double),
        ("t_analyze", C.c_double), ("t_ilu1t", C.c_double), ("t_factor_device", C.c_double),
        ("t_aggregate", C.c_double), ("t_factor", C.c_double),
        ("dev_ms_factor", C.c_double), ("dev_ms_apply", C.c_double), ("dev_ms_spmv", C.c_double),
        ("n_factor_launches", C.c_int64), ("n_apply", C.c_int64), ("n_spmv", C.c_int64),
        ("bytes_factor", C.c_double), ("t_phase", C.c_double * 8),
        ("apply_faults", C.c_int64), ("heap_regrows", C.c_int64), ("r_kept", C.c_double),
        ("drops_rows", C.c_int64), ("drops_cols", C.c_int64), ("drop_margin_min", C.c_double),
        ("drop_log_count", C.c_int64), ("tuning_applied", C.c_int64),
        ("max_width_initial", C.c_int64),
        ("ilu1t_host", C.c_int64),
    ]


class FactorsHost(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("nblocks", C.c_int64), ("nblocks_initial", C.c_int64),
        ("perm", C.POINTER(C.c_int64)), ("starts", C.POINTER(C.c_int64)),
        ("starts_initial", C.POINTER(C.c_int64)), ("group_starts", C.POINTER(C.c_int64)),
        ("ngroups", C.c_int64),
        ("r_ptr", C.POINTER(C.c_int64)), ("r_idx", C.POINTER(C.c_int32)),
        ("c_ptr", C.POINTER(C.c_int64)), ("c_idx", C.POINTER(C.c_int32)),
        ("l_val", C.POINTER(C.c_double)), ("w_val", C.POINTER(C.c_double)),
        ("d_val", C.POINTER(C.c_double)),
        ("ndrop_log", C.c_int64), ("drop_block", C.POINTER(C.c_int64)),
        ("drop_index", C.POINTER(C.c_int64)), ("drop_norm", C.POINTER(C.c_double)),
    ]


EXPORTED = [
    "bilu_default_options", "bilu_create", "bilu_analyze", "bilu_factor", "bilu_apply",
    "bilu_spmv", "bilu_fgmres_solve", "bilu_get_stats", "bilu_export_factors",
    "bilu_free_factors", "bilu_destroy", "bilu_status_string", "bilu_last_error",
    "bilu_preprocess", "bilu_sync", "bilu_export_trace", "bilu_factor_batched", "bilu_mwm",
    "bilu_analyze_device", "bilu_refactor", "bilu_kept_residual", "bilu_apply_noalloc",
    "bilu_load_tuning", "bilu_tuning_entries", "bilu_refactor_frozen", "bilu_sqmr_solve",
]

_lib = None


def load(path: str = LIB_PATH):
    """Load libbilu.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_1908_10169_amd/build.py")
    lib = C.CDLL(path)
    vp = C.c_void_p
    lib.bilu_default_options.argtypes = [C.POINTER(Options)]
    lib.bilu_create.argtypes = [C.POINTER(vp), C.POINTER(Options), vp]
    lib.bilu_analyze.argtypes = [vp, C.c_int64, vp, vp, vp]
    lib.bilu_factor.argtypes = [vp, C.c_double]
    lib.bilu_factor_batched.argtypes = [C.POINTER(vp), C.c_int, C.POINTER(C.c_double)]
    lib.bilu_apply.argtypes = [vp, vp, vp]
    lib.bilu_apply_noalloc.argtypes = [vp, vp, vp]
    lib.bilu_spmv.argtypes = [vp, vp, vp]
    lib.bilu_fgmres_solve.argtypes = [vp, vp, vp, C.c_int, C.c_double, C.c_int,
                                      C.POINTER(SolveInfo)]
    lib.bilu_sqmr_solve.argtypes = [vp, vp, vp, C.c_double, C.c_int, C.POINTER(SolveInfo),
                                    C.POINTER(C.c_double)]
    lib.bilu_sqmr_solve.restype = C.c_int
    lib.bilu_get_stats.argtypes = [vp, C.POINTER(Stats)]
    lib.bilu_export_factors.argtypes = [vp, C.POINTER(FactorsHost)]
    lib.bilu_free_factors.argtypes = [C.POINTER(FactorsHost)]
    lib.bilu_destroy.argtypes = [vp]
    lib.bilu_destroy.restype = None
    lib.bilu_status_string.argtypes = [C.c_int]
    lib.bilu_status_string.restype = C.c_char_p
    lib.bilu_last_error.argtypes = [vp]
    lib.bilu_last_error.restype = C.c_char_p
    lib.bilu_sync.argtypes = [vp]
    lib.bilu_export_trace.argtypes = [vp, vp, C.c_int64, C.POINTER(C.c_int64),
                                      C.POINTER(C.c_double)]
    lib.bilu_export_trace.restype = C.c_int
    lib.bilu_mwm.argtypes = [C.c_int64, vp, vp, vp, vp, vp, vp]
    lib.bilu_analyze_device.argtypes = [vp, C.c_int64, vp, vp, vp]
    lib.bilu_refactor.argtypes = [vp, C.c_double, vp]
    lib.bilu_refactor_frozen.argtypes = [vp, vp]
    lib.bilu_kept_residual.argtypes = [vp, C.POINTER(C.c_double)]
    lib.bilu_load_tuning.argtypes = [C.c_char_p]
    lib.bilu_load_tuning.restype = C.c_int
    lib.bilu_tuning_entries.argtypes = []
    lib.bilu_tuning_entries.restype = C.c_int64
    lib.bilu_preprocess.argtypes = [C.POINTER(Options), C.c_int64, vp, vp, vp, C.c_double,
                                    vp, vp, C.POINTER(C.c_int64), vp, C.POINTER(C.c_int64)]
    for f in ("bilu_create", "bilu_analyze", "bilu_analyze_device", "bilu_refactor",
              "bilu_refactor_frozen", "bilu_factor",
              "bilu_factor_batched", "bilu_apply", "bilu_apply_noalloc",
              "bilu_spmv", "bilu_kept_residual",
              "bilu_fgmres_solve", "bilu_get_stats", "bilu_export_factors", "bilu_preprocess",
              "bilu_sync"):
        getattr(lib, f).restype = C.c_int
    _lib = lib
    return lib


class BiluError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{load().bilu_status_string(status).decode()}: {msg}")
        self.status = status


def default_options(**kw) -> Options:
    o = Options()
    load().bilu_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, int(v) if isinstance(v, bool) else v)
    return o


@dataclass
class Factors:
    perm: np.ndarray
    starts: np.ndarray
    starts_initial: np.ndarray
    group_starts: np.ndarray
    R: list
    L: list
    C: list
    W: list
    D: list
    drop_log: dict | None = None


def _check_tensor(t, name, dtype, numel=None):
    """Reject what would make a kernel read or write out of bounds: the
    library takes raw device pointers and cannot check them itself."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    if t.dtype != dtype:
        raise ValueError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name}: {t.numel()} elements, expected {numel}")
    if not t.is_cuda:
        raise ValueError(f"{name}: must be a device (cuda) tensor")
    return t.data_ptr()


def _check_vectors(n, *named):
    """Every (name, tensor) is a contiguous float64 device vector of n
    entries; outputs (the last one) share no memory with the inputs."""
    import torch
    out_name, out = named[-1]
    for name, t in named[:-1]:
        if isinstance(t, torch.Tensor) and isinstance(out, torch.Tensor):
            a0, a1 = t.data_ptr(), t.data_ptr() + t.element_size() * t.numel()
            b0, b1 = out.data_ptr(), out.data_ptr() + out.element_size() * out.numel()
            if a0 < b1 and b0 < a1:
                raise ValueError(f"{out_name} overlaps {name}")
    return [_check_tensor(t, name, torch.float64, n) for name, t in named]


def _stream_ptr(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return stream


def factor_batched(handles, taus):
    """Factor analyzed handles in one launch (bilu_factor_batched)."""
    lib = load()
    hs = (C.c_void_p * len(handles))(*[h._h.value for h in handles])
    ts = (C.c_double * len(handles))(*[float(t) for t in taus])
    st = lib.bilu_factor_batched(hs, len(handles), ts)
    if st not in (BILU_OK, BILU_WARN_PERTURBED):
        errs = "; ".join(lib.bilu_last_error(h._h).decode() for h in handles)
        raise BiluError(st, f"bilu_factor_batched: {errs}")
    return st


def load_tuning(path: str | None):
    """bilu_load_tuning: the process-wide table of tuned kernel settings
    (None or "" clears it); returns the number of entries."""
    lib = load()
    st = lib.bilu_load_tuning(path.encode() if path else None)
    if st != BILU_OK:
        raise BiluError(st, f"bilu_load_tuning({path!r})")
    return lib.bilu_tuning_entries()


def preprocess(a, tau: float, pre_perm=None, **kw):
    """Host-only structural preprocessing: (perm, group_starts, block_starts)."""
    lib = load()
    opts = default_options(**kw)
    pp = None
    if pre_perm is not None:
        pp = np.ascontiguousarray(pre_perm, dtype=np.int64)
        opts.pre_perm = pp.ctypes.data
    rp = np.ascontiguousarray(a.rowptr, dtype=np.int64)
    ci = np.ascontiguousarray(a.colind, dtype=np.int32)
    v = np.ascontiguousarray(a.val, dtype=np.float64)
    perm = np.empty(a.n, dtype=np.int64)
    gs = np.empty(a.n + 1, dtype=np.int64)
    bs = np.empty(a.n + 1, dtype=np.int64)
    ng, nb = C.c_int64(), C.c_int64()
    st = lib.bilu_preprocess(C.byref(opts), a.n, rp.ctypes.data, ci.ctypes.data, v.ctypes.data,
                             tau, perm.ctypes.data, gs.ctypes.data, C.byref(ng), bs.ctypes.data,
                             C.byref(nb))
    if st != BILU_OK:
        raise BiluError(st, "bilu_preprocess")
    return perm, gs[:ng.value + 1].copy(), bs[:nb.value + 1].copy()


def mwm(a):
    """Sec. 3.1 maximum weight matching on the host: (sigma, dl, dr) with
    D_l A D_r Pi of unit diagonal magnitudes, Pi[sigma(i), i] = 1."""
    lib = load()
    rp = np.ascontiguousarray(a.rowptr, dtype=np.int64)
    ci = np.ascontiguousarray(a.colind, dtype=np.int32)
    v = np.ascontiguousarray(a.val, dtype=np.float64)
    sigma = np.empty(a.n, dtype=np.int64)
    dl = np.empty(a.n)
    dr = np.empty(a.n)
    st = lib.bilu_mwm(C.c_int64(a.n), rp.ctypes.data, ci.ctypes.data, v.ctypes.data,
                      sigma.ctypes.data, dl.ctypes.data, dr.ctypes.data)
    if st != BILU_OK:
        raise BiluError(st, "bilu_mwm")
    return sigma, dl, dr


class Bilu:
    """One BILU preconditioner handle (one matrix)."""

    def __init__(self, options: Options | None = None, stream=None, **kw):
        self._lib = load()
        self._h = C.c_void_p()
        self.n = None  # set by analyze; before it the library reports BILU_ERR_STATE
        opts = options if options is not None else default_options(**kw)
        self._pre = None
        if kw.get("pre_perm") is not None:
            raise ValueError("pass pre_perm to analyze()")
        self._opts = opts
        st = self._lib.bilu_create(C.byref(self._h), C.byref(opts), C.c_void_p(_stream_ptr(stream)))
        if st != BILU_OK:
            raise BiluError(st, "bilu_create")

    def _check(self, st, what, ok=(BILU_OK,)):
        if st not in ok:
            raise BiluError(st, f"{what}: {self._lib.bilu_last_error(self._h).decode()}")
        return st

    def close(self):
        if self._h:
            self._lib.bilu_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ API
    def analyze(self, a, pre_perm=None):
        rp = np.ascontiguousarray(a.rowptr, dtype=np.int64)
        ci = np.ascontiguousarray(a.colind, dtype=np.int32)
        v = np.ascontiguousarray(a.val, dtype=np.float64)
        if pre_perm is not None:
            self._pre = np.ascontiguousarray(pre_perm, dtype=np.int64)
            self._opts.pre_perm = self._pre.ctypes.data
        else:
            self._opts.pre_perm = None
        # options are copied at create: rebuild the handle with the permutation
        self.close()
        st = self._lib.bilu_create(C.byref(self._h), C.byref(self._opts),
                                   C.c_void_p(_stream_ptr(None)))
        if st != BILU_OK:
            raise BiluError(st, "bilu_create")
        self.n = a.n
        return self._check(self._lib.bilu_analyze(self._h, a.n, rp.ctypes.data, ci.ctypes.data,
                                                  v.ctypes.data), "bilu_analyze")

    def analyze_device(self, n, rowptr, colind, val, pre_perm=None):
        """bilu_analyze_device: rowptr (int64, n+1), colind (int32) and val
        (float64) are device tensors."""
        if pre_perm is not None:
            self._pre = np.ascontiguousarray(pre_perm, dtype=np.int64)
            self._opts.pre_perm = self._pre.ctypes.data
        else:
            self._opts.pre_perm = None
        self.close()
        st = self._lib.bilu_create(C.byref(self._h), C.byref(self._opts),
                                   C.c_void_p(_stream_ptr(None)))
        if st != BILU_OK:
            raise BiluError(st, "bilu_create")
        import torch
        _check_tensor(rowptr, "rowptr", torch.int64, n + 1)
        _check_tensor(colind, "colind", torch.int32)
        _check_tensor(val, "val", torch.float64, colind.numel())
        nnz = int(rowptr[-1].item())
        if nnz != colind.numel():
            raise ValueError(f"rowptr[n] = {nnz} but colind and val hold {colind.numel()} entries")
        self.n = n
        return self._check(self._lib.bilu_analyze_device(self._h, n, rowptr.data_ptr(),
                                                         colind.data_ptr(), val.data_ptr()),
                           "bilu_analyze_device")

    def factor(self, tau: float):
        return self._check(self._lib.bilu_factor(self._h, tau), "bilu_factor",
                           ok=(BILU_OK, BILU_WARN_PERTURBED))

    def refactor(self, tau: float, val):
        """bilu_refactor: val is a float64 device tensor of nnz values in the
        analyzed matrix's entry order."""
        import torch
        _check_tensor(val, "val", torch.float64, self.stats()["nnz_a"])
        return self._check(self._lib.bilu_refactor(self._h, tau, val.data_ptr()), "bilu_refactor",
                           ok=(BILU_OK, BILU_WARN_PERTURBED))

    def refactor_frozen(self, val):
        """bilu_refactor_frozen: val as for refactor; the last factor's
        blocks and patterns stay, its values are recomputed."""
        import torch
        _check_tensor(val, "val", torch.float64, self.stats()["nnz_a"])
        return self._check(self._lib.bilu_refactor_frozen(self._h, val.data_ptr()),
                           "bilu_refactor_frozen", ok=(BILU_OK, BILU_WARN_PERTURBED))

    def apply(self, x, y):
        """y = M^{-1} x; x, y: torch float64 CUDA tensors of length n."""
        px, py = _check_vectors(self.n, ("x", x), ("y", y))
        return self._check(self._lib.bilu_apply(self._h, px, py), "bilu_apply")

    def kept_residual(self) -> float:
        """||(L S U - A)_Omega||_F / ||A||_F of the last factor (bilu_kept_residual)."""
        r = C.c_double()
        self._check(self._lib.bilu_kept_residual(self._h, C.byref(r)), "bilu_kept_residual")
        return r.value

    def apply_noalloc(self, x, y):
        """bilu_apply_noalloc: y = M^{-1} x with the library's fixed device
        array as workspace (no allocation; n <= 2^21)."""
        px, py = _check_vectors(self.n, ("x", x), ("y", y))
        return self._check(self._lib.bilu_apply_noalloc(self._h, px, py), "bilu_apply_noalloc")

    def trace(self):
        """Per-block factor trace (collect_timing=2): (records x 24 uint64, ticks/s)."""
        m, tps = C.c_int64(), C.c_double()
        self._check(self._lib.bilu_export_trace(self._h, None, 0, C.byref(m), C.byref(tps)),
                    "bilu_export_trace")
        out = np.zeros(m.value * 24, dtype=np.uint64)
        self._check(self._lib.bilu_export_trace(self._h, out.ctypes.data, out.size, C.byref(m),
                                                C.byref(tps)), "bilu_export_trace")
        return out.reshape(m.value, 24), tps.value

    def sync(self):
        """Wait for the stream; raise if an asynchronous call reported an error."""
        return self._check(self._lib.bilu_sync(self._h), "bilu_sync")

    def spmv(self, x, y):
        px, py = _check_vectors(self.n, ("x", x), ("y", y))
        return self._check(self._lib.bilu_spmv(self._h, px, py), "bilu_spmv")

    def fgmres(self, b, x, restart=30, rtol=1e-8, maxit=2000):
        pb, px = _check_vectors(self.n, ("b", b), ("x", x))
        info = SolveInfo()
        st = self._lib.bilu_fgmres_solve(self._h, pb, px, restart, rtol, maxit, C.byref(info))
        self._check(st, "bilu_fgmres_solve", ok=(BILU_OK, BILU_WARN_NOT_CONVERGED))
        return dict(iterations=info.iterations, restarts=info.restarts,
                    rel_residual=info.rel_residual, seconds=info.seconds,
                    converged=bool(info.converged))

    def sqmr(self, b, x, tol=1e-6, maxit=2000):
        """Simplified QMR for symmetric A (bilu_sqmr_solve); stops on the
        infinity-norm backward error.  Returns iterations (steps),
        rel_residual, eta (backward error), seconds, converged."""
        pb, px = _check_vectors(self.n, ("b", b), ("x", x))
        info = SolveInfo()
        eta = C.c_double(0.0)
        st = self._lib.bilu_sqmr_solve(self._h, pb, px, tol, maxit, C.byref(info), C.byref(eta))
        self._check(st, "bilu_sqmr_solve", ok=(BILU_OK, BILU_WARN_NOT_CONVERGED))
        return dict(iterations=info.iterations, rel_residual=info.rel_residual, eta=eta.value,
                    seconds=info.seconds, converged=bool(info.converged))

    def stats(self) -> dict:
        s = Stats()
        self._check(self._lib.bilu_get_stats(self._h, C.byref(s)), "bilu_get_stats")
        out = {f: getattr(s, f) for f, _ in Stats._fields_}
        out["t_phase"] = list(s.t_phase)
        return out

    def export(self) -> Factors:
        fh = FactorsHost()
        self._check(self._lib.bilu_export_factors(self._h, C.byref(fh)), "bilu_export_factors")
        try:
            n, nb = fh.n, fh.nblocks
            arr = lambda p, m, dt: np.ctypeslib.as_array(p, shape=(m,)).astype(dt, copy=True)  # noqa
            starts = arr(fh.starts, nb + 1, np.int64)
            rp = arr(fh.r_ptr, nb + 1, np.int64)
            cp = arr(fh.c_ptr, nb + 1, np.int64)
            q = np.diff(starts)
            tr, tc = int(rp[-1]), int(cp[-1])
            ridx = arr(fh.r_idx, max(tr, 1), np.int64)[:tr]
            cidx = arr(fh.c_idx, max(tc, 1), np.int64)[:tc]
            lv = arr(fh.l_val, max(int((np.diff(rp) * q).sum()), 1), np.float64)
            wv = arr(fh.w_val, max(int((np.diff(cp) * q).sum()), 1), np.float64)
            dv = arr(fh.d_val, max(int((q * q).sum()), 1), np.float64)
            f = Factors(arr(fh.perm, n, np.int64), starts,
                        arr(fh.starts_initial, fh.nblocks_initial + 1, np.int64),
                        arr(fh.group_starts, fh.ngroups + 1, np.int64), [], [], [], [], [])
            if fh.ndrop_log > 0:
                m = fh.ndrop_log
                f.drop_log = dict(block=arr(fh.drop_block, m, np.int64),
                                  index=arr(fh.drop_index, m, np.int64),
                                  norm=arr(fh.drop_norm, m, np.float64))
            lo = wo = do = 0
            for k in range(nb):
                qk = int(q[k])
                mr, mc = int(rp[k + 1] - rp[k]), int(cp[k + 1] - cp[k])
                f.R.append(ridx[rp[k]:rp[k + 1]])
                f.C.append(cidx[cp[k]:cp[k + 1]])
                f.L.append(lv[lo:lo + mr * qk].reshape(mr, qk)); lo += mr * qk
                f.W.append(wv[wo:wo + mc * qk].reshape(mc, qk).T); wo += mc * qk
                f.D.append(dv[do:do + qk * qk].reshape(qk, qk)); do += qk * qk
            return f
        finally:
            self._lib.bilu_free_factors(C.byref(fh))
