"""ctypes wrapper of the FP64 CPU oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

from . import build as _build

_lib = None

_I64P = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_I32P = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_F64P = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


class _Opts(C.Structure):
    _fields_ = [
        ("use_cosine", C.c_int), ("use_ilu1t", C.c_int), ("use_aggregation", C.c_int),
        ("max_block", C.c_int), ("tau", C.c_double), ("cos_eps", C.c_double),
        ("pert_tau", C.c_double), ("pert_rho", C.c_double), ("pivot_eps", C.c_double),
        ("beta_one", C.c_int), ("drop_norm", C.c_int), ("sym_perturb", C.c_int),
    ]


class _Info(C.Structure):
    _fields_ = [("iterations", C.c_int64), ("restarts", C.c_int64),
                ("rel_residual", C.c_double), ("converged", C.c_int)]


def load():
    global _lib
    if _lib is not None:
        return _lib
    path = _build.LIB
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
        _build.build()
    lib = C.CDLL(path)
    vp = C.c_void_p
    lib.orc_create.restype = vp
    lib.orc_destroy.argtypes = [vp]
    lib.orc_default_options.argtypes = [C.POINTER(_Opts)]
    lib.orc_run.argtypes = [vp, C.c_int64, _I64P, _I32P, _F64P, vp, C.POINTER(_Opts)]
    lib.orc_run.restype = C.c_int
    lib.orc_run_units.argtypes = [vp, C.c_int64, _I64P, _I32P, _F64P, vp, C.c_int64, vp, vp,
                                  C.POINTER(_Opts)]
    lib.orc_run_units.restype = C.c_int
    lib.orc_run_partition.argtypes = [vp, C.c_int64, _I64P, _I32P, _F64P, vp, C.c_int64,
                                      _I64P, C.POINTER(_Opts)]
    lib.orc_run_partition.restype = C.c_int
    lib.orc_cosine.argtypes = [C.c_int64, _I64P, _I32P, C.c_double, C.c_int, _I64P, _I64P,
                               C.POINTER(C.c_int64)]
    lib.orc_cosine.restype = C.c_int64
    lib.orc_ilu1t.argtypes = [C.c_int64, _I64P, _I32P, _F64P, C.c_int64, _I64P, C.c_double,
                              C.c_int, _I64P]
    lib.orc_ilu1t.restype = C.c_int64
    lib.orc_ilu1t_sets.argtypes = [C.c_int64, _I64P, _I32P, _F64P, C.c_int64, C.c_double,
                                   _I64P, C.POINTER(C.c_int64), _I64P, C.POINTER(C.c_int64)]
    lib.orc_ilu1t_sets.restype = C.c_int64
    lib.orc_perturb_invert.argtypes = [C.c_int, _F64P, C.c_double, C.POINTER(_Opts), _F64P,
                                       _F64P]
    lib.orc_perturb_invert.restype = C.c_int
    for name in ("orc_n", "orc_nblocks", "orc_nblocks_initial"):
        getattr(lib, name).argtypes = [vp]
        getattr(lib, name).restype = C.c_int64
    lib.orc_get_perm.argtypes = [vp, _I64P]
    lib.orc_get_starts.argtypes = [vp, _I64P]
    lib.orc_get_starts_initial.argtypes = [vp, _I64P]
    lib.orc_get_group_starts.argtypes = [vp, vp, C.POINTER(C.c_int64)]
    lib.orc_get_counts.argtypes = [vp, _I64P, _I64P]
    lib.orc_get_factors.argtypes = [vp, _I64P, _F64P, _I64P, _F64P, _F64P]
    lib.orc_get_stats.argtypes = [vp, _I64P]
    lib.orc_get_droplog.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.orc_get_droplog.restype = C.c_int64
    lib.orc_get_mergelog.argtypes = [vp, vp]
    lib.orc_get_mergelog.restype = C.c_int64
    lib.orc_apply.argtypes = [vp, _F64P, _F64P]
    lib.orc_fgmres.argtypes = [vp, _F64P, _F64P, C.c_int, C.c_double, C.c_int, C.POINTER(_Info)]
    lib.orc_fgmres_hist.argtypes = [vp, _F64P, _F64P, C.c_int, C.c_double, C.c_int,
                                    C.POINTER(_Info), _F64P]
    lib.orc_fgmres_plain.argtypes = [C.c_int64, _I64P, _I32P, _F64P, _F64P, _F64P, C.c_int,
                                     C.c_double, C.c_int, C.POINTER(_Info), _F64P]
    lib.orc_sqmr.argtypes = [vp, _F64P, _F64P, C.c_double, C.c_int, C.POINTER(_Info),
                             C.POINTER(C.c_double), _F64P]
    lib.orc_sqmr_plain.argtypes = [C.c_int64, _I64P, _I32P, _F64P, _F64P, _F64P, C.c_double,
                                   C.c_int, C.POINTER(_Info), C.POINTER(C.c_double), _F64P]
    lib.orc_kept_residual.argtypes = [vp]
    lib.orc_kept_residual.restype = C.c_double
    lib.orc_final_residual.argtypes = [vp]
    lib.orc_final_residual.restype = C.c_double
    lib.orc_refactor_frozen.argtypes = [vp, _F64P]
    lib.orc_refactor_frozen.restype = C.c_int
    lib.orc_lsu_matvec.argtypes = [vp, _F64P, _F64P]
    lib.orc_get_times.argtypes = [vp, _F64P]
    lib.orc_plant.argtypes = [vp, C.c_int, C.c_int64, C.c_int64, C.c_double]
    lib.orc_plant.restype = C.c_int
    _lib = lib
    return lib


@dataclass
class OracleOptions:
    use_cosine: bool = True
    use_ilu1t: bool = True
    use_aggregation: bool = True
    max_block: int = 128
    tau: float = 1e-2
    cos_eps: float = 0.8
    pert_tau: float = 1e-2
    pert_rho: float = 1e-1
    pivot_eps: float = 1e-12
    beta_one: bool = False
    drop_norm: int = 0
    sym_perturb: bool = False

    def c(self) -> _Opts:
        o = _Opts()
        for f, _ in _Opts._fields_:
            v = getattr(self, f)
            setattr(o, f, int(v) if isinstance(v, bool) else v)
        return o


@dataclass
class Factors:
    perm: np.ndarray
    starts: np.ndarray
    starts_initial: np.ndarray
    R: list = field(default_factory=list)
    L: list = field(default_factory=list)
    C: list = field(default_factory=list)
    W: list = field(default_factory=list)
    D: list = field(default_factory=list)


class Oracle:
    """One oracle run: preprocessing + sequential block Crout sweep."""

    def __init__(self):
        self._lib = load()
        self._h = self._lib.orc_create()

    def __del__(self):
        try:
            self._lib.orc_destroy(self._h)
        except Exception:
            pass

    def run(self, a, opts: OracleOptions | None = None, pre_perm=None, unit_starts=None,
            partner=None) -> int:
        """The full pipeline; unit_starts (in the pre-permuted numbering)
        gives the units of the symmetric variant that groups never split;
        partner (final numbering) the 2x2 pivots when the units are
        coarser than them."""
        opts = opts or OracleOptions()
        self.n = a.n
        self.a = a
        pp = None if pre_perm is None else np.ascontiguousarray(pre_perm, dtype=np.int64)
        self._pp = pp
        us = None if unit_starts is None else np.ascontiguousarray(unit_starts, dtype=np.int64)
        pt = None if partner is None else np.ascontiguousarray(partner, dtype=np.int64)
        rc = self._lib.orc_run_units(self._h, a.n, a.rowptr, a.colind, a.val,
                                     pp.ctypes.data if pp is not None else None,
                                     0 if us is None else len(us) - 1,
                                     us.ctypes.data if us is not None else None,
                                     pt.ctypes.data if pt is not None else None,
                                     C.byref(opts.c()))
        return rc

    def run_partition(self, a, starts, opts: OracleOptions | None = None, perm=None) -> int:
        opts = opts or OracleOptions()
        self.n = a.n
        self.a = a
        starts = np.ascontiguousarray(starts, dtype=np.int64)
        pp = None if perm is None else np.ascontiguousarray(perm, dtype=np.int64)
        self._pp = pp
        return self._lib.orc_run_partition(self._h, a.n, a.rowptr, a.colind, a.val,
                                           pp.ctypes.data if pp is not None else None,
                                           len(starts) - 1, starts, C.byref(opts.c()))

    # ---------------- results
    def perm(self):
        p = np.empty(self.n, dtype=np.int64)
        self._lib.orc_get_perm(self._h, p)
        return p

    def starts(self):
        nb = self._lib.orc_nblocks(self._h)
        s = np.empty(nb + 1, dtype=np.int64)
        self._lib.orc_get_starts(self._h, s)
        return s

    def starts_initial(self):
        nb = self._lib.orc_nblocks_initial(self._h)
        s = np.empty(nb + 1, dtype=np.int64)
        self._lib.orc_get_starts_initial(self._h, s)
        return s

    def group_starts(self):
        ng = C.c_int64()
        self._lib.orc_get_group_starts(self._h, None, C.byref(ng))
        s = np.empty(ng.value + 1, dtype=np.int64)
        self._lib.orc_get_group_starts(self._h, s.ctypes.data, C.byref(ng))
        return s

    def stats(self) -> dict:
        s = np.zeros(16, dtype=np.int64)
        self._lib.orc_get_stats(self._h, s)
        keys = ["nblocks_initial", "nblocks", "merges", "perturbed_blocks", "nnz_L", "nnz_W",
                "nnz_D", "max_width", "ngroups", "ignored", "singular", "nnz_A"]
        return {k: int(s[i]) for i, k in enumerate(keys)}

    def factors(self) -> Factors:
        st = self.starts()
        nb = len(st) - 1
        nR = np.empty(nb, dtype=np.int64)
        nC = np.empty(nb, dtype=np.int64)
        self._lib.orc_get_counts(self._h, nR, nC)
        q = np.diff(st)
        R = np.empty(int(nR.sum()), dtype=np.int64)
        Cc = np.empty(int(nC.sum()), dtype=np.int64)
        L = np.empty(int((nR * q).sum()), dtype=np.float64)
        W = np.empty(int((nC * q).sum()), dtype=np.float64)
        D = np.empty(int((q * q).sum()), dtype=np.float64)
        self._lib.orc_get_factors(self._h, R, L, Cc, W, D)
        f = Factors(self.perm(), st, self.starts_initial())
        r0 = c0 = l0 = w0 = d0 = 0
        for k in range(nb):
            qk, mr, mc = int(q[k]), int(nR[k]), int(nC[k])
            f.R.append(R[r0:r0 + mr]); r0 += mr
            f.C.append(Cc[c0:c0 + mc]); c0 += mc
            f.L.append(L[l0:l0 + mr * qk].reshape(mr, qk)); l0 += mr * qk
            # stored column-major q x |C|: element (t, j) at j*q + t
            f.W.append(W[w0:w0 + mc * qk].reshape(mc, qk).T); w0 += mc * qk
            f.D.append(D[d0:d0 + qk * qk].reshape(qk, qk)); d0 += qk * qk
        return f

    def droplog(self):
        m = self._lib.orc_get_droplog(self._h, None, None, None, None, None)
        blk = np.empty(m, dtype=np.int64)
        idx = np.empty(m, dtype=np.int64)
        kind = np.empty(m, dtype=np.int32)
        nrm = np.empty(m, dtype=np.float64)
        kept = np.empty(m, dtype=np.int32)
        self._lib.orc_get_droplog(self._h, blk.ctypes.data, idx.ctypes.data, kind.ctypes.data,
                                  nrm.ctypes.data, kept.ctypes.data)
        return dict(block=blk, index=idx, kind=kind, norm=nrm, kept=kept.astype(bool))

    def mergelog(self):
        m = self._lib.orc_get_mergelog(self._h, None)
        rec = np.empty(6 * m, dtype=np.int64)
        self._lib.orc_get_mergelog(self._h, rec.ctypes.data)
        return rec.reshape(m, 6)

    def apply(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.empty_like(x)
        self._lib.orc_apply(self._h, x, y)
        return y

    def lsu_matvec(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.empty_like(x)
        self._lib.orc_lsu_matvec(self._h, x, y)
        return y

    def fgmres(self, b, x0=None, restart=30, rtol=1e-8, maxit=2000, history=False):
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
        info = _Info()
        hist = np.zeros(max(maxit, 1))
        self._lib.orc_fgmres_hist(self._h, b, x, restart, rtol, maxit, C.byref(info), hist)
        out = dict(iterations=info.iterations, restarts=info.restarts,
                   rel_residual=info.rel_residual, converged=bool(info.converged))
        if history:
            return x, out, hist[:info.iterations].copy()
        return x, out

    def sqmr(self, b, x0=None, tol=1e-6, maxit=2000, history=False):
        """Simplified QMR with M from the run (A and M symmetric); stops on
        the infinity-norm backward error.  Returns x and a dict with
        iterations, rel_residual (true 2-norm), eta (true backward error),
        converged; with history also the quasi-residual norms tau_k."""
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
        info = _Info()
        eta = C.c_double(0.0)
        hist = np.zeros(max(maxit, 1))
        self._lib.orc_sqmr(self._h, b, x, tol, maxit, C.byref(info), C.byref(eta), hist)
        out = dict(iterations=info.iterations, rel_residual=info.rel_residual,
                   eta=eta.value, converged=bool(info.converged))
        if history:
            return x, out, hist[:info.iterations].copy()
        return x, out

    def kept_residual(self) -> float:
        return self._lib.orc_kept_residual(self._h)

    def final_residual(self) -> float:
        """||(L S U - A)_Omega|| / ||A|| over the final blocks' positions."""
        return self._lib.orc_final_residual(self._h)

    def refactor_frozen(self, val) -> int:
        """New values of A (entry order of the matrix last run, same pattern);
        the final blocks and patterns stay, L, W, D are recomputed."""
        v = np.ascontiguousarray(val, dtype=np.float64)
        return self._lib.orc_refactor_frozen(self._h, v)

    def plant(self, which: str, block: int, pos: int, delta: float) -> None:
        """Test hook: add delta to one stored value of L_K ("L") or W_K ("W")."""
        if self._lib.orc_plant(self._h, {"L": 0, "W": 1}[which], block, pos, delta) != 0:
            raise IndexError((which, block, pos))

    def times(self):
        t = np.zeros(3)
        self._lib.orc_get_times(self._h, t)
        return dict(analyze=t[0], ilu1t=t[1], factor=t[2])


def cosine_groups(a, cos_eps=0.8, max_block=128):
    lib = load()
    perm = np.empty(a.n, dtype=np.int64)
    gs = np.empty(a.n + 1, dtype=np.int64)
    nig = C.c_int64()
    ng = lib.orc_cosine(a.n, a.rowptr, a.colind, cos_eps, max_block, perm, gs, C.byref(nig))
    return perm, gs[:ng + 1].copy(), nig.value


def ilu1t_blocks(a, unit_starts, tau, max_block=128):
    lib = load()
    us = np.ascontiguousarray(unit_starts, dtype=np.int64)
    bs = np.empty(a.n + 1, dtype=np.int64)
    nb = lib.orc_ilu1t(a.n, a.rowptr, a.colind, a.val, len(us) - 1, us, tau, max_block, bs)
    return bs[:nb + 1].copy()


def ilu1t_sets(a, k, tau):
    lib = load()
    I = np.empty(a.n, dtype=np.int64)
    J = np.empty(a.n, dtype=np.int64)
    nI, nJ = C.c_int64(), C.c_int64()
    lib.orc_ilu1t_sets(a.n, a.rowptr, a.colind, a.val, k, tau, I, C.byref(nI), J, C.byref(nJ))
    return I[:nI.value].copy(), J[:nJ.value].copy()


def perturb_invert(s, alpha, opts: OracleOptions | None = None):
    lib = load()
    opts = opts or OracleOptions()
    s = np.ascontiguousarray(s, dtype=np.float64)
    q = s.shape[0]
    su = np.empty_like(s)
    di = np.empty_like(s)
    r = lib.orc_perturb_invert(q, s.ravel(), alpha, C.byref(opts.c()), su.ravel(), di.ravel())
    return r, su, di


def fgmres_plain(a, b, restart=30, rtol=1e-8, maxit=2000):
    lib = load()
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    info = _Info()
    hist = np.zeros(maxit + 1)
    lib.orc_fgmres_plain(a.n, a.rowptr, a.colind, a.val, b, x, restart, rtol, maxit,
                         C.byref(info), hist)
    return x, dict(iterations=info.iterations, restarts=info.restarts,
                   rel_residual=info.rel_residual, converged=bool(info.converged)), \
        hist[:info.iterations]


def sqmr_plain(a, b, tol=1e-6, maxit=2000, x0=None):
    """Simplified QMR with M = I on a CSR matrix; returns x, info, tau_k."""
    lib = load()
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    info = _Info()
    eta = C.c_double(0.0)
    hist = np.zeros(max(maxit, 1))
    lib.orc_sqmr_plain(a.n, a.rowptr, a.colind, a.val, b, x, tol, maxit, C.byref(info),
                       C.byref(eta), hist)
    return x, dict(iterations=info.iterations, rel_residual=info.rel_residual,
                   eta=eta.value, converged=bool(info.converged)), hist[:info.iterations].copy()
