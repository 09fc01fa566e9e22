"""Simplified QMR on the GPU (bilu_sqmr_solve) against the oracle's SQMR,
on symmetric elasticity-like operators: positive definite (shift 0.1) and
indefinite (negative shifts put eigenvalues below zero), unperturbed so the
matrix and the block factorization are symmetric.

Parity: after a fixed number of steps (tol = 0) the iterates agree to
rounding; with a tolerance both sides stop at the same step, meet the
backward-error bar with the true residual and agree on it.
"""
import ctypes as C
import sys

import numpy as np
import pytest

from paper_1908_10169_amd import matgen as mg

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _system(side, shift):
    a = mg.grid3d_elasticity(side, 3, seed=2, pert=0.0, shift=shift)
    perm = mg.node_perm_to_scalar(
        mg.grid_nd_node_order((side,) * 3, dissect_separators=False), 3)
    return a, perm


def _pair(a, perm, tau, agg=True):
    from oracle import Oracle, OracleOptions
    from paper_1908_10169_amd import bilu
    o = Oracle()
    assert o.run(a, OracleOptions(tau=tau, use_aggregation=agg), pre_perm=perm) == 0
    h = bilu.Bilu(ordering=bilu.ORDER_NATURAL, use_aggregation=agg)
    h.analyze(a, pre_perm=perm)
    h.factor(tau)
    return o, h


def _eta(a, b, x):
    r = b - a.matvec(x)
    an = max(np.abs(a.val[a.rowptr[i]:a.rowptr[i + 1]]).sum() for i in range(a.n))
    return np.abs(r).max() / (an * np.abs(x).max() + np.abs(b).max())


CASES = [
    # (side, shift, tau, aggregation): M well conditioned, so a relative
    # change of 1e-13 in M^{-1} moves the fifth iterate by 1e-11 or less
    (10, 0.1, 1e-2, True),
    (10, -0.05, 1e-2, True),
    (10, -0.1, 3e-3, True),
    (10, -0.3, 3e-3, False),
    (16, 0.1, 1e-2, True),
]
# Indefinite cases whose factor is close to singular: ||M^{-1}|| is large,
# and a relative change of 1e-13 in M^{-1} moves the fifth iterate by 2e-7
# (first) and 5e-9 (second, 140 to 190 steps), so the GPU's rounding
# (another summation order in the products) moves the stopping step; both
# sides must still converge to the bar, in about as many steps.
SENSITIVE = [(10, -0.1, 1e-2, True), (12, -0.2, 1e-2, False)]


def _ids(cases):
    return [f"el3d{c[0]}-shift{c[1]}-tau{c[2]}-{'agg' if c[3] else 'plain'}" for c in cases]


IDS = _ids(CASES)


@pytest.mark.parametrize("side,shift,tau,agg", CASES, ids=IDS)
def test_sqmr_fixed_steps_iterates(side, shift, tau, agg):
    """tol = 0, five steps: the GPU iterate is the oracle's to rounding."""
    torch = _torch()
    a, perm = _system(side, shift)
    say(f"[sqmr-steps] side={side} shift={shift} tau={tau} agg={agg}")
    o, h = _pair(a, perm, tau, agg)
    b = a.matvec(np.ones(a.n))
    x_o, info_o = o.sqmr(b, tol=0.0, maxit=5)
    bd = torch.from_numpy(b).cuda()
    xd = torch.zeros_like(bd)
    info = h.sqmr(bd, xd, tol=0.0, maxit=5)
    x = xd.cpu().numpy()
    assert info["iterations"] == info_o["iterations"] == 5
    assert not info["converged"]
    assert np.linalg.norm(x - x_o) <= 1e-9 * np.linalg.norm(x_o)
    assert abs(info["eta"] - info_o["eta"]) <= 1e-7 * info_o["eta"]
    h.close()


@pytest.mark.parametrize("tol", [1e-6, 1e-10])
@pytest.mark.parametrize("side,shift,tau,agg", CASES + SENSITIVE, ids=_ids(CASES + SENSITIVE))
def test_sqmr_converges_like_the_oracle(side, shift, tau, agg, tol):
    torch = _torch()
    a, perm = _system(side, shift)
    say(f"[sqmr] side={side} shift={shift} tau={tau} agg={agg} tol={tol}")
    o, h = _pair(a, perm, tau, agg)
    b = a.matvec(np.linspace(-1.0, 2.0, a.n))
    _, info_o = o.sqmr(b, tol=tol, maxit=1000)
    assert info_o["converged"]
    bd = torch.from_numpy(b).cuda()
    xd = torch.zeros_like(bd)
    info = h.sqmr(bd, xd, tol=tol, maxit=1000)
    x = xd.cpu().numpy()
    assert info["converged"]
    if (side, shift, tau, agg) in SENSITIVE:
        # 140 to 190 steps on the long case; measured 187 against 177
        it_o = info_o["iterations"]
        assert abs(info["iterations"] - it_o) <= max(2, 0.1 * it_o)
    else:
        assert info["iterations"] == info_o["iterations"]
    # the residual of a converged x is formed with cancellation: its
    # rounding error, relative to ||A|| ||x||, is a few dozen ulps
    eta = _eta(a, b, x)
    assert eta <= tol and info["eta"] <= tol
    assert abs(eta - info["eta"]) <= 1e-6 * eta + 1e-14
    res = np.linalg.norm(b - a.matvec(x)) / np.linalg.norm(b)
    assert abs(res - info["rel_residual"]) <= 1e-6 * res + 1e-13
    assert h.stats()["apply_faults"] == 0
    h.close()


def test_sqmr_maxit_and_exact_start():
    """maxit = 1 stops unconverged with the oracle's backward error; an
    exact initial guess takes no step."""
    torch = _torch()
    from paper_1908_10169_amd import bilu
    a, perm = _system(10, -0.1)
    say("[sqmr-maxit] side=10 shift=-0.1")
    o, h = _pair(a, perm, 1e-2)
    b = a.matvec(np.ones(a.n))
    _, info_o = o.sqmr(b, tol=1e-8, maxit=1)
    bd = torch.from_numpy(b).cuda()
    xd = torch.zeros_like(bd)
    info = bilu.SolveInfo()
    eta = C.c_double(0.0)
    st = bilu.load().bilu_sqmr_solve(h._h, bd.data_ptr(), xd.data_ptr(), 1e-8, 1,
                                     C.byref(info), C.byref(eta))
    assert st == bilu.BILU_WARN_NOT_CONVERGED
    assert info.iterations == 1 and info.restarts == 0 and not info.converged
    assert not info_o["converged"] and info_o["iterations"] == 1
    assert abs(eta.value - info_o["eta"]) <= 1e-8 * info_o["eta"]
    xd = torch.ones_like(bd)
    out = h.sqmr(bd, xd, tol=1e-12, maxit=10)
    assert out["converged"] and out["iterations"] == 0
    assert torch.equal(xd, torch.ones_like(bd))
    h.close()


def test_sqmr_below_rounding_runs_to_maxit():
    """A tolerance below the rounding floor: the updated residual passes it
    while the true one cannot, so the solver confirms, resumes the stopped
    step and goes on until maxit."""
    torch = _torch()
    a, perm = _system(8, 0.1)
    say("[sqmr-floor] side=8 tol=1e-17")
    o, h = _pair(a, perm, 1e-2)
    b = a.matvec(np.ones(a.n))
    _, info_o = o.sqmr(b, tol=1e-17, maxit=60)
    bd = torch.from_numpy(b).cuda()
    xd = torch.zeros_like(bd)
    info = h.sqmr(bd, xd, tol=1e-17, maxit=60)
    assert not info_o["converged"] and info_o["iterations"] == 60
    assert not info["converged"] and info["iterations"] == 60
    assert info["eta"] <= 1e-14 and info_o["eta"] <= 1e-14
    h.close()


def test_sqmr_refuses_the_nonsymmetric_matching():
    torch = _torch()
    from paper_1908_10169_amd import bilu
    a, perm = _system(6, 0.1)
    say("[sqmr-mwm] side=6")
    h = bilu.Bilu(ordering=bilu.ORDER_NATURAL, use_mwm=1)
    h.analyze(a, pre_perm=perm)
    h.factor(1e-2)
    bd = torch.from_numpy(a.matvec(np.ones(a.n))).cuda()
    xd = torch.zeros_like(bd)
    st = bilu.load().bilu_sqmr_solve(h._h, bd.data_ptr(), xd.data_ptr(), 1e-6, 10, None, None)
    assert st == bilu.BILU_ERR_INVALID
    h.close()


# ---------------------------------------------------------------------------
# The symmetric matching (use_mwm = 2) on saddle-point matrices whose
# constraint rows carry no diagonal and come before their unknowns.
# ---------------------------------------------------------------------------
def _kkt_pair(side, tau, agg):
    from oracle import Oracle, OracleOptions, symmetric_units
    from paper_1908_10169_amd import bilu
    a, order, m = mg.kkt_elasticity(side)
    sigma, dl, dr = bilu.mwm(a)
    d, uorder, us = symmetric_units(a, sigma, dl, dr, pre=order)
    rows = np.repeat(np.arange(a.n), np.diff(a.rowptr))
    ah = mg.Csr(a.n, a.rowptr, a.colind, (d[rows] * a.val) * d[a.colind])
    o = Oracle()
    assert o.run(ah, OracleOptions(tau=tau, use_aggregation=agg, sym_perturb=True),
                 pre_perm=uorder,
                 unit_starts=us) == 0
    h = bilu.Bilu(ordering=bilu.ORDER_NATURAL, use_aggregation=agg, use_mwm=2)
    h.analyze(a, pre_perm=order)
    h.factor(tau)
    return a, order, d, o, h


@pytest.mark.parametrize("side,tau,agg", [(5, 1e-2, False), (6, 1e-2, True), (6, 1e-3, True)])
def test_symmetric_matching_factor_parity(side, tau, agg):
    """The library's factor of D A D with the 2x2 pivots kept whole equals
    the oracle's (same numbering, blocks and patterns; values to 1e-10)."""
    _torch()
    say(f"[symmwm] kkt side={side} tau={tau} agg={agg}")
    a, order, d, o, h = _kkt_pair(side, tau, agg)
    fo, fl = o.factors(), h.export()
    assert np.array_equal(fl.perm, fo.perm)
    assert np.array_equal(fl.starts_initial, fo.starts_initial)
    assert np.array_equal(fl.starts, fo.starts)
    for k in range(len(fo.starts) - 1):
        assert np.array_equal(fl.R[k], fo.R[k]) and np.array_equal(fl.C[k], fo.C[k]), k
    for name in ("L", "W", "D"):
        num = sum(float(np.sum((x - y) ** 2)) for x, y in zip(getattr(fl, name), getattr(fo, name)))
        den = sum(float(np.sum(y ** 2)) for y in getattr(fo, name))
        assert np.sqrt(num / max(den, 1e-300)) <= 1e-10, name
    assert h.stats()["perturbed_blocks"] == o.stats()["perturbed_blocks"] == 0
    # the 2x2 pivots' thresholds keep the sets within the device kernels
    assert h.stats()["ilu1t_host"] == 0
    h.close()


def test_symmetric_matching_sqmr_and_fgmres():
    """SQMR on A x = b through the scaled system: five steps give the
    oracle's iterate (x = D x^); to 1e-8 it converges in A's own backward
    error, in a tenth of the steps the plain factorization needs (which
    perturbs pivot blocks); FGMRES runs on the same handle."""
    torch = _torch()
    from oracle import Oracle, OracleOptions
    from paper_1908_10169_amd import bilu
    say("[symmwm-sqmr] kkt side=6 tau=1e-2")
    a, order, d, o, h = _kkt_pair(6, 1e-2, True)
    b = a.matvec(np.ones(a.n))
    xh_o, _ = o.sqmr(d * b, tol=0.0, maxit=5)
    bd = torch.from_numpy(b).cuda()
    xd = torch.zeros_like(bd)
    h.sqmr(bd, xd, tol=0.0, maxit=5)
    x5 = xd.cpu().numpy()
    assert np.linalg.norm(x5 - d * xh_o) <= 1e-9 * np.linalg.norm(d * xh_o)
    xd = torch.zeros_like(bd)
    info = h.sqmr(bd, xd, tol=1e-8, maxit=1000)
    x = xd.cpu().numpy()
    eta = _eta(a, b, x)
    assert info["converged"] and eta <= 1e-8
    assert abs(eta - info["eta"]) <= 1e-6 * eta + 1e-14
    g = bilu.Bilu(ordering=bilu.ORDER_NATURAL, use_aggregation=True)
    g.analyze(a, pre_perm=order)
    g.factor(1e-2)
    xd = torch.zeros_like(bd)
    plain = g.sqmr(bd, xd, tol=1e-8, maxit=2000)
    assert g.stats()["perturbed_blocks"] > 0
    assert plain["converged"] and info["iterations"] * 10 < plain["iterations"]
    xd = torch.zeros_like(bd)
    fg = h.fgmres(bd, xd, restart=30, rtol=1e-8)
    res = np.linalg.norm(b - a.matvec(xd.cpu().numpy())) / np.linalg.norm(b)
    assert fg["converged"] and res <= 1.5e-8
    say(f"[symmwm-sqmr] steps {info['iterations']} (plain {plain['iterations']}), "
        f"FGMRES {fg['iterations']}")
    h.close()
    g.close()


@pytest.mark.parametrize("ordering", ["nd", "multilevel"])
def test_symmetric_matching_with_the_library_ordering(ordering):
    """The symmetric workload's configuration (use_mwm = 2 with the
    library's nested dissection of the compressed graph, multilevel as the
    benchmark runs it): the analysis equals the host preprocessing, and the
    factor equals the oracle's sweep of D A D on that numbering with the
    library's groups as units."""
    torch = _torch()
    from oracle import Oracle, OracleOptions
    from paper_1908_10169_amd import bilu
    order_id = {"nd": bilu.ORDER_ND, "multilevel": bilu.ORDER_ND_MULTILEVEL}[ordering]
    a, order, m = mg.kkt_elasticity(8)
    tau = 1e-2
    say(f"[symmwm-{ordering}] kkt side=8 n={a.n}")
    perm, gs, bs = bilu.preprocess(a, tau, pre_perm=order, ordering=order_id, use_mwm=2)
    h = bilu.Bilu(ordering=order_id, use_aggregation=True, use_mwm=2)
    h.analyze(a, pre_perm=order)
    h.factor(tau)
    fl = h.export()
    assert np.array_equal(fl.perm, perm) and np.array_equal(fl.starts_initial, bs)
    from oracle import symmetric_units
    sigma, dl, dr = bilu.mwm(a)
    d, uorder, us = symmetric_units(a, sigma, dl, dr, pre=order)
    # the 2x2 pivots in the library's numbering (its groups are the units
    # here, coarser than the pivots)
    pos = np.empty(a.n, dtype=np.int64)
    pos[perm] = np.arange(a.n)
    partner = np.full(a.n, -1, dtype=np.int64)
    for u in range(len(us) - 1):
        if us[u + 1] - us[u] == 2:
            p0, p1 = pos[uorder[us[u]]], pos[uorder[us[u] + 1]]
            partner[p0], partner[p1] = p1, p0
    rows = np.repeat(np.arange(a.n), np.diff(a.rowptr))
    ah = mg.Csr(a.n, a.rowptr, a.colind, (d[rows] * a.val) * d[a.colind])
    o = Oracle()
    assert o.run(ah, OracleOptions(tau=tau, use_aggregation=True, use_cosine=False,
                                   sym_perturb=True),
                 pre_perm=perm, unit_starts=gs, partner=partner) == 0
    fo = o.factors()
    assert np.array_equal(fo.perm, fl.perm)
    assert np.array_equal(fo.starts_initial, fl.starts_initial)
    assert np.array_equal(fo.starts, fl.starts)
    for k in range(len(fo.starts) - 1):
        assert np.array_equal(fl.R[k], fo.R[k]) and np.array_equal(fl.C[k], fo.C[k]), k
    for name in ("L", "W", "D"):
        num = sum(float(np.sum((x - y) ** 2)) for x, y in zip(getattr(fl, name), getattr(fo, name)))
        den = sum(float(np.sum(y ** 2)) for y in getattr(fo, name))
        assert np.sqrt(num / max(den, 1e-300)) <= 1e-10, name
    b = a.matvec(np.ones(a.n))
    bd = torch.from_numpy(b).cuda()
    xd = torch.zeros_like(bd)
    info = h.sqmr(bd, xd, tol=1e-6, maxit=500)
    assert info["converged"] and _eta(a, b, xd.cpu().numpy()) <= 1e-6
    h.close()


def test_symmetric_matching_analyze_device_equals_host():
    """bilu_analyze_device with use_mwm = 2 takes the host route and leaves
    the handle as bilu_analyze does: the factors agree bit for bit."""
    torch = _torch()
    from paper_1908_10169_amd import bilu
    a, order, m = mg.kkt_elasticity(6)
    say(f"[symmwm-device] kkt side=6 n={a.n}")
    h = bilu.Bilu(ordering=bilu.ORDER_ND, use_mwm=2)
    h.analyze(a, pre_perm=order)
    h.factor(1e-2)
    g = bilu.Bilu(ordering=bilu.ORDER_ND, use_mwm=2)
    g.analyze_device(a.n, torch.from_numpy(np.asarray(a.rowptr, dtype=np.int64)).cuda(),
                     torch.from_numpy(np.asarray(a.colind, dtype=np.int32)).cuda(),
                     torch.from_numpy(np.asarray(a.val, dtype=np.float64)).cuda(), pre_perm=order)
    g.factor(1e-2)
    fh, fg = h.export(), g.export()
    assert np.array_equal(fh.perm, fg.perm) and np.array_equal(fh.starts, fg.starts)
    for name in ("L", "W", "D"):
        assert b"".join(x.tobytes() for x in getattr(fh, name)) == \
            b"".join(x.tobytes() for x in getattr(fg, name)), name
    h.close()
    g.close()


def test_symmetric_workload_full_size_parity():
    """The benchmark's symmetric line at its own size (kkt_32, n = 114,688,
    the symmetric matching, multilevel ND, aggregation): partition, every
    pattern and every value against the oracle's sweep of D A D on the
    library's numbering, no perturbed block, and SQMR to the benchmark's
    backward error of 1e-6."""
    torch = _torch()
    from oracle import Oracle, OracleOptions, symmetric_units
    from paper_1908_10169_amd import bilu
    a, order, m = mg.kkt_elasticity(32)
    tau = 1e-2
    say(f"[symmwm-full] kkt side=32 n={a.n} nnz={a.nnz}")
    h = bilu.Bilu(ordering=bilu.ORDER_ND_MULTILEVEL, use_aggregation=True, use_mwm=2)
    h.analyze(a, pre_perm=order)
    h.factor(tau)
    fl = h.export()
    assert h.stats()["ilu1t_host"] == 0
    perm, gs, bs = bilu.preprocess(a, tau, pre_perm=order, ordering=bilu.ORDER_ND_MULTILEVEL,
                                   use_mwm=2)
    assert np.array_equal(fl.perm, perm) and np.array_equal(fl.starts_initial, bs)
    sigma, dl, dr = bilu.mwm(a)
    d, uorder, us = symmetric_units(a, sigma, dl, dr, pre=order)
    pos = np.empty(a.n, dtype=np.int64)
    pos[perm] = np.arange(a.n)
    partner = np.full(a.n, -1, dtype=np.int64)
    for u in range(len(us) - 1):
        if us[u + 1] - us[u] == 2:
            p0, p1 = pos[uorder[us[u]]], pos[uorder[us[u] + 1]]
            partner[p0], partner[p1] = p1, p0
    rows = np.repeat(np.arange(a.n), np.diff(a.rowptr))
    ah = mg.Csr(a.n, a.rowptr, a.colind, (d[rows] * a.val) * d[a.colind])
    say("[symmwm-full] oracle sweep")
    o = Oracle()
    assert o.run(ah, OracleOptions(tau=tau, use_aggregation=True, use_cosine=False,
                                   sym_perturb=True),
                 pre_perm=perm, unit_starts=gs, partner=partner) == 0
    fo = o.factors()
    assert np.array_equal(fo.starts_initial, fl.starts_initial)
    assert np.array_equal(fo.starts, fl.starts)
    for k in range(len(fo.starts) - 1):
        assert np.array_equal(fl.R[k], fo.R[k]) and np.array_equal(fl.C[k], fo.C[k]), k
    for name in ("L", "W", "D"):
        num = sum(float(np.sum((x - y) ** 2)) for x, y in zip(getattr(fl, name), getattr(fo, name)))
        den = sum(float(np.sum(y ** 2)) for y in getattr(fo, name))
        assert np.sqrt(num / max(den, 1e-300)) <= 1e-10, name
    assert h.stats()["perturbed_blocks"] == o.stats()["perturbed_blocks"] == 0
    b = a.matvec(np.ones(a.n))
    bd = torch.from_numpy(b).cuda()
    xd = torch.zeros_like(bd)
    info = h.sqmr(bd, xd, tol=1e-6, maxit=2000)
    eta = _eta(a, b, xd.cpu().numpy())
    say(f"[symmwm-full] SQMR {info['iterations']} steps, eta {eta:.2e}")
    assert info["converged"] and eta <= 1e-6
    assert abs(eta - info["eta"]) <= 1e-6 * eta + 1e-14
    h.close()


def _singular_pair_elasticity(side):
    """The unperturbed elasticity operator with unknown 1 a copy of unknown
    0 (row and column): node 0's pivot block is singular."""
    a = mg.grid3d_elasticity(side, 3, seed=2, pert=0.0, shift=0.1)
    A = a.to_dense()
    mask = np.zeros_like(A, dtype=bool)
    mask[np.repeat(np.arange(a.n), np.diff(a.rowptr)), a.colind] = True
    A[1, :] = A[0, :]
    A[:, 1] = A[:, 0]
    A[1, 1] = A[0, 0]
    return mg.dense_to_csr(A, mask=mask)


def test_symmetric_matching_perturbs_symmetrically():
    """A singular pivot block under the symmetric matching: the library
    perturbs it with the symmetric rule, as the oracle does with
    sym_perturb (same patterns, values to 1e-10), and not as the
    column-then-row rule would."""
    _torch()
    from oracle import Oracle, OracleOptions, symmetric_units
    from paper_1908_10169_amd import bilu
    a = _singular_pair_elasticity(4)
    order = mg.node_perm_to_scalar(mg.grid_nd_node_order((4,) * 3, dissect_separators=False), 3)
    say(f"[symmwm-perturb] n={a.n}")
    h = bilu.Bilu(ordering=bilu.ORDER_NATURAL, use_mwm=2)
    h.analyze(a, pre_perm=order)
    h.factor(1e-2)
    fl = h.export()
    sigma, dl, dr = bilu.mwm(a)
    d, uorder, us = symmetric_units(a, sigma, dl, dr, pre=order)
    rows = np.repeat(np.arange(a.n), np.diff(a.rowptr))
    ah = mg.Csr(a.n, a.rowptr, a.colind, (d[rows] * a.val) * d[a.colind])
    fo = {}
    for sp in (True, False):
        o = Oracle()
        assert o.run(ah, OracleOptions(tau=1e-2, sym_perturb=sp), pre_perm=uorder,
                     unit_starts=us) == 0
        assert o.stats()["perturbed_blocks"] == 1
        fo[sp] = o.factors()
    assert h.stats()["perturbed_blocks"] == 1
    f = fo[True]
    assert np.array_equal(fl.perm, f.perm) and np.array_equal(fl.starts, f.starts)
    for k in range(len(f.starts) - 1):
        assert np.array_equal(fl.R[k], f.R[k]) and np.array_equal(fl.C[k], f.C[k]), k
    for name in ("L", "W", "D"):
        num = sum(float(np.sum((x - y) ** 2)) for x, y in zip(getattr(fl, name), getattr(f, name)))
        den = sum(float(np.sum(y ** 2)) for y in getattr(f, name))
        assert np.sqrt(num / max(den, 1e-300)) <= 1e-10, name
    other = max(float(np.abs(x - y).max()) for x, y in zip(fl.D, fo[False].D))
    assert other > 1e-6
    h.close()
