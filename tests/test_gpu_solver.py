"""Solver-level behaviour through the C ABI: restarted FGMRES cycles against
the oracle, the maxit stop, a factor heap that has to grow, and the apply
fault counter.

Restarts: every parity workload converges inside its first FGMRES cycle, so
these cases use a loose drop tolerance and a short restart length to force
several cycles; the GPU solver must take the oracle's iteration and restart
counts and reach the same true residual bar.
"""
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


RESTART_CASES = [
    # (workload, tau, restart, aggregation): 3 to 13 cycles in the oracle
    ("cd2d_32x32_b3", 1e-1, 2, False),
    ("cd2d_32x32_b3", 3e-1, 4, True),
    ("cd3d_12_b4", 1e-1, 3, True),
    ("el3d_10_b3", 5e-2, 3, False),
]


@pytest.mark.parametrize("name,tau,restart,agg", RESTART_CASES,
                         ids=[f"{c[0]}-m{c[2]}-{'agg' if c[3] else 'plain'}" for c in RESTART_CASES])
def test_restarted_fgmres_parity(name, tau, restart, agg):
    torch = _torch()
    from oracle import Oracle, OracleOptions
    from paper_1908_10169_amd import bilu
    w = mg.workload(name)
    say(f"[restart] {name} tau={tau} m={restart} aggregation={agg}")
    o = Oracle()
    assert o.run(w.a, OracleOptions(tau=tau, use_aggregation=agg), pre_perm=w.perm) == 0
    b = w.a.matvec(np.ones(w.a.n))
    _, info_o = o.fgmres(b, restart=restart, rtol=1e-8)
    assert info_o["converged"] and info_o["restarts"] > 1
    h = bilu.Bilu(ordering=bilu.ORDER_NATURAL, use_aggregation=agg)
    h.analyze(w.a, pre_perm=w.perm)
    h.factor(tau)
    bd = torch.from_numpy(b).cuda()
    xd = torch.zeros_like(bd)
    info = h.fgmres(bd, xd, restart=restart, rtol=1e-8)
    assert info["converged"]
    assert info["iterations"] == info_o["iterations"]
    assert info["restarts"] == info_o["restarts"]
    x = xd.cpu().numpy()
    res = np.linalg.norm(b - w.a.matvec(x)) / np.linalg.norm(b)
    assert res <= 1e-8 and info["rel_residual"] <= 1e-8
    assert abs(res - info["rel_residual"]) <= 1e-3 * res
    assert h.stats()["apply_faults"] == 0
    h.close()


def test_maxit_stops_unconverged():
    """maxit = 1: one Arnoldi step, BILU_WARN_NOT_CONVERGED, and the same
    residual after that step as the oracle's."""
    torch = _torch()
    from oracle import Oracle, OracleOptions
    from paper_1908_10169_amd import bilu
    w = mg.workload("cd2d_32x32_b3")
    say("[maxit] cd2d_32x32_b3 maxit=1")
    o = Oracle()
    assert o.run(w.a, OracleOptions(tau=w.tau, use_aggregation=True), pre_perm=w.perm) == 0
    b = w.a.matvec(np.ones(w.a.n))
    _, info_o = o.fgmres(b, restart=30, rtol=1e-8, maxit=1)
    h = bilu.Bilu(ordering=bilu.ORDER_NATURAL)
    h.analyze(w.a, pre_perm=w.perm)
    h.factor(w.tau)
    bd = torch.from_numpy(b).cuda()
    xd = torch.zeros_like(bd)
    lib = bilu.load()
    info = bilu.SolveInfo()
    import ctypes as C
    st = lib.bilu_fgmres_solve(h._h, bd.data_ptr(), xd.data_ptr(), 30, 1e-8, 1, C.byref(info))
    assert st == bilu.BILU_WARN_NOT_CONVERGED
    assert info.iterations == 1 and info.restarts == 1 and not info.converged
    assert not info_o["converged"] and info_o["iterations"] == 1
    assert abs(info.rel_residual - info_o["rel_residual"]) <= 1e-8 * info_o["rel_residual"]
    assert info.rel_residual > 1e-8
    h.close()


def test_small_heap_grows_and_resumes():
    """A factor heap far too small (heap_bytes = 1 KiB) is grown and the
    sweep run again: the result equals the one with the default size, bit
    for bit."""
    _torch()
    from paper_1908_10169_amd import bilu
    w = mg.workload("cd3d_12_b4")
    say("[heap] cd3d_12_b4 heap_bytes=1024")
    outs = []
    for hb in (0, 1024):
        h = bilu.Bilu(ordering=bilu.ORDER_NATURAL, heap_bytes=hb)
        h.analyze(w.a, pre_perm=w.perm)
        h.factor(w.tau)
        f = h.export()
        outs.append((f.starts.tobytes(), b"".join(r.tobytes() for r in f.R + f.C),
                     b"".join(x.tobytes() for x in f.L + f.W + f.D)))
        h.close()
    assert outs[0] == outs[1]
