"""The maximum weight matching step (Sec. 3.1, eq. (mwm)) in the GPU
pipeline (use_mwm).

The handle factors A^ = D_l A D_r Pi, with sigma, D_l, D_r from bilu_mwm
(which equals the oracle's matching, tests/test_mwm_native.py).  Checked:

* its factor is bit-identical to the one of a plain handle given A^ formed
  independently on the host, and within the parity tolerance of the
  oracle's factor of A^;
* spmv still multiplies by A, and apply equals D_r Pi M^{-1} D_l x;
* FGMRES solves A x = b to 1e-8 in A's own residual, on a matrix whose
  rows were shuffled so that its diagonal is poor.
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from paper_1908_10169_amd import matgen as mg

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def shuffled_rows(a, seed):
    """P_r A for a random row permutation P_r (the diagonal is lost)."""
    rng = np.random.default_rng(seed)
    p = rng.permutation(a.n)
    s = sp.csr_matrix((a.val, a.colind, a.rowptr), shape=(a.n, a.n))[p]
    s.sort_indices()
    return mg.Csr(a.n, s.indptr.astype(np.int64), s.indices.astype(np.int32), s.data.copy())


def scaled(a, sigma, dl, dr):
    """A^ = D_l A D_r Pi on the host, rows sorted by the new column index."""
    pos = np.empty(a.n, dtype=np.int64)
    pos[sigma] = np.arange(a.n)
    r = np.repeat(np.arange(a.n), np.diff(a.rowptr))
    v = (dl[r] * a.val) * dr[a.colind]
    s = sp.csr_matrix((v, pos[a.colind], a.rowptr), shape=(a.n, a.n))
    s.sort_indices()
    return mg.Csr(a.n, s.indptr.astype(np.int64), s.indices.astype(np.int32), s.data.copy())


def factor_bytes(f):
    return (f.perm.tobytes(), f.starts.tobytes(), [r.tobytes() for r in f.R],
            [c.tobytes() for c in f.C], b"".join(x.tobytes() for x in f.L + f.W + f.D))


CASES = [
    ("cd3d_12_b4_shuffled", lambda: shuffled_rows(mg.workload("cd3d_12_b4", nd=False).a, 3), 1e-2),
    ("cd2d_32x32_b3_shuffled", lambda: shuffled_rows(mg.workload("cd2d_32x32_b3", nd=False).a, 4), 1e-2),
]


@pytest.mark.parametrize("name,make,tau", CASES, ids=[c[0] for c in CASES])
def test_mwm_pipeline(name, make, tau):
    torch = _torch()
    from oracle import Oracle, OracleOptions
    from paper_1908_10169_amd import bilu
    a = make()
    say(f"[mwm] {name} n={a.n} nnz={a.nnz}")
    sigma, dl, dr = bilu.mwm(a)
    ah = scaled(a, sigma, dl, dr)
    # the pipeline with use_mwm against a plain handle on A^
    h = bilu.Bilu(ordering=bilu.ORDER_NATURAL, use_aggregation=False, use_mwm=True)
    h.analyze(a)
    h.factor(tau)
    g = bilu.Bilu(ordering=bilu.ORDER_NATURAL, use_aggregation=False)
    g.analyze(ah)
    g.factor(tau)
    assert factor_bytes(h.export()) == factor_bytes(g.export())
    # the oracle's factor of A^
    o = Oracle()
    assert o.run(ah, OracleOptions(tau=tau, use_aggregation=False)) == 0
    fo, fl = o.factors(), h.export()
    assert np.array_equal(fl.perm, fo.perm) and np.array_equal(fl.starts, fo.starts)
    for name_ in ("L", "W", "D"):
        num = sum(float(np.sum((x - y) ** 2)) for x, y in zip(getattr(fl, name_), getattr(fo, name_)))
        den = sum(float(np.sum(y ** 2)) for y in getattr(fo, name_))
        assert np.sqrt(num / max(den, 1e-300)) <= TOL, name_
    # spmv is A, apply is D_r Pi M^-1 D_l
    rng = np.random.default_rng(5)
    x = rng.standard_normal(a.n)
    xd = torch.from_numpy(x).cuda()
    yd = torch.empty_like(xd)
    h.spmv(xd, yd)
    ax = a.matvec(x)
    assert np.linalg.norm(yd.cpu().numpy() - ax) <= 1e-12 * np.linalg.norm(ax)
    h.apply(xd, yd)
    zd = torch.empty_like(xd)
    g.apply(torch.from_numpy(dl * x).cuda(), zd)
    z = zd.cpu().numpy()
    want = np.empty(a.n)
    want[sigma] = dr[sigma] * z
    got = yd.cpu().numpy()
    assert np.linalg.norm(got - want) <= 1e-12 * np.linalg.norm(want)
    # FGMRES on A x = b, checked in A's own residual
    b = a.matvec(np.ones(a.n))
    bd = torch.from_numpy(b).cuda()
    xs = torch.zeros_like(bd)
    info = h.fgmres(bd, xs, restart=30, rtol=1e-8)
    res = np.linalg.norm(b - a.matvec(xs.cpu().numpy())) / np.linalg.norm(b)
    say(f"[mwm] {name}: {info['iterations']} iterations, true residual {res:.2e}")
    assert info["converged"] and res <= 1.5e-8
    assert info["rel_residual"] == pytest.approx(res, rel=1e-3, abs=1e-14)
    h.close()
    g.close()
