"""bilu_refactor: new values of the analyzed pattern, the block Crout sweep
of Sec. 2.2 again on the initial blocks of the last factor.

Reference: the oracle's sweep over a given partition (run_partition) with
the handle's permutation and initial blocks on the new matrix.  Bar as in
the parity tests: partition and every pattern identical, L, W, D and the
apply within 1e-10 relative.  Also: the same values give the same factor bit
for bit; a refactor keeps the stored matrix consistent (a following
bilu_factor equals a fresh handle's); both analyze routes refactor alike;
errors leave the previous factor in place.
"""
import sys

import numpy as np
import pytest

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


def new_values(a, seed, spread=0.3):
    """Same pattern, every value scaled by 1 + spread * U(-1, 1)."""
    rng = np.random.default_rng(seed)
    return mg.Csr(a.n, a.rowptr, a.colind, a.val * (1.0 + spread * rng.uniform(-1.0, 1.0, a.nnz)))


def factor_bytes(f):
    return (f.perm.tobytes(), f.starts.tobytes(), f.starts_initial.tobytes(),
            b"".join(r.tobytes() for r in f.R), b"".join(c.tobytes() for c in f.C),
            b"".join(x.tobytes() for x in f.L + f.W + f.D))


def compare_with_oracle(o, fl):
    fo = o.factors()
    assert np.array_equal(fl.perm, fo.perm)
    assert np.array_equal(fl.starts, fo.starts)
    for k in range(len(fo.starts) - 1):
        assert np.array_equal(fl.R[k], fo.R[k]), f"rows of block {k}"
        assert np.array_equal(fl.C[k], fo.C[k]), f"cols of block {k}"
    for name in ("L", "W", "D"):
        num = sum(float(np.sum((x - y) ** 2)) for x, y in zip(getattr(fl, name), getattr(fo, name)))
        den = sum(float(np.sum(y ** 2)) for y in getattr(fo, name))
        assert np.sqrt(num / max(den, 1e-300)) <= TOL, name


CASES = [
    ("cd3d_12_b4_nd", "cd3d_12_b4", False),
    ("cd3d_12_b4_nd_agg", "cd3d_12_b4", True),
    ("el3d_10_b3_nd_agg", "el3d_10_b3", True),
    ("cd2d_32x32_b3_agg", "cd2d_32x32_b3", True),
]


@pytest.mark.parametrize("name,wl,agg", CASES, ids=[c[0] for c in CASES])
def test_refactor_matches_oracle(name, wl, agg):
    torch = _torch()
    from oracle import Oracle, OracleOptions
    from paper_1908_10169_amd import bilu
    w = mg.workload(wl)
    say(f"[refactor] {name} n={w.a.n}")
    h = bilu.Bilu(ordering=bilu.ORDER_NATURAL, use_aggregation=agg)
    h.analyze(w.a, pre_perm=w.perm)
    h.factor(w.tau)
    f0 = h.export()
    a2 = new_values(w.a, 5)
    h.refactor(w.tau, torch.from_numpy(a2.val).cuda())
    fl = h.export()
    assert np.array_equal(fl.starts_initial, f0.starts_initial)
    o = Oracle()
    assert o.run_partition(a2, f0.starts_initial, OracleOptions(tau=w.tau, use_aggregation=agg),
                           perm=f0.perm) == 0
    compare_with_oracle(o, fl)
    # apply and solve on the new matrix
    rng = np.random.default_rng(7)
    x = rng.standard_normal(a2.n)
    yo = o.apply(x)
    xd = torch.from_numpy(x).cuda()
    yd = torch.empty_like(xd)
    h.apply(xd, yd)
    h.sync()
    assert np.linalg.norm(yd.cpu().numpy() - yo) <= TOL * np.linalg.norm(yo)
    b = a2.matvec(np.ones(a2.n))
    bd = torch.from_numpy(b).cuda()
    xs = torch.zeros_like(bd)
    info = h.fgmres(bd, xs, restart=w.restart, rtol=1e-8)
    res = np.linalg.norm(b - a2.matvec(xs.cpu().numpy())) / np.linalg.norm(b)
    say(f"[refactor] {name}: {info['iterations']} iterations, true residual {res:.2e}")
    assert info["converged"] and res <= 1.5e-8
    h.close()


def test_refactor_same_values_and_consistency():
    """Same values: the same factor bit for bit.  New values: a following
    bilu_factor equals a fresh handle analyzed and factored on them."""
    torch = _torch()
    from paper_1908_10169_amd import bilu
    w = mg.workload("cd3d_12_b4")
    h = bilu.Bilu(ordering=bilu.ORDER_NATURAL)
    h.analyze(w.a, pre_perm=w.perm)
    h.factor(w.tau)
    f0 = factor_bytes(h.export())
    h.refactor(w.tau, torch.from_numpy(w.a.val).cuda())
    assert factor_bytes(h.export()) == f0
    a2 = new_values(w.a, 8)
    h.refactor(w.tau, torch.from_numpy(a2.val).cuda())
    h.factor(w.tau)
    g = bilu.Bilu(ordering=bilu.ORDER_NATURAL)
    g.analyze(a2, pre_perm=w.perm)
    g.factor(w.tau)
    assert factor_bytes(h.export()) == factor_bytes(g.export())
    h.close()
    g.close()


def test_refactor_host_route():
    torch = _torch()
    from paper_1908_10169_amd import bilu
    w = mg.workload("el3d_10_b3")
    a2 = new_values(w.a, 9)
    v2 = torch.from_numpy(a2.val).cuda()
    out = []
    for path in (0, 1):
        h = bilu.Bilu(analyze_path=path)
        h.analyze(w.a)
        h.factor(w.tau)
        h.refactor(w.tau, v2)
        out.append(factor_bytes(h.export()))
        h.close()
    assert out[0] == out[1]


def test_refactor_errors():
    torch = _torch()
    from paper_1908_10169_amd import bilu
    w = mg.workload("cd3d_8_b2")
    v = torch.from_numpy(w.a.val).cuda()
    h = bilu.Bilu(ordering=bilu.ORDER_NATURAL)
    h.analyze(w.a, pre_perm=w.perm)
    with pytest.raises(bilu.BiluError) as e:
        h.refactor(w.tau, v)
    assert e.value.status == bilu.BILU_ERR_STATE
    h.factor(w.tau)
    x = torch.from_numpy(np.random.default_rng(1).standard_normal(w.a.n)).cuda()
    y0 = torch.empty_like(x)
    h.apply(x, y0)
    bad = w.a.val.copy()
    bad[11] = np.inf
    with pytest.raises(bilu.BiluError) as e:
        h.refactor(w.tau, torch.from_numpy(bad).cuda())
    assert e.value.status == bilu.BILU_ERR_INVALID and "non-finite" in str(e.value)
    y1 = torch.empty_like(x)
    h.apply(x, y1)
    h.sync()
    assert y0.cpu().numpy().tobytes() == y1.cpu().numpy().tobytes()
    h.close()
    m = bilu.Bilu(use_mwm=1)
    m.analyze(w.a)
    m.factor(w.tau)
    with pytest.raises(bilu.BiluError) as e:
        m.refactor(w.tau, v)
    assert e.value.status == bilu.BILU_ERR_INVALID
    m.close()


def test_refactor_full_size():
    """cd3d_64_b4 (n = 1048576) in the benchmark's configuration: a refactor
    with the same values reproduces the factor (apply output bit for bit)."""
    torch = _torch()
    import time
    from paper_1908_10169_amd import bilu
    w = mg.workload("cd3d_64_b4")
    h = bilu.Bilu(ordering=bilu.ORDER_NATURAL)
    h.analyze(w.a, pre_perm=w.perm)
    h.factor(w.tau)
    s0 = h.stats()
    x = torch.from_numpy(np.random.default_rng(3).standard_normal(w.a.n)).cuda()
    y0 = torch.empty_like(x)
    h.apply(x, y0)
    v = torch.from_numpy(w.a.val).cuda()
    torch.cuda.synchronize()
    t = time.perf_counter()
    h.refactor(w.tau, v)
    dt = time.perf_counter() - t
    s1 = h.stats()
    y1 = torch.empty_like(x)
    h.apply(x, y1)
    h.sync()
    say(f"[refactor] cd3d_64_b4: factor {s0['t_factor']:.4f} s, refactor {dt:.4f} s")
    for k in ("nblocks", "nblocks_initial", "nnz_l", "nnz_w", "nnz_d"):
        assert s0[k] == s1[k], k
    assert y0.cpu().numpy().tobytes() == y1.cpu().numpy().tobytes()
    h.close()


# ---------------------------------------------------------------------------
# bilu_refactor_frozen: the last factor's blocks and patterns stay, the
# values follow the new matrix.  Reference: the oracle's frozen
# refactorization of its own factor of the first matrix (the two factors
# have the same blocks and patterns by the parity tests).
# ---------------------------------------------------------------------------
FROZEN_CASES = [
    ("cd2d_32x32_b3", "cd2d_32x32_b3", False),
    ("cd2d_32x32_b3_agg", "cd2d_32x32_b3", True),
    ("cd3d_12_b4_agg", "cd3d_12_b4", True),
    ("el3d_10_b3", "el3d_10_b3", False),
    ("el3d_10_b3_agg", "el3d_10_b3", True),
]


@pytest.mark.parametrize("name,wl,agg", FROZEN_CASES, ids=[c[0] for c in FROZEN_CASES])
def test_refactor_frozen_matches_oracle(name, wl, agg):
    torch = _torch()
    from oracle import Oracle, OracleOptions
    from paper_1908_10169_amd import bilu
    w = mg.workload(wl)
    say(f"[frozen] {name} n={w.a.n}")
    o = Oracle()
    assert o.run(w.a, OracleOptions(tau=w.tau, use_aggregation=agg), pre_perm=w.perm) == 0
    h = bilu.Bilu(ordering=bilu.ORDER_NATURAL, use_aggregation=agg)
    h.analyze(w.a, pre_perm=w.perm)
    h.factor(w.tau)
    a2 = new_values(w.a, 9)
    assert o.refactor_frozen(a2.val) == 0
    h.refactor_frozen(torch.from_numpy(a2.val).cuda())
    fl = h.export()
    compare_with_oracle(o, fl)
    # the apply with the new values, and a solve of the new system
    rng = np.random.default_rng(3)
    x = rng.standard_normal(w.a.n)
    y = torch.empty(w.a.n, dtype=torch.float64, device="cuda")
    h.apply(torch.from_numpy(x).cuda(), y)
    yo = o.apply(x)
    assert np.linalg.norm(y.cpu().numpy() - yo) <= TOL * np.linalg.norm(yo)
    b = a2.matvec(np.ones(w.a.n))
    bd = torch.from_numpy(b).cuda()
    xd = torch.zeros_like(bd)
    info = h.fgmres(bd, xd, restart=w.restart, rtol=1e-8)
    assert info["converged"]
    assert np.linalg.norm(b - a2.matvec(xd.cpu().numpy())) <= 1e-8 * np.linalg.norm(b)
    assert h.stats()["apply_faults"] == 0
    if not agg:  # the kept-pattern identity on the new values
        assert h.kept_residual() <= 1e-13
    h.close()


def test_refactor_frozen_same_values_and_errors():
    """The same values give the factor back (to rounding, no merges); the
    kept-pattern residual is refused after merges; a non-finite value
    changes nothing; a call before bilu_factor is a state error."""
    torch = _torch()
    from paper_1908_10169_amd import bilu
    w = mg.workload("cd3d_12_b4")
    h = bilu.Bilu(ordering=bilu.ORDER_NATURAL, use_aggregation=False)
    h.analyze(w.a, pre_perm=w.perm)
    with pytest.raises(bilu.BiluError) as e:
        h.refactor_frozen(torch.from_numpy(w.a.val).cuda())
    assert e.value.status == bilu.BILU_ERR_STATE
    h.factor(w.tau)
    f0 = h.export()
    h.refactor_frozen(torch.from_numpy(w.a.val).cuda())
    f1 = h.export()
    for name in ("L", "W", "D"):
        x = np.concatenate([v.ravel() for v in getattr(f1, name)])
        y = np.concatenate([v.ravel() for v in getattr(f0, name)])
        assert np.linalg.norm(x - y) <= 1e-13 * np.linalg.norm(y), name
    bad = w.a.val.copy()
    bad[7] = np.nan
    with pytest.raises(bilu.BiluError) as e:
        h.refactor_frozen(torch.from_numpy(bad).cuda())
    assert e.value.status == bilu.BILU_ERR_INVALID
    f2 = h.export()
    assert all(np.array_equal(x, y) for x, y in zip(f1.L + f1.W + f1.D, f2.L + f2.W + f2.D))
    h.close()
    g = bilu.Bilu(ordering=bilu.ORDER_NATURAL, use_aggregation=True)
    g.analyze(w.a, pre_perm=w.perm)
    g.factor(w.tau)
    if g.stats()["merges"] > 0:
        g.refactor_frozen(torch.from_numpy(new_values(w.a, 2).val).cuda())
        with pytest.raises(bilu.BiluError) as e:
            g.kept_residual()
        assert e.value.status == bilu.BILU_ERR_STATE
    g.close()
