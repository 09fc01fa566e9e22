"""The device analyze (Sec. 3.2-3.3 with the matrix in HBM) against the host
analyze, through the C ABI.

Both routes must leave the handle identical bit for bit: permutation, cosine
groups, and the permuted matrix (checked through the factor it produces, and
at full size through the apply).  The host route equals the oracle's
permutation and groups (tests/test_gpu_parity.py runs the default route, the
device one, against the oracle as well).  Cases cover a caller permutation,
both orderings, the integer and the floating cosine test, a small max_block,
rows past the LDS hash table (an arrow matrix), the cosine step switched off,
the MWM route, device-array input, and the error paths.
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


def arrow(n, seed):
    """Tridiagonal-plus-neighbours pattern with a dense last row and column:
    every seed reaches every later row through the last column, so most seeds
    have more later rows than the LDS table holds."""
    rng = np.random.default_rng(seed)
    rows = []
    for i in range(n):
        cols = {i, n - 1}
        for d in (-7, -1, 1, 7):
            if 0 <= i + d < n:
                cols.add(i + d)
        if i == n - 1:
            cols = set(range(n))
        rows.append(sorted(cols))
    rp = np.zeros(n + 1, dtype=np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    ci = np.concatenate([np.array(r, dtype=np.int32) for r in rows])
    v = rng.uniform(-1.0, 1.0, len(ci))
    for i in range(n):
        k = rp[i] + rows[i].index(i)
        v[k] = 8.0 + rng.random()
    return mg.Csr(n, rp, ci, v)


def twin_rows(n, seed):
    """Random pattern where rows come in pairs and triples with equal or
    nearly equal patterns, so the floating cosine test has borderline pairs."""
    rng = np.random.default_rng(seed)
    rows = []
    i = 0
    while i < n:
        g = min(n - i, int(rng.integers(1, 4)))
        base = set(rng.choice(n, size=int(rng.integers(3, 12)), replace=False).tolist())
        for t in range(g):
            cols = set(base)
            if rng.random() < 0.5:
                cols.add(int(rng.integers(n)))
            cols.add(i + t)
            rows.append(sorted(cols))
        i += g
    rp = np.zeros(n + 1, dtype=np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    ci = np.concatenate([np.array(r, dtype=np.int32) for r in rows])
    v = rng.uniform(-1.0, 1.0, len(ci))
    for r in range(n):
        v[rp[r] + rows[r].index(r)] = 20.0
    return mg.Csr(n, rp, ci, v)


def factor_bytes(f):
    return (f.perm.tobytes(), f.group_starts.tobytes(), f.starts.tobytes(),
            b"".join(r.tobytes() for r in f.R), b"".join(c.tobytes() for c in f.C),
            b"".join(x.tobytes() for x in f.L + f.W + f.D))


def both(a, tau, pre_perm=None, **kw):
    from paper_1908_10169_amd import bilu
    out = []
    for path in (0, 1):
        h = bilu.Bilu(analyze_path=path, **kw)
        h.analyze(a, pre_perm=pre_perm)
        h.factor(tau)
        out.append(h)
    return out


CASES = [
    ("cd3d_12_b4_nd_natural", lambda: mg.workload("cd3d_12_b4"), dict(ordering=1), True),
    ("cd3d_12_b4_own_nd", lambda: mg.workload("cd3d_12_b4", nd=False), dict(), False),
    ("cd2d_32x32_b3_eps06_mb2", lambda: mg.workload("cd2d_32x32_b3", nd=False),
     dict(cos_eps=0.6, max_block=2), False),
    ("twin_rows_eps07", lambda: mg.Workload("twin", twin_rows(3000, 3), 1, (3000,), 1e-2, 30, None),
     dict(cos_eps=0.7, ordering=1), False),
    ("twin_rows_eps08_nd", lambda: mg.Workload("twin", twin_rows(2500, 4), 1, (2500,), 1e-2, 30,
                                               np.random.default_rng(9).permutation(2500)),
     dict(), True),
    ("arrow_overflow", lambda: mg.Workload("arrow", arrow(2000, 5), 1, (2000,), 1e-2, 30, None),
     dict(ordering=1), False),
    ("el3d_10_no_cosine_nd", lambda: mg.workload("el3d_10_b3"), dict(use_cosine=0), True),
    ("irregular_mesh_multilevel_nd",
     lambda: mg.Workload("rgg", mg.random_geometric(1200, k=7, dim=3, b=3, seed=6), 3, (1200,),
                         1e-2, 30, None),
     dict(ordering=2), False),
]


@pytest.mark.parametrize("name,make,kw,use_pre", CASES, ids=[c[0] for c in CASES])
def test_device_analyze_equals_host(name, make, kw, use_pre):
    _torch()
    w = make()
    say(f"[analyze] {name} n={w.a.n} nnz={w.a.nnz} {kw}")
    hd, hh = both(w.a, w.tau, pre_perm=w.perm if use_pre else None, use_aggregation=0, **kw)
    fd, fh = hd.export(), hh.export()
    assert factor_bytes(fd) == factor_bytes(fh)
    sd, sh = hd.stats(), hh.stats()
    assert sd["ngroups"] == sh["ngroups"]
    say(f"[analyze] {name}: {sd['ngroups']} groups, device {sd['t_analyze']:.3f} s, "
        f"host {sh['t_analyze']:.3f} s")
    hd.close()
    hh.close()


def test_device_analyze_matches_oracle_groups():
    """The device route's permutation and groups against the oracle on a
    floating-threshold case (the integer case runs in the parity tests)."""
    _torch()
    from oracle import Oracle, OracleOptions
    from paper_1908_10169_amd import bilu
    a = twin_rows(600, 11)
    o = Oracle()
    assert o.run(a, OracleOptions(tau=1e-2, use_aggregation=False, cos_eps=0.7)) == 0
    h = bilu.Bilu(ordering=bilu.ORDER_NATURAL, use_aggregation=False, cos_eps=0.7)
    h.analyze(a)
    h.factor(1e-2)
    fl = h.export()
    assert np.array_equal(fl.perm, o.perm())
    assert np.array_equal(fl.group_starts, o.group_starts())
    assert np.array_equal(fl.starts, o.starts())
    h.close()


def test_analyze_device_arrays():
    """bilu_analyze_device on torch tensors equals bilu_analyze on host
    arrays, with a caller permutation and with the MWM route."""
    torch = _torch()
    from paper_1908_10169_amd import bilu
    w = mg.workload("cd3d_12_b4")
    a = w.a
    rp = torch.from_numpy(a.rowptr).cuda()
    ci = torch.from_numpy(a.colind).cuda()
    v = torch.from_numpy(a.val).cuda()
    for kw in (dict(ordering=1), dict(use_mwm=1)):
        g = bilu.Bilu(use_aggregation=0, **kw)
        g.analyze_device(a.n, rp, ci, v, pre_perm=w.perm)
        g.factor(w.tau)
        r = bilu.Bilu(use_aggregation=0, **kw)
        r.analyze(a, pre_perm=w.perm)
        r.factor(w.tau)
        assert factor_bytes(g.export()) == factor_bytes(r.export()), kw
        g.close()
        r.close()


def bad_matrices():
    a = mg.workload("cd3d_8_b2", nd=False).a
    out = []
    ci = a.colind.copy()
    ci[a.rowptr[6] - 1] = a.n  # last entry of row 5: out of range, order intact
    out.append(("column index out of range", mg.Csr(a.n, a.rowptr, ci, a.val)))
    ci = a.colind.copy()
    r = 3
    ci[a.rowptr[r]], ci[a.rowptr[r] + 1] = ci[a.rowptr[r] + 1], ci[a.rowptr[r]]
    out.append(("column indices not strictly increasing", mg.Csr(a.n, a.rowptr, ci, a.val)))
    v = a.val.copy()
    v[17] = np.nan
    out.append(("non-finite value", mg.Csr(a.n, a.rowptr, a.colind, v)))
    return a, out


def test_device_analyze_errors():
    """Invalid entries and a bad caller permutation give the host route's
    status and message."""
    _torch()
    from paper_1908_10169_amd import bilu
    a, cases = bad_matrices()
    for msg, m in cases:
        for path in (0, 1):
            h = bilu.Bilu(analyze_path=path)
            with pytest.raises(bilu.BiluError) as e:
                h.analyze(m)
            assert e.value.status == bilu.BILU_ERR_INVALID and msg in str(e.value), (path, msg)
            h.close()
    bad = np.arange(a.n)
    bad[4] = 3
    for path in (0, 1):
        h = bilu.Bilu(analyze_path=path)
        with pytest.raises(bilu.BiluError) as e:
            h.analyze(a, pre_perm=bad)
        assert "pre_perm" in str(e.value)
        h.close()


def test_device_analyze_full_size():
    """cd3d_64_b4 (n = 1048576) in the configuration the benchmark times: the
    device and host routes give the same groups, blocks and apply output bit
    for bit."""
    torch = _torch()
    from paper_1908_10169_amd import bilu
    w = mg.workload("cd3d_64_b4")
    outs = []
    for path in (0, 1):
        h = bilu.Bilu(ordering=bilu.ORDER_NATURAL, analyze_path=path)
        h.analyze(w.a, pre_perm=w.perm)
        h.factor(w.tau)
        s = h.stats()
        x = torch.from_numpy(np.random.default_rng(3).standard_normal(w.a.n)).cuda()
        y = torch.empty_like(x)
        h.apply(x, y)
        h.sync()
        outs.append((s, y.cpu().numpy()))
        say(f"[analyze] cd3d_64_b4 path {path}: {s['t_analyze']:.3f} s, {s['ngroups']} groups, "
            f"{s['nblocks']} blocks")
        h.close()
    (s0, y0), (s1, y1) = outs
    for k in ("ngroups", "nblocks", "nblocks_initial", "nnz_l", "nnz_w", "nnz_d"):
        assert s0[k] == s1[k], k
    assert y0.tobytes() == y1.tobytes()
