"""GPU path vs the FP64 oracle, element by element (through the C ABI).

Bar (FP64 mode): block partition and every row/column pattern identical;
L, W, D within 1e-10 relative (Frobenius, per factor); apply within 1e-10
relative; equal FGMRES iteration counts and true residual <= rtol.
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


def run_pair(a, tau, pre_perm=None, agg=False, update_mfma=0, deterministic=1, **blocking):
    from oracle import Oracle, OracleOptions
    from paper_1908_10169_amd import bilu
    o = Oracle()
    rc = o.run(a, OracleOptions(tau=tau, use_aggregation=agg, **blocking), pre_perm=pre_perm)
    assert rc == 0
    h = bilu.Bilu(ordering=bilu.ORDER_NATURAL, use_aggregation=agg, update_mfma=update_mfma,
                  deterministic=deterministic, **blocking)
    h.analyze(a, pre_perm=pre_perm)
    h.factor(tau)
    return o, h


def compare_factors(o, h):
    fo = o.factors()
    fl = h.export()
    assert np.array_equal(fl.perm, fo.perm)
    assert np.array_equal(fl.starts_initial, fo.starts_initial)
    assert np.array_equal(fl.starts, fo.starts)
    num = {"L": 0.0, "W": 0.0, "D": 0.0}
    den = {"L": 0.0, "W": 0.0, "D": 0.0}
    for k in range(len(fo.starts) - 1):
        assert np.array_equal(fl.R[k], fo.R[k]), f"rows of block {k}"
        assert np.array_equal(fl.C[k], fo.C[k]), f"cols of block {k}"
        for name in ("L", "W", "D"):
            x, y = getattr(fl, name)[k], getattr(fo, name)[k]
            num[name] += float(np.sum((x - y) ** 2))
            den[name] += float(np.sum(y ** 2))
    for name in num:
        rel = np.sqrt(num[name] / max(den[name], 1e-300))
        assert rel <= TOL, (name, rel)
    worst = max_block_error(fl, fo)
    assert worst <= BLOCK_TOL, worst
    return fl


BLOCK_TOL = 1e-8  # per block: one wrong block stands out of the global norm


def check_drop_counts(o, h, tau):
    """The sweep's drop statistics equal the oracle's decision log: the
    number of dropped rows and columns exactly, the smallest margin
    |norm - tau| / tau to rounding."""
    log = o.droplog()
    st = h.stats()
    assert st["drops_rows"] == int(np.sum((log["kind"] == 0) & ~log["kept"]))
    assert st["drops_cols"] == int(np.sum((log["kind"] == 1) & ~log["kept"]))
    if tau > 0 and len(log["norm"]):
        m = float(np.min(np.abs(log["norm"] - tau) / tau))
        assert abs(st["drop_margin_min"] - m) <= 1e-9 * max(m, 1e-300) + 1e-15, (st, m)


def max_block_error(fl, fo):
    """Largest relative difference of any single block's L, W or D."""
    worst = 0.0
    for name in ("L", "W", "D"):
        for x, y in zip(getattr(fl, name), getattr(fo, name)):
            if y.size:
                worst = max(worst, float(np.linalg.norm(x - y)) / max(float(np.linalg.norm(y)),
                                                                       1e-300))
    return worst


def check_apply_and_solve(o, h, a, restart=30):
    torch = _torch()
    rng = np.random.default_rng(7)
    x = rng.standard_normal(a.n)
    yo = o.apply(x)
    xd = torch.from_numpy(x).cuda()
    yd = torch.empty_like(xd)
    h.apply(xd, yd)
    h.sync()
    yl = yd.cpu().numpy()
    assert np.linalg.norm(yl - yo) <= TOL * np.linalg.norm(yo)
    b = a.matvec(np.ones(a.n))
    xo, info_o = o.fgmres(b, restart=restart, rtol=1e-8)
    bd = torch.from_numpy(b).cuda()
    xl = torch.zeros_like(bd)
    info_l = h.fgmres(bd, xl, restart=restart, rtol=1e-8)
    assert info_l["converged"] and info_o["converged"]
    assert info_l["iterations"] == info_o["iterations"]
    xh = xl.cpu().numpy()
    res = np.linalg.norm(b - a.matvec(xh)) / np.linalg.norm(b)
    assert res <= 1e-8
    assert info_l["rel_residual"] <= 1e-8


CASES = [
    ("cd2d_natural", lambda: (mg.grid2d_random_blocks(32, 3, 4.5, seed=0), None), 1e-2, {}),
    ("cd2d_nd", lambda: (mg.workload("cd2d_32x32_b3").a, mg.workload("cd2d_32x32_b3").perm),
     1e-2, {}),
    ("cd2d_scalar", lambda: (mg.grid2d_random_blocks(20, 3, 4.5, seed=0), None), 1e-2,
     dict(use_cosine=False, use_ilu1t=False)),
    ("cd2d_cosine_only", lambda: (mg.grid2d_random_blocks(24, 2, 3.5, seed=4), None), 3e-2,
     dict(use_ilu1t=False)),
    ("cd3d_12_nd", lambda: (mg.workload("cd3d_12_b4").a, mg.workload("cd3d_12_b4").perm), 1e-2, {}),
    ("el3d_10_nd", lambda: (mg.workload("el3d_10_b3").a, mg.workload("el3d_10_b3").perm), 5e-3, {}),
    ("random_sparse", lambda: (mg.random_sparse(400, 0.01, seed=5, diag_shift=3.0), None), 1e-2, {}),
    # dense rows: ILU(1,tau) grows blocks wider than 64 (pivots outside LDS)
    ("wide_blocks", lambda: (mg.random_sparse(200, 0.5, seed=3, diag_shift=8.0), None), 1e-2, {}),
]


@pytest.mark.parametrize("name,make,tau,blocking", CASES, ids=[c[0] for c in CASES])
def test_factor_parity(name, make, tau, blocking):
    _torch()
    a, perm = make()
    say(f"[parity] {name} n={a.n} nnz={a.nnz} tau={tau} {blocking}")
    o, h = run_pair(a, tau, perm, **blocking)
    compare_factors(o, h)
    check_drop_counts(o, h, tau)
    # the kept-pattern identity (Sec. 2.2) on the device, as in the oracle
    rk, rk_o = h.kept_residual(), o.kept_residual()
    assert rk <= 1e-12 and rk_o <= 1e-12, (rk, rk_o)
    check_apply_and_solve(o, h, a)
    h.close()


MFMA_CASES = [c for c in CASES if c[0] in ("cd2d_nd", "cd3d_12_nd", "el3d_10_nd", "random_sparse")]


@pytest.mark.parametrize("name,make,tau,blocking", MFMA_CASES, ids=[c[0] for c in MFMA_CASES])
def test_factor_parity_matrix_cores(name, make, tau, blocking):
    """FP64 update terms as 16x16x4 matrix-core tiles (update_mfma = 1): the
    products round differently, so the bar is the parity bar (patterns
    identical, values within the tolerance, equal iterations)."""
    _torch()
    a, perm = make()
    say(f"[parity mfma] {name} n={a.n} tau={tau}")
    o, h = run_pair(a, tau, perm, update_mfma=1, **blocking)
    compare_factors(o, h)
    check_apply_and_solve(o, h, a)
    h.close()


@pytest.mark.parametrize("name,make,tau,blocking", MFMA_CASES, ids=[c[0] for c in MFMA_CASES])
def test_factor_parity_atomic_accumulation(name, make, tau, blocking):
    """deterministic = 0: the update terms are subtracted with atomic adds in
    whatever order they arrive; the parity bar still holds."""
    _torch()
    a, perm = make()
    say(f"[parity atomic] {name} n={a.n} tau={tau}")
    o, h = run_pair(a, tau, perm, deterministic=0, **blocking)
    compare_factors(o, h)
    check_apply_and_solve(o, h, a)
    h.close()


AGG_CASES = [c for c in CASES if c[0] in ("cd2d_nd", "cd2d_scalar", "cd3d_12_nd", "el3d_10_nd",
                                          "random_sparse", "wide_blocks")]


@pytest.mark.parametrize("name,make,tau,blocking", AGG_CASES, ids=[c[0] for c in AGG_CASES])
def test_aggregated_parity(name, make, tau, blocking):
    """Progressive aggregation (Sec. 3.5): the final partition and patterns
    equal the oracle's (which merges during its sweep), the merged factors
    agree within the tolerance, and the solver takes the same iterations."""
    _torch()
    a, perm = make()
    say(f"[agg] {name} n={a.n} tau={tau} {blocking}")
    o, h = run_pair(a, tau, perm, agg=True, **blocking)
    assert h.stats()["merges"] == o.stats()["merges"]
    fl = compare_factors(o, h)
    assert len(fl.starts) < len(fl.starts_initial) or o.stats()["merges"] == 0
    check_apply_and_solve(o, h, a)
    h.close()


def test_aggregation_to_the_cap():
    """Diagonal input (everything kept): every block merges with the next
    until the width cap, as the closed form of the decision says."""
    _torch()
    from paper_1908_10169_amd import bilu
    n = 300
    a = mg.dense_to_csr(np.diag(np.linspace(1.0, 2.0, n)))
    say(f"[agg] diagonal n={n}")
    o, h = run_pair(a, 0.0, None, agg=True, use_cosine=False, use_ilu1t=False)
    st = h.export().starts
    assert np.array_equal(np.diff(st), [128, 128, 44])
    compare_factors(o, h)
    del bilu


def test_tau_zero_is_exact_lu():
    torch = _torch()
    a = mg.grid2d_random_blocks(12, 2, 4.0, seed=2)
    say(f"[parity] tau0 n={a.n}")
    o, h = run_pair(a, 0.0)
    compare_factors(o, h)
    b = a.matvec(np.ones(a.n)) + np.arange(a.n) / a.n
    bd = torch.from_numpy(b).cuda()
    yd = torch.empty_like(bd)
    h.apply(bd, yd)
    h.sync()
    x_ref = np.linalg.solve(a.to_dense(), b)
    assert np.linalg.norm(yd.cpu().numpy() - x_ref) <= 1e-12 * np.linalg.norm(x_ref)
    xl = torch.zeros_like(bd)
    info = h.fgmres(bd, xl, restart=30, rtol=1e-8)
    assert info["iterations"] == 1


def test_perturbed_pivot_blocks():
    torch = _torch()
    # a few nodes get a singular (all-ones) diagonal block and exact-zero
    # couplings to earlier nodes, so their pivot block is that singular
    # block; one more gets an all-zero diagonal block (zero column path)
    a = mg.grid2d_random_blocks(10, 2, 3.0, seed=9)
    A = a.to_dense()
    for node, val in ((0, 0.0), (17, 1.0), (40, 1.0), (63, -2.0)):
        s = slice(2 * node, 2 * node + 2)
        A[s, s] = val
        A[s, :2 * node] = 0.0
        A[:2 * node, s] = 0.0
    mask = a.to_dense() != 0
    b = mg.dense_to_csr(A, mask)
    say(f"[parity] perturbed n={b.n}")
    o, h = run_pair(b, 1e-2, use_ilu1t=False)
    assert o.stats()["perturbed_blocks"] == 4
    assert h.stats()["perturbed_blocks"] == o.stats()["perturbed_blocks"]
    compare_factors(o, h)
    # the perturbations are what is left of A on the kept pattern: the
    # device and the oracle measure the same defect
    rk, rk_o = h.kept_residual(), o.kept_residual()
    assert rk_o > 1e-6 and abs(rk - rk_o) <= 1e-10 * rk_o, (rk, rk_o)


def test_tiny_and_ragged():
    _torch()
    for n in (1, 2, 5, 37):
        a = mg.random_sparse(n, 0.3, seed=n, diag_shift=2.0)
        say(f"[parity] tiny n={n}")
        o, h = run_pair(a, 1e-2)
        compare_factors(o, h)
        check_apply_and_solve(o, h, a, restart=5)


def test_deterministic_rerun():
    torch = _torch()
    w = mg.workload("cd3d_12_b4")
    from paper_1908_10169_amd import bilu
    outs = []
    for _ in range(2):
        h = bilu.Bilu(ordering=bilu.ORDER_NATURAL, use_aggregation=False)
        h.analyze(w.a, pre_perm=w.perm)
        h.factor(w.tau)
        f = h.export()
        outs.append(b"".join(x.tobytes() for x in f.L + f.W + f.D))
        h.close()
    assert outs[0] == outs[1]
    del torch


@pytest.mark.parametrize("name", ["cd3d_12_b4", "el3d_10_b3", "cd2d_32x32_b3"])
def test_fast_and_general_paths_identical(name):
    """The staged path for narrow blocks (data in LDS, or in global scratch)
    and the general path perform the same arithmetic in the same order: the
    factors agree bit for bit."""
    _torch()
    from paper_1908_10169_amd import bilu
    w = mg.workload(name)
    say(f"[paths] {name} n={w.a.n}")
    outs = []
    for path in (0, 1, 2):
        h = bilu.Bilu(ordering=bilu.ORDER_NATURAL, use_aggregation=False, factor_path=path)
        h.analyze(w.a, pre_perm=w.perm)
        h.factor(w.tau)
        f = h.export()
        outs.append((f.starts.tobytes(), [r.tobytes() for r in f.R], [c.tobytes() for c in f.C],
                     b"".join(x.tobytes() for x in f.L + f.W + f.D)))
        h.close()
    assert outs[0] == outs[1] == outs[2]


@pytest.mark.parametrize("name", ["cd3d_12_b4", "cd3d_24_b4", "el3d_16_b3"])
def test_apply_paths_identical(name):
    """The apply as one dataflow launch (blocks in workgroup order, or by
    ticket) and as one launch per dependency level give the same bits, and
    no dataflow wait timed out."""
    torch = _torch()
    from paper_1908_10169_amd import bilu
    w = mg.workload(name)
    say(f"[apply paths] {name} n={w.a.n}")
    rng = np.random.default_rng(11)
    x = torch.from_numpy(rng.standard_normal(w.a.n)).cuda()
    outs = []
    for path in (0, 1, 2):
        h = bilu.Bilu(ordering=bilu.ORDER_NATURAL, apply_path=path)
        h.analyze(w.a, pre_perm=w.perm)
        h.factor(w.tau)
        y = torch.empty_like(x)
        for _ in range(2):  # a second call reuses the plan and buffers
            h.apply(x, y)
        h.sync()
        assert h.stats()["apply_faults"] == 0
        outs.append(y.cpu().numpy().tobytes())
        h.close()
    assert outs[0] == outs[1] == outs[2]


def test_state_errors():
    torch = _torch()
    from paper_1908_10169_amd import bilu
    h = bilu.Bilu()
    x = torch.zeros(10, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(bilu.BiluError) as e:
        h.apply(x, y)
    assert e.value.status == bilu.BILU_ERR_STATE
    with pytest.raises(bilu.BiluError) as e:
        h.factor(1e-2)
    assert e.value.status == bilu.BILU_ERR_STATE


@pytest.mark.parametrize("agg,det", [(False, 1), (True, 1), (True, 0)],
                         ids=["plain", "aggregated", "aggregated-atomic"])
def test_full_size_cd3d_64(agg, det):
    """The 64^3 x 4 convection-diffusion workload at full size, in the
    benchmark's configuration: partition, every pattern, factors within the
    tolerance and the FGMRES iteration count equal the oracle's."""
    torch = _torch()
    from oracle import Oracle, OracleOptions
    from paper_1908_10169_amd import bilu
    w = mg.workload("cd3d_64_b4")
    say(f"[full] cd3d_64_b4 n={w.a.n} nnz={w.a.nnz} aggregation={agg} deterministic={det}")
    h = bilu.Bilu(ordering=bilu.ORDER_NATURAL, use_aggregation=agg, deterministic=det)
    h.analyze(w.a, pre_perm=w.perm)
    h.factor(w.tau)
    o = Oracle()
    assert o.run(w.a, OracleOptions(tau=w.tau, use_aggregation=agg), pre_perm=w.perm) == 0
    assert h.stats()["ilu1t_host"] == 0  # the partition came from the device kernels
    assert h.stats()["merges"] == o.stats()["merges"]
    say("[full] oracle done")
    fl, fo = h.export(), o.factors()
    assert np.array_equal(fl.perm, fo.perm)
    assert np.array_equal(fl.starts_initial, fo.starts_initial)
    assert np.array_equal(fl.starts, fo.starts)
    for name in ("R", "C"):
        x, y = getattr(fl, name), getattr(fo, name)
        assert np.array_equal([len(v) for v in x], [len(v) for v in y]), name
        assert np.array_equal(np.concatenate(x), np.concatenate(y)), name
    for name in ("L", "W", "D"):
        x = np.concatenate([v.ravel() for v in getattr(fl, name)])
        y = np.concatenate([v.ravel() for v in getattr(fo, name)])
        assert np.linalg.norm(x - y) <= TOL * np.linalg.norm(y), name
    worst = max_block_error(fl, fo)
    say(f"[full] largest per-block relative difference {worst:.2e}")
    assert worst <= BLOCK_TOL
    b = w.a.matvec(np.ones(w.a.n))
    _, info_o = o.fgmres(b, restart=w.restart, rtol=1e-8)
    bd = torch.from_numpy(b).cuda()
    xd = torch.zeros_like(bd)
    info_l = h.fgmres(bd, xd, restart=w.restart, rtol=1e-8)
    assert info_l["converged"] and info_l["iterations"] == info_o["iterations"]
    h.close()


@pytest.mark.parametrize("name", ["cd2d_32x32_b3", "el3d_10_b3"])
def test_drop_log_equals_oracle(name):
    """drop_log_margin: the logged near-tie decisions (block, candidate,
    norm) are the oracle's decisions within that margin of tau."""
    _torch()
    from oracle import Oracle, OracleOptions
    from paper_1908_10169_amd import bilu
    w = mg.workload(name)
    margin = 0.05
    say(f"[drop log] {name} margin={margin}")
    h = bilu.Bilu(ordering=bilu.ORDER_NATURAL, use_aggregation=False, drop_log_margin=margin)
    h.analyze(w.a, pre_perm=w.perm)
    h.factor(w.tau)
    fl = h.export()
    o = Oracle()
    assert o.run(w.a, OracleOptions(tau=w.tau, use_aggregation=False), pre_perm=w.perm) == 0
    log = o.droplog()
    rel = np.abs(log["norm"] - w.tau) / w.tau
    sel = rel <= margin
    edge = np.abs(rel - margin) <= 1e-9  # rounding may put these on either side
    want = {(int(b), int(i) if k == 0 else ~int(i)): nrm
            for b, i, k, nrm, s_, e in zip(log["block"], log["index"], log["kind"], log["norm"],
                                           sel, edge) if s_ and not e}
    got = {}
    assert fl.drop_log is not None and len(want) > 0
    for b, i, nrm in zip(fl.drop_log["block"], fl.drop_log["index"], fl.drop_log["norm"]):
        got[(int(b), int(i))] = float(nrm)
    edge_keys = {(int(b), int(i) if k == 0 else ~int(i))
                 for b, i, k, e in zip(log["block"], log["index"], log["kind"], edge) if e}
    assert set(got) - edge_keys == set(want)
    for key, nrm in want.items():
        assert abs(got[key] - nrm) <= 1e-10 * nrm
    assert h.stats()["drop_log_count"] == len(got)
    h.close()


def test_multilevel_nd_ordering_parity():
    """The multilevel nested dissection option on an irregular mesh: the
    library's own analysis orders as the host preprocessing does, and the
    sweep on that order matches the oracle (which takes it as the caller's
    permutation)."""
    _torch()
    from paper_1908_10169_amd import bilu
    a = mg.random_geometric(1500, k=7, dim=3, b=3, seed=8)
    tau = 1e-2
    say(f"[multilevel nd] irregular mesh n={a.n} nnz={a.nnz}")
    perm, _, _ = bilu.preprocess(a, tau, ordering=bilu.ORDER_ND_MULTILEVEL)
    h = bilu.Bilu(ordering=bilu.ORDER_ND_MULTILEVEL, use_aggregation=True)
    h.analyze(a)
    h.factor(tau)
    assert np.array_equal(h.export().perm, perm)
    h.close()
    o, h2 = run_pair(a, tau, pre_perm=perm, agg=True)
    compare_factors(o, h2)
    h2.close()
