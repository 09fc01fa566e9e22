"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Every test here runs on the CPU.  None of them re-types the oracle's own
formulas: each checks a closed form, an invariant, a textbook special case
or an independent brute-force computation (dense NumPy).
"""
import numpy as np
import pytest

from oracle import Oracle, OracleOptions, cosine_groups, ilu1t_blocks, perturb_invert, \
    fgmres_plain, sqmr_plain
from paper_1908_10169_amd import matgen as mg

NO_BLOCKING = dict(use_cosine=False, use_ilu1t=False, use_aggregation=False)


# ---------------------------------------------------------------------------
# helpers: dense assembly of the oracle's factors (independent of its code)
# ---------------------------------------------------------------------------
def assemble(o: Oracle):
    """Dense L (unit), S (block diag, S_K = D_K^{-1}), U (unit) and perm."""
    f = o.factors()
    n = o.n
    L = np.eye(n)
    U = np.eye(n)
    S = np.zeros((n, n))
    for k in range(len(f.starts) - 1):
        a, b = f.starts[k], f.starts[k + 1]
        S[a:b, a:b] = np.linalg.inv(f.D[k])
        if len(f.R[k]):
            L[np.ix_(f.R[k], np.arange(a, b))] = f.L[k]
        if len(f.C[k]):
            U[np.ix_(np.arange(a, b), f.C[k])] = f.D[k] @ f.W[k]
    return L, S, U, f


def permuted_dense(a, perm):
    A = a.to_dense()
    return A[np.ix_(perm, perm)]


def scalar_crout_ilu(A, mask, tau):
    """Alg. 1 of the paper (Crout ILU), dense arrays with a pattern mask.

    Column k of L and row k of U are formed from the already computed parts;
    l_ik is dropped when |l_ik| <= tau |l_kk|, u_ki when |u_ki| <= tau |u_kk|.
    Returns unit L, upper U (with pivots) and their kept masks."""
    n = A.shape[0]
    L = np.zeros((n, n)); Lm = np.zeros((n, n), bool)
    U = np.zeros((n, n)); Um = np.zeros((n, n), bool)
    for k in range(n):
        col = {i: A[i, k] for i in range(k, n) if mask[i, k]}
        for j in range(k):
            if Um[j, k]:
                for i in range(k, n):
                    if Lm[i, j]:
                        col[i] = col.get(i, 0.0) - L[i, j] * U[j, k]
        lkk = col.get(k, 0.0)
        for i, v in col.items():
            if i > k and abs(v) > tau * abs(lkk):
                L[i, k] = v / lkk
                Lm[i, k] = True
        L[k, k] = 1.0
        Lm[k, k] = True
        row = {i: A[k, i] for i in range(k, n) if mask[k, i]}
        for j in range(k):
            if Lm[k, j]:
                for i in range(k, n):
                    if Um[j, i]:
                        row[i] = row.get(i, 0.0) - L[k, j] * U[j, i]
        ukk = row.get(k, 0.0)
        U[k, k] = ukk
        Um[k, k] = True
        for i, v in row.items():
            if i > k and abs(v) > tau * abs(ukk):
                U[k, i] = v
                Um[k, i] = True
    return L, Lm, U, Um


def tridiag(n, seed, diag=4.0):
    rng = np.random.default_rng(seed)
    A = np.diag(diag + rng.uniform(0, 1, n))
    A += np.diag(rng.choice([-1.0, 1.0], n - 1) * rng.uniform(0.5, 1, n - 1), 1)
    A += np.diag(rng.choice([-1.0, 1.0], n - 1) * rng.uniform(0.5, 1, n - 1), -1)
    return A


# ---------------------------------------------------------------------------
# P1: tau = 0 keeps every nonzero: the factorization is exact LU
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("blocking", [NO_BLOCKING, {}])
def test_p1_tau0_is_exact_lu(blocking):
    a = mg.random_sparse(200, 0.03, seed=3, diag_shift=8.0)
    o = Oracle()
    assert o.run(a, OracleOptions(tau=0.0, **blocking)) == 0
    A = a.to_dense()
    b = A @ np.ones(a.n) + np.arange(a.n) / a.n
    y = o.apply(b)
    x_ref = np.linalg.solve(A, b)
    assert np.linalg.norm(y - x_ref) <= 1e-12 * np.linalg.norm(x_ref)
    L, S, U, f = assemble(o)
    P = permuted_dense(a, f.perm)
    assert np.linalg.norm(L @ S @ U - P) <= 1e-14 * np.linalg.norm(P) * 10
    _, info = o.fgmres(A @ np.ones(a.n), restart=30, rtol=1e-8)
    assert info["converged"] and info["iterations"] == 1


# ---------------------------------------------------------------------------
# P2: with scalar blocks and no blocking strategy BILU is the scalar Crout ILU
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("tau", [1e-1, 1e-2, 1e-3])
@pytest.mark.parametrize("seed", [11, 12])
def test_p2_scalar_blocks_equal_alg1(tau, seed):
    a = mg.random_sparse(90, 0.06, seed=seed, diag_shift=3.0)
    A = a.to_dense()
    mask = np.zeros_like(A, bool)
    rows = np.repeat(np.arange(a.n), np.diff(a.rowptr))
    mask[rows, a.colind] = True
    Lr, Lm, Ur, Um = scalar_crout_ilu(A, mask, tau)
    o = Oracle()
    assert o.run_partition(a, np.arange(a.n + 1), OracleOptions(tau=tau, **NO_BLOCKING)) == 0
    f = o.factors()
    for k in range(a.n):
        ref_rows = np.flatnonzero(Lm[k + 1:, k]) + k + 1
        assert np.array_equal(f.R[k], ref_rows)
        assert np.allclose(f.L[k][:, 0], Lr[ref_rows, k], rtol=1e-13, atol=1e-15)
        ref_cols = np.flatnonzero(Um[k, k + 1:]) + k + 1
        assert np.array_equal(f.C[k], ref_cols)
        assert np.allclose(f.W[k][0], Ur[k, ref_cols], rtol=1e-13, atol=1e-15)
        assert abs(f.D[k][0, 0] * Ur[k, k] - 1.0) < 1e-13


# ---------------------------------------------------------------------------
# P3: banded input with nothing dropped: BILU equals (block) LU
# ---------------------------------------------------------------------------
def test_p3_tridiagonal_equals_lu():
    A = tridiag(120, seed=5)
    a = mg.dense_to_csr(A)
    o = Oracle()
    assert o.run(a, OracleOptions(tau=1e-3)) == 0
    log = o.droplog()
    assert log["kept"][np.flatnonzero(log["norm"] > 0)].all()
    b = np.sin(np.arange(a.n))
    assert np.linalg.norm(o.apply(b) - np.linalg.solve(A, b)) <= 1e-13 * np.linalg.norm(b)


def test_p3_block_tridiagonal_equals_block_lu():
    rng = np.random.default_rng(9)
    nb, bs = 40, 3
    n = nb * bs
    A = np.zeros((n, n))
    for k in range(nb):
        s = slice(k * bs, (k + 1) * bs)
        A[s, s] = rng.uniform(-1, 1, (bs, bs)) + 6 * np.eye(bs)
        if k + 1 < nb:
            t = slice((k + 1) * bs, (k + 2) * bs)
            A[s, t] = rng.uniform(-1, 1, (bs, bs))
            A[t, s] = rng.uniform(-1, 1, (bs, bs))
    a = mg.dense_to_csr(A)
    o = Oracle()
    assert o.run(a, OracleOptions(tau=1e-4)) == 0
    b = np.cos(np.arange(n))
    assert np.linalg.norm(o.apply(b) - np.linalg.solve(A, b)) <= 1e-13 * np.linalg.norm(b)


# ---------------------------------------------------------------------------
# P4: fill stays inside the structural recurrence and the symbolic LU
# ---------------------------------------------------------------------------
def symbolic_block_lu(P, starts):
    """Boolean block LU of the pattern of P: kept patterns with no dropping."""
    n = P.shape[0]
    F = P != 0
    nb = len(starts) - 1
    for k in range(nb):
        a, b = starts[k], starts[k + 1]
        rows = np.flatnonzero(F[b:, a:b].any(axis=1)) + b
        cols = np.flatnonzero(F[a:b, b:].any(axis=0)) + b
        F[np.ix_(rows, cols)] = True
    return F


@pytest.mark.parametrize("tau", [1e-1, 1e-2])
def test_p4_fill_bound(tau):
    a = mg.grid3d_convdiff(b=2, dims=(5, 5, 4), seed=4)
    perm = mg.node_perm_to_scalar(mg.grid_nd_node_order((5, 5, 4)), 2)
    o = Oracle()
    assert o.run(a, OracleOptions(tau=tau, use_aggregation=False), pre_perm=perm) == 0
    f = o.factors()
    P = permuted_dense(a, f.perm)
    F = symbolic_block_lu(P, f.starts)
    for k in range(len(f.starts) - 1):
        s, e = f.starts[k], f.starts[k + 1]
        assert F[np.ix_(f.R[k], np.arange(s, e))].any(axis=1).all()
        assert F[np.ix_(np.arange(s, e), f.C[k])].any(axis=0).all()
        # local recurrence: rows of A(:,K) below K plus rows of the J that update K
        allowed = set(np.flatnonzero((P[e:, s:e] != 0).any(axis=1)) + e)
        for j in range(k):
            if np.any((f.C[j] >= s) & (f.C[j] < e)):
                allowed |= set(int(i) for i in f.R[j] if i >= e)
        assert set(int(i) for i in f.R[k]) <= allowed


# ---------------------------------------------------------------------------
# P5: (L S U)_Omega = A_Omega on the computed pattern, for any tau
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("tau", [3e-1, 1e-2, 1e-4])
@pytest.mark.parametrize("agg", [False, True])
def test_p5_kept_pattern_identity(tau, agg):
    a = mg.grid2d_random_blocks(12, 3, 4.5, seed=1)
    o = Oracle()
    assert o.run(a, OracleOptions(tau=tau, use_aggregation=agg)) == 0
    assert o.kept_residual() <= 1e-13


# ---------------------------------------------------------------------------
# P6: every dropped row/column is at or below tau, every kept one above,
# recomputed densely from the factors (Schur complement of the leading part)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("tau", [2e-1, 3e-2])
@pytest.mark.parametrize("norm", ["inf", "two"])
def test_p6_drop_rule(tau, norm):
    a = mg.grid2d_random_blocks(8, 2, 3.0, seed=2)
    o = Oracle()
    assert o.run(a, OracleOptions(tau=tau, use_aggregation=False,
                                  drop_norm=0 if norm == "inf" else 1)) == 0
    rnorm = (lambda X, ax: np.abs(X).max(axis=ax)) if norm == "inf" else \
        (lambda X, ax: np.sqrt((X * X).sum(axis=ax)))
    L, S, U, f = assemble(o)
    P = permuted_dense(a, f.perm)
    W = S @ U
    n = a.n
    checked = differs = 0
    for k in range(len(f.starts) - 1):
        s, e = f.starts[k], f.starts[k + 1]
        D = f.D[k]
        Cpan = P[e:, s:e] - L[e:, :s] @ W[:s, s:e]
        Lc = Cpan @ D
        nr = rnorm(Lc, 1)
        kept = np.zeros(n - e, bool)
        kept[f.R[k] - e] = True
        margin = 1e-12 * max(1.0, np.abs(Lc).max(initial=0))
        assert np.all(nr[kept] > tau - margin)
        assert np.all(nr[~kept] <= tau + margin)
        assert np.allclose(f.L[k], Lc[kept], rtol=1e-11, atol=1e-13)
        Rpan = P[s:e, e:] - L[s:e, :s] @ W[:s, e:]
        Uc = D @ Rpan
        nc = rnorm(Uc, 0)
        keptc = np.zeros(n - e, bool)
        keptc[f.C[k] - e] = True
        assert np.all(nc[keptc] > tau - margin)
        assert np.all(nc[~keptc] <= tau + margin)
        assert np.allclose(f.W[k], Rpan[:, keptc], rtol=1e-11, atol=1e-13)
        checked += (~kept).sum() + (~keptc).sum()
        # kept by the 2-norm although the max-abs norm is below tau
        differs += int(np.sum(kept & (np.abs(Lc).max(axis=1) <= tau)))
        differs += int(np.sum(keptc & (np.abs(Uc).max(axis=0) <= tau)))
    assert checked > 0
    assert (differs > 0) == (norm == "two")


# ---------------------------------------------------------------------------
# P7: cosine blocking recovers the node partition of node-blocked stencils
# ---------------------------------------------------------------------------
def _stencil_pattern(dims, offs, b, numbering, seed=0):
    dims = np.asarray(dims)
    N = int(np.prod(dims))
    coords = np.stack(np.unravel_index(np.arange(N), tuple(dims[::-1])), axis=1)[:, ::-1]
    rng = np.random.default_rng(seed)
    node_label = np.arange(N) if numbering != "random" else rng.permutation(N)
    idx = {tuple(c): i for i, c in enumerate(coords)}
    n = N * b

    def sid(v, c):
        lv = node_label[v]
        return c * N + lv if numbering == "component" else b * lv + c

    M = np.zeros((n, n), bool)
    for v, c in enumerate(coords):
        for o in offs:
            w = idx.get(tuple(c + o))
            if w is None:
                continue
            for c1 in range(b):
                for c2 in range(b):
                    M[sid(v, c1), sid(w, c2)] = True
    nodes = [frozenset(sid(v, c) for c in range(b)) for v in range(N)]
    return M, set(nodes)


TRI = [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1), (1, -1), (-1, 1)]


@pytest.mark.parametrize("kind,dims", [("star", (6, 5)), ("star", (4, 4, 3)), ("box", (5, 5, 5)),
                                       ("tri", (6, 6))])
@pytest.mark.parametrize("b", [1, 2, 3, 4])
@pytest.mark.parametrize("numbering", ["node", "component", "random"])
def test_p7_cosine_node_partition(kind, dims, b, numbering):
    if kind == "tri":
        offs = np.array(TRI)
    else:
        offs = mg._offsets(len(dims), kind)
    M, nodes = _stencil_pattern(dims, offs, b, numbering)
    a = mg.dense_to_csr(M.astype(float), M)
    perm, gs, nig = cosine_groups(a)
    assert nig == 0
    groups = {frozenset(int(x) for x in perm[gs[g]:gs[g + 1]]) for g in range(len(gs) - 1)}
    if b == 1:
        # scalar stencils: a group may only join rows with identical or near patterns;
        # no two grid points of a star/box/tri stencil satisfy the test
        assert all(len(g) == 1 for g in groups)
    else:
        assert groups == nodes


def test_p7_cosine_filter_ignores_dense_rows():
    # an arrow matrix: the dense row/column exceed mu + 2 sigma and stay alone
    n = 40
    M = np.eye(n, dtype=bool)
    M[0, :] = True
    M[:, 0] = True
    for i in range(1, n - 1, 2):
        M[i, i + 1] = M[i + 1, i] = True
    a = mg.dense_to_csr(M.astype(float), M)
    perm, gs, nig = cosine_groups(a)
    assert nig == 1
    g0 = [list(perm[gs[g]:gs[g + 1]]) for g in range(len(gs) - 1) if 0 in perm[gs[g]:gs[g + 1]]]
    assert g0 == [[0]]


# ---------------------------------------------------------------------------
# P8: ILU(1,tau) growth closed forms
# ---------------------------------------------------------------------------
def test_p8_diagonal_blocks_of_five():
    # diagonal: r = s = 0, c = l, f = l^2: grow iff l' <= 5
    a = mg.dense_to_csr(np.diag(np.arange(1.0, 24.0)))
    bs = ilu1t_blocks(a, np.arange(a.n + 1), 1e-2)
    assert list(np.diff(bs)) == [5, 5, 5, 5, 3]


def test_p8_tridiagonal_blocks_of_five():
    # large off-diagonals: r = s = 1, c = 3l, f = (l+2) l: grow iff l' <= 5
    n = 23
    A = 4 * np.eye(n) + np.eye(n, k=1) + np.eye(n, k=-1)
    bs = ilu1t_blocks(mg.dense_to_csr(A), np.arange(n + 1), 1e-2)
    assert list(np.diff(bs)) == [5, 5, 5, 5, 3]


@pytest.mark.parametrize("n,bmax", [(40, 128), (40, 16)])
def test_p8_dense_single_block(n, bmax):
    # dense with all entries above tau|a_kk|: f = c, always grows (up to the cap)
    A = np.ones((n, n)) + n * np.eye(n)
    bs = ilu1t_blocks(mg.dense_to_csr(A), np.arange(n + 1), 1e-2, max_block=bmax)
    expect = [bmax] * (n // bmax) + ([n % bmax] if n % bmax else [])
    assert list(np.diff(bs)) == expect


# ---------------------------------------------------------------------------
# P9: progressive aggregation closed forms: nu - mu = 2p <= 2(p+q)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind", ["diag", "tri"])
def test_p9_aggregation_to_cap(kind):
    n, bmax = 30, 8
    A = 4 * np.eye(n)
    if kind == "tri":
        A += np.eye(n, k=1) + np.eye(n, k=-1)
    o = Oracle()
    opts = OracleOptions(tau=1e-2, use_cosine=False, use_ilu1t=False, use_aggregation=True,
                         max_block=bmax)
    assert o.run(mg.dense_to_csr(A), opts) == 0
    assert list(np.diff(o.starts())) == [8, 8, 8, 6]
    rec = o.mergelog()
    # every test with a width-1 block K: mu, nu as the closed form says
    for k, p, q, mu, nu, merged in rec:
        assert q == 1
        if kind == "diag":
            assert (mu, nu) == (p * p + 1, (p + 1) ** 2)
        else:
            lastblk = k == n - 1
            if not lastblk:
                assert (mu, nu) == (p * p + 2 * p + 3, (p + 1) * (p + 3))
        assert merged == (p + q <= bmax)


# ---------------------------------------------------------------------------
# P10: merging preserves L S U and keeps D^ = S^{-1}
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("tau", [1e-1, 1e-2])
def test_p10_merge_preserves_product(tau):
    a = mg.grid2d_random_blocks(10, 2, 3.5, seed=6)
    o0, o1 = Oracle(), Oracle()
    opts0 = OracleOptions(tau=tau, use_aggregation=False, use_ilu1t=False)
    opts1 = OracleOptions(tau=tau, use_aggregation=True, use_ilu1t=False)
    assert o0.run(a, opts0) == 0 and o1.run(a, opts1) == 0
    assert o1.stats()["merges"] > 0
    assert np.array_equal(o0.perm(), o1.perm())
    L0, S0, U0, _ = assemble(o0)
    L1, S1, U1, _ = assemble(o1)
    M0 = L0 @ S0 @ U0
    M1 = L1 @ S1 @ U1
    assert np.linalg.norm(M1 - M0) <= 1e-14 * np.linalg.norm(M0) * 10
    # apply (uses D) inverts the product (uses S) on random vectors
    rng = np.random.default_rng(0)
    perm = o1.perm()
    for _ in range(3):
        x = rng.standard_normal(a.n)
        xp = np.empty_like(x)
        xp[perm] = o1.lsu_matvec(x[perm])
        assert np.linalg.norm(o1.apply(xp) - x) <= 1e-12 * np.linalg.norm(x)


# ---------------------------------------------------------------------------
# P11: perturbation of singular pivot blocks
# ---------------------------------------------------------------------------
def test_p11_zero_column():
    s = np.array([[2.0, 0.0, 1.0], [1.0, 0.0, 3.0], [0.5, 0.0, 1.0]])
    r, su, di = perturb_invert(s, alpha=7.0)
    assert r >= 1
    assert su[1, 1] == pytest.approx(1e-2 * 7.0, rel=0, abs=1e-15)
    assert np.allclose(su @ di, np.eye(3), atol=1e-12)


def test_p11_all_ones_2x2():
    s = np.ones((2, 2))
    r, su, di = perturb_invert(s, alpha=1.0)
    assert r == 1
    # columns: 1*1.1+0.01 = 1.11 on both diagonals; rows: 1.11*1.111+0.01
    assert np.allclose(su, [[1.24321, 1.0], [1.0, 1.24321]], rtol=0, atol=1e-14)
    assert np.allclose(su @ di, np.eye(2), atol=1e-13)


def test_p11_beta_one_reading():
    s = np.ones((2, 2))
    r, su, _ = perturb_invert(s, alpha=1.0, opts=OracleOptions(beta_one=True))
    # beta = 1: columns 1*1.1+0.01 = 1.11; rows 1.11*1.1+0.01 = 1.231
    assert np.allclose(su, [[1.231, 1.0], [1.0, 1.231]], rtol=0, atol=1e-14)


def test_p11_regular_block_untouched():
    s = np.array([[4.0, 1.0], [2.0, 3.0]])
    r, su, di = perturb_invert(s, alpha=4.0)
    assert r == 0 and np.array_equal(su, s)
    assert np.allclose(di, np.linalg.inv(s), rtol=1e-15, atol=1e-15)


# ---------------------------------------------------------------------------
# P12: apply = dense solve with the assembled preconditioner
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("agg", [False, True])
def test_p12_apply_dense(agg):
    a = mg.grid2d_random_blocks(9, 3, 4.5, seed=8)
    o = Oracle()
    assert o.run(a, OracleOptions(tau=5e-2, use_aggregation=agg)) == 0
    L, S, U, f = assemble(o)
    M = L @ S @ U
    Pm = np.eye(a.n)[:, f.perm]     # (Pm x)[perm[i]] = x[i]
    Morig = Pm @ M @ Pm.T
    x = np.random.default_rng(1).standard_normal(a.n)
    y = o.apply(x)
    assert np.linalg.norm(y - np.linalg.solve(Morig, x)) <= 1e-12 * np.linalg.norm(y)


# ---------------------------------------------------------------------------
# P13: FGMRES with M = I minimises the residual over the Krylov space
# ---------------------------------------------------------------------------
def test_p13_fgmres_minimal_residual():
    a = mg.random_sparse(60, 0.1, seed=21, diag_shift=1.5)
    A = a.to_dense()
    b = np.random.default_rng(2).standard_normal(a.n)
    m = 10
    _, info, hist = fgmres_plain(a, b, restart=m, rtol=1e-14, maxit=m)
    assert len(hist) == m
    K = np.zeros((a.n, m))
    v = b / np.linalg.norm(b)
    for j in range(m):          # orthonormal Krylov basis by repeated QR
        K[:, j] = v
        Q, _ = np.linalg.qr(K[:, :j + 1])
        v = A @ Q[:, j]
    for j in range(1, m + 1):
        Q, _ = np.linalg.qr(K[:, :j])
        AQ = A @ Q
        y, *_ = np.linalg.lstsq(AQ, b, rcond=None)
        rmin = np.linalg.norm(b - AQ @ y)
        assert hist[j - 1] == pytest.approx(rmin, rel=1e-8)
    assert np.all(np.diff(hist) <= 1e-12 * hist[0])


def _krylov_cycle(Op, r, m):
    """Residuals after 1..m steps of the minimal-residual method from residual
    r over the Krylov space K_m(Op, r), by dense least squares on an
    orthonormal basis built by repeated QR; also the coefficient vector in
    that basis after m steps.  Independent of any Givens/Hessenberg code."""
    K = np.zeros((len(r), m))
    v = r / np.linalg.norm(r)
    for j in range(m):
        K[:, j] = v
        Q, _ = np.linalg.qr(K[:, :j + 1])
        v = Op @ Q[:, j]
    res = []
    for j in range(1, m + 1):
        Q, _ = np.linalg.qr(K[:, :j])
        y, *_ = np.linalg.lstsq(Op @ Q, r, rcond=None)
        res.append(np.linalg.norm(r - Op @ (Q @ y)))
    return np.array(res), Q @ y


# ---------------------------------------------------------------------------
# P13b: restarted FGMRES(m) with M = I.  Every cycle restarts from its own
# true residual b - A x_c and minimises over K_m(A, r_c); x_{c+1} is the
# minimiser.  Several full cycles, then a partial one.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("m", [2, 3, 5])
def test_p13_restart_cycles_plain(m):
    a = mg.random_sparse(70, 0.08, seed=31, diag_shift=0.6)
    A = a.to_dense()
    b = np.random.default_rng(5).standard_normal(a.n)
    cycles = 4
    maxit = cycles * m + (m - 1 if m > 1 else 0)
    x_o, info, hist = fgmres_plain(a, b, restart=m, rtol=1e-15, maxit=maxit)
    assert info["iterations"] == maxit
    assert info["restarts"] == cycles + (1 if maxit % m else 0)
    x = np.zeros(a.n)
    it = 0
    for c in range(info["restarts"]):
        steps = min(m, maxit - it)
        r = b - A @ x
        res, d = _krylov_cycle(A, r, steps)
        # the Givens estimate of every step equals the cycle's least-squares
        # minimum from its own starting residual
        assert hist[it:it + steps] == pytest.approx(res, rel=1e-7)
        assert np.all(np.diff(res) <= 1e-12 * res[0])
        it += steps
        x = x + d
        # the next cycle restarts from the true residual of the minimiser
        assert np.linalg.norm(b - A @ x) == pytest.approx(res[-1], rel=1e-7)
    assert np.linalg.norm(x_o - x) <= 1e-7 * np.linalg.norm(x)
    assert info["rel_residual"] == pytest.approx(np.linalg.norm(b - A @ x) / np.linalg.norm(b),
                                                 rel=1e-6)
    # restarting stagnates above what unrestarted GMRES reaches in as many steps
    _, info_full, hist_full = fgmres_plain(a, b, restart=maxit, rtol=1e-15, maxit=maxit)
    assert info_full["restarts"] == 1
    assert hist_full[-1] <= hist[-1] * (1 + 1e-9)


# ---------------------------------------------------------------------------
# P13c: restarted FGMRES with the block ILU as (fixed) right preconditioner:
# cycle c minimises ||r_c - A M^{-1} Q y|| over K_m(A M^{-1}, r_c) and moves x
# by M^{-1} Q y, with M assembled densely from the factors (as in P12)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("m", [2, 3])
def test_p13_restart_cycles_preconditioned(m):
    a = mg.grid2d_random_blocks(8, 3, 3.0, seed=12)
    o = Oracle()
    assert o.run(a, OracleOptions(tau=3e-1, use_aggregation=True)) in (0,)
    L, S, U, f = assemble(o)
    Pm = np.eye(a.n)[:, f.perm]
    Minv = np.linalg.inv(Pm @ (L @ S @ U) @ Pm.T)
    A = a.to_dense()
    b = A @ np.ones(a.n)
    maxit = 4 * m + 1
    x_o, info, hist = o.fgmres(b, restart=m, rtol=1e-15, maxit=maxit, history=True)
    assert info["iterations"] == maxit and info["restarts"] == 5
    x = np.zeros(a.n)
    it = 0
    AM = A @ Minv
    for c in range(info["restarts"]):
        steps = min(m, maxit - it)
        r = b - A @ x
        res, d = _krylov_cycle(AM, r, steps)
        assert hist[it:it + steps] == pytest.approx(res, rel=1e-6)
        it += steps
        x = x + Minv @ d
    assert np.linalg.norm(x_o - x) <= 1e-6 * np.linalg.norm(x)
    # and to convergence: several cycles, true residual confirmed
    x_c, info_c = o.fgmres(b, restart=m, rtol=1e-8, maxit=500)
    assert info_c["converged"] and info_c["restarts"] >= 2
    assert np.linalg.norm(b - A @ x_c) <= 1e-8 * np.linalg.norm(b)
    assert info_c["rel_residual"] == pytest.approx(
        np.linalg.norm(b - A @ x_c) / np.linalg.norm(b), rel=1e-6)


# ---------------------------------------------------------------------------
# P5b: the kept-pattern residual itself, against a dense computation of
# ||(L S U - A)_Omega||_F / ||A||_F from the exported factors, also with a
# defect planted in one stored value (so a zero sum or a wrong Omega fails)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("which", ["L", "W"])
def test_p5_kept_residual_dense(which):
    a = mg.grid2d_random_blocks(7, 2, 3.0, seed=4)
    o = Oracle()
    assert o.run(a, OracleOptions(tau=5e-2, use_aggregation=False)) == 0

    def dense_kept():
        L, S, U, f = assemble(o)
        P = permuted_dense(a, f.perm)
        omega = np.zeros((a.n, a.n), bool)
        for k in range(len(f.starts) - 1):
            s_, e_ = f.starts[k], f.starts[k + 1]
            omega[s_:e_, s_:e_] = True
            omega[np.ix_(f.R[k], np.arange(s_, e_))] = True
            omega[np.ix_(np.arange(s_, e_), f.C[k])] = True
        E = (L @ S @ U - P)[omega]
        return np.linalg.norm(E) / np.linalg.norm(a.val), omega, P

    base, omega, P = dense_kept()
    assert base <= 1e-13 and o.kept_residual() <= 1e-13
    # Omega is strictly smaller than the full pattern of L S U (dropping)
    f = o.factors()
    k = next(k for k in range(len(f.starts) - 1) if (len(f.R[k]) if which == "L" else len(f.C[k])))
    o.plant(which, k, 0, 1e-3)
    planted, _, _ = dense_kept()
    assert planted > 1e-6
    assert o.kept_residual() == pytest.approx(planted, rel=1e-9)


# ---------------------------------------------------------------------------
# P14: determinism
# ---------------------------------------------------------------------------
def test_p14_deterministic():
    a = mg.grid2d_random_blocks()
    outs = []
    for _ in range(2):
        o = Oracle()
        assert o.run(a, OracleOptions()) == 0
        f = o.factors()
        outs.append((f.starts.tobytes(), b"".join(x.tobytes() for x in f.L),
                     b"".join(x.tobytes() for x in f.W), b"".join(x.tobytes() for x in f.D)))
    assert outs[0] == outs[1]


# ---------------------------------------------------------------------------
# The small workload converges (checked before any GPU work)
# ---------------------------------------------------------------------------
def test_cd2d_workload_converges():
    a = mg.grid2d_random_blocks(32, 3, 4.5, seed=0)
    o = Oracle()
    assert o.run(a, OracleOptions(tau=1e-2)) == 0
    b = a.matvec(np.ones(a.n))
    x, info = o.fgmres(b, restart=30, rtol=1e-8)
    assert info["converged"] and info["rel_residual"] <= 1e-8
    assert np.abs(x - 1).max() < 1e-6


# ---------------------------------------------------------------------------
# P8 (sets): at tau = 0 the ILU(1,tau) estimate is the textbook ILU(1)
# pattern: original entries plus fill created by two original entries
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [0, 1])
def test_p8_sets_tau0_are_ilu1_pattern(seed):
    from oracle import ilu1t_sets
    a = mg.random_sparse(70, 0.05, seed=seed, diag_shift=2.0)
    Pm = a.to_dense() != 0
    n = a.n
    lower = np.tril(Pm, -1).astype(int)
    upper = np.triu(Pm, 1).astype(int)
    lev1 = Pm | ((lower @ upper) > 0)   # fill (i,k) via some j < min(i,k)
    for k in range(n):
        I, J = ilu1t_sets(a, k, 0.0)
        assert np.array_equal(I, np.flatnonzero(lev1[k + 1:, k]) + k + 1)
        assert np.array_equal(J, np.flatnonzero(lev1[k, k + 1:]) + k + 1)


@pytest.mark.parametrize("tau,expect_fill,expect_orig", [(0.05, True, True), (0.07, False, True),
                                                        (0.3, False, False)])
def test_p8_sets_5point_thresholds(tau, expect_fill, expect_orig):
    # 5-point Laplacian (4, -1) on a 6x6 grid, natural order: the level-1 fill
    # at (k+nx-1, k) has size |(-1)(-1)/4| = 1/4, compared with tau*4;
    # original neighbours have size 1, compared with tau*4.
    from oracle import ilu1t_sets
    nx = 6
    n = nx * nx
    A = 4 * np.eye(n)
    for i in range(n):
        x, y = i % nx, i // nx
        if x + 1 < nx:
            A[i, i + 1] = A[i + 1, i] = -1
        if y + 1 < nx:
            A[i, i + nx] = A[i + nx, i] = -1
    a = mg.dense_to_csr(A)
    k = 2 * nx + 2                   # interior point
    I, J = ilu1t_sets(a, k, tau)
    exp = set()
    if expect_orig:
        exp |= {k + 1, k + nx}
    if expect_fill:
        exp |= {k + nx - 1}
    assert set(I.tolist()) == exp
    assert set(J.tolist()) == exp      # symmetric matrix: J~ mirrors I~


def test_p11_negative_block_sign():
    s = -np.ones((2, 2))
    r, su, _ = perturb_invert(s, alpha=1.0)
    assert r == 1
    assert np.allclose(su, [[-1.24321, -1.0], [-1.0, -1.24321]], rtol=0, atol=1e-14)


def test_p8_sets_use_the_pivot_diagonal():
    # The fill a_ki a_ij (i < k) is measured against |a_ii a_kk|: raising the
    # diagonal of the intermediate index i = k-1 to 8 makes the fill 1/(8*4)
    # of the product, below tau = 0.05 (it would pass against a_jj = 4).
    from oracle import ilu1t_sets
    nx = 6
    n = nx * nx
    A = 4 * np.eye(n)
    for i in range(n):
        x, y = i % nx, i // nx
        if x + 1 < nx:
            A[i, i + 1] = A[i + 1, i] = -1
        if y + 1 < nx:
            A[i, i + nx] = A[i + nx, i] = -1
    k = 2 * nx + 2
    A[k - 1, k - 1] = 8.0
    I, J = ilu1t_sets(mg.dense_to_csr(A), k, 0.05)
    assert set(I.tolist()) == {k + 1, k + nx}
    assert set(J.tolist()) == {k + 1, k + nx}
    I, J = ilu1t_sets(mg.dense_to_csr(A), k, 0.03)
    assert set(I.tolist()) == {k + 1, k + nx, k + nx - 1}
    assert set(J.tolist()) == {k + 1, k + nx, k + nx - 1}


# ---------------------------------------------------------------------------
# P15: refactorization with frozen patterns (a variant for matrix sequences)
# ---------------------------------------------------------------------------
def _new_values(a, seed):
    """The same pattern, values scaled entrywise by 1 + 0.3 U(-1, 1)."""
    rng = np.random.default_rng(seed)
    return a.val * (1.0 + 0.3 * rng.uniform(-1.0, 1.0, a.val.size))


@pytest.mark.parametrize("blocking", [NO_BLOCKING, {}])
def test_p15_frozen_tau0_is_exact_lu_of_the_new_matrix(blocking):
    """With tau = 0 the stored pattern is the full LU fill, so the frozen
    refactorization on new values is the exact LU of the new matrix."""
    a = mg.random_sparse(200, 0.03, seed=3, diag_shift=8.0)
    o = Oracle()
    assert o.run(a, OracleOptions(tau=0.0, **blocking)) == 0
    v2 = _new_values(a, 5)
    assert o.refactor_frozen(v2) == 0
    a2 = mg.Csr(a.n, a.rowptr, a.colind, v2)
    A2 = a2.to_dense()
    b = A2 @ np.ones(a.n)
    y = o.apply(b)
    x_ref = np.linalg.solve(A2, b)
    assert np.linalg.norm(y - x_ref) <= 1e-11 * np.linalg.norm(x_ref)
    assert o.final_residual() <= 1e-14


@pytest.mark.parametrize("tau,agg", [(1e-2, False), (1e-1, False), (1e-2, True), (1e-1, True)])
def test_p15_frozen_keeps_the_pattern_identity(tau, agg):
    """For any tau, with or without merged blocks: the new factor reproduces
    the new matrix on the stored positions, (L S U)_Omega = A_Omega, and
    the patterns are the old ones."""
    w = mg.workload("cd2d_32x32_b3")
    o = Oracle()
    assert o.run(w.a, OracleOptions(tau=tau, use_aggregation=agg), pre_perm=w.perm) == 0
    f0 = o.factors()
    assert o.refactor_frozen(_new_values(w.a, 7)) == 0
    f1 = o.factors()
    assert np.array_equal(f0.starts, f1.starts)
    for k in range(len(f0.starts) - 1):
        assert np.array_equal(f0.R[k], f1.R[k]) and np.array_equal(f0.C[k], f1.C[k])
    assert o.final_residual() <= 1e-13
    # and a plain definition of the identity, entry by entry on a sample
    L, S, U, f = assemble(o)
    a2 = mg.Csr(w.a.n, w.a.rowptr, w.a.colind, _new_values(w.a, 7))
    P = permuted_dense(a2, f.perm)
    M = L @ S @ U
    K0 = 5
    q = f1.starts[K0 + 1] - f1.starts[K0]
    for r in range(f1.starts[K0], f1.starts[K0] + q):
        for j in f1.C[K0]:
            assert abs(M[r, j] - P[r, j]) <= 1e-12 * np.abs(P).max()


def test_p15_frozen_with_the_same_values_reproduces_the_factor():
    """Without merges the sweep's kept values are the Crout values on its
    own pattern, so the frozen refactorization of the same matrix gives
    them back (to rounding)."""
    w = mg.workload("cd2d_32x32_b3")
    o = Oracle()
    assert o.run(w.a, OracleOptions(tau=1e-2, use_aggregation=False), pre_perm=w.perm) == 0
    f0 = o.factors()
    assert o.refactor_frozen(w.a.val) == 0
    f1 = o.factors()
    for name in ("L", "W", "D"):
        x = np.concatenate([v.ravel() for v in getattr(f1, name)])
        y = np.concatenate([v.ravel() for v in getattr(f0, name)])
        assert np.linalg.norm(x - y) <= 1e-13 * np.linalg.norm(y), name


# ---------------------------------------------------------------------------
# P16: simplified QMR (Sec. 5), the Krylov solver for symmetric A and M.
# Pins: (a) for symmetric A and M, QMR with the two-sided Lanczos process
# and right preconditioner M (SciPy's qmr, an independent implementation
# with its own recurrences) produces the same iterates in exact
# arithmetic; (b) finite termination after as many steps as A has distinct
# eigenvalues; (c) the QMR bound ||b - A x_k||_2 <= sqrt(k + 1) tau_k;
# (d) an exact preconditioner (tau = 0) solves in one step; (e) the stop is
# taken at the first step whose backward error meets the tolerance.
# ---------------------------------------------------------------------------
def _sym_indefinite(n, eigs, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return Q @ np.diag(eigs) @ Q.T, rng.standard_normal(n)


def _sym_elasticity(side, shift):
    a = mg.grid3d_elasticity(side, 3, seed=2, pert=0.0, shift=shift)
    perm = mg.node_perm_to_scalar(
        mg.grid_nd_node_order((side,) * 3, dissect_separators=False), 3)
    return a, perm


def _scipy_qmr(A, b, k, prec=None):
    import scipy.sparse.linalg as sla
    kw = {}
    if prec is not None:
        n = len(b)
        eye = sla.LinearOperator((n, n), matvec=lambda v: v, rmatvec=lambda v: v)
        M2 = sla.LinearOperator((n, n), matvec=prec, rmatvec=prec)
        kw = dict(M1=eye, M2=M2)
    x, _ = sla.qmr(A, b, maxiter=k, rtol=1e-300, atol=0.0, **kw)
    return x


@pytest.mark.parametrize("k", [1, 2, 4, 8, 12])
def test_p16_sqmr_plain_matches_qmr(k):
    rng = np.random.default_rng(11)
    eigs = np.concatenate([rng.uniform(1.0, 5.0, 32), -rng.uniform(1.0, 3.0, 8)])
    A, b = _sym_indefinite(40, eigs, 4)
    x, info, _ = sqmr_plain(mg.dense_to_csr(A), b, tol=0.0, maxit=k)
    assert info["iterations"] == k and not info["converged"]
    xs = _scipy_qmr(A, b, k)
    assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)


@pytest.mark.parametrize("k", [1, 3, 6])
def test_p16_sqmr_preconditioned_matches_qmr(k):
    """M from the block ILU of a symmetric indefinite matrix: the sweep on
    symmetric data is symmetric (L^T and U share their patterns), so M is
    symmetric up to rounding and QMR with right preconditioner M agrees."""
    a, perm = _sym_elasticity(6, -0.1)
    o = Oracle()
    assert o.run(a, OracleOptions(tau=1e-2, use_aggregation=True), pre_perm=perm) == 0
    st = o.stats()
    assert st["nnz_L"] == st["nnz_W"]
    b = a.matvec(np.linspace(-1.0, 1.0, a.n))
    x, info = o.sqmr(b, tol=0.0, maxit=k)
    assert info["iterations"] == k
    xs = _scipy_qmr(a.to_dense(), b, k, prec=o.apply)
    assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)


def test_p16_sqmr_finite_termination():
    """Three distinct eigenvalues, one of them negative: the Krylov space
    stops growing after three steps, where the QMR iterate is the solution."""
    A, b = _sym_indefinite(30, np.repeat([2.0, -1.0, 5.0], 10), 6)
    a = mg.dense_to_csr(A)
    _, info2, _ = sqmr_plain(a, b, tol=1e-12, maxit=2)
    assert not info2["converged"] and info2["rel_residual"] > 1e-3
    x, info, _ = sqmr_plain(a, b, tol=1e-12, maxit=10)
    assert info["converged"] and info["iterations"] == 3
    assert np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-11 * np.linalg.norm(x)


def test_p16_sqmr_quasi_residual_bound():
    a, perm = _sym_elasticity(5, -0.2)
    o = Oracle()
    assert o.run(a, OracleOptions(tau=3e-2), pre_perm=perm) == 0
    b = a.matvec(np.ones(a.n))
    A = a.to_dense()
    _, info, taus = o.sqmr(b, tol=0.0, maxit=12, history=True)
    assert len(taus) == 12
    for k in range(1, 13):
        x, _ = o.sqmr(b, tol=0.0, maxit=k)
        r = np.linalg.norm(b - A @ x)
        assert r <= np.sqrt(k + 1) * taus[k - 1] * (1 + 1e-10), k


def test_p16_sqmr_exact_preconditioner_one_step():
    a, perm = _sym_elasticity(4, -0.3)
    o = Oracle()
    assert o.run(a, OracleOptions(tau=0.0), pre_perm=perm) == 0
    b = a.matvec(np.cos(np.arange(a.n)))
    x, info = o.sqmr(b, tol=1e-12, maxit=5)
    assert info["converged"] and info["iterations"] == 1


def test_p16_sqmr_stops_at_the_first_step_below_tol():
    """The returned eta is the infinity-norm backward error of the returned
    x (checked with the Rigal-Gaches perturbation built from it), it meets
    the tolerance, and one step fewer does not."""
    a, perm = _sym_elasticity(6, 0.1)
    o = Oracle()
    assert o.run(a, OracleOptions(tau=1e-2), pre_perm=perm) == 0
    b = a.matvec(np.ones(a.n))
    A = a.to_dense()
    tol = 1e-6
    x, info = o.sqmr(b, tol=tol)
    k = info["iterations"]
    assert info["converged"] and info["eta"] <= tol and k > 1
    # (A + E) x = b + f with ||E|| = eta ||A||, ||f|| = eta ||b|| (inf-norms)
    r = b - A @ x
    an = np.abs(A).sum(axis=1).max()
    den = an * np.abs(x).max() + np.abs(b).max()
    j = int(np.argmax(np.abs(x)))
    z = np.zeros(a.n)
    z[j] = np.sign(x[j])
    E = np.outer(r, z) * (an / den)
    f = -r * (np.abs(b).max() / den)
    assert np.abs((A + E) @ x - (b + f)).max() <= 1e-12 * np.abs(b).max()
    assert np.isclose(np.abs(E).sum(axis=1).max(), info["eta"] * an, rtol=1e-8)
    assert np.isclose(np.abs(f).max(), info["eta"] * np.abs(b).max(), rtol=1e-8)
    _, info1 = o.sqmr(b, tol=tol, maxit=k - 1)
    assert not info1["converged"] and info1["eta"] > tol


# ---------------------------------------------------------------------------
# P17: the symmetric matching of Sec. 5 (eq. (smwm)) and groups built on the
# compressed companion matrix.  Pins: (a) the Duff-Pralet property: the
# symmetrized scaling of a maximum product matching keeps every |a^_ij| <= 1
# and the matched entries, hence the 2x2 pivots' off-diagonal entries and
# the fixed points' diagonal entries, at magnitude one; (b) the cycle rule on
# hand-solved 3x3 cases; (c) all-1x1 units reduce the unit pipeline to the
# plain one; (d) no group or block splits a unit.
# ---------------------------------------------------------------------------
def _scaled_dense(a, d):
    return d[:, None] * a.to_dense() * d[None, :]


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_p17_symmetric_scaling_duff_pralet(seed):
    from oracle import mwm_scalings, symmetric_units
    rng = np.random.default_rng(seed)
    n = 40
    A = rng.standard_normal((n, n)) * (rng.uniform(size=(n, n)) < 0.15)
    A = A + A.T + np.diag(np.where(rng.uniform(size=n) < 0.6, 0.0, rng.standard_normal(n)))
    A[np.arange(n), np.arange(n)] = np.where(np.abs(np.diag(A)) > 0, np.diag(A), 0.0)
    a = mg.dense_to_csr(A, mask=(A != 0))
    sigma, dl, dr = mwm_scalings(a)
    d, order, us = symmetric_units(a, sigma, dl, dr)
    Ah = _scaled_dense(a, d)
    assert np.abs(Ah).max() <= 1.0 + 1e-12
    assert np.allclose(np.abs(Ah[np.arange(n), sigma]), 1.0, atol=1e-12)
    assert np.array_equal(np.sort(order), np.arange(n))
    w = np.diff(us)
    assert set(w.tolist()) <= {1, 2}
    for u in range(len(w)):
        idx = order[us[u]:us[u + 1]]
        if len(idx) == 2:
            assert abs(abs(Ah[idx[0], idx[1]]) - 1.0) <= 1e-12
            assert idx[0] < idx[1]
        elif sigma[idx[0]] == idx[0]:
            assert abs(abs(Ah[idx[0], idx[0]]) - 1.0) <= 1e-12


def test_p17_odd_cycle_rule():
    """[[0,1,1],[1,0,1],[1,1,c]]: for c = 0.5 the best transversal is a
    3-cycle (product 1 against 0.5 for (0 1)(2)); its member with the
    largest scaled diagonal (index 2) is the 1x1 pivot, {0, 1} the 2x2 one.
    For c = 0 all diagonals tie and the first in cycle order (0) stays."""
    from oracle import mwm_scalings, symmetric_units
    for c, want_order, want_starts in ((0.5, [0, 1, 2], [0, 2, 3]), (0.0, [0, 1, 2], [0, 1, 3])):
        A = np.array([[0.0, 1.0, 1.0], [1.0, 0.0, 1.0], [1.0, 1.0, c]])
        a = mg.dense_to_csr(A, mask=(A != 0))
        sigma, dl, dr = mwm_scalings(a)
        assert sorted(sigma.tolist()) == [0, 1, 2] and all(sigma[i] != i for i in range(3))
        _, order, us = symmetric_units(a, sigma, dl, dr)
        assert order.tolist() == want_order and us.tolist() == want_starts, c


def test_p17_singleton_units_reduce_to_the_plain_run():
    w = mg.workload("cd2d_32x32_b3")
    o1, o2 = Oracle(), Oracle()
    opts = OracleOptions(tau=1e-2, use_aggregation=True)
    assert o1.run(w.a, opts, pre_perm=w.perm) == 0
    assert o2.run(w.a, opts, pre_perm=w.perm, unit_starts=np.arange(w.a.n + 1)) == 0
    f1, f2 = o1.factors(), o2.factors()
    assert np.array_equal(f1.perm, f2.perm) and np.array_equal(f1.starts, f2.starts)
    assert np.array_equal(o1.group_starts(), o2.group_starts())
    for x, y in zip(f1.L + f1.W + f1.D, f2.L + f2.W + f2.D):
        assert np.array_equal(x, y)


def _kkt_symmetric(side, tau, agg=True):
    from oracle import mwm_scalings, symmetric_units
    a, order, m = mg.kkt_elasticity(side)
    sigma, dl, dr = mwm_scalings(a)
    d, uorder, us = symmetric_units(a, sigma, dl, dr, pre=order)
    # D A D on A's own pattern (stored zeros stay)
    rows = np.repeat(np.arange(a.n), np.diff(a.rowptr))
    ah = mg.Csr(a.n, a.rowptr, a.colind, (d[rows] * a.val) * d[a.colind])
    o = Oracle()
    assert o.run(ah, OracleOptions(tau=tau, use_aggregation=agg), pre_perm=uorder,
                 unit_starts=us) == 0
    return a, order, o, d, uorder, us


def test_p17_units_stay_whole():
    a, _, o, d, uorder, us = _kkt_symmetric(5, 1e-2)
    perm = o.factors().perm
    pos = np.empty(a.n, dtype=np.int64)
    pos[perm] = np.arange(a.n)
    for bounds in (o.group_starts(), o.factors().starts_initial, o.factors().starts):
        block_of = np.searchsorted(bounds, np.arange(a.n), side="right") - 1
        for u in range(len(us) - 1):
            idx = uorder[us[u]:us[u + 1]]
            assert len(set(block_of[pos[idx]].tolist())) == 1
            assert np.all(np.diff(pos[idx]) == 1)   # contiguous, in unit order


def test_p17_matching_removes_the_perturbations():
    """Constraints ordered before their unknowns: the plain factorization
    meets zero pivots (perturbed blocks) and SQMR needs hundreds of steps;
    with the symmetric matching the 2x2 pivots keep every block regular."""
    a, order, m = mg.kkt_elasticity(6)
    b = a.matvec(np.ones(a.n))
    o = Oracle()
    assert o.run(a, OracleOptions(tau=1e-2), pre_perm=order) == 0
    _, plain = o.sqmr(b, tol=1e-8, maxit=1000)
    assert o.stats()["perturbed_blocks"] > 0
    a, _, o2, d, _, _ = _kkt_symmetric(6, 1e-2)
    assert o2.stats()["perturbed_blocks"] == 0
    xh, sym = o2.sqmr(d * b, tol=1e-8, maxit=1000)
    assert sym["converged"] and plain["converged"]
    assert sym["iterations"] * 10 < plain["iterations"]
    x = d * xh
    assert np.linalg.norm(b - a.matvec(x)) <= 1e-6 * np.linalg.norm(b)


def _ilu1t_partition_dense(P, mask, dvec, ustart, tau, max_block=128):
    """The ILU(1,tau) block guess of Sec. 3.4 written from its definition
    on dense arrays (independent of the oracle's sparse loops): the
    estimated rows I_k of column k of L and columns J_k of row k of U,
    then units added while the dense count stays within the scalar one."""
    n = P.shape[0]

    def sets(k):
        I, J = set(), set()
        for i in range(k + 1, n):
            if mask[i, k] and abs(P[i, k]) >= tau * abs(dvec[k]):
                I.add(i)
            if mask[k, i] and abs(P[k, i]) >= tau * abs(dvec[k]):
                J.add(i)
        for j in range(k):
            if mask[j, k]:
                for i in range(k + 1, n):
                    if mask[i, j] and abs(P[i, j] * P[j, k]) >= tau * abs(dvec[j] * dvec[k]):
                        I.add(i)
            if mask[k, j]:
                for i in range(k + 1, n):
                    if mask[j, i] and abs(P[k, j] * P[j, i]) >= tau * abs(dvec[j] * dvec[k]):
                        J.add(i)
        return I, J

    nu = len(ustart) - 1
    starts = [0]
    u = 0
    while u < nu:
        s0, e0 = ustart[u], ustart[u + 1]
        rows, cols, c = set(), set(), 0
        for k in range(s0, e0):
            I, J = sets(k)
            rows |= {i for i in I if i >= e0}
            cols |= {j for j in J if j >= e0}
            c += len(I) + len(J) + 1
        width = e0 - s0
        u += 1
        while u < nu:
            s1, e1 = ustart[u], ustart[u + 1]
            w2 = width + (e1 - s1)
            if w2 > max_block:
                break
            rows2 = {i for i in rows if i >= e1}
            cols2 = {j for j in cols if j >= e1}
            c2 = c
            for k in range(s1, e1):
                I, J = sets(k)
                rows2 |= {i for i in I if i >= e1}
                cols2 |= {j for j in J if j >= e1}
                c2 += len(I) + len(J) + 1
            f2 = (len(rows2) + len(cols2) + w2) * w2
            if 3 * f2 <= 4 * c2 or f2 <= c2 + 4 * w2:
                rows, cols, c, width = rows2, cols2, c2, w2
                u += 1
            else:
                break
        starts.append(starts[-1] + width)
    return np.array(starts)


@pytest.mark.parametrize("tau", [1e-2, 1e-1])
def test_p17_ilu1t_thresholds_of_2x2_pivots(tau):
    """The reading for 2x2 pivots (Sec. 5): both scalars of a 2x2 pivot take
    the pivot block's largest magnitude in place of |a_kk|.  The oracle's
    partition of a saddle point (units = the symmetric matching's pivots,
    no cosine step) equals the dense definition with that reading, and
    differs from the one with the scalar diagonals (constraint rows have
    none)."""
    from oracle import mwm_scalings, symmetric_units
    a, order, m = mg.kkt_elasticity(4)
    sigma, dl, dr = mwm_scalings(a)
    d, uorder, us = symmetric_units(a, sigma, dl, dr, pre=order)
    rows = np.repeat(np.arange(a.n), np.diff(a.rowptr))
    ah = mg.Csr(a.n, a.rowptr, a.colind, (d[rows] * a.val) * d[a.colind])
    o = Oracle()
    assert o.run(ah, OracleOptions(tau=tau, use_cosine=False, use_aggregation=False),
                 pre_perm=uorder, unit_starts=us) == 0
    assert np.array_equal(o.perm(), uorder)
    mask_full = np.zeros((a.n, a.n), dtype=bool)
    mask_full[rows, a.colind] = True
    Pd = ah.to_dense()[np.ix_(uorder, uorder)]
    mask = mask_full[np.ix_(uorder, uorder)]
    scalar = np.diag(Pd).copy()
    paired = scalar.copy()
    for u in range(len(us) - 1):
        if us[u + 1] - us[u] == 2:
            i, p = us[u], us[u] + 1
            blk = np.abs(Pd[np.ix_([i, p], [i, p])])
            paired[i] = paired[p] = blk.max()
    want = _ilu1t_partition_dense(Pd, mask, paired, us, tau)
    assert np.array_equal(o.starts_initial(), want)
    other = _ilu1t_partition_dense(Pd, mask, scalar, us, tau)
    assert not np.array_equal(other, want)


@pytest.mark.parametrize("k", [2, 5])
def test_p16_sqmr_with_the_symmetric_matching_matches_qmr(k):
    """M from the symmetric variant's pipeline (D A D of a saddle point,
    2x2 pivots as units): still symmetric up to rounding, so SQMR equals
    QMR with right preconditioner M on the scaled system."""
    a, order, o, d, uorder, us = _kkt_symmetric(4, 1e-2)
    rows = np.repeat(np.arange(a.n), np.diff(a.rowptr))
    ah = mg.Csr(a.n, a.rowptr, a.colind, (d[rows] * a.val) * d[a.colind])
    b = d * a.matvec(np.ones(a.n))
    x, info = o.sqmr(b, tol=0.0, maxit=k)
    assert info["iterations"] == k
    xs = _scipy_qmr(ah.to_dense(), b, k, prec=o.apply)
    assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)


# P11b: the symmetrized perturbation (Sec. 5, sym_perturb): each column's
# selected entry and its mirror take the same value, so a symmetric pivot
# block stays symmetric.
def test_p11_symmetric_all_ones_2x2():
    """[[1,1],[1,1]] is singular; column 0 selects its diagonal (2|1| >= |1|),
    column 1 too, each becomes 1 (1 + rho beta) + tau alpha with beta = 1."""
    s = np.ones((2, 2))
    alpha, rho, tau = 3.0, 1e-1, 1e-2
    r, su, di = perturb_invert(s, alpha=alpha, opts=OracleOptions(sym_perturb=True))
    d = 1.0 * (1.0 + rho * 1.0) + tau * alpha
    assert r == 1
    assert np.array_equal(su, np.array([[d, 1.0], [1.0, d]]))
    assert np.allclose(di @ su, np.eye(2), atol=1e-14)


def test_p11_symmetric_keeps_symmetry():
    """A symmetric singular 3x3 block whose row 2 is twice row 1: the
    symmetric rule perturbs each column's diagonal once (2|m_jj| >= the
    column's largest entry), so S stays symmetric bit for bit and matches
    the closed form; the column-then-row rule perturbs the diagonals a
    second time in its row pass."""
    s = np.array([[4.0, 1.0, 2.0], [1.0, 10.0, 20.0], [2.0, 20.0, 40.0]])
    alpha, rho, tau = 1.0, 1e-1, 1e-2
    r, su, di = perturb_invert(s, alpha=alpha, opts=OracleOptions(sym_perturb=True))
    assert r == 1 and np.array_equal(su, su.T)
    want = s.copy()
    for j in range(3):
        beta = np.abs(s[:, j]).max()
        want[j, j] = s[j, j] * (1.0 + rho * beta) + tau * alpha
    assert np.array_equal(su, want)
    assert np.allclose(su @ di, np.eye(3), atol=1e-12)
    r2, su2, _ = perturb_invert(s, alpha=alpha)
    assert r2 == 1 and not np.array_equal(su2, su)
