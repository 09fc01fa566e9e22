"""Pins of the maximum weight matching oracle (Sec. 3.1, eq. (mwm)).

None re-types the oracle: optimality is checked by brute force over all
permutations, against SciPy's sparse assignment solver, and by linear
programming duality (dual feasibility plus complementary slackness certify
an optimal assignment); eq. (mwm)'s properties are checked on the scaled
matrix itself.
"""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import min_weight_full_bipartite_matching

from oracle.mwm import apply_mwm, mwm, mwm_scalings
from paper_1908_10169_amd import matgen as mg


def random_csr(n, density, seed, zero_diag=False, spread=6.0):
    """Nonsymmetric sparse matrix with magnitudes over ~spread decades and a
    random permutation guaranteeing a perfect matching."""
    rng = np.random.default_rng(seed)
    mask = rng.random((n, n)) < density
    mask[np.arange(n), rng.permutation(n)] = True
    if zero_diag:
        mask[np.arange(n), np.arange(n)] = False
        mask[np.arange(n), (np.arange(n) + 1) % n] = True
    vals = rng.choice([-1.0, 1.0], size=(n, n)) * 10.0 ** rng.uniform(-spread / 2, spread / 2, (n, n))
    A = np.where(mask, vals, 0.0)
    return dense_to_csr(A), A


def dense_to_csr(A):
    s = sp.csr_matrix(A)
    s.sort_indices()
    return mg.Csr(A.shape[0], s.indptr.astype(np.int64), s.indices.astype(np.int32),
                  s.data.astype(np.float64))


def brute_force_cost(A):
    n = A.shape[0]
    absA = np.abs(A)
    colmax = absA.max(axis=0)
    best = np.inf
    for p in itertools.permutations(range(n)):
        vals = absA[np.arange(n), p]
        if np.all(vals > 0):
            best = min(best, float(np.sum(np.log(colmax[list(p)]) - np.log(vals))))
    return best


@pytest.mark.parametrize("seed", range(6))
def test_mwm_brute_force(seed):
    a, A = random_csr(6, 0.45, seed)
    sigma, u, v, colmax, cost = mwm(a)
    assert sorted(sigma.tolist()) == list(range(6))
    assert cost == pytest.approx(brute_force_cost(A), abs=1e-10)


@pytest.mark.parametrize("n,seed,zd", [(40, 1, False), (120, 2, True), (300, 3, False)])
def test_mwm_matches_scipy(n, seed, zd):
    a, A = random_csr(n, 6.0 / n, seed, zero_diag=zd)
    sigma, _, _, colmax, cost = mwm(a)
    absA = np.abs(A)
    cm = absA.max(axis=0)
    rows, cols = np.nonzero(absA)
    # +1 on every cost: the optimum is unchanged (n edges in every
    # assignment) and no cost is the solver's implicit zero
    c = np.log(cm[cols]) - np.log(absA[rows, cols]) + 1.0
    g = sp.csr_matrix((c, (rows, cols)), shape=(n, n))
    r_ind, c_ind = min_weight_full_bipartite_matching(g)
    scipy_cost = float(np.sum(g[r_ind, c_ind])) - n
    assert cost == pytest.approx(scipy_cost, abs=1e-9 * max(1.0, abs(scipy_cost)))


@pytest.mark.parametrize("n,seed", [(50, 4), (200, 5)])
def test_mwm_duality_certificate(n, seed):
    """u_i + v_j <= c_ij on every entry and = on the matching: an optimal
    assignment by LP duality."""
    a, A = random_csr(n, 5.0 / n, seed, zero_diag=True)
    sigma, u, v, colmax, cost = mwm(a)
    absA = np.abs(A)
    rows, cols = np.nonzero(absA)
    c = np.log(colmax[cols]) - np.log(absA[rows, cols])
    slack = c - u[rows] - v[cols]
    assert slack.min() >= -1e-9
    assert np.abs(c_matched(absA, colmax, sigma) - u - v[sigma]).max() <= 1e-9
    # the dual objective equals the primal cost
    assert float(u.sum() + v.sum()) == pytest.approx(cost, abs=1e-8)


def c_matched(absA, colmax, sigma):
    n = absA.shape[0]
    return np.log(colmax[sigma]) - np.log(absA[np.arange(n), sigma])


@pytest.mark.parametrize("n,seed", [(30, 6), (150, 7)])
def test_mwm_scaled_matrix(n, seed):
    """eq. (mwm): |a^_ij| <= 1 and |a^_ii| = 1 for D_l A D_r Pi."""
    a, A = random_csr(n, 6.0 / n, seed, zero_diag=True)
    sigma, dl, dr = mwm_scalings(a)
    H = np.abs(apply_mwm(a, sigma, dl, dr))
    assert H.max() <= 1.0 + 1e-12
    assert np.abs(np.diag(H) - 1.0).max() <= 1e-12


def test_mwm_identity_on_diagonally_maximal():
    """A diagonal that holds every column maximum (far above the rest) is
    the matching, at cost 0."""
    a, A = random_csr(25, 0.2, 8)
    A = A.copy()
    np.fill_diagonal(A, 1e9 * (1.0 + np.arange(25)))
    sigma, u, v, colmax, cost = mwm(dense_to_csr(A))
    assert np.array_equal(sigma, np.arange(25))
    assert cost == pytest.approx(0.0, abs=1e-12)


def test_mwm_structurally_singular():
    # rows 1 and 2 reach columns 0 and 1 only, row 0 also column 2: matched
    A = np.array([[1.0, 2.0, 1.0], [3.0, 4.0, 0.0], [5.0, 6.0, 0.0]])
    sigma, *_ = mwm(dense_to_csr(A))
    assert sorted(sigma.tolist()) == [0, 1, 2]
    assert sigma[0] == 2
    # rows 0 and 1 both reach column 0 only: no perfect matching
    B = np.array([[1.0, 0.0, 0.0], [2.0, 0.0, 0.0], [3.0, 4.0, 5.0]])
    with pytest.raises(ValueError):
        mwm(dense_to_csr(B))
