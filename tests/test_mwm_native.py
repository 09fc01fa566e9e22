"""The library's host maximum weight matching (bilu_mwm, Sec. 3.1) against
the oracle and against eq. (mwm)'s properties.  CPU only: no GPU is used.

For random real magnitudes the optimal matching is unique, so the library
and the oracle must return the same permutation and the same optimal cost;
the duals (hence the scalings) are not unique, so each side's scalings are
checked against eq. (mwm) itself.
"""
import numpy as np
import pytest

from oracle.mwm import apply_mwm, mwm as oracle_mwm
from paper_1908_10169_amd import bilu
from test_oracle_mwm import dense_to_csr, random_csr


def cost_of(A, sigma):
    absA = np.abs(A)
    cm = absA.max(axis=0)
    n = A.shape[0]
    return float(np.sum(np.log(cm[sigma]) - np.log(absA[np.arange(n), sigma])))


@pytest.mark.parametrize("n,seed,zd", [(6, 0, False), (40, 1, True), (300, 2, False), (800, 3, True)])
def test_mwm_native_equals_oracle(n, seed, zd):
    a, A = random_csr(n, min(0.45, 6.0 / n), seed, zero_diag=zd)
    sig_o, _, _, _, cost_o = oracle_mwm(a)
    sigma, dl, dr = bilu.mwm(a)
    assert np.array_equal(np.sort(sigma), np.arange(n))
    assert cost_of(A, sigma) == pytest.approx(cost_o, abs=1e-9 * max(1.0, abs(cost_o)))
    assert np.array_equal(sigma, sig_o)
    H = np.abs(apply_mwm(a, sigma, dl, dr))
    assert H.max() <= 1.0 + 1e-12
    assert np.abs(np.diag(H) - 1.0).max() <= 1e-12


def test_mwm_native_larger():
    """A 20,000-row nonsymmetric stencil-like matrix with zero diagonal
    entries: eq. (mwm) holds on every stored entry."""
    rng = np.random.default_rng(9)
    n = 20000
    rows, cols = [], []
    for d in (-101, -3, -1, 1, 2, 97):
        i = np.arange(max(0, -d), min(n, n - d))
        rows.append(i)
        cols.append(i + d)
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = rng.choice([-1.0, 1.0], rows.size) * 10.0 ** rng.uniform(-3, 3, rows.size)
    import scipy.sparse as sp
    s = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    s.sort_indices()
    from paper_1908_10169_amd import matgen as mg
    a = mg.Csr(n, s.indptr.astype(np.int64), s.indices.astype(np.int32), s.data)
    sigma, dl, dr = bilu.mwm(a)
    assert np.array_equal(np.sort(sigma), np.arange(n))
    r = np.repeat(np.arange(n), np.diff(a.rowptr))
    mag = np.abs(a.val) * dl[r] * dr[a.colind]
    assert mag.max() <= 1.0 + 1e-12
    on = a.colind == sigma[r]
    assert np.abs(mag[on] - 1.0).max() <= 1e-12 and on.sum() == n


def test_mwm_native_singular_and_invalid():
    B = np.array([[1.0, 0.0, 0.0], [2.0, 0.0, 0.0], [3.0, 4.0, 5.0]])
    with pytest.raises(bilu.BiluError) as e:
        bilu.mwm(dense_to_csr(B))
    assert e.value.status == bilu.BILU_ERR_SINGULAR
