"""CPU checks of the C-ABI library: it loads, exports every declared symbol,
and its host-only structural preprocessing equals the oracle's."""
import os
import re

import numpy as np
import pytest

from paper_1908_10169_amd import bilu, matgen as mg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "bilu.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bilu_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = bilu.load()
    names = declared_symbols()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(bilu.EXPORTED) == names


def test_default_options_are_the_papers():
    o = bilu.default_options()
    assert (o.use_cosine, o.use_ilu1t, o.use_aggregation) == (1, 1, 1)
    assert o.cos_eps == 0.8 and o.perturb_tau == 1e-2 and o.perturb_rho == 1e-1
    assert o.max_block == 128


WORKLOADS = ["cd2d_32x32_b3", "cd3d_12_b4", "el3d_10_b3"]


@pytest.mark.parametrize("name", WORKLOADS)
@pytest.mark.parametrize("blocking", [dict(), dict(use_cosine=False),
                                      dict(use_ilu1t=False)])
def test_preprocess_matches_oracle(name, blocking):
    from oracle import Oracle, OracleOptions
    w = mg.workload(name)
    perm, gs, bs = bilu.preprocess(w.a, w.tau, pre_perm=w.perm, ordering=bilu.ORDER_NATURAL,
                                   **blocking)
    o = Oracle()
    assert o.run(w.a, OracleOptions(tau=w.tau, use_aggregation=False, **blocking),
                 pre_perm=w.perm) == 0
    assert np.array_equal(perm, o.perm())
    assert np.array_equal(gs, o.group_starts())
    assert np.array_equal(bs, o.starts_initial())


@pytest.mark.parametrize("tau", [0.0, 1e-3, 1e-1])
def test_preprocess_tau_and_natural_numbering(tau):
    from oracle import Oracle, OracleOptions
    a = mg.grid2d_random_blocks(16, 2, 3.0, seed=5)
    perm, gs, bs = bilu.preprocess(a, tau, ordering=bilu.ORDER_NATURAL)
    o = Oracle()
    assert o.run(a, OracleOptions(tau=tau, use_aggregation=False)) == 0
    assert np.array_equal(perm, o.perm()) and np.array_equal(bs, o.starts_initial())


def test_nested_dissection_ordering_is_a_block_permutation():
    a = mg.grid3d_convdiff(b=2, dims=(9, 8, 7), seed=3)
    perm, gs, bs = bilu.preprocess(a, 1e-2, ordering=bilu.ORDER_ND)
    assert np.array_equal(np.sort(perm), np.arange(a.n))
    # every cosine group is one node: its members are consecutive old indices
    for g in range(len(gs) - 1):
        mem = perm[gs[g]:gs[g + 1]]
        assert len(mem) == 2 and mem[1] == mem[0] + 1 and mem[0] % 2 == 0


def test_nested_dissection_reduces_fill():
    """The project ordering should beat the lexicographic one on a 3D grid
    in exact (symbolic) block LU fill of the compressed graph."""
    dims = (8, 8, 8)
    a = mg.grid3d_convdiff(b=1, dims=dims, seed=3)
    perm_nd, _, _ = bilu.preprocess(a, 1e-2, ordering=bilu.ORDER_ND, use_cosine=False)
    A = a.to_dense() != 0

    def fill(p):
        F = A[np.ix_(p, p)].copy()
        n = len(p)
        for k in range(n):
            rows = np.flatnonzero(F[k + 1:, k]) + k + 1
            cols = np.flatnonzero(F[k, k + 1:]) + k + 1
            F[np.ix_(rows, cols)] = True
        return F.sum()

    assert fill(perm_nd) < 0.8 * fill(np.arange(a.n))


@pytest.mark.parametrize("bad", ["unsorted", "oob", "nan", "perm"])
def test_invalid_input_is_rejected(bad):
    a = mg.grid2d_random_blocks(4, 2, 3.0, seed=1)
    rp, ci, v = a.rowptr.copy(), a.colind.copy(), a.val.copy()
    pre = None
    if bad == "unsorted":
        ci[0], ci[1] = ci[1], ci[0]
    elif bad == "oob":
        ci[3] = a.n
    elif bad == "nan":
        v[5] = np.nan
    else:
        pre = np.zeros(a.n, dtype=np.int64)
    b = mg.Csr(a.n, rp, ci, v)
    with pytest.raises(bilu.BiluError) as e:
        bilu.preprocess(b, 1e-2, pre_perm=pre)
    assert e.value.status == bilu.BILU_ERR_INVALID


def test_geometric_nd_orders():
    """The workloads' geometric nested dissection is a permutation of the grid
    nodes in both separator forms, and it is a nested dissection: the last
    nodes (the top separator plane) split the rest into two groups that no
    stencil couples (all 27 neighbours)."""
    dims = (9, 8, 7)
    n = int(np.prod(dims))
    coords = np.stack(np.unravel_index(np.arange(n), dims[::-1]), axis=1)[:, ::-1]
    for sep in (True, False):
        order = mg.grid_nd_node_order(dims, dissect_separators=sep)
        assert np.array_equal(np.sort(order), np.arange(n))
        # top separator: the middle plane of the longest axis, ordered last
        ax = int(np.argmax(dims))
        mid = dims[ax] // 2
        plane = coords[:, ax] == mid
        k = int(plane.sum())
        assert np.array_equal(np.sort(order[-k:]), np.flatnonzero(plane))
        left = set(np.flatnonzero(coords[:, ax] < mid).tolist())
        first = order[:-k]
        pos = {v: i for i, v in enumerate(first)}
        # every node below the plane comes before every node above it
        above = [pos[v] for v in first if v not in left]
        below = [pos[v] for v in first if v in left]
        assert max(below) < min(above)
    # the two forms differ only inside separators
    a = mg.grid_nd_node_order(dims, dissect_separators=True)
    b = mg.grid_nd_node_order(dims, dissect_separators=False)
    assert not np.array_equal(a, b)


def test_binding_rejects_bad_tensors():
    """The binding refuses tensors that would make a kernel access memory out
    of bounds, before anything reaches the library (raw pointers cross it)."""
    import torch
    from paper_1908_10169_amd.bilu import _check_vectors
    n = 16
    ok = torch.zeros(n, dtype=torch.float64)
    cases = [
        ((("x", torch.zeros(n, dtype=torch.float32)), ("y", ok.clone())), "dtype"),
        ((("x", torch.zeros(n + 1, dtype=torch.float64)), ("y", ok.clone())), "elements"),
        ((("x", torch.zeros(2 * n, dtype=torch.float64)[::2]), ("y", ok.clone())), "contiguous"),
        ((("x", ok), ("y", ok)), "overlaps"),
        ((("x", torch.zeros(2 * n, dtype=torch.float64)[:n]), ("y", ok.clone())), "device"),
        ((("x", np.zeros(n)), ("y", ok.clone())), "torch tensor"),
    ]
    for named, what in cases:
        with pytest.raises((ValueError, TypeError), match=what):
            _check_vectors(n, *named)
    buf = torch.zeros(2 * n, dtype=torch.float64)
    with pytest.raises(ValueError, match="overlaps"):
        _check_vectors(n, ("x", buf[:n]), ("y", buf[n // 2:n // 2 + n]))


def test_tuning_table_reader(tmp_path):
    """bilu_load_tuning reads the tuner's JSON (flat numeric entries, other
    keys ignored), rejects out-of-range fields without touching the loaded
    table, and clears with an empty path."""
    import json
    from paper_1908_10169_amd import bilu
    good = {"version": 1, "entries": [
        dict(precision=0, width_class=0, reproducible=1, workers_per_cu=0, update_mfma=0,
             factor_path=0, apply_path=0, deterministic=1, relative_time=1.0),
        dict(precision=1, width_class=0, reproducible=0, workers_per_cu=1, update_mfma=1,
             factor_path=2, apply_path=1, deterministic=0, relative_time=0.9)],
        "notes": [{"workloads": ["x"], "default_ms": {"x": 1.0}}]}
    p = tmp_path / "t.json"
    p.write_text(json.dumps(good))
    assert bilu.load_tuning(str(p)) == 2
    bad = dict(good, entries=[dict(good["entries"][0], apply_path=7)])
    q = tmp_path / "bad.json"
    q.write_text(json.dumps(bad))
    with pytest.raises(bilu.BiluError):
        bilu.load_tuning(str(q))
    # a reproducible entry must keep the ordered accumulation
    bad2 = dict(good, entries=[dict(good["entries"][0], deterministic=0)])
    q.write_text(json.dumps(bad2))
    with pytest.raises(bilu.BiluError):
        bilu.load_tuning(str(q))
    assert bilu.load().bilu_tuning_entries() == 2
    with pytest.raises(bilu.BiluError):
        bilu.load_tuning(str(tmp_path / "missing.json"))
    assert bilu.load_tuning(None) == 0


def _symbolic_fill(a, p):
    A = a.to_dense() != 0
    F = A[np.ix_(p, p)].copy()
    for k in range(len(p)):
        rows = np.flatnonzero(F[k + 1:, k]) + k + 1
        cols = np.flatnonzero(F[k, k + 1:]) + k + 1
        F[np.ix_(rows, cols)] = True
    return int(F.sum())


def test_multilevel_nd_is_a_block_permutation_and_deterministic():
    a = mg.random_geometric(700, k=7, dim=2, b=2, seed=4)
    p1, gs, _ = bilu.preprocess(a, 1e-2, ordering=bilu.ORDER_ND_MULTILEVEL)
    p2, _, _ = bilu.preprocess(a, 1e-2, ordering=bilu.ORDER_ND_MULTILEVEL)
    assert np.array_equal(p1, p2)
    assert np.array_equal(np.sort(p1), np.arange(a.n))
    # the ordering only moves the cosine groups: the same groups as in the
    # natural order, each contiguous
    pn, gsn, _ = bilu.preprocess(a, 1e-2, ordering=bilu.ORDER_NATURAL)
    groups = lambda p, s: {frozenset(p[s[g]:s[g + 1]].tolist()) for g in range(len(s) - 1)}
    assert groups(p1, gs) == groups(pn, gsn)


def test_multilevel_nd_beats_level_structure_on_an_irregular_mesh():
    """On a k-nearest-neighbour mesh (no grid structure for breadth-first
    levels to follow) the multilevel separators give clearly less exact
    block-LU fill than the level-structure ones, and both far less than the
    natural order."""
    a = mg.random_geometric(900, k=7, dim=2, b=1, seed=2)
    fills = {}
    for name, o in (("natural", bilu.ORDER_NATURAL), ("level", bilu.ORDER_ND),
                    ("multilevel", bilu.ORDER_ND_MULTILEVEL)):
        perm, _, _ = bilu.preprocess(a, 1e-2, ordering=o, use_cosine=False)
        fills[name] = _symbolic_fill(a, perm)
    assert fills["multilevel"] < 0.85 * fills["level"], fills
    assert fills["level"] < 0.3 * fills["natural"], fills


def _sym_cases():
    rng = np.random.default_rng(12)
    n = 41   # odd, zero diagonal: the matching must hold an odd cycle
    A = rng.standard_normal((n, n)) * (rng.uniform(size=(n, n)) < 0.12)
    A = np.triu(A, 1)
    A = A + A.T
    A[np.arange(n - 1), np.arange(1, n)] = A[np.arange(1, n), np.arange(n - 1)] = 0.7
    zd = mg.dense_to_csr(A)
    kkt5 = mg.kkt_elasticity(5)
    kkt6 = mg.kkt_elasticity(6, constraints_first=False)
    return {"zero_diagonal_41": (zd, None), "kkt5": (kkt5[0], kkt5[1]),
            "kkt6_after": (kkt6[0], kkt6[1])}


@pytest.mark.parametrize("name", ["zero_diagonal_41", "kkt5", "kkt6_after"])
@pytest.mark.parametrize("max_block,use_cosine", [(128, True), (5, True), (128, False)])
def test_symmetric_matching_preprocess_matches_oracle(name, max_block, use_cosine):
    """use_mwm = 2: the library's symmetric matching, unit-aware cosine
    groups and ILU(1,tau) partition equal the oracle's on D A D, with the
    library's matching (sigma, D_l, D_r from bilu_mwm; the duals are not
    unique) handed to the oracle's pivot rule."""
    from oracle import Oracle, OracleOptions, symmetric_units
    a, order = _sym_cases()[name]
    tau = 1e-2
    sigma, dl, dr = bilu.mwm(a)
    d, uorder, us = symmetric_units(a, sigma, dl, dr, pre=order)
    # D A D on A's own pattern (stored zeros stay)
    rows = np.repeat(np.arange(a.n), np.diff(a.rowptr))
    ah = mg.Csr(a.n, a.rowptr, a.colind, (d[rows] * a.val) * d[a.colind])
    o = Oracle()
    assert o.run(ah, OracleOptions(tau=tau, use_aggregation=False, max_block=max_block,
                                   use_cosine=use_cosine),
                 pre_perm=uorder, unit_starts=us) == 0
    perm, gs, bs = bilu.preprocess(a, tau, pre_perm=order, ordering=bilu.ORDER_NATURAL,
                                   use_mwm=2, max_block=max_block, use_cosine=use_cosine)
    assert np.array_equal(perm, o.perm())
    assert np.array_equal(gs, o.group_starts())
    assert np.array_equal(bs, o.starts_initial())
    if name == "zero_diagonal_41":
        assert (np.diff(us) == 1).sum() >= 1   # an odd cycle left a 1x1 pivot
    assert np.diff(gs).max() <= max_block


def test_symmetric_matching_errors():
    """use_mwm = 2 on a structurally singular matrix (an empty row and
    column): BILU_ERR_SINGULAR from the matching; a bad use_mwm value:
    BILU_ERR_INVALID."""
    A = np.array([[2.0, 1.0, 0.0], [1.0, 3.0, 0.0], [0.0, 0.0, 0.0]])
    mask = A != 0
    a = mg.dense_to_csr(A, mask=mask)
    with pytest.raises(bilu.BiluError) as e:
        bilu.preprocess(a, 1e-2, use_mwm=2)
    assert e.value.status == bilu.BILU_ERR_SINGULAR
    good = mg.dense_to_csr(np.array([[2.0, 1.0], [1.0, 3.0]]))
    with pytest.raises(bilu.BiluError) as e:
        bilu.preprocess(good, 1e-2, use_mwm=3)
    assert e.value.status == bilu.BILU_ERR_INVALID
