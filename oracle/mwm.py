"""Maximum weight matching of Sec. 3.1 (eq. (mwm)): the oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A maximum product transversal of A is a permutation sigma maximizing
prod_i |a_{i,sigma(i)}|.  With colmax_j = max_i |a_ij| and, for every stored
entry with a_ij != 0,

    c_ij = log(colmax_j) - log|a_ij|  (>= 0),

it is the linear assignment problem  min sum_i c_{i,sigma(i)}  on the
bipartite graph of rows and columns.  Its dual (u rows, v columns) has
u_i + v_j <= c_ij on every entry, with equality on the matching.  The
scalings

    D_l = diag(exp(u)),  D_r = diag(exp(v) / colmax),

give  |(D_l A D_r)_ij| = exp(u_i + v_j - c_ij) <= 1, equal to 1 on the
matching, and with Pi[sigma(i), i] = 1 the matrix  D_l A D_r Pi  has unit
diagonal magnitudes (the property eq. (mwm) asks for).

The assignment is solved by successive shortest augmenting paths (the
sparse Kuhn-Munkres scheme the paper refers to): for each row, Dijkstra on
the reduced costs c_ij - u_i - v_j >= 0 finds the nearest free column over
alternating paths; the duals of the rows and columns reached before it move
by their distance deficit, which keeps every reduced cost non-negative and
makes the path tight; the path is then flipped.  Plain Python loops: for the
small matrices of the tests.
"""
from __future__ import annotations

import heapq

import numpy as np


def mwm(a):
    """Return (sigma, u, v, colmax, cost) for the square Csr matrix a.

    sigma[i] is the column matched to row i.  Raises ValueError when A is
    structurally singular (no perfect matching on its nonzero entries)."""
    n = a.n
    rp, ci, val = a.rowptr, a.colind, a.val
    absv = np.abs(val)
    colmax = np.zeros(n)
    np.maximum.at(colmax, ci, absv)
    if np.any(colmax == 0.0):
        raise ValueError("a column without nonzero entries")
    rows = []  # per row: (columns, costs) of its nonzero entries
    for i in range(n):
        cols, costs = [], []
        for m in range(rp[i], rp[i + 1]):
            if absv[m] != 0.0:
                j = int(ci[m])
                cols.append(j)
                costs.append(float(np.log(colmax[j]) - np.log(absv[m])))
        rows.append((cols, costs))
    u = np.array([min(c) if c else np.inf for _, c in rows])
    if np.any(~np.isfinite(u)):
        raise ValueError("a row without nonzero entries")
    v = np.zeros(n)
    row_of = [-1] * n  # column -> matched row
    col_of = [-1] * n  # row -> matched column
    for r in range(n):
        dist = {}       # tentative distances of columns
        pred = {}       # column -> row it was reached from
        done = {}       # finalized columns -> distance
        heap = []
        d_row = {r: 0.0}
        cols, costs = rows[r]
        for j, c in zip(cols, costs):
            d = c - u[r] - v[j]
            if d < dist.get(j, np.inf):
                dist[j] = d
                pred[j] = r
                heapq.heappush(heap, (d, j))
        free = -1
        delta = 0.0
        while heap:
            d, j = heapq.heappop(heap)
            if j in done or d > dist[j]:
                continue
            done[j] = d
            if row_of[j] < 0:
                free, delta = j, d
                break
            i = row_of[j]
            d_row[i] = d
            for k, c in zip(*rows[i]):
                if k in done:
                    continue
                nd = d + c - u[i] - v[k]
                if nd < dist.get(k, np.inf):
                    dist[k] = nd
                    pred[k] = i
                    heapq.heappush(heap, (nd, k))
        if free < 0:
            raise ValueError("structurally singular: no perfect matching")
        # duals: rows and columns reached closer than delta move by the deficit
        for i, di in d_row.items():
            if di < delta:
                u[i] += delta - di
        for j, dj in done.items():
            if dj < delta:
                v[j] -= delta - dj
        # flip the alternating path ending at the free column
        j = free
        while True:
            i = pred[j]
            prev = col_of[i]
            row_of[j] = i
            col_of[i] = j
            if i == r:
                break
            j = prev
    sigma = np.array(col_of, dtype=np.int64)
    cost = float(sum(np.log(colmax[sigma[i]]) - np.log(_entry(a, i, sigma[i])) for i in range(n)))
    return sigma, u, v, colmax, cost


def _entry(a, i, j):
    for m in range(a.rowptr[i], a.rowptr[i + 1]):
        if a.colind[m] == j:
            return abs(a.val[m])
    return 0.0


def mwm_scalings(a):
    """(sigma, dl, dr): the matching and the scalings of eq. (mwm)."""
    sigma, u, v, colmax, _ = mwm(a)
    return sigma, np.exp(u), np.exp(v) / colmax


def apply_mwm(a, sigma, dl, dr):
    """Dense D_l A D_r Pi (column i of the result is column sigma(i))."""
    A = a.to_dense()
    return (dl[:, None] * A * dr[None, :])[:, sigma]


def symmetric_units(a, sigma, dl, dr, pre=None):
    """Sec. 5, eq. (smwm): the symmetric matching of the BILDL variant
    (Duff and Pralet, SIAM J. Matrix Anal. Appl. 27, 2005).

    For symmetric A and a maximum product matching (sigma, D_l, D_r) the
    symmetric scaling d_i = sqrt(dl_i dr_i) keeps |(D A D)_ij| <= 1 with
    the matched entries of magnitude one.  The matching's cycles give the
    pivots: a fixed point a 1x1 pivot, a 2-cycle a 2x2 pivot; a longer
    cycle c_0 -> c_1 -> ... (c_0 its smallest index, c_{k+1} = sigma(c_k))
    is cut into consecutive pairs (c_0, c_1), (c_2, c_3), ...; an odd one
    first leaves out as a 1x1 pivot the member with the largest |(D A D)_ii|
    (the first in cycle order on ties) and pairs the rest from the member
    after it on.  Readings: the two pairings of an even cycle are both made
    of matched entries, the one starting at c_0 is taken; a pair lists its
    smaller index first.

    Returns (d, order, unit_starts): order (new -> old) lists the units in
    the order their first index is met along pre (identity when None),
    unit_starts their boundaries in that numbering."""
    n = a.n
    sigma = np.asarray(sigma, dtype=np.int64)
    d = np.sqrt(np.asarray(dl) * np.asarray(dr))
    diag = np.zeros(n)
    for i in range(n):
        diag[i] = _entry(a, i, i) * d[i] * d[i]
    unit = np.full(n, -1, dtype=np.int64)
    units = []
    for s in range(n):
        if unit[s] >= 0:
            continue
        cyc = [s]
        j = int(sigma[s])
        while j != s:
            cyc.append(j)
            j = int(sigma[j])
        L = len(cyc)
        first = len(units)
        if L % 2 == 1:
            best = max(range(L), key=lambda k: (diag[cyc[k]], -k))
            units.append([cyc[best]])
            rest = [cyc[(best + 1 + t) % L] for t in range(L - 1)]
        else:
            rest = cyc
        for t in range(0, len(rest), 2):
            units.append(sorted(rest[t:t + 2]))
        for k in range(first, len(units)):
            for i in units[k]:
                unit[i] = k
    pre = np.arange(n) if pre is None else np.asarray(pre, dtype=np.int64)
    done = np.zeros(len(units), dtype=bool)
    order, starts = [], [0]
    for i in pre:
        u = unit[i]
        if done[u]:
            continue
        done[u] = True
        order.extend(units[u])
        starts.append(len(order))
    return d, np.array(order, dtype=np.int64), np.array(starts, dtype=np.int64)
