"""Seeded synthetic test matrices shaped like the paper's workloads.

This module is shared by the oracle-side tests and the GPU path.  It holds
no arithmetic of the factorization method: it only builds sparse matrices
(CSR, sorted column indices), right-hand sides and node orderings.

The paper evaluates on SuiteSparse matrices with n >= 50,000 and between
1.6 and 78.9 nonzeros per row (Section 4 and the appendix).  Those files
are not available, so node-blocked stencil matrices stand in for them:

* ``grid2d_random_blocks``: 2D grid, 5-point coupling, every coupled node
  pair carries a dense b x b block drawn from U(-1, 1); diagonal node blocks
  are shifted by ``shift * I``.
* ``grid3d_convdiff``: 3D grid, 7-point first-order upwind
  convection-diffusion with cell Peclet number ``pe`` on every axis,
  node blocks ``s_vw * (I + G)`` with G ~ N(0, sigma), then every row's
  diagonal entry is set to ``dom`` times its off-diagonal absolute row sum.
* ``grid3d_elasticity``: 3D grid, 27-point graph Laplacian with weights
  1, 1/2, 1/3 (face, edge, corner) tensored with ``I + d d^T``, shifted by
  ``0.1 * mean(diag)``, then every off-diagonal entry scaled by
  ``1 + 0.05 * xi`` with xi ~ U(-1, 1).

Unknowns are numbered node-major (row = b * node + component) with nodes in
lexicographic order (x fastest).  Stencils are truncated at the grid
boundary (Dirichlet).

``grid_nd_node_order`` returns a geometric nested-dissection order of the
grid nodes (recursive bisection with one-node-thick separator planes,
separators ordered last and themselves dissected, or left lexicographic as
the elasticity workloads use), which stands in for the fill-reducing
ordering that the paper obtains from METIS.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class Csr:
    n: int
    rowptr: np.ndarray  # int64[n+1]
    colind: np.ndarray  # int32[nnz]
    val: np.ndarray     # float64[nnz]

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_dense(self) -> np.ndarray:
        a = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.rowptr))
        a[rows, self.colind] = self.val
        return a

    def matvec(self, x: np.ndarray) -> np.ndarray:
        rows = np.repeat(np.arange(self.n), np.diff(self.rowptr))
        y = np.zeros(self.n)
        np.add.at(y, rows, self.val * x[self.colind])
        return y


# ---------------------------------------------------------------------------
# generic node-blocked stencil assembly
# ---------------------------------------------------------------------------

def _offsets(dim: int, kind: str) -> np.ndarray:
    """Stencil offsets (including the centre) sorted by linear index shift."""
    if kind == "star":  # 5-point (2D) / 7-point (3D)
        offs = [np.zeros(dim, dtype=np.int64)]
        for d in range(dim):
            for s in (-1, 1):
                o = np.zeros(dim, dtype=np.int64)
                o[d] = s
                offs.append(o)
    elif kind == "box":  # 9-point (2D) / 27-point (3D)
        grids = np.meshgrid(*([np.array([-1, 0, 1])] * dim), indexing="ij")
        offs = list(np.stack([g.ravel() for g in grids], axis=1))
    else:
        raise ValueError(kind)
    offs = np.array(offs, dtype=np.int64)
    # linear shift with x fastest: sort key z, y, x
    key = np.zeros(len(offs), dtype=np.int64)
    for d in reversed(range(dim)):
        key = key * 4 + (offs[:, d] + 1)
    return offs[np.argsort(key, kind="stable")]


def _assemble(dims, b, offs, blocks, valid) -> Csr:
    """Assemble node blocks into CSR.

    dims   : grid extents (x fastest)
    b      : unknowns per node
    offs   : (O, dim) offsets sorted by linear shift
    blocks : (N, O, b, b) block values, blocks[v, o] couples node v to v+offs[o]
    valid  : (N, O) boolean, neighbour inside the grid
    """
    dims = np.asarray(dims, dtype=np.int64)
    N = int(np.prod(dims))
    O = offs.shape[0]
    strides = np.cumprod(np.concatenate([[1], dims[:-1]]))
    shift = offs @ strides                                  # (O,)
    w = np.arange(N, dtype=np.int64)[:, None] + shift[None, :]   # (N, O)
    # columns for row (v, cr): for o valid: b*w + cc
    cols = (b * w)[:, None, :, None] + np.arange(b)[None, None, None, :]  # (N,1,O,b)
    cols = np.broadcast_to(cols, (N, b, O, b))
    vals = np.transpose(blocks, (0, 2, 1, 3))               # (N, b(cr), O, b(cc))
    mask = np.broadcast_to(valid[:, None, :, None], (N, b, O, b))
    colind = cols[mask].astype(np.int32)
    val = np.ascontiguousarray(vals[mask], dtype=np.float64)
    per_row = (valid.sum(axis=1) * b).astype(np.int64)      # (N,)
    row_counts = np.repeat(per_row, b)
    rowptr = np.zeros(N * b + 1, dtype=np.int64)
    np.cumsum(row_counts, out=rowptr[1:])
    return Csr(N * b, rowptr, colind, val)


def _valid(dims, offs) -> np.ndarray:
    dims = np.asarray(dims, dtype=np.int64)
    N = int(np.prod(dims))
    coords = np.stack(np.unravel_index(np.arange(N), tuple(dims[::-1])), axis=1)[:, ::-1]
    nb = coords[:, None, :] + offs[None, :, :]
    return np.all((nb >= 0) & (nb < dims[None, None, :]), axis=2)


# ---------------------------------------------------------------------------
# the workload families
# ---------------------------------------------------------------------------

def grid2d_random_blocks(side: int = 32, b: int = 3, shift: float = 4.5,
                         seed: int = 0, kind: str = "star") -> Csr:
    """2D grid, dense U(-1,1) node blocks on every coupled pair, centre += shift*I."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    dims = (side, side)
    offs = _offsets(2, kind)
    valid = _valid(dims, offs)
    N = side * side
    blocks = rng.uniform(-1.0, 1.0, size=(N, len(offs), b, b))
    centre = int(np.flatnonzero(np.all(offs == 0, axis=1))[0])
    blocks[:, centre] += shift * np.eye(b)
    return _assemble(dims, b, offs, blocks, valid)


def grid3d_convdiff(side: int = 64, b: int = 4, pe: float = 10.0,
                    sigma: float = 0.3, dom: float = 1.1, seed: int = 1,
                    dims=None) -> Csr:
    """3D 7-point upwind convection-diffusion with random node blocks."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    dims = tuple(dims) if dims is not None else (side, side, side)
    dim = len(dims)
    offs = _offsets(dim, "star")
    valid = _valid(dims, offs)
    N = int(np.prod(dims))
    coef = np.empty(len(offs))
    for o, off in enumerate(offs):
        s = int(off.sum())
        if not off.any():
            coef[o] = 2 * dim + dim * pe
        elif s < 0:   # upwind neighbour (flow towards +axis)
            coef[o] = -(1.0 + pe)
        else:
            coef[o] = -1.0
    g = rng.normal(0.0, sigma, size=(N, len(offs), b, b))
    blocks = coef[None, :, None, None] * (np.eye(b)[None, None] + g)
    a = _assemble(dims, b, offs, blocks, valid)
    _set_dominant_diagonal(a, dom)
    return a


def grid3d_elasticity(side: int = 80, b: int = 3, seed: int = 2,
                      pert: float = 0.05, dims=None, shift: float = 0.1) -> Csr:
    """27-point elasticity-like operator plus shift * (mean diagonal) * I,
    its entries randomly perturbed by up to ``pert``.  pert = 0 keeps it
    symmetric: positive definite for shift > 0, indefinite for a negative
    shift inside the spectrum."""
    if b != 3:
        raise ValueError("elasticity-like operator uses 3 unknowns per node")
    rng = np.random.default_rng(np.random.PCG64(seed))
    dims = tuple(dims) if dims is not None else (side, side, side)
    offs = _offsets(3, "box")
    valid = _valid(dims, offs)
    N = int(np.prod(dims))
    O = len(offs)
    centre = int(np.flatnonzero(np.all(offs == 0, axis=1))[0])
    mats = np.zeros((O, 3, 3))
    for o, off in enumerate(offs):
        k = int(np.abs(off).sum())
        if k == 0:
            continue
        d = off / np.linalg.norm(off)
        mats[o] = (1.0 / k) * (np.eye(3) + np.outer(d, d))
    blocks = np.zeros((N, O, 3, 3))
    offmask = valid.copy()
    offmask[:, centre] = False
    blocks[:] = -mats[None]
    blocks *= offmask[:, :, None, None]
    blocks[:, centre] = np.einsum("no,oij->nij", offmask.astype(np.float64), mats)
    mean_diag = float(np.mean(np.diagonal(blocks[:, centre], axis1=1, axis2=2)))
    blocks[:, centre] += shift * mean_diag * np.eye(3)
    xi = rng.uniform(-1.0, 1.0, size=(N, O, 3, 3))
    scale = 1.0 + pert * xi
    scale[:, centre, np.arange(3), np.arange(3)] = 1.0   # keep scalar diagonal
    blocks *= scale
    return _assemble(dims, b, offs, blocks, valid)


def kkt_elasticity(side: int = 8, ncon: int | None = None, seed: int = 7,
                   shift: float = 0.1, constraints_first: bool = True):
    """Symmetric indefinite saddle-point matrix [[K, B^T], [B, 0]]: K the
    unperturbed elasticity-like operator (positive definite), B holds ncon
    constraints (default: one per two nodes), each coupling the 3 unknowns
    of a random node and of its neighbour along the first axis with
    U(-1, 1) weights; the constraint rows store no diagonal.  Returned with
    a node-major ordering in which each constraint sits just before (or,
    constraints_first=False, just after) the unknowns of its node: (Csr,
    order new->old, number of constraints)."""
    import scipy.sparse as sp
    K = grid3d_elasticity(side, 3, seed=2, pert=0.0, shift=shift)
    nodes = side ** 3
    m = nodes // 2 if ncon is None else ncon
    rng = np.random.default_rng(np.random.PCG64(seed))
    node = rng.integers(0, nodes, size=m)
    x = node % side
    nb = np.where(x + 1 < side, node + 1, node - 1)
    cols = np.concatenate([3 * node[:, None] + np.arange(3), 3 * nb[:, None] + np.arange(3)], axis=1)
    vals = rng.uniform(-1.0, 1.0, size=cols.shape)
    B = sp.csr_matrix((vals.ravel(), (np.repeat(np.arange(m), 6), cols.ravel())),
                      shape=(m, K.n))
    Ks = sp.csr_matrix((K.val, K.colind, K.rowptr), shape=(K.n, K.n))
    S = sp.bmat([[Ks, B.T], [B, None]], format="csr")
    S.sort_indices()
    a = Csr(S.shape[0], S.indptr.astype(np.int64), S.indices.astype(np.int32), S.data.copy())
    by_node = [[] for _ in range(nodes)]
    for r in range(m):
        by_node[node[r]].append(K.n + r)
    order = []
    for v in range(nodes):
        dofs = [3 * v, 3 * v + 1, 3 * v + 2]
        order.extend(by_node[v] + dofs if constraints_first else dofs + by_node[v])
    return a, np.array(order, dtype=np.int64), m


def _set_dominant_diagonal(a: Csr, dom: float) -> None:
    rows = np.repeat(np.arange(a.n), np.diff(a.rowptr))
    diag = a.colind == rows
    offsum = np.zeros(a.n)
    np.add.at(offsum, rows[~diag], np.abs(a.val[~diag]))
    a.val[diag] = dom * offsum[rows[diag]]


def random_sparse(n: int, density: float, seed: int, diag_shift: float = 0.0,
                  symmetric_pattern: bool = False) -> Csr:
    """Random sparse matrix with a full diagonal, U(-1,1) values."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    mask = rng.random((n, n)) < density
    if symmetric_pattern:
        mask = mask | mask.T
    np.fill_diagonal(mask, True)
    vals = rng.uniform(-1.0, 1.0, size=(n, n))
    vals[np.arange(n), np.arange(n)] += diag_shift
    return dense_to_csr(np.where(mask, vals, 0.0), mask)


def random_geometric(nodes: int, k: int = 8, dim: int = 2, b: int = 2, seed: int = 0,
                     dom: float = 1.2) -> Csr:
    """Irregular mesh-like matrix: ``nodes`` points uniform in the unit
    square (cube), each coupled to its k nearest neighbours (symmetrized
    pattern); every coupled node pair gets a dense b x b block ~U(-1,1), and
    each row's diagonal is ``dom`` times the sum of its off-diagonal
    magnitudes.  Node-major numbering (row = b * node + component)."""
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(np.random.PCG64(seed))
    pts = rng.random((nodes, dim))
    _, nb = cKDTree(pts).query(pts, k + 1)
    adj = np.zeros((nodes, nodes), dtype=bool)
    rows = np.repeat(np.arange(nodes), k)
    cols = nb[:, 1:].ravel()
    adj[rows, cols] = True
    adj |= adj.T
    np.fill_diagonal(adj, True)
    n = nodes * b
    mask = np.kron(adj, np.ones((b, b), dtype=bool))
    vals = np.where(mask, rng.uniform(-1.0, 1.0, size=(n, n)), 0.0)
    np.fill_diagonal(vals, 0.0)
    np.fill_diagonal(vals, dom * np.abs(vals).sum(axis=1) + 1.0)
    return dense_to_csr(vals, mask)


def dense_to_csr(a: np.ndarray, mask: np.ndarray | None = None) -> Csr:
    """CSR of a dense array; ``mask`` selects structural entries (default a != 0)."""
    a = np.asarray(a, dtype=np.float64)
    if mask is None:
        mask = a != 0.0
    n = a.shape[0]
    counts = mask.sum(axis=1).astype(np.int64)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    r, c = np.nonzero(mask)
    return Csr(n, rowptr, c.astype(np.int32), a[r, c].astype(np.float64))


# ---------------------------------------------------------------------------
# orderings
# ---------------------------------------------------------------------------

def grid_nd_node_order(dims, leaf: int = 8, dissect_separators: bool = True) -> np.ndarray:
    """Geometric nested dissection of a grid: returns new->old node numbering.

    Recursively splits the longest axis at its middle plane; the two halves
    are ordered first, the one-node-thick separator plane last.  Separator
    planes are themselves dissected as lower-dimensional boxes, or, with
    ``dissect_separators=False``, kept in lexicographic order.  Boxes with
    at most ``leaf`` nodes, or too thin to split, keep lexicographic order.
    """
    dims = tuple(int(d) for d in dims)
    strides = np.cumprod((1,) + dims[:-1])
    out: list[np.ndarray] = []

    def lex(lo, hi):
        rng = [np.arange(l, h) for l, h in zip(lo, hi)]
        grids = np.meshgrid(*rng[::-1], indexing="ij")       # slowest axis first
        idx = sum(g.ravel() * strides[len(dims) - 1 - k] for k, g in enumerate(grids))
        return np.asarray(idx, dtype=np.int64)

    stack = [(tuple(0 for _ in dims), dims, 0)]
    # explicit recursion with a post-order emit: (lo, hi, state)
    def rec(lo, hi):
        ext = [h - l for l, h in zip(lo, hi)]
        vol = int(np.prod(ext))
        if vol == 0:
            return
        ax = int(np.argmax(ext))
        if vol <= leaf or ext[ax] < 3:
            out.append(lex(lo, hi))
            return
        mid = lo[ax] + ext[ax] // 2
        lhi = list(hi); lhi[ax] = mid
        rlo = list(lo); rlo[ax] = mid + 1
        slo = list(lo); slo[ax] = mid
        shi = list(hi); shi[ax] = mid + 1
        rec(tuple(lo), tuple(lhi))
        rec(tuple(rlo), tuple(hi))
        if dissect_separators:
            rec(tuple(slo), tuple(shi))
        else:
            out.append(lex(tuple(slo), tuple(shi)))

    del stack
    rec(tuple(0 for _ in dims), dims)
    order = np.concatenate(out)
    assert order.size == int(np.prod(dims))
    return order


def node_perm_to_scalar(node_order: np.ndarray, b: int) -> np.ndarray:
    """Expand a node ordering (new->old) to the node-major scalar numbering."""
    node_order = np.asarray(node_order, dtype=np.int64)
    return (b * node_order[:, None] + np.arange(b)[None, :]).ravel()


# ---------------------------------------------------------------------------
# named workloads
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    a: Csr
    b_node: int
    dims: tuple
    tau: float
    restart: int
    perm: np.ndarray | None   # scalar new->old ordering, None = natural


def workload(name: str, nd: bool = True) -> Workload:
    """The named synthetic workloads (sizes as in the hot-path scope table)."""
    if name == "cd2d_32x32_b3":
        a = grid2d_random_blocks(32, 3, 4.5, seed=0)
        dims, b, tau, m = (32, 32), 3, 1e-2, 30
    elif name == "cd3d_64_b4":
        a = grid3d_convdiff(64, 4, seed=1)
        dims, b, tau, m = (64, 64, 64), 4, 1e-2, 50
    elif name == "el3d_80_b3":
        a = grid3d_elasticity(80, 3, seed=2)
        dims, b, tau, m = (80, 80, 80), 3, 5e-3, 30
    elif name.startswith("cd3d_"):       # cd3d_<side>_b<b>
        side = int(name.split("_")[1])
        b = int(name.split("_b")[1])
        a = grid3d_convdiff(side, b, seed=1)
        dims, tau, m = (side, side, side), 1e-2, 50
    elif name.startswith("el3d_"):
        side = int(name.split("_")[1])
        a = grid3d_elasticity(side, 3, seed=2)
        dims, b, tau, m = (side, side, side), 3, 5e-3, 30
    else:
        raise KeyError(name)
    # the 27-point elasticity stencils factor with far shorter dependency
    # chains when the separator planes stay lexicographic
    sep = not name.startswith("el3d_")
    perm = node_perm_to_scalar(grid_nd_node_order(dims, dissect_separators=sep), b) if nd else None
    return Workload(name, a, b, dims, tau, m, perm)


def batch_workloads(master_seed: int = 5, count: int = 64):
    """Seeded descriptors of a batch of independent stencil systems.

    For i in range(count): dim in {2, 3}, b in 1..6, n log-uniform on
    [20k, 300k] (side = round((n/b)^(1/dim))), star stencil, the
    convection-diffusion value model, tau in {1e-2, 1e-3}.
    """
    rng = np.random.default_rng(np.random.PCG64(master_seed))
    out = []
    for i in range(count):
        dim = int(rng.integers(2, 4))
        b = int(rng.integers(1, 7))
        n = math.exp(rng.uniform(math.log(20_000), math.log(300_000)))
        side = max(3, int(round((n / b) ** (1.0 / dim))))
        tau = float(rng.choice([1e-2, 1e-3]))
        out.append(dict(index=i, dim=dim, b=b, side=side, tau=tau, seed=5000 + i))
    return out


def batch_matrix(desc) -> Workload:
    dims = (desc["side"],) * desc["dim"]
    a = grid3d_convdiff(b=desc["b"], seed=desc["seed"], dims=dims)
    perm = node_perm_to_scalar(grid_nd_node_order(dims), desc["b"])
    return Workload(f"batch{desc['index']}", a, desc["b"], dims, desc["tau"], 30, perm)
