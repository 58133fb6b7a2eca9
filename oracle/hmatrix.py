"""Compressed EFIE blocks: hierarchical matrices whose far blocks are
low-rank factors from adaptive cross approximation (ACA).

Sec. 4 (the Fokker example) compresses the two parts of the EFIE operator
separately with ACA at tolerance 1e-4 and states nothing else about the
compression.  Readings taken here (the paper is silent on them):

* clusters: a set of indices (RWG edges for T_A, cells for V), each with a
  point (edge midpoint, cell centroid), is split at the median of the longest
  axis of the points' bounding box, the first part taking
  leaf * max(1, round(n / (2 leaf))) indices in the sorted order along that
  axis, until a cluster has at most `leaf` indices;
* supports: a cluster's box is the bounding box of the vertices of every
  cell its basis functions live on (both cells of an edge, the cell itself);
* admissibility of a pair of clusters: min(diam) <= eta * dist of their
  boxes, and dist >= 2 * (longest edge of the mesh) * (1 + 1e-9), so that no
  near cell pair (quadrature spec) lies in a compressed block;
* the block partition: an admissible pair is a low-rank block; an
  inadmissible pair of leaves is a dense block; otherwise both clusters are
  split (a leaf is kept whole against the other's children);
* ACA with partial pivoting (Bebendorf 2000): the residual row of the pivot
  row, its largest entry as the column pivot, the residual column, and the
  next pivot row where the new column is largest among the rows not yet
  taken; stop when |u_k| |v_k| <= tol |S_k|_F (Frobenius norm of the
  approximation so far), or at full rank.

Test infrastructure only: nothing in the library imports this module.  The
entries come from a dense matrix the oracle has assembled, so every value
here is the plain definition of the compressed operator.
"""

import numpy as np

__all__ = ["Cluster", "cluster_tree", "edge_boxes", "cell_boxes", "partition", "aca", "HMatrix",
           "near_distance"]


class Cluster:
    """Indices idx (original numbering), bounding box lo/hi of their supports,
    children (empty for a leaf)."""

    def __init__(self, idx, lo, hi, children=()):
        self.idx = np.asarray(idx, dtype=np.int64)
        self.lo = lo
        self.hi = hi
        self.children = list(children)

    @property
    def diam(self):
        return float(np.linalg.norm(self.hi - self.lo))


def edge_boxes(top):
    """Per RWG edge: its point (midpoint) and the box of both its cells."""
    cells = np.stack([top.cplus, top.cminus], axis=1)        # [N, 2]
    v = top.xyz[top.tri[cells]].reshape(top.N, 6, 3)        # both cells' vertices
    mid = 0.5 * (top.xyz[top.edges[:, 0]] + top.xyz[top.edges[:, 1]])
    return mid, v.min(axis=1), v.max(axis=1)


def cell_boxes(top):
    """Per cell: its centroid and the box of its vertices."""
    v = top.xyz[top.tri]                                     # [C, 3, 3]
    return top.centroid, v.min(axis=1), v.max(axis=1)


def near_distance(top):
    """The separation below which a cell pair may be near (quadrature spec:
    centroid distance < 2 max(longest edge of either cell) (1 + 1e-9))."""
    e = top.xyz[top.tri[:, [1, 2, 0]]] - top.xyz[top.tri]
    return 2.0 * float(np.sqrt((e ** 2).sum(axis=2)).max()) * (1.0 + 1e-9)


def cluster_tree(points, lo, hi, leaf):
    """Recursive bisection of indices 0..n-1 (see the module docstring)."""
    def build(idx):
        blo = lo[idx].min(axis=0)
        bhi = hi[idx].max(axis=0)
        n = len(idx)
        if n <= leaf:
            return Cluster(idx, blo, bhi)
        p = points[idx]
        ax = int(np.argmax(p.max(axis=0) - p.min(axis=0)))
        order = idx[np.argsort(p[:, ax], kind="stable")]
        n1 = leaf * max(1, int(round(n / (2.0 * leaf))))
        n1 = min(n1, n - 1)
        return Cluster(idx, blo, bhi, [build(order[:n1]), build(order[n1:])])
    return build(np.arange(len(points)))


def box_distance(a, b):
    gap = np.maximum(0.0, np.maximum(a.lo - b.hi, b.lo - a.hi))
    return float(np.linalg.norm(gap))


def admissible(a, b, eta, dnear):
    d = box_distance(a, b)
    return d >= dnear and min(a.diam, b.diam) <= eta * d


def partition(rows, cols, eta, dnear):
    """Blocks (row cluster, column cluster, admissible) covering the matrix."""
    out = []

    def rec(a, b):
        if admissible(a, b, eta, dnear):
            out.append((a, b, True))
        elif not a.children and not b.children:
            out.append((a, b, False))
        elif not a.children:
            for bb in b.children:
                rec(a, bb)
        elif not b.children:
            for aa in a.children:
                rec(aa, b)
        else:
            for aa in a.children:
                for bb in b.children:
                    rec(aa, bb)
    rec(rows, cols)
    return out


def aca(row, col, m, n, tol, kmax=None):
    """M (m x n) ~ U V^T from rows row(i) and columns col(j) of M.  Returns
    U [m, k], V [n, k] (complex128)."""
    kmax = min(m, n) if kmax is None else min(kmax, m, n)
    U = np.zeros((m, 0), dtype=np.complex128)
    V = np.zeros((n, 0), dtype=np.complex128)
    taken = np.zeros(m, dtype=bool)
    i = 0
    while U.shape[1] < kmax:
        r = row(i) - U[i, :] @ V.T                            # residual row i
        taken[i] = True
        j = int(np.argmax(np.abs(r)))
        if abs(r[j]) == 0.0:
            # row i is already represented: try another row
            free = np.flatnonzero(~taken)
            if len(free) == 0:
                break
            i = int(free[0])
            continue
        v = r / r[j]
        u = col(j) - U @ V[j, :]                             # residual column j
        U = np.concatenate([U, u[:, None]], axis=1)
        V = np.concatenate([V, v[:, None]], axis=1)
        S = np.linalg.norm(U @ V.T)
        if np.linalg.norm(u) * np.linalg.norm(v) <= tol * S:
            break
        free = np.flatnonzero(~taken)
        if len(free) == 0:
            break
        i = int(free[np.argmax(np.abs(u[free]))])
    return U, V


class HMatrix:
    """Compressed form of a dense square matrix M over the cluster tree
    `tree` (rows and columns alike): dense blocks copied, admissible blocks
    as ACA factors at tolerance tol."""

    def __init__(self, M, tree, eta, dnear, tol):
        self.n = M.shape[0]
        self.blocks = []
        for a, b, adm in partition(tree, tree, eta, dnear):
            if adm:
                sub = M[np.ix_(a.idx, b.idx)]
                U, V = aca(lambda i: sub[i, :], lambda j: sub[:, j], len(a.idx), len(b.idx), tol)
                self.blocks.append((a.idx, b.idx, "lr", (U, V)))
            else:
                self.blocks.append((a.idx, b.idx, "dense", M[np.ix_(a.idx, b.idx)].copy()))

    def dense(self):
        out = np.zeros((self.n, self.n), dtype=np.complex128)
        for ri, ci, kind, data in self.blocks:
            out[np.ix_(ri, ci)] = data if kind == "dense" else data[0] @ data[1].T
        return out

    def matvec(self, x):
        y = np.zeros(self.n, dtype=np.complex128)
        for ri, ci, kind, data in self.blocks:
            y[ri] += (data @ x[ci]) if kind == "dense" else data[0] @ (data[1].T @ x[ci])
        return y

    def entries(self):
        """Stored complex entries (dense blocks, and k (m + n) per low-rank
        block)."""
        s = 0
        for ri, ci, kind, data in self.blocks:
            s += data.size if kind == "dense" else data[0].size + data[1].size
        return s

    def ranks(self):
        return [data[0].shape[1] for _, _, kind, data in self.blocks if kind == "lr"]
