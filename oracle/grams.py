"""Gram matrices and the cell graph Laplacian (Sec. 2 and Sec. 3 of the paper).

* G_ll: Gram matrix of the primal piecewise-linear hats (eq. pwlf), the P1
  mass matrix: int lambda_i lambda_j over a cell of area A is A/6 for i = j and
  A/12 otherwise.
* G_pp: Gram matrix of the cell functions p_n = 1/A_n (eq. patchstddef), which
  is diag(1/A).
* G_tp: mixed Gram matrix of the dual hats and the cell functions, the closed
  form stated in Sec. 3 right after the definition of the middle matrix.
* L = Sigma^T Sigma, the cell (dual) graph Laplacian inside the projectors.
"""

import numpy as np

__all__ = ["gram_ll", "gram_pp", "gram_tp", "laplacian"]


def gram_ll(top):
    """P1 mass matrix, dense [V,V]."""
    G = np.zeros((top.V, top.V))
    for c in range(top.C):
        A = top.area[c]
        for i in range(3):
            for j in range(3):
                G[top.tri[c, i], top.tri[c, j]] += A / 6.0 if i == j else A / 12.0
    return G


def gram_pp(top):
    """diag(1/A) as a dense [C,C] matrix."""
    return np.diag(1.0 / top.area)


def gram_tp(top):
    """Closed form of the dual-hat / cell mixed Gram matrix, dense [C,C].

    diagonal:            (2/18) (9/2 + sum_i 1/NoC(v_i))  over the cell's vertices
    cells sharing edge:  (2/18) (1/2 + 1/NoC(e+) + 1/NoC(e-))  over the edge's vertices
    sharing one vertex:  (2/18) (1/NoC(v))
    """
    G = np.zeros((top.C, top.C))
    inv = 1.0 / top.noc
    cells_at = [[] for _ in range(top.V)]
    for c in range(top.C):
        for v in top.tri[c]:
            cells_at[v].append(c)
    for m in range(top.C):
        vm = set(top.tri[m].tolist())
        G[m, m] = (2.0 / 18.0) * (4.5 + sum(inv[v] for v in vm))
        neigh = set()
        for v in vm:
            neigh.update(cells_at[v])
        neigh.discard(m)
        for n in neigh:
            shared = vm & set(top.tri[n].tolist())
            if len(shared) == 2:
                a, b = shared
                G[m, n] = (2.0 / 18.0) * (0.5 + inv[a] + inv[b])
            elif len(shared) == 1:
                (v,) = shared
                G[m, n] = (2.0 / 18.0) * inv[v]
    return G


def laplacian(top):
    """L = Sigma^T Sigma (dense [C,C])."""
    return top.Sigma.T @ top.Sigma
