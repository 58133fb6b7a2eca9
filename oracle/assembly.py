"""Dense Galerkin blocks T_A and V of the EFIE, complex128 (Sec. 2 of the paper).

Definitions (Sec. 2, eqs. for [T_A]_mn and [T_Phi]_mn, with the RWG of
eq. RWGdef and the n x f testing, which folds away for tangential fields):

  [T_A]_mn = int int f_m(r) . f_n(r') G_k(|r - r'|) dS dS'
  V_cc'    = (A_c A_c')^-1 int_c int_c' G_k dS dS'        (so T_Phi = Sigma V Sigma^T)
  G_k(R)   = exp(i k R) / (4 pi R)

On cell c, f_m = sigma (r - r_m^c)/(2 A_c) with sigma = Sigma[m, c] and r_m^c
the free vertex, so T_A = E B E^T where E sums the two cell pieces of each
RWG and the cell-pair block is

  B[(c,i),(c',j)] = sigma sigma' / (4 A_c A_c') int_c int_c' (r - r_i^c).(r' - r_j^c') G_k.

Quadrature spec (the paper is silent; the GPU library implements the same
written spec independently):
* far pairs: the 7-point degree-5 rule on both cells (7 x 7 products);
* near pairs (centroid distance below near_factor times the longer of the two
  cells' longest edges, with a 1e-9 relative slack so that exact ties on
  structured meshes are near): outer 7-point rule on the lower-indexed cell,
  the 1/(4 pi R) part integrated over the other cell in closed form
  (``singular.potentials``) and the bounded remainder (exp(ikR) - 1)/(4 pi R)
  with the 7 x 7 rule, evaluated as (-2 sin^2(kR/2) + i sin(kR))/R (limit ik at
  R = 0).  The block of the mirrored pair is the transpose; the 3 x 3 block of
  a self pair is replaced by its symmetric part.  Both blocks are therefore
  exactly complex-symmetric.
"""

import numpy as np

from .quadrature import tri7_points
from .singular import potentials

__all__ = ["near_mask", "assemble", "near_block", "cell_embedding", "far_rows", "block_rows", "ta_rows"]


def near_mask(top, near_factor=2.0):
    """Boolean [C,C]: pairs that take the singular-extraction path."""
    h = top.longest_edge()
    d = np.linalg.norm(top.centroid[:, None, :] - top.centroid[None, :, :], axis=-1)
    thr = near_factor * np.maximum(h[:, None], h[None, :]) * (1.0 + 1e-9)
    return d < thr


def cell_embedding(top):
    """E [N, 3C]: E[m, 3c+i] = 1 when local edge i of cell c is RWG m."""
    E = np.zeros((top.N, 3 * top.C))
    for c in range(top.C):
        for i in range(3):
            E[top.cell_edges[c, i], 3 * c + i] = 1.0
    return E


def _g_smooth(k, R):
    """(exp(ikR) - 1)/R without cancellation; ik at R = 0."""
    x = k * R
    re = -0.5 * k * x * np.sinc(x / (2.0 * np.pi)) ** 2   # -2 sin^2(x/2)/R
    im = k * np.sinc(x / np.pi)                          # sin(x)/R
    return re + 1j * im


def near_block(top, c, cp, k, pts, w):
    """Singular-extraction block for outer cell c and inner cell cp.

    Returns (B [3,3] complex, v complex): B[i,j] for local edges i of c and j
    of cp (sign factors included), v = V_{c,cp}.
    """
    rp = pts[c]            # [7,3] outer points
    rq = pts[cp]           # [7,3] inner points
    Pin = top.xyz[top.tri[cp]]
    Ain = top.area[cp]
    S, Vv = potentials(Pin, rp)                       # [7], [7,3]
    R = np.linalg.norm(rp[:, None, :] - rq[None, :, :], axis=-1)
    g = _g_smooth(k, R)                                # [7,7]
    four_pi = 4.0 * np.pi
    v = np.sum(w * S) / (four_pi * Ain) + np.einsum("p,q,pq->", w, w, g) / four_pi
    a = rp[:, None, :] - top.xyz[top.tri[c]][None, :, :]    # [7,3(i),3]
    b = rq[:, None, :] - top.xyz[top.tri[cp]][None, :, :]   # [7,3(j),3]
    # inner closed form of int (r' - r_j)/R = Vvec + (r_p - r_j) S
    inner = Vv[:, None, :] + (rp[:, None, :] - top.xyz[top.tri[cp]][None, :, :]) * S[:, None, None]
    sing = np.einsum("p,pid,pjd->ij", w, a, inner) / (four_pi * Ain)
    smooth = np.einsum("p,q,pq,pid,qjd->ij", w, w, g, a, b) / four_pi
    sig = np.outer(top.cell_sign[c], top.cell_sign[cp]) / 4.0
    return sig * (sing + smooth), v


def far_rows(top, k, cs, pts, w):
    """7x7-point quadrature of every pair (c, c'), c in the test cells cs
    (an index array or slice), c' any cell: (V rows [len(cs), C],
    cell-slot block rows [len(cs), 3, C, 3]).  Near pairs get values here
    too; assemble() overwrites them."""
    vert = top.xyz[top.tri]                                  # [C,3,3]
    arm = pts[:, :, None, :] - vert[:, None, :, :]           # [C,7,3(i),3]: r_p - r_i
    sig = top.cell_sign / 2.0                                # sigma/2 per (c,i)
    ww = np.outer(w, w)
    R = np.linalg.norm(pts[cs, :, None, None, :] - pts[None, None, :, :, :], axis=-1)  # [cc,7,C,7]
    with np.errstate(divide="ignore", invalid="ignore"):
        G = np.exp(1j * k * R) / (4.0 * np.pi * R)
    G[~np.isfinite(G)] = 0.0          # only self pairs, replaced by the near path
    Gw = G * ww[None, :, None, :]
    v = Gw.sum(axis=(1, 3))
    blk = np.einsum("apid,apbq,bqjd->aibj", arm[cs], Gw, arm, optimize=True)
    return v, blk * sig[cs][:, :, None, None] * sig[None, None, :, :]


def assemble(top, k, near_factor=2.0, chunk=32, return_blocks=False):
    """Dense (T_A [N,N], V [C,C]) complex128 by the quadrature spec."""
    pts, w = tri7_points(top.xyz, top.tri)
    C = top.C
    near = near_mask(top, near_factor)
    B = np.zeros((C, 3, C, 3), dtype=np.complex128)
    Vm = np.zeros((C, C), dtype=np.complex128)
    for s in range(0, C, chunk):
        cs = slice(s, min(C, s + chunk))
        Vm[cs], B[cs] = far_rows(top, k, cs, pts, w)
    for c in range(C):
        for cp in range(c, C):
            if not near[c, cp]:
                continue
            blk, v = near_block(top, c, cp, k, pts, w)
            if c == cp:
                blk = 0.5 * (blk + blk.T)
            B[c, :, cp, :] = blk
            B[cp, :, c, :] = blk.T
            Vm[c, cp] = v
            Vm[cp, c] = v
    E = cell_embedding(top)
    Bm = B.reshape(3 * C, 3 * C)
    TA = E @ Bm @ E.T
    if return_blocks:
        return TA, Vm, Bm
    return TA, Vm


def block_rows(top, k, cells, near_factor=2.0):
    """Rows ``cells`` of V and of the cell-slot block matrix B, by the same
    spec as ``assemble`` but without forming the C x C matrices (for
    sampled checks on large meshes): (V rows [len, C], B rows [len, 3, C, 3]).

    The near test uses the criterion of ``near_mask`` for the given rows
    only; a near pair (c, c') takes the outer rule on the lower-indexed cell,
    so for c' < c the row holds the transpose of the (c', c) block."""
    cells = np.asarray(cells)
    pts, w = tri7_points(top.xyz, top.tri)
    Vr, Br = far_rows(top, k, cells, pts, w)
    h = top.longest_edge()
    for a, c in enumerate(cells):
        d = np.linalg.norm(top.centroid - top.centroid[c], axis=1)
        thr = near_factor * np.maximum(h[c], h) * (1.0 + 1e-9)
        for cp in np.nonzero(d < thr)[0]:
            if cp >= c:
                blk, v = near_block(top, c, cp, k, pts, w)
                if cp == c:
                    blk = 0.5 * (blk + blk.T)
            else:
                blk, v = near_block(top, cp, c, k, pts, w)
                blk = blk.T
            Br[a, :, cp, :] = blk
            Vr[a, cp] = v
    return Vr, Br


def ta_rows(top, k, edges, near_factor=2.0):
    """Rows ``edges`` of T_A (complex128 [len, N]) from T_A = E B E^T: row m
    sums the block rows of the two cell slots of RWG m, and each column n
    collects the slots of RWG n."""
    edges = np.asarray(edges)
    cells = np.unique(np.concatenate([top.cplus[edges], top.cminus[edges]]))
    _, Br = block_rows(top, k, cells, near_factor)
    row_of = {int(c): a for a, c in enumerate(cells)}
    out = np.zeros((len(edges), top.N), dtype=np.complex128)
    for r, m in enumerate(edges):
        acc = np.zeros((top.C, 3), dtype=np.complex128)
        for c in (int(top.cplus[m]), int(top.cminus[m])):
            i = int(np.nonzero(top.cell_edges[c] == m)[0][0])
            acc += Br[row_of[c], i]
        np.add.at(out[r], top.cell_edges.ravel(), acc.ravel())
    return out
