"""Pins of the oracle's compressed operator (oracle/hmatrix.py): ACA against
exact low-rank matrices and against the truncated SVD of a kernel block
(numpy's SVD as the independent reference), the block partition against a
brute-force count and the quadrature spec's near pairs, the compressed EFIE
blocks against the dense ones, and the RF-CMP solution with compressed
blocks against the dense solution.  Planted mistakes in ACA fail the pins."""
import numpy as np
import pytest

import synth
from oracle import assembly, hmatrix as hm, rfcmp
from oracle.topology import Topology


def _rng(seed):
    return np.random.default_rng(seed)


def _crandn(g, *shape):
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


def _kernel_block(k=2.0, m=200, n=150, gap=3.0, seed=1):
    g = _rng(seed)
    x = g.random((m, 3))
    y = g.random((n, 3)) + np.array([1.0 + gap, 0.0, 0.0])
    R = np.linalg.norm(x[:, None, :] - y[None, :, :], axis=2)
    return np.exp(1j * k * R) / (4 * np.pi * R)


def _aca_dense(M, tol, fn=None):
    fn = fn or hm.aca
    return fn(lambda i: M[i, :], lambda j: M[:, j], M.shape[0], M.shape[1], tol)


def _aca_without_residual_row(row, col, m, n, tol, kmax=None):
    """ACA with a plausible slip: the pivot row is not reduced by the
    approximation so far."""
    U = np.zeros((m, 0), dtype=np.complex128)
    V = np.zeros((n, 0), dtype=np.complex128)
    taken = np.zeros(m, dtype=bool)
    i = 0
    while U.shape[1] < min(m, n):
        r = row(i)
        taken[i] = True
        j = int(np.argmax(np.abs(r)))
        v = r / r[j]
        u = col(j) - U @ V[j, :]
        U = np.concatenate([U, u[:, None]], axis=1)
        V = np.concatenate([V, v[:, None]], axis=1)
        if np.linalg.norm(u) * np.linalg.norm(v) <= tol * np.linalg.norm(U @ V.T):
            break
        free = np.flatnonzero(~taken)
        if len(free) == 0:
            break
        i = int(free[np.argmax(np.abs(u[free]))])
    return U, V


def _aca_pivot_not_normalised(row, col, m, n, tol, kmax=None):
    """ACA with another slip: v is not divided by the pivot entry."""
    U = np.zeros((m, 0), dtype=np.complex128)
    V = np.zeros((n, 0), dtype=np.complex128)
    taken = np.zeros(m, dtype=bool)
    i = 0
    while U.shape[1] < min(m, n):
        r = row(i) - U[i, :] @ V.T
        taken[i] = True
        j = int(np.argmax(np.abs(r)))
        v = r
        u = col(j) - U @ V[j, :]
        U = np.concatenate([U, u[:, None]], axis=1)
        V = np.concatenate([V, v[:, None]], axis=1)
        if np.linalg.norm(u) * np.linalg.norm(v) <= tol * np.linalg.norm(U @ V.T):
            break
        free = np.flatnonzero(~taken)
        if len(free) == 0:
            break
        i = int(free[np.argmax(np.abs(u[free]))])
    return U, V


def _exact_low_rank_error(fn):
    g = _rng(3)
    r = 5
    M = _crandn(g, 80, r) @ _crandn(g, r, 60)
    U, V = _aca_dense(M, 1e-12, fn)
    return U.shape[1], np.linalg.norm(M - U @ V.T) / np.linalg.norm(M)


def test_aca_recovers_exact_low_rank():
    k, err = _exact_low_rank_error(None)
    assert k <= 6
    assert err < 1e-12


@pytest.mark.parametrize("tol", [1e-2, 1e-4, 1e-6])
def test_aca_error_and_rank_against_svd(tol):
    M = _kernel_block()
    U, V = _aca_dense(M, tol)
    err = np.linalg.norm(M - U @ V.T) / np.linalg.norm(M)
    assert err < 10 * tol
    # the optimal rank for the error ACA reached (truncated SVD)
    s = np.linalg.svd(M, compute_uv=False)
    tail = np.sqrt(np.cumsum((s ** 2)[::-1])[::-1]) / np.linalg.norm(s)   # tail[r] = error of rank r
    r_opt = int(np.argmax(tail <= err)) if np.any(tail <= err) else len(s)
    assert U.shape[1] <= 2 * r_opt + 2


@pytest.mark.parametrize("slip", [_aca_without_residual_row, _aca_pivot_not_normalised])
def test_aca_slips_fail_the_pins(slip):
    k, err = _exact_low_rank_error(slip)
    M = _kernel_block()
    U, V = _aca_dense(M, 1e-4, slip)
    err2 = np.linalg.norm(M - U @ V.T) / np.linalg.norm(M)
    assert err > 1e-12 or err2 > 1e-3


def _ico2():
    xyz, tri = synth.icosphere(2)
    return Topology(xyz, tri)


@pytest.fixture(scope="module")
def ico2_blocks():
    top = _ico2()
    TA, V = assembly.assemble(top, 1.0)
    return top, TA, V


@pytest.mark.parametrize("what", ["edges", "cells"])
def test_partition_covers_once_and_keeps_near_pairs_dense(what):
    top = _ico2()
    p, lo, hi = hm.edge_boxes(top) if what == "edges" else hm.cell_boxes(top)
    tree = hm.cluster_tree(p, lo, hi, 16)
    dn = hm.near_distance(top)
    blocks = hm.partition(tree, tree, 2.0, dn)
    n = len(p)
    count = np.zeros((n, n), dtype=np.int64)
    for a, b, adm in blocks:
        count[np.ix_(a.idx, b.idx)] += 1
    assert np.all(count == 1)
    near = assembly.near_mask(top)
    # the cells each index lives on
    cells = (np.stack([top.cplus, top.cminus], axis=1) if what == "edges" else np.arange(top.C)[:, None])
    nadm = 0
    for a, b, adm in blocks:
        if not adm:
            assert not a.children and not b.children
            continue
        nadm += 1
        ca = np.unique(cells[a.idx].ravel())
        cb = np.unique(cells[b.idx].ravel())
        assert not near[np.ix_(ca, cb)].any()
        # every vertex of one support at least dnear from every vertex of the other
        va = top.xyz[top.tri[ca]].reshape(-1, 3)
        vb = top.xyz[top.tri[cb]].reshape(-1, 3)
        dmin = np.sqrt(((va[:, None, :] - vb[None, :, :]) ** 2).sum(axis=2)).min()
        assert dmin >= dn * (1 - 1e-12)
    assert nadm > 0


@pytest.mark.parametrize("tol", [1e-2, 1e-4])
def test_compressed_efie_blocks(ico2_blocks, tol):
    top, TA, V = ico2_blocks
    dn = hm.near_distance(top)
    for M, (p, lo, hi) in ((TA, hm.edge_boxes(top)), (V, hm.cell_boxes(top))):
        H = hm.HMatrix(M, hm.cluster_tree(p, lo, hi, 16), 2.0, dn, tol)
        D = H.dense()
        assert np.linalg.norm(D - M) / np.linalg.norm(M) < 10 * tol
        assert any(kind == "lr" for _, _, kind, _ in H.blocks)
        x = _crandn(_rng(5), M.shape[0])
        assert np.linalg.norm(H.matvec(x) - D @ x) <= 1e-13 * np.linalg.norm(D @ x)


def test_compressed_solution(ico2_blocks):
    top, TA, V = ico2_blocks
    k, tol = 1.0, 1e-4
    dn = hm.near_distance(top)
    HA = hm.HMatrix(TA, hm.cluster_tree(*hm.edge_boxes(top), 16), 2.0, dn, tol).dense()
    HV = hm.HMatrix(V, hm.cluster_tree(*hm.cell_boxes(top), 16), 2.0, dn, tol).dense()
    kh, pol = synth.default_plane_wave()
    from oracle import rhs
    e = rhs.planewave(top, k, kh, pol)[0]
    sols = []
    for A_, V_ in ((TA, V), (HA, HV)):
        P = rfcmp.Preconditioner(top, A_, V_, k)
        P.k_scalings()
        b = P.rhs(e)
        i = rfcmp.cg(P.apply, b, 1e-12, 500)[0]
        sols.append(P.recover(i))
    err = np.linalg.norm(sols[1] - sols[0]) / np.linalg.norm(sols[0])
    assert err < 30 * tol
