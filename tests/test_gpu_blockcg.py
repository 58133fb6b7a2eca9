"""Block CG over a shared Krylov space (options.block_cg = 1) through the C
ABI: the solutions of many right-hand sides against the oracle's dense
solutions (the same tolerances as the independent CGs: 1e-5 on the
complex64/FP64 path, 1e-6 after BF16x3 refinement), a rank-deficient block
(repeated right-hand sides, which the search block must drop), and the
iteration counts against the independent CGs at full size."""
import functools

import numpy as np
import pytest

import synth
from oracle import assembly, rfcmp, rhs
from oracle.topology import Topology

from ._meshes import rel

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=None)
def _oracle(lvl, k):
    top = Topology(*synth.icosphere(lvl))
    TA, V = assembly.assemble(top, k)
    pre = rfcmp.Preconditioner(top, TA, V, k)
    pre.power_scalings(synth.complex_start(top.N, 11), 30)
    return top, pre


def _gpu():
    import torch
    import paper_1803_08333_amd as rf
    assert torch.cuda.is_available()
    return torch, rf


@functools.lru_cache(maxsize=None)
def _mesh(lvl):
    torch, rf = _gpu()
    return rf.Mesh(*synth.icosphere(lvl))


@functools.lru_cache(maxsize=None)
def _op(lvl, k, precision, block):
    torch, rf = _gpu()
    m = _mesh(lvl)
    start = torch.from_numpy(synth.complex_start(m.N, 11)).cuda()
    return rf.Operator(m, k, power_start=start, precision=precision, block_cg=block)


@pytest.mark.parametrize("precision,bound", [(0, 1e-5), (1, 1e-6)])
def test_block_cg_matches_oracle(precision, bound):
    torch, rf = _gpu()
    k = 1.0
    top, pre = _oracle(2, k)
    kh, pol = synth.plane_waves(16, 4)
    E = rhs.planewave(top, k, kh, pol)
    A = pre.system_split()
    op = _op(2, k, precision, 1)
    j, st, info = op.solve(torch.from_numpy(E).cuda(), tol=1e-8, maxit=500)
    assert st == 0
    J = j.cpu().numpy()
    errs = [rel(J[r], pre.recover(np.linalg.solve(A, pre.rhs(E[r])))) for r in range(len(E))]
    its = [i["iters"] for i in info]
    print("precision", precision, "max error", max(errs), "iterations", its[0], "residual",
          max(i["rel_residual"] for i in info))
    assert max(errs) < bound
    assert all(i["rel_residual"] <= 1e-8 for i in info)


def test_block_cg_repeated_right_hand_sides():
    """Eight right-hand sides of which only three are distinct (and one is a
    multiple of another): the block drops the dependent directions and every
    column converges to the solution of the independent CGs."""
    torch, rf = _gpu()
    k = 1.0
    kh, pol = synth.plane_waves(3, 9)
    opb = _op(2, k, 0, 1)
    opi = _op(2, k, 0, 0)
    e = opb.rhs_planewave(kh, pol)
    E = torch.stack([e[0], e[1], e[0], e[2], 2.5 * e[1], e[2], e[0], e[1]]).contiguous()
    jb, stb, infob = opb.solve(E, tol=1e-8, maxit=500)
    ji, sti, infoi = opi.solve(E, tol=1e-8, maxit=500)
    assert stb == 0 and sti == 0
    err = float(torch.linalg.norm(jb - ji) / torch.linalg.norm(ji))
    print("repeated right-hand sides: block vs independent", err, infob[0]["iters"], infoi[0]["iters"])
    assert err < 1e-6
    assert all(i["rel_residual"] <= 1e-8 for i in infob)


@pytest.mark.parametrize("precision", [0, 1])
def test_block_cg_full_size(precision):
    """Level-4 sphere, 32 plane waves, ka = 2: the block solutions against the
    independent ones (both to 1e-6), and no more iterations."""
    torch, rf = _gpu()
    opb = _op(4, 2.0, precision, 1)
    opi = _op(4, 2.0, precision, 0)
    kh, pol = synth.plane_waves(32, 4)
    e = opi.rhs_planewave(kh, pol)
    jb, stb, infob = opb.solve(e, tol=1e-6, maxit=500)
    ji, sti, infoi = opi.solve(e, tol=1e-6, maxit=500)
    assert stb == 0 and sti == 0
    err = float(torch.linalg.norm(jb - ji) / torch.linalg.norm(ji))
    itb, iti = infob[0]["iters"], max(i["iters"] for i in infoi)
    print("level 4, precision", precision, "block vs independent", err, "iterations", itb, iti)
    assert err < 1e-5
    assert itb <= iti
