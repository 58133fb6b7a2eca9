"""Element-wise parity at the bench's full sizes, for the kernels it times.

The level-4 sphere (N = 7680, C = 5120) takes the 256-wide symmetric-block
products (chosen above n = 6912), the FP64 matrix-core products of 8 and
more right-hand sides, the paired T_A + V launches of the operator and the
power iteration, and the level-5 sphere with 64 right-hand sides the BF16x3
GEMM at the precision study's shape.  References:
* dense complex128 products of the exported complex64 blocks (exact
  conversion; only the summation order differs: 1e-13);
* the FP64 oracle's preconditioner built on the exported blocks, for the
  operator, the right-hand side, the recovery and the power scalings;
* the static closed forms of a PEC sphere at ka = 1e-4, the oracle's own
  physics pin, whose discretisation error falls with h (levels 1-3 of the
  oracle: loop part 1.4e-2, 7.1e-3, 2.6e-3; charge 6.6e-2, 1.9e-2, 6.0e-3).
"""
import functools

import numpy as np
import pytest

import synth
from oracle import rfcmp
from oracle.topology import Topology

from ._meshes import rel

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    import paper_1803_08333_amd as rf
    assert torch.cuda.is_available()
    return torch, rf


def _np(t):
    return t.detach().cpu().numpy()


def _cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).cuda()


@functools.lru_cache(maxsize=1)
def _ico4():
    torch, rf = _gpu()
    xyz, tri = synth.icosphere(4)
    top = Topology(xyz, tri)
    m = rf.Mesh(xyz, tri)
    return top, m


@functools.lru_cache(maxsize=2)
def _ico4_op(k):
    """Operator at power-iteration scalings (30 fixed steps), its exported
    blocks and the oracle's preconditioner on those blocks."""
    torch, rf = _gpu()
    top, m = _ico4()
    start = _cuda(synth.complex_start(m.N, 11))
    op = rf.Operator(m, k, power_start=start, power_tol=0.0)
    gTA, gV = op.export()
    pre = rfcmp.Preconditioner(top, _np(gTA).astype(np.complex128), _np(gV).astype(np.complex128), k)
    a, b, g, _ = op.scalings()
    pre.set_scalings(a, b, g)
    return op, gTA, gV, pre


@pytest.mark.parametrize("nrhs", [1, 2, 3, 4, 5, 8, 13, 16, 21, 32, 45])
@pytest.mark.parametrize("conj", [False, True])
def test_symv_256_blocks_match_complex128(nrhs, conj):
    """rfcmp_matvec which 0 (T_A, n = 7680) and 1 (V, n = 5120) at level 4:
    1 to 5 right-hand sides on the symmetric streaming products (the 4 + 1
    split included), 8 and more on the FP64 matrix-core products (up to 32
    per pass in groups of 16: 13, 21 and 45 = 32 + 13 leave a ragged group;
    they read the lower triangle that the symmetric products never do), with
    and without conjugation, against complex128 products of the exported
    blocks, as a whole and per right-hand side."""
    torch, rf = _gpu()
    op, gTA, gV, _ = _ico4_op(1.0)
    for which, M in ((0, gTA), (1, gV)):
        n = M.shape[0]
        x = _cuda(np.stack([synth.complex_start(n, 50 + r) for r in range(nrhs)]))
        M128 = M.to(torch.complex128)
        if conj:
            M128 = M128.conj().resolve_conj()
        ref = (M128 @ x.T).T
        got = op.matvec(which, x, conj)
        err = (torch.linalg.norm(got - ref) / torch.linalg.norm(ref)).item()
        col = (torch.linalg.norm(got - ref, dim=1) / torch.linalg.norm(ref, dim=1)).max().item()
        del M128
        assert err < 1e-13 and col < 1e-13, (which, err, col)


@pytest.mark.parametrize("k", [1.0, 1e-4])
def test_operator_steps_full_size(k):
    """rfcmp_apply, rfcmp_precond_rhs and rfcmp_recover at level 4 against
    the oracle's dense preconditioner on the exported blocks."""
    op, _, _, pre = _ico4_op(k)
    N = pre.top.N
    x = np.stack([synth.complex_start(N, 61 + r) for r in range(3)])
    assert rel(_np(op.apply(_cuda(x))), pre.apply(x.T).T) < 1e-11
    e = np.stack([synth.complex_start(N, 71)])
    assert rel(_np(op.precond_rhs(_cuda(e))), pre.rhs(e.T).T) < 1e-11
    assert rel(_np(op.recover(_cuda(x))), pre.recover(x.T).T) < 1e-12


def test_power_scalings_full_size():
    """The power iteration's paired T_A + V launches (two plus one columns)
    at level 4: 30 fixed steps against the oracle's power iteration on the
    exported blocks, from the same start vector."""
    op, _, _, pre = _ico4_op(1.0)
    ref = pre.power_scalings(synth.complex_start(pre.top.N, 11), 30)
    a, b, g, lam = op.scalings()
    assert op.power_steps() == 30
    for got, want in zip((a, b, g), ref[:3]):
        assert abs(got - want) < 1e-10 * want
    # leave the scalings of the operator as they are for the other tests
    pre.set_scalings(a, b, g)


def test_static_limit_full_size():
    """Level 4 at ka = 1e-4 (the bench's low-frequency case): the solution's
    loop part against (3/2) Lambda y and its cell charges Sigma^T j against
    3 i k A_c x_c, the statics of a PEC sphere for khat = z, pol = x.  The
    oracle's second-order trend (loop 2.6e-3, charge 6.0e-3 at level 3,
    falling about 2.8x and 3.1x per level) puts level 4 near 1e-3 and 2e-3."""
    torch, rf = _gpu()
    k = 1e-4
    op, _, _, pre = _ico4_op(k)
    top, m = _ico4()
    kh, pol = synth.default_plane_wave()
    j, st, info = op.solve(op.rhs_planewave(kh, pol), tol=1e-8, maxit=500)
    assert st == 0
    jl = _np(op.project(rf.PROJ_LH, j))[0]
    q = _np(op.project(rf.PROJ_SIGMA_T, j))[0]
    loop_ref = 1.5 * (top.Lambda @ top.xyz[:, 1])
    charge_ref = 3j * k * top.area * top.centroid[:, 0]
    el, eq = rel(jl, loop_ref), rel(q, charge_ref)
    print(f"level 4, ka = 1e-4: loop part {el:.2e}, charge {eq:.2e}")
    assert el < 2e-3 and eq < 4e-3


def test_bf16x3_gemm_full_size_sampled_rows():
    """The BF16x3 GEMM at the precision study's shape (level 5, N = 30720,
    C = 20480, 64 right-hand sides): seeded sampled rows of T_A X and V X,
    plain and conjugated, against complex128 products of the exported rows
    (3e-5, the per-product bound of the split: hi.hi + hi.lo + lo.hi in
    FP32).  The same rows of the FP64 matrix-core products (which 0 and 1:
    32 right-hand sides per pass, the headline's K slices), which form the
    right-hand side and the refinement residuals, to 1e-13 (FP64 sums of
    exactly widened entries; only the order differs)."""
    torch, rf = _gpu()
    xyz, tri = synth.icosphere(5)
    m = rf.Mesh(xyz, tri)
    op = rf.Operator(m, 2.0, scaling=1, precision=1)
    gTA, gV = op.export()
    rng = np.random.default_rng(23)
    for which, M, n in ((2, gTA, m.N), (3, gV, m.C), (0, gTA, m.N), (1, gV, m.C)):
        bound = 3e-5 if which >= 2 else 1e-13
        x = _cuda(np.stack([synth.complex_start(n, 400 + r) for r in range(64)]))
        rows = np.unique(np.r_[0, n - 1, rng.integers(0, n, 62)])
        ridx = torch.from_numpy(rows).cuda()
        R = M[ridx].to(torch.complex128)
        for conj in (False, True):
            Rc = R.conj().resolve_conj() if conj else R
            ref = (Rc @ x.T).T                      # [64][rows]
            got = op.matvec(which, x, conj)[:, ridx]
            err = (torch.linalg.norm(got - ref) / torch.linalg.norm(ref)).item()
            col = (torch.linalg.norm(got - ref, dim=1) / torch.linalg.norm(ref, dim=1)).max().item()
            print(f"which {which} conj {conj}: sampled-row rel err {err:.2e}, worst right-hand side {col:.2e}")
            assert err < bound and col < 10 * bound
        del R
    del gTA, gV
    op.close()
    m.close()
