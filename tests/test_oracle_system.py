"""Pins of the oracle's RF-CMP system, solver and solution (CPU only)."""
import numpy as np
import pytest

import synth
from oracle import assembly, rfcmp, rhs
from oracle.topology import Topology

from ._meshes import blocks, excitation, precond, rel, topo


# ---------------------------------------------------------------- projectors
@pytest.mark.parametrize("name", ["ico1", "torus_small"])
def test_projector_identities(name):
    """P_S^2 = P_S = P_S^T, P_S P_LH = 0, P_S + P_LH = I (Sec. 2)."""
    pre = precond(name, 0.5)
    PS, PL = pre.P_S, pre.P_LH
    assert np.abs(PS @ PS - PS).max() < 1e-12
    assert np.abs(PS - PS.T).max() < 1e-12
    assert np.abs(PS @ PL).max() < 1e-12
    assert np.abs(PS + PL - np.eye(len(PS))).max() == 0.0
    top = pre.top
    assert np.abs(PS @ top.Lambda).max() < 1e-12       # loops are solenoidal
    assert np.abs(PS @ top.Sigma - top.Sigma).max() < 1e-12


def test_gram_weighted_star_map():
    """P_gS has the range of Sigma, kills loops, but is not idempotent."""
    pre = precond("ico1", 0.5)
    P = pre.P_gS
    assert np.abs(P @ pre.top.Lambda).max() < 1e-12
    assert np.abs(pre.P_LH @ P).max() < 1e-12
    assert np.abs(P @ P - P).max() > 1e-3


# ---------------------------------------------------------------- system
@pytest.mark.parametrize("name,k", [("ico1", 0.5), ("ico2", 1.0), ("torus_small", 0.5)])
@pytest.mark.parametrize("star", ["sigma", "gsigma"])
def test_direct_equals_split(name, k, star):
    pre = precond(name, k, star)
    A1 = pre.system_direct()
    A2 = pre.system_split()
    assert rel(A2, A1) < 1e-11


@pytest.mark.parametrize("k", [1e-4, 0.5])
def test_hermitian_positive_definite(k):
    """Remark of Sec. 3.1/3.3: the system matrix is HPD."""
    pre = precond("ico1", k)
    A = pre.system_split()
    assert np.abs(A - A.conj().T).max() < 1e-12 * np.abs(A).max()
    assert np.linalg.eigvalsh(0.5 * (A + A.conj().T))[0] > 0.05


def test_adjoint_by_conjugation():
    """T^H x = conj(T conj(x)) for the complex-symmetric EFIE matrix (Sec. 3.4)."""
    pre = precond("ico1", 0.5)
    T = pre.T()
    x = synth.complex_start(pre.top.N, 3)
    assert rel(np.conj(T @ np.conj(x)), T.conj().T @ x) < 1e-12


def _expansion_terms(k):
    pre = precond("ico1", k, "gsigma", "k")
    TA, TP = pre.TA, pre.TPhi
    H = lambda M: M.conj().T
    Plh, Pgs = pre.P_LH, pre.P_gS
    PmL = pre.ML_hat + pre.P_LH        # P_mL of Sec. 3 (unscaled)
    PmS = pre.MS_hat                   # bar P_mS of Sec. 3 (unscaled)
    printed = (H(Plh) @ H(TA) @ PmL @ TA @ Plh + H(Pgs) @ H(TP) @ PmS @ TP @ Pgs
               + k ** 2 * H(Pgs) @ H(TA) @ PmL @ TA @ Pgs + k ** 4 * H(Pgs) @ H(TA) @ PmS @ TA @ Pgs
               + 1j * k * H(Plh) @ H(TA) @ PmL @ TA @ Pgs - 1j * k * H(Pgs) @ H(TA) @ PmL @ TA @ Plh
               + 1j * k ** 3 * H(Plh) @ H(TA) @ PmS @ TA @ Pgs - 1j * k ** 3 * H(Pgs) @ H(TA) @ PmS @ TA @ Plh
               - 1j * k * H(Plh) @ H(TA) @ PmS @ TP @ Pgs + 1j * k * H(Pgs) @ H(TP) @ PmS @ TA @ Plh)
    missing = (k ** 2 * H(Plh) @ H(TA) @ PmS @ TA @ Plh - k ** 2 * H(Pgs) @ H(TA) @ PmS @ TP @ Pgs
               - k ** 2 * H(Pgs) @ H(TP) @ PmS @ TA @ Pgs)
    return pre.system_direct(), printed, missing


def test_k_explicit_expansion():
    """Eq. LastProofBigUmformung (alpha = sqrt(k), beta = 1/sqrt(k), gamma = k,
    Gram-weighted star map).  Multiplying out X^H P_m X with
    X = T P_o = i sqrt(k) T_A P_LH - k^1.5 T_A P_gS + k^-0.5 T_Phi P_gS gives the
    ten printed terms plus three O(k^2) terms the printed expansion omits:
    k^2 P_LH^H T_A^H P_mS T_A P_LH - k^2 P_gS^H T_A^H P_mS T_Phi P_gS
    - k^2 P_gS^H T_Phi^H P_mS T_A P_gS.  With them the expansion is exact; the
    printed ten terms alone differ by O(k^2), which leaves the static limit
    of the proof unchanged."""
    A, printed, missing = _expansion_terms(0.5)
    assert rel(printed + missing, A) < 1e-11
    e1 = rel(printed, A)
    A2, printed2, missing2 = _expansion_terms(0.05)
    assert rel(printed2 + missing2, A2) < 1e-9
    e2 = rel(printed2, A2)
    assert 50 < e1 / e2 < 200           # O(k^2)


def test_static_limit_principal_part():
    """Sec. 3.3: the system tends to its two principal terms as k -> 0, with
    an O(k) remainder."""
    r = []
    for k in (1e-2, 1e-3):
        pre = precond("ico1", k, "gsigma", "k")
        H = lambda M: M.conj().T
        princ = (H(pre.P_LH) @ H(pre.TA) @ (pre.ML_hat + pre.P_LH) @ pre.TA @ pre.P_LH
                 + H(pre.P_gS) @ H(pre.TPhi) @ pre.MS_hat @ pre.TPhi @ pre.P_gS)
        r.append(rel(pre.system_split(), princ))
    assert r[0] < 0.1
    assert 0.05 < r[1] / r[0] < 0.2


def test_condition_flat_in_k_and_h():
    """Main claim (Sec. 3.3 proposition; Figs. SphereF/SphereH): cond(A)
    bounded independently of k and h."""
    conds = []
    for name in ("ico1", "ico2"):
        for k in (1e-1, 1e-3, 1e-6):
            A = precond(name, k).system_split()
            ev = np.linalg.eigvalsh(0.5 * (A + A.conj().T))
            conds.append(ev[-1] / ev[0])
    assert max(conds) < 20 and max(conds) / min(conds) < 2.0


@pytest.mark.parametrize("k", [1e-4, 0.5])
def test_cg_iteration_bound(k):
    """Eq. Niter: CG needs at most ceil(1/2 sqrt(cond) log(2/eps)) iterations."""
    pre = precond("ico1", k)
    A = pre.system_split()
    ev = np.linalg.eigvalsh(0.5 * (A + A.conj().T))
    b = pre.rhs(excitation("ico1", k))
    eps = 1e-10
    _, its, res = rfcmp.cg(pre.apply, b, eps, 500)
    assert res <= eps
    assert its <= rfcmp.iteration_bound(ev[-1] / ev[0], eps)


def test_power_iteration_converges_to_norm():
    pre = precond("ico1", 0.5)
    Oa, Ob, Og = pre.scaling_operators()
    for op in (Oa, Ob, Og):
        M = op(np.eye(pre.top.N, dtype=complex))
        lam = np.linalg.eigvalsh(0.5 * (M + M.conj().T))[-1]
        est = rfcmp.power_norm(op, synth.complex_start(pre.top.N, 4), 30)
        # an estimate from below; the sphere's near-degenerate top eigenvalues
        # (gap ~1 %) limit 30 steps to ~3e-3
        assert est <= lam * (1 + 1e-12) and (lam - est) / lam < 1e-2


# ---------------------------------------------------------------- solution
@pytest.mark.parametrize("name,k", [("ico1", 0.5), ("ico2", 1.0), ("torus_small", 0.5)])
def test_three_routes_agree(name, k):
    """R1 (plain Galerkin LU), R2 (dense RF-CMP) and R3 (RF-CMP + CG)."""
    pre = precond(name, k)
    e = excitation(name, k)
    j1 = -np.linalg.solve(pre.T(), e)
    i2 = np.linalg.solve(pre.system_split(), pre.rhs(e))
    j2 = pre.recover(i2)
    i3, _, _ = rfcmp.cg(pre.apply, pre.rhs(e), 1e-12, 500)
    j3 = pre.recover(i3)
    assert rel(j2, j1) < 1e-9 and rel(j3, j2) < 1e-10


def test_low_frequency_routes():
    """At ka = 1e-4, R2 = R3 to the solve tolerance, for both star maps."""
    k = 1e-4
    js = []
    for star in ("sigma", "gsigma"):
        pre = precond("ico1", k, star)
        e = excitation("ico1", k)
        j2 = pre.recover(np.linalg.solve(pre.system_split(), pre.rhs(e)))
        i3, _, res = rfcmp.cg(pre.apply, pre.rhs(e), 1e-11, 500)
        assert res <= 1e-11
        assert rel(pre.recover(i3), j2) < 1e-9
        js.append(j2)
    assert rel(js[1], js[0]) < 1e-8


def test_solution_independent_of_scalings():
    """App.: j = -T^-1 e for every admissible alpha, beta, gamma and P_s."""
    k = 0.3
    e = excitation("ico1", k)
    ref = None
    for star, scal in (("sigma", "power"), ("gsigma", "power"), ("sigma", "k"), ("gsigma", "k")):
        pre = precond("ico1", k, star, scal)
        j = pre.recover(np.linalg.solve(pre.system_split(), pre.rhs(e)))
        if ref is None:
            ref = j
        assert rel(j, ref) < 1e-10


def _static_errors(name, k):
    pre = precond(name, k)
    e = excitation(name, k)
    i, _, _ = rfcmp.cg(pre.apply, pre.rhs(e), 1e-10, 500)
    j = pre.recover(i)
    top = pre.top
    loop_ref = 1.5 * top.Lambda @ top.xyz[:, 1]
    charge_ref = 3j * k * top.area * top.centroid[:, 0]
    return rel(pre.P_LH @ j, loop_ref), rel(top.Sigma.T @ j, charge_ref)


def test_static_limit_physics():
    """Unit PEC sphere, khat = z, pol = x, k -> 0: magnetostatic current
    j = (3/2) n x y_hat = (3/2) Lam y and electrostatic charge
    div j = 3 i k x (textbook statics of a conducting sphere); the
    discretisation error falls with h."""
    l1, q1 = _static_errors("ico1", 1e-4)
    l2, q2 = _static_errors("ico2", 1e-4)
    assert l2 < 0.02 and q2 < 0.04
    assert l2 < 0.75 * l1 and q2 < 0.5 * q1


def test_torus_global_loops_solved():
    """Genus-1 torus: the harmonic part of j is non-zero and captured
    without any global-loop search (Sec. 2, the reason for projectors)."""
    pre = precond("torus_small", 0.5)
    top = pre.top
    e = excitation("torus_small", 0.5)
    j = pre.recover(np.linalg.solve(pre.system_split(), pre.rhs(e)))
    PL = top.Lambda @ np.linalg.pinv(top.Lambda.T @ top.Lambda) @ top.Lambda.T
    PH = np.eye(top.N) - pre.P_S - PL
    assert np.linalg.norm(PH @ j) > 1e-3 * np.linalg.norm(j)
    assert rel(j, -np.linalg.solve(pre.T(), e)) < 1e-9


# ---------------------------------------------------------------- planted mistakes
def _mutant_static_errors(k=1e-4):
    top = Topology(*synth.icosphere(1))
    TA, V = assembly.assemble(top, k)
    pre = rfcmp.Preconditioner(top, TA, V, k)
    pre.power_scalings(synth.complex_start(top.N, 11), 30)
    kh, pol = synth.default_plane_wave()
    e = rhs.planewave(top, k, kh, pol)[0]
    j = pre.recover(np.linalg.solve(pre.system_split(), pre.rhs(e)))
    loop = rel(pre.P_LH @ j, 1.5 * top.Lambda @ top.xyz[:, 1])
    charge = rel(top.Sigma.T @ j, 3j * k * top.area * top.centroid[:, 0])
    return max(loop, charge)


def _half_scalar_potential(real):
    def f(P, r):
        S, Vv = real(P, r)
        return 0.5 * S, Vv
    return f


def _flipped_rhs(real):
    def f(top, k, kh, pol):
        return -real(top, k, kh, pol)
    return f


def _wrong_smooth_sign(real):
    def f(k, R):
        return -real(k, R)
    return f


def _gram_ll_times_two(real):
    def f(top):
        return 2.0 * real(top)
    return f


def _near_far_mismatch(k=1.0):
    """Largest relative gap between the singular-extraction and the plain
    7x7 path on well-separated pairs (the pin of test_oracle_blocks)."""
    from oracle import quadrature
    top = topo("ico1")
    pts, w = quadrature.tri7_points(top.xyz, top.tri)
    near = assembly.near_mask(top)
    _, Vm = assembly.assemble(top, k)
    worst = 0.0
    pairs = [(c, cp) for c in (0, 3, 10) for cp in range(top.C) if not near[c, cp]][::17][:6]
    for c, cp in pairs:
        _, vn = assembly.near_block(top, c, cp, k, pts, w)
        worst = max(worst, abs(vn - Vm[c, cp]) / abs(Vm[c, cp]))
    return worst


MUTATIONS = [
    ("assembly", "potentials", _half_scalar_potential, _mutant_static_errors),  # wrong factor
    ("rhs", "planewave", _flipped_rhs, _mutant_static_errors),                  # wrong sign of e
    ("assembly", "_g_smooth", _wrong_smooth_sign, _near_far_mismatch),          # wrong sign of a term
]


@pytest.mark.parametrize("mod,attr,mut,pin", MUTATIONS)
def test_pins_catch_planted_mistakes(monkeypatch, mod, attr, mut, pin):
    """A plausible mistake planted in the oracle (wrong factor, wrong sign)
    must fail a pin that the correct oracle passes."""
    good = pin()
    import oracle
    target = getattr(oracle, mod)
    monkeypatch.setattr(target, attr, mut(getattr(target, attr)))
    bad = pin()
    assert good < 0.07 and bad > 3 * good


def test_middle_gram_mistake_changes_system_not_solution(monkeypatch):
    """A wrong Gram matrix inside P_m (G_ll doubled) changes the system
    matrix A but not j = -T^-1 e: A i = b is equivalent to T P_o i = -e for
    any HPD middle matrix.  So the planted mistake must move A by far more
    than rounding while the recovered j stays put; the graded-mesh
    conditioning pin below is what catches a wrong Gram there."""
    from oracle import grams
    k = 0.5
    top = topo("ico1")
    TA, V = blocks("ico1", k)
    e = excitation("ico1", k)

    def solve():
        pre = rfcmp.Preconditioner(top, TA, V, k)
        pre.set_scalings(1.0, 1.0, 1.0)
        A = pre.system_split()
        return A, pre.recover(np.linalg.solve(A, pre.rhs(e)))

    A_good, j_good = solve()
    monkeypatch.setattr(grams, "gram_ll", _gram_ll_times_two(grams.gram_ll))
    A_bad, j_bad = solve()
    assert rel(A_bad, A_good) > 1e-2
    assert rel(j_bad, j_good) < 1e-10


def _graded_condition(k=1e-3):
    """cond(A) on a strongly graded sphere (areas spread 15x)."""
    top = Topology(*synth.graded_sphere(1, 0.8))
    TA, V = assembly.assemble(top, k)
    pre = rfcmp.Preconditioner(top, TA, V, k)
    pre.power_scalings(synth.complex_start(top.N, 11), 40)
    A = pre.system_split()
    ev = np.linalg.eigvalsh(0.5 * (A + A.conj().T))
    return ev[-1] / ev[0]


def test_condition_bounded_on_graded_mesh():
    """The star middle matrix P_mS = Sigma L^+ G_pp^-1 L^+ Sigma^T (Sec. 3)
    must weigh each cell by its area (G_pp^-1 = diag(A), the inverse Gram of
    the cell functions 1/A) for the Calderon pairing with T_Phi to hold
    independently of the local mesh size.  On a sphere graded to a 15x spread
    of cell areas, cond(A) stays at the uniform mesh's level (about 10 against
    6.8); a middle matrix with diag(1/A) instead leaves cond(A) above 1000."""
    assert _graded_condition() < 15.0


def test_graded_pin_catches_inverted_cell_gram(monkeypatch):
    """Plant G_pp = diag(A) (so that P_mS carries diag(1/A)): the graded-mesh
    pin must fail."""
    from oracle import grams
    monkeypatch.setattr(grams, "gram_pp", lambda top: np.diag(top.area))
    assert _graded_condition() > 100.0


@pytest.mark.parametrize("name,k", [("ico1", 1e-3), ("ico1", 0.5), ("torus_small", 0.5)])
def test_scaled_principal_terms_unit_norm(name, k):
    """Reading of the Sec. 4 norms with the EFIE's k factors (i k T_A and
    T_Phi/(i k)): with the power-iteration scalings, each principal term of
    the system, formed here from the dense matrices,
      (k^2/alpha^4)   P_LH^H T_A^H Lam G_ll^-1 Lam^T T_A P_LH,
      1/(k^2 beta^4)  P_S^H T_Phi^H (bar P_mS) T_Phi P_S,
      k^2/(alpha^2 gamma) P_LH^H T_A^H P_LH T_A P_LH,
    has unit 2-norm.  The power iteration approaches each norm from below, so
    each term's norm is at least 1 and, after 60 steps, within 2 %.  Without
    the k factors the terms would be off by k^-2, k^2 and k^-2 (the test uses
    k != 1)."""
    top = topo(name)
    TA, V = blocks(name, k)
    pre = rfcmp.Preconditioner(top, TA, V, k)
    al, be, ga, *_ = pre.power_scalings(synth.complex_start(top.N, 11), 60)
    H = lambda M: M.conj().T
    terms = [(k * k / al ** 4) * H(pre.P_LH) @ H(TA) @ pre.ML_hat @ TA @ pre.P_LH,
             (1.0 / (k * k * be ** 4)) * H(pre.P_S) @ H(pre.TPhi) @ pre.MS_hat @ pre.TPhi @ pre.P_S,
             (k * k / (al ** 2 * ga)) * H(pre.P_LH) @ H(TA) @ pre.P_LH @ TA @ pre.P_LH]
    for t in terms:
        assert 1.0 - 1e-9 <= np.linalg.norm(t, 2) < 1.02


@pytest.mark.parametrize("name,k", [("ico2", 1.0), ("ico2", 1e-4), ("torus_small", 0.5)])
def test_power_iteration_early_stop(name, k):
    """The adaptive stop of the power iteration: with tol = 0 the three
    operators iterated side by side give exactly the separate power_norm
    estimates; with tol = 1e-2 it stops at a check (a multiple of 5 steps,
    at least 10), every scaling within 3e-2 of its 60-step value, and CG
    needs the same number of iterations on the resulting system."""
    top = topo(name)
    TA, V = blocks(name, k)
    start = synth.complex_start(top.N, 11)
    pre = rfcmp.Preconditioner(top, TA, V, k)
    Oa, Ob, Og = pre.scaling_operators()
    *_, lam, n = pre.power_scalings(start, 30)
    assert n == 30 and lam == tuple(rfcmp.power_norm(o, start, 30) for o in (Oa, Ob, Og))
    e = rhs.planewave(top, k, *synth.default_plane_wave())[0]
    ref = pre.power_scalings(start, 60)[:3]
    it_ref = rfcmp.cg(lambda x: pre.system_split() @ x, pre.rhs(e), 1e-6, 1000)[1]
    a, b, g, _, n = pre.power_scalings(start, 30, tol=1e-2)
    assert n % rfcmp.POWER_CHECK == 0 and 2 * rfcmp.POWER_CHECK <= n < 30, n
    assert all(abs(x - y) < 3e-2 * y for x, y in zip((a, b, g), ref))
    A = pre.system_split()
    assert rfcmp.cg(lambda x: A @ x, pre.rhs(e), 1e-6, 1000)[1] == it_ref


def test_efie_condition_grows_as_kh_minus_two():
    """Introduction: cond(T) of the plain EFIE grows as (k h)^-2: a tenfold
    smaller k multiplies it by about 100 (low-frequency breakdown), and halving
    h (icosphere level 1 -> 2) by about 4 (dense-discretisation breakdown),
    while cond(A) of the RF-CMP system stays put (test_condition_flat_in_k_and_h)."""
    c = {}
    for name in ("ico1", "ico2"):
        for k in (1e-2, 1e-3):
            TA, V = blocks(name, k)
            c[name, k] = rfcmp.efie_condition(topo(name), TA, V, k)
    for name in ("ico1", "ico2"):
        assert 80 < c[name, 1e-3] / c[name, 1e-2] < 120
    assert 2.5 < c["ico2", 1e-3] / c["ico1", 1e-3] < 6.0
