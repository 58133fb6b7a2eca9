"""Pins of the oracle's singular potentials, Galerkin blocks and excitation."""
import numpy as np
import pytest
from scipy import integrate

import synth
from oracle import assembly, quadrature, rhs, singular
from oracle.topology import Topology

from ._meshes import blocks, topo

FOUR_PI = 4.0 * np.pi


# ---------------------------------------------------------------- brute force
def _polar_potentials(P, r):
    """S and int (r'-r)/R by adaptive quadrature in polar coordinates about
    the projection of r (signed sub-triangles), independent of the closed
    forms."""
    n = np.cross(P[1] - P[0], P[2] - P[0])
    n /= np.linalg.norm(n)
    d = (r - P[0]) @ n
    rho = r - d * n
    S, W = 0.0, np.zeros(3)
    for i in range(3):
        a, b = P[i], P[(i + 1) % 3]
        e1, e2 = a - rho, b - rho
        sgn = np.sign(np.cross(e1, e2) @ n)
        if sgn == 0:
            continue
        J = np.linalg.norm(np.cross(e1, e2))

        def f(u, v, comp):
            x = u * (e1 + v * (e2 - e1))
            val = u * J / np.sqrt(x @ x + d * d)
            return val if comp < 0 else val * x[comp]

        opts = dict(epsabs=1e-13, epsrel=1e-13)
        S += sgn * integrate.dblquad(lambda u, v: f(u, v, -1), 0, 1, 0, 1, **opts)[0]
        for comp in range(3):
            W[comp] += sgn * integrate.dblquad(lambda u, v, c=comp: f(u, v, c), 0, 1, 0, 1, **opts)[0]
    return S, W - d * n * S


TRI = np.array([[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.2, 0.9, 0.0]])
POINTS = [
    [0.3, 0.3, 0.0],      # inside, in plane (the self-pair case)
    [0.3, 0.3, 0.2],      # above the inside
    [0.4, 0.3, -1e-3],    # just below the inside
    [1.5, 0.15, 0.0],     # in plane, outside
    [1.1, -0.2, 0.05],    # near a vertex, off plane
    [2.0, -1.0, 0.5],     # far
]


@pytest.mark.parametrize("r", POINTS)
def test_singular_potentials_vs_polar_quadrature(r):
    r = np.array(r)
    S, Vv = singular.potentials(TRI, r[None])
    Sb, Vb = _polar_potentials(TRI, r)
    assert abs(S[0] - Sb) < 1e-12
    assert np.abs(Vv[0] - Vb).max() < 1e-12


def test_singular_potentials_on_edge_line():
    """Point on the extension of an edge line (coplanar neighbours)."""
    P = TRI
    r = P[0] + 1.7 * (P[1] - P[0])
    S, Vv = singular.potentials(P, r[None])
    Sb, Vb = _polar_potentials(P, r)
    assert abs(S[0] - Sb) < 1e-11 and np.abs(Vv[0] - Vb).max() < 1e-11


# ---------------------------------------------------------------- blocks
def _subdivide(P, levels):
    tris = [P]
    for _ in range(levels):
        nxt = []
        for a, b, c in tris:
            ab, bc, ca = (a + b) / 2, (b + c) / 2, (c + a) / 2
            nxt += [np.array([a, ab, ca]), np.array([b, bc, ab]), np.array([c, ca, bc]), np.array([ab, bc, ca])]
        tris = nxt
    return tris


def _fine_rule(P, levels=2):
    """Points and absolute weights of the degree-5 rule on 4^levels pieces."""
    bary, w = quadrature.tri7_barycentric()
    pts, wts = [], []
    for t in _subdivide(P, levels):
        A = 0.5 * np.linalg.norm(np.cross(t[1] - t[0], t[2] - t[0]))
        pts.append(bary @ t)
        wts.append(A * w)
    return np.concatenate(pts), np.concatenate(wts)


def _block_by_definition(top, c, cp, k, levels=2):
    """sigma sigma'/(4 A A') int int (r - r_i).(r' - r_j) G and V_cc' directly
    from the definitions, on subdivided cells (far pairs only)."""
    x, wx = _fine_rule(top.xyz[top.tri[c]], levels)
    y, wy = _fine_rule(top.xyz[top.tri[cp]], levels)
    R = np.linalg.norm(x[:, None] - y[None], axis=-1)
    G = np.exp(1j * k * R) / (FOUR_PI * R) * wx[:, None] * wy[None]
    B = np.zeros((3, 3), dtype=complex)
    for i in range(3):
        for j in range(3):
            ai = x - top.xyz[top.tri[c, i]]
            bj = y - top.xyz[top.tri[cp, j]]
            B[i, j] = np.sum(G * (ai @ bj.T))
    B *= np.outer(top.cell_sign[c], top.cell_sign[cp]) / (4 * top.area[c] * top.area[cp])
    return B, G.sum() / (top.area[c] * top.area[cp])


@pytest.mark.parametrize("k", [0.3, 2.0])
def test_far_blocks_vs_refined_definition(k):
    top = topo("ico2")
    TA, V, Bm = assembly.assemble(top, k, return_blocks=True)
    near = assembly.near_mask(top)
    rng = np.random.default_rng(1)
    checked = 0
    while checked < 6:
        c, cp = rng.integers(0, top.C, 2)
        if near[c, cp]:
            continue
        B, v = _block_by_definition(top, c, cp, k)
        got = Bm[3 * c:3 * c + 3, 3 * cp:3 * cp + 3]
        assert np.abs(got - B).max() < 2e-5 * np.abs(B).max()
        assert abs(V[c, cp] - v) < 2e-5 * abs(v)
        checked += 1


@pytest.mark.parametrize("k", [1e-3, 1.0])
def test_near_path_equals_far_path_when_separated(k):
    """The singular-extraction path and the plain 7x7 path compute the same
    integral; on well-separated cells they must agree to quadrature error."""
    top = topo("ico2")
    pts, w = quadrature.tri7_points(top.xyz, top.tri)
    _, _, Bm = assembly.assemble(top, k, return_blocks=True)
    _, Vm = blocks("ico2", k)
    near = assembly.near_mask(top)
    rng = np.random.default_rng(2)
    n = 0
    while n < 6:
        c, cp = sorted(rng.integers(0, top.C, 2))
        if near[c, cp]:
            continue
        Bn, vn = assembly.near_block(top, c, cp, k, pts, w)
        Bf = Bm[3 * c:3 * c + 3, 3 * cp:3 * cp + 3]
        assert np.abs(Bn - Bf).max() < 1e-5 * np.abs(Bf).max()
        assert abs(vn - Vm[c, cp]) < 1e-5 * abs(vn)
        n += 1


def test_touching_pairs_vs_refined_outer_rule():
    """Spec-Q accuracy on touching pairs: the outer 7-point rule against a
    subdivided outer rule (inner integral identical).  Reported bound: 2e-2."""
    top = topo("ico1")
    k = 1.0
    pts, w = quadrature.tri7_points(top.xyz, top.tri)
    near = assembly.near_mask(top)
    worst = 0.0
    for c in range(0, top.C, 9):
        for cp in np.nonzero(near[c])[0]:
            if cp == c:
                continue
            _, v = assembly.near_block(top, c, cp, k, pts, w)
            x, wx = _fine_rule(top.xyz[top.tri[c]], 3)
            S, _ = singular.potentials(top.xyz[top.tri[cp]], x)
            y = pts[cp]
            R = np.linalg.norm(x[:, None] - y[None], axis=-1)
            g = (np.exp(1j * k * R) - 1) / R
            ref = (np.sum(wx * S) / FOUR_PI + top.area[cp] * np.sum(wx[:, None] * w[None] * g) / FOUR_PI)
            ref /= top.area[c] * top.area[cp]
            worst = max(worst, abs(v - ref) / abs(ref))
    assert worst < 2e-2


@pytest.mark.parametrize("name", ["ico1", "torus_small", "cube2"])
def test_blocks_complex_symmetric(name):
    """T_A = T_A^T and V = V^T (used by the adjoint-by-conjugation identity of
    Sec. 3.4); equal up to summation-order rounding in the oracle."""
    TA, V = blocks(name, 0.7)
    assert np.abs(TA - TA.T).max() <= 1e-14 * np.abs(TA).max()
    assert np.abs(V - V.T).max() <= 1e-14 * np.abs(V).max()


@pytest.mark.parametrize("name", ["ico1", "torus_small"])
def test_tphi_annihilates_loops(name):
    top = topo(name)
    TA, V = blocks(name, 0.7)
    TPhi = top.Sigma @ V @ top.Sigma.T
    assert np.abs(TPhi @ top.Lambda).max() < 1e-13 * np.abs(TPhi).max()


@pytest.mark.parametrize("name", ["ico1", "cube2"])
def test_small_k_imaginary_parts(name):
    """Im G_k = k/(4 pi) + O(k^3 R^2): Im V_cc' = k/(4 pi) + O(k^3) and
    Im T_A[m,n] = (k/4pi) (int f_m).(int f_n) + O(k^3) with
    int f_m = sum_c sigma/2 (centroid_c - r_m^c)."""
    top = topo(name)
    k = 1e-3
    TA, V = blocks(name, k)
    assert np.abs(V.imag - k / FOUR_PI).max() < 10 * k ** 3
    F = np.zeros((top.N, 3))
    for c in range(top.C):
        for i in range(3):
            F[top.cell_edges[c, i]] += top.cell_sign[c, i] / 2 * (top.centroid[c] - top.xyz[top.tri[c, i]])
    ref = k / FOUR_PI * F @ F.T
    assert np.abs(TA.imag - ref).max() < 10 * k ** 3


# ---------------------------------------------------------------- excitation
@pytest.mark.parametrize("name", ["ico1", "cube2"])
def test_rhs_static_closed_form(name):
    """At k = 0: int f_n . p = -(Sigma (p . centroid))_n (integration by parts
    on the closed surface; exact for the degree-5 rule)."""
    top = topo(name)
    pol = np.array([[0.3, -0.5, 0.8]])
    e = rhs.planewave(top, 0.0, np.array([[0.0, 0.0, 1.0]]), pol)[0]
    ref = -(top.Sigma @ (top.centroid @ pol[0]))
    assert np.abs(e - ref).max() < 1e-14


def test_rhs_vs_refined_quadrature():
    top = topo("ico1")
    k = 2.0
    kh = np.array([0.0, 0.6, 0.8])
    pol = np.array([1.0, 0.0, 0.0])
    e = rhs.planewave(top, k, kh[None], pol[None])[0]
    ref = np.zeros(top.N, dtype=complex)
    for c in range(top.C):
        x, wx = _fine_rule(top.xyz[top.tri[c]], 3)
        for i in range(3):
            f = top.cell_sign[c, i] * (x - top.xyz[top.tri[c, i]]) / (2 * top.area[c])
            ref[top.cell_edges[c, i]] += np.sum(wx * (f @ pol) * np.exp(1j * k * (x @ kh)))
    assert np.abs(e - ref).max() < 1e-6 * np.abs(ref).max()


def test_sampled_rows_equal_full_assembly():
    """block_rows / ta_rows (used for sampled checks of full-size GPU blocks)
    reproduce the rows of the full assembly exactly: same spec, same
    functions, including near pairs on both sides of the diagonal."""
    xyz, tri = synth.torus(12, 8, jitter=0.01, seed=3)
    top = Topology(xyz, tri)
    TA, V = assembly.assemble(top, 0.7)
    cells = [0, 5, 17, top.C - 1]
    Vr, _ = assembly.block_rows(top, 0.7, cells)
    assert np.array_equal(Vr, V[cells])
    edges = [0, 3, 50, top.N - 1]
    assert np.array_equal(assembly.ta_rows(top, 0.7, edges), TA[edges])
