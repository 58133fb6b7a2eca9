"""Pins of the oracle's quadrature rule, topology and Gram matrices (CPU only).

Each check compares the oracle with something the paper or mathematics fixes
independently of the oracle's own formulas.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import grams, quadrature
from oracle.topology import MeshError, Topology

from ._meshes import mesh, topo

MESHES = ["ico0", "ico1", "ico2", "torus_small", "cube2", "ellipsoid1"]


# ---------------------------------------------------------------- quadrature
def test_tri7_exact_to_degree5():
    """Closed form int_T x^a y^b = a! b! / (a+b+2)! on the unit right triangle."""
    bary, w = quadrature.tri7_barycentric()
    # vertices (0,0), (1,0), (0,1); area 1/2
    x, y = bary[:, 1], bary[:, 2]
    for deg in range(6):
        for a in range(deg + 1):
            b = deg - a
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            got = 0.5 * np.sum(w * x ** a * y ** b)
            assert abs(got - exact) < 1e-15, (a, b)
    # and not exact at degree 6 (so it is the degree-5 rule, not a higher one)
    got = 0.5 * np.sum(w * x ** 6)
    assert abs(got - math.factorial(6) / math.factorial(8)) > 1e-6


def test_tri7_points_inside_and_symmetric():
    bary, w = quadrature.tri7_barycentric()
    assert np.all(bary > 0) and np.allclose(bary.sum(1), 1.0)
    assert abs(w.sum() - 1.0) < 1e-15 and np.all(w > 0)


# ---------------------------------------------------------------- topology
@pytest.mark.parametrize("name", MESHES)
def test_euler_and_genus(name):
    top = topo(name)
    assert top.V - top.N + top.C == 2 - 2 * top.genus
    assert top.genus == (1 if name.startswith("torus") else 0)
    assert 2 * top.N == 3 * top.C


@pytest.mark.parametrize("name", MESHES)
def test_null_vectors_and_orthogonality(name):
    """Lambda 1 = 0, Sigma 1 = 0 and Lambda^T Sigma = 0, exactly in integers."""
    top = topo(name)
    assert np.all(top.Lambda @ np.ones(top.V) == 0)
    assert np.all(top.Sigma @ np.ones(top.C) == 0)
    assert np.all(top.Lambda.T @ top.Sigma == 0)


@pytest.mark.parametrize("name", ["ico1", "torus_small", "cube2"])
def test_harmonic_projector_rank(name):
    """P_H = I - P_Lambda - P_Sigma is the projector on the 2g global loops."""
    top = topo(name)
    PS = top.Sigma @ np.linalg.pinv(top.Sigma.T @ top.Sigma) @ top.Sigma.T
    PL = top.Lambda @ np.linalg.pinv(top.Lambda.T @ top.Lambda) @ top.Lambda.T
    PH = np.eye(top.N) - PS - PL
    assert abs(np.trace(PH) - 2 * top.genus) < 1e-8
    assert np.abs(PH @ PH - PH).max() < 1e-9


def test_rwg_divergence_and_flux():
    """div f_n = Sigma[n,c]/A_c and the flux of f_n across edge n is 1."""
    top = topo("ico1")
    for n in range(0, top.N, 7):
        cp, lp = top.cplus[n], top.lplus[n]
        a, b = top.xyz[top.edges[n, 0]], top.xyz[top.edges[n, 1]]
        rp = top.xyz[top.free_plus[n]]
        mid = 0.5 * (a + b)
        f = (mid - rp) / (2 * top.area[cp])
        # outward normal of c+ across the edge, in the cell plane
        t = (b - a) / np.linalg.norm(b - a)
        m = np.cross(t, top.normal[cp])
        assert abs(np.dot(f, m) * np.linalg.norm(b - a) - 1.0) < 1e-12
        assert top.tri[cp, lp] == top.free_plus[n]


def test_mesh_errors():
    xyz, tri = mesh("ico0")
    with pytest.raises(MeshError):
        Topology(xyz, tri[:-1])                      # open
    bad = tri.copy()
    bad[0] = bad[0][[0, 2, 1]]
    with pytest.raises(MeshError):
        Topology(xyz, bad)                           # orientation
    deg = xyz.copy()
    t0 = tri[0]
    deg[t0[2]] = 0.5 * (deg[t0[0]] + deg[t0[1]])
    with pytest.raises(MeshError):
        Topology(deg, tri)                           # zero-area cell


# ---------------------------------------------------------------- Grams
def _dual_hat_nodes(top, m, n):
    """Nodal values of the dual hat of cell m on cell n, from its definition.

    Partition of unity: 1 at the own barycentre, 1/2 at the own edge
    midpoints (two dual hats meet there), 1/NoC(v) at the own vertices, zero
    on the boundary of the support (other barycentres and midpoints of edges
    not of cell m).  Returns (bary, {vertex: value}, {edge(a,b): value}).
    """
    vm = set(top.tri[m].tolist())
    bc = 1.0 if m == n else 0.0
    vals = {}
    for v in top.tri[n]:
        vals[int(v)] = 1.0 / top.noc[v] if v in vm else 0.0
    mids = {}
    for i in range(3):
        a, b = int(top.tri[n, (i + 1) % 3]), int(top.tri[n, (i + 2) % 3])
        mids[(a, b)] = 0.5 if (a in vm and b in vm) else 0.0
    return bc, vals, mids


def _gram_tp_by_integration(top):
    """(1/A_n) int_{c_n} dual_hat_m, on the 6 barycentric sub-triangles where
    the dual hat is linear, with the degree-5 rule (exact for linear)."""
    bary, w = quadrature.tri7_barycentric()
    G = np.zeros((top.C, top.C))
    cells_at = [[] for _ in range(top.V)]
    for c in range(top.C):
        for v in top.tri[c]:
            cells_at[v].append(c)
    for m in range(top.C):
        neigh = set()
        for v in top.tri[m]:
            neigh.update(cells_at[v])
        for n in neigh:
            bc, vals, mids = _dual_hat_nodes(top, m, n)
            total = 0.0
            for i in range(3):
                a, b = int(top.tri[n, (i + 1) % 3]), int(top.tri[n, (i + 2) % 3])
                for v in (a, b):
                    nodes = np.array([bc, vals[v], mids[(a, b)]])
                    sub_area = top.area[n] / 6.0
                    total += sub_area * np.sum(w * (bary @ nodes))
            G[m, n] = total / top.area[n]
    return G


@pytest.mark.parametrize("name", ["ico1", "torus_small", "cube2", "ellipsoid1"])
def test_gram_tp_closed_form_vs_integration(name):
    top = topo(name)
    assert np.abs(grams.gram_tp(top) - _gram_tp_by_integration(top)).max() < 1e-14


@pytest.mark.parametrize("name", MESHES)
def test_gram_tp_column_sums(name):
    """Lemma mixedGramEig: 1 is an eigenvector of G_tp^-T (column sums are 1)."""
    G = grams.gram_tp(topo(name))
    assert np.abs(G.sum(axis=0) - 1.0).max() < 1e-14
    assert np.abs(np.linalg.solve(G.T, np.ones(len(G))) - 1.0).max() < 1e-12
    # corollary: G^-1 maps mean-free vectors to mean-free vectors
    x = np.random.default_rng(0).normal(size=len(G))
    x -= x.mean()
    assert abs(np.linalg.solve(G, x).sum()) < 1e-12


def test_dual_hat_figure_values(root):
    """Figure DPLF: the dual hat is 1 at the barycentre, 1/2 at the midpoints
    and 1/NoC at the vertices (NoC = 5, 6, 4 in the figure)."""
    with open(os.path.join(root, "tests", "golden", "fig_dplf_dual_hat.json")) as f:
        gold = json.load(f)
    # a closed mesh with a cell whose vertices meet 5, 6 and 4 cells: flip
    # edges of a level-1 icosphere until one appears.
    xyz, tri = mesh("ico1")
    tri = tri.astype(np.int64).copy()
    want = sorted(gold["vertex_cell_counts"])
    found = None
    for attempt in range(len(tri)):
        top = Topology(xyz, tri)
        for c in range(top.C):
            if sorted(top.noc[top.tri[c]].tolist()) == want:
                found = (top, c)
                break
        if found:
            break
        # flip edge 'attempt' (a valid flip keeps the mesh closed and oriented)
        n = attempt
        cp, cm = top.cplus[n], top.cminus[n]
        a, b = top.edges[n]
        p, q = top.free_plus[n], top.free_minus[n]
        # c+ = (a, b, p) and c- = (b, a, q) are CCW, so the quad a, q, b, p is
        # CCW; its other diagonal gives (a, q, p) and (q, b, p).
        if any(set((p, q)) <= set(t.tolist()) for t in tri):
            continue
        tri[cp] = (a, q, p)
        tri[cm] = (q, b, p)
    assert found, "no cell with the figure's vertex counts"
    top, c = found
    bc, vals, mids = _dual_hat_nodes(top, c, c)
    assert bc == gold["barycentre"]
    assert all(v == gold["edge_midpoint"] for v in mids.values())
    got = sorted(vals.values())
    exp = sorted(1.0 / x for x in gold["vertex_cell_counts"])
    assert np.allclose(got, exp, rtol=0, atol=1e-15)
    assert sorted(gold["vertex_values"]) == pytest.approx(exp, abs=1e-15)


@pytest.mark.parametrize("name", MESHES)
def test_gram_ll(name):
    """P1 mass matrix: 1^T G 1 = surface area, and entries equal the 7-point
    integral of the hat products (exact: degree 2)."""
    top = topo(name)
    G = grams.gram_ll(top)
    assert abs(G.sum() - top.area.sum()) < 1e-12 * top.area.sum()
    bary, w = quadrature.tri7_barycentric()
    H = np.zeros_like(G)
    for c in range(top.C):
        for i in range(3):
            for j in range(3):
                H[top.tri[c, i], top.tri[c, j]] += top.area[c] * np.sum(w * bary[:, i] * bary[:, j])
    assert np.abs(G - H).max() < 1e-15


@pytest.mark.parametrize("name", ["ico1", "cube2", "ellipsoid1"])
def test_gram_pp_by_quadrature(name):
    """G_pp of the cell functions p_n = 1/A_n on cell n, zero elsewhere
    (Sec. 2): every entry integrated with the 7-point rule over every cell,
    sum_c A_c sum_q w_q p_m(x_q) p_n(x_q).  Supports meet only on the
    diagonal, where the integrand is the constant 1/A_c^2."""
    top = topo(name)
    G = grams.gram_pp(top)
    bary, w = quadrature.tri7_barycentric()
    H = np.zeros_like(G)
    for c in range(top.C):
        # p_m evaluated at cell c's points: 1/A_c for m == c, else 0
        vals = np.zeros((top.C, len(w)))
        vals[c, :] = 1.0 / top.area[c]
        H += top.area[c] * np.einsum("q,mq,nq->mn", w, vals, vals)
    assert np.abs(G - H).max() <= 1e-14 * np.abs(H).max()
    assert np.all(np.diag(G) > 0)


@pytest.mark.parametrize("name", ["ico1", "torus_small", "cube2"])
def test_laplacian_pseudo_inverse_identity(name):
    """(Sig^T Sig + 1 1^T/C)^-1 = (Sig^T Sig)^+ + 1 1^T/C (Sec. 3.2)."""
    top = topo(name)
    L = grams.laplacian(top)
    C = top.C
    J = np.full((C, C), 1.0 / C)
    lhs = np.linalg.inv(L + J)
    rhs = np.linalg.pinv(L) + J
    assert np.abs(lhs - rhs).max() < 1e-11 * np.abs(rhs).max()
    assert np.all(np.diag(L) == 3)


def test_uneven_batch_recipe():
    """The seeded uneven batch: 32 closed meshes of the three kinds with the
    recipe's size ranges, reproducible, and 4 unit plane waves per item with
    polarisations orthogonal to their directions."""
    from synth import batch
    objs = batch.uneven_objects()
    again = batch.uneven_objects()
    assert len(objs) == 32
    for o, p in zip(objs, again):
        assert o["kind"] == p["kind"] and np.array_equal(o["xyz"], p["xyz"]) and np.array_equal(o["tri"], p["tri"])
        top = Topology(o["xyz"], o["tri"])
        assert top.genus == 0
        if o["kind"] == "cube":
            n = int(o["param"].split()[1])
            assert 8 <= n <= 32 and top.C == 12 * n * n
        else:
            level = int(o["param"].split(",")[0].split()[1])
            assert 2 <= level <= 4 and top.C == 20 * 4 ** level
        if o["kind"] == "ellipsoid":
            axes = [float(a) for a in o["param"].split("axes")[1].split(",")]
            assert all(0.5 <= a <= 1.5 for a in axes)
    assert {o["kind"] for o in objs} == {"icosphere", "cube", "ellipsoid"}
    ks = batch.sweep_wavenumbers()
    assert len(ks) == 8 and ks[0] == 1e-3 and abs(ks[-1] - 5.0) < 1e-12
    kh, pol = batch.sweep_waves(3, 5)
    assert kh.shape == (4, 3) and np.allclose(np.linalg.norm(kh, axis=1), 1) and np.allclose(np.sum(kh * pol, 1), 0)
