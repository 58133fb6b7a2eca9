"""Pins of the voltage-gap excitation (oracle.rhs.voltage_gap; the second
source of the Fokker example, Sec. 4) against what the physics fixes: the
delta gap as the limit of a narrow strip of uniform field, conservation of
energy (the power the gap delivers is the power the far field carries away)
and reciprocity."""

import numpy as np
import pytest

from oracle import farfield, rhs
from ._meshes import precond, topo


def _strip_excitation(top, m, V, t):
    """Brute force: int f_n . E dS for the field V/w n_hat on the strip of
    width w = 2 t h_c (t a fraction of each cell's height h_c over edge m)
    on both cells of edge m, n_hat the in-plane normal of the edge pointing
    from c+ into c-.  Each half-strip {barycentric of the free vertex <= t}
    is a trapezoid, split into two triangles; f_n is linear, so the centroid
    rule is exact on them.  Returns {n: e_n}."""
    a, b = top.xyz[top.edges[m, 0]], top.xyz[top.edges[m, 1]]
    out = {}
    for c, into in ((top.cplus[m], False), (top.cminus[m], True)):
        loc = [i for i in range(3) if top.cell_edges[c, i] == m][0]
        p = top.xyz[top.tri[c, loc]]                       # free vertex of edge m in c
        ab = b - a
        foot = a + np.dot(p - a, ab) / np.dot(ab, ab) * ab
        h = np.linalg.norm(p - foot)
        nh = (p - foot) / h if into else (foot - p) / h    # c+ -> c- direction, in the cell's plane
        w = 2.0 * t * h
        a2, b2 = a + t * (p - a), b + t * (p - b)
        for T in ((a, b, b2), (a, b2, a2)):
            area = 0.5 * np.linalg.norm(np.cross(T[1] - T[0], T[2] - T[0]))
            g = (T[0] + T[1] + T[2]) / 3.0
            for i in range(3):
                n = top.cell_edges[c, i]
                f = top.cell_sign[c, i] * (g - top.xyz[top.tri[c, i]]) / (2.0 * top.area[c])
                out[n] = out.get(n, 0.0) + area * np.dot(f, nh) * V / w
    return out


@pytest.mark.parametrize("m", [0, 17, 101])
def test_gap_is_the_narrow_strip_limit(m):
    """As the strip narrows the brute-force excitation tends to V on the gap
    edge (at first order in the width) and to 0 on the other four RWG
    functions of its two cells; the oracle's e is that limit (jittered torus,
    so the two cells have unequal heights and are not coplanar)."""
    top = topo("torus_small")
    V = 0.7 - 0.4j
    e = rhs.voltage_gap(top, [m], [V])[0]
    errs = []
    for t in (1e-2, 1e-3):
        s = _strip_excitation(top, m, V, t)
        assert set(np.flatnonzero(e)) == {m}
        errs.append(max(abs(s[n] - e[n]) for n in s))
    assert errs[1] < 2e-3 * abs(V) and 5.0 < errs[0] / errs[1] < 20.0, errs


def _directions(nt):
    mu, wmu = np.polynomial.legendre.leggauss(nt)
    ph = 2 * np.pi * np.arange(2 * nt) / (2 * nt)
    MU, PH = np.meshgrid(mu, ph, indexing="ij")
    d = np.stack([np.sqrt(1 - MU ** 2) * np.cos(PH), np.sqrt(1 - MU ** 2) * np.sin(PH), MU], -1).reshape(-1, 3)
    return d, (wmu[:, None] * np.full(2 * nt, np.pi / nt)[None, :]).reshape(-1)


@pytest.mark.parametrize("name,k", [("ico1", 1.0), ("ico1", 1e-2), ("ico2", 0.3)])
def test_gap_power_balance(name, k):
    """Energy conservation on a perfect conductor: the gap's input power
    Re(V conj(j_m)) (j = eta J, in units of 1/(2 eta)) equals the radiated
    power (1/(4 pi)) int sigma dOmega of the far field, sigma the bistatic RCS
    form of the far field (Gauss-Legendre x trapezoid over the directions).
    For the Galerkin solution of T j = -e the identity holds up to the
    quadrature of the far field, so it fixes the gap's scale and sign, the
    sign of the system and the far-field normalisation together."""
    top = topo(name)
    pre = precond(name, k)
    m, V = 5, 1.0 - 0.5j
    j = -np.linalg.solve(pre.T(), rhs.voltage_gap(top, [m], [V])[0])
    d, w = _directions(16)
    s = farfield.rcs(k, farfield.far_field(top, k, j, d)[0], d)
    p_rad = np.sum(w * s) / (4 * np.pi)
    p_in = np.real(V * np.conj(j[m]))
    assert p_in > 0 and abs(p_rad / p_in - 1) < 1e-7, (p_in, p_rad)


def test_gap_reciprocity():
    """Mutual admittances are symmetric: the current on edge b driven by a unit
    gap on edge a equals the current on a driven by a unit gap on b."""
    top = topo("ico1")
    pre = precond("ico1", 1.0)
    a, b = 3, 40
    e = rhs.voltage_gap(top, [[a], [b]], [[1.0], [1.0]])
    J = -np.linalg.solve(pre.T(), e.T).T
    assert abs(J[0, b] - J[1, a]) <= 1e-12 * abs(J[0, b])


def test_gap_duplicates_add_and_range():
    top = topo("ico1")
    e = rhs.voltage_gap(top, [[2, 9, 2]], [[1.0, 2.0j, 0.5]])[0]
    assert e[2] == 1.5 and e[9] == 2.0j and np.count_nonzero(e) == 2
    with pytest.raises(ValueError):
        rhs.voltage_gap(top, [top.N], [1.0])


def _power_mismatch():
    top = topo("ico1")
    pre = precond("ico1", 1.0)
    m, V = 5, 1.0
    j = -np.linalg.solve(pre.T(), rhs.voltage_gap(top, [m], [V])[0])
    d, w = _directions(12)
    p_rad = np.sum(w * farfield.rcs(1.0, farfield.far_field(top, 1.0, j, d)[0], d)) / (4 * np.pi)
    return abs(p_rad / np.real(V * np.conj(j[m])) - 1)


@pytest.mark.parametrize("scale", [0.5, -1.0, 2.0])
def test_power_balance_catches_planted_mistakes(monkeypatch, scale):
    """A gap excitation with a wrong factor (V shared between the two cells,
    or V times the edge's flux counted twice) or a wrong sign (field from c-
    into c+) fails the power balance that the oracle's passes."""
    good = _power_mismatch()
    real = rhs.voltage_gap
    monkeypatch.setattr(rhs, "voltage_gap", lambda top, e, v: scale * real(top, e, v))
    assert good < 1e-7 and _power_mismatch() > 0.3
