"""Pins of the far-field and RCS oracle (oracle/farfield.py) against what the
mathematics fixes: the Mie fields themselves far from the sphere, the
Rayleigh limit, and the far-field integral of the exact Mie surface current."""

import numpy as np
import pytest

import synth
from oracle import farfield, mie
from oracle.topology import Topology


def _dirs(th, ph):
    th, ph = np.asarray(th, float), np.asarray(ph, float)
    return np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], axis=1)


DIRS = _dirs([0.0, 0.3, 1.0, 1.6, 2.0, 2.9, np.pi], [0.0, 0.0, 0.7, 1.2, 2.5, 4.0, 0.0])


@pytest.mark.parametrize("ka", [0.5, 1.0, 2.0])
def test_mie_rcs_is_the_far_limit_of_the_mie_fields(ka):
    """4 pi r^2 |E^s|^2 of the Mie field expansion (oracle.mie, itself pinned)
    tends to the amplitude-function RCS: the largest difference over the
    directions falls at least at first order in 1/(k r) from kr = 25 to 50 to
    100 (the field's near-zone corrections), and is below 5 % at kr = 100."""
    k = ka
    ref = farfield.mie_rcs(k, 1.0, DIRS)
    err = []
    for kr in (25.0, 50.0, 100.0):
        r = kr / k
        Es, _ = mie.fields(k, 1.0, r * DIRS, "scattered")
        err.append(np.abs(4 * np.pi * np.sum(np.abs(r * Es) ** 2, axis=1) / ref - 1))
    m = [e.max() for e in err]
    assert m[1] <= 0.56 * m[0] and m[2] <= 0.56 * m[1] and m[2] < 0.05, m


def test_mie_rcs_rayleigh_limit():
    """Backscatter of a small PEC sphere: sigma = 9 pi a^2 (ka)^4 (1 + O(ka^2))."""
    for x in (1e-2, 1e-3):
        s = farfield.mie_rcs(x, 1.0, np.array([[0.0, 0.0, -1.0]]))[0]
        assert abs(s / (9 * np.pi * x ** 4) - 1) < 0.5 * x * x


@pytest.mark.parametrize("ka", [0.3, 1.0, 3.0])
def test_far_field_of_the_exact_mie_current(ka):
    """The far-field formula (F, the transverse part, k^2 / (4 pi)) applied to
    the exact Mie surface current, integrated by Gauss-Legendre in cos(theta)
    times the trapezoid rule in phi, reproduces the Mie RCS."""
    k = ka
    mu, wmu = np.polynomial.legendre.leggauss(48)
    ph = 2 * np.pi * np.arange(96) / 96
    MU, PH = np.meshgrid(mu, ph, indexing="ij")
    pts = np.stack([np.sqrt(1 - MU ** 2) * np.cos(PH), np.sqrt(1 - MU ** 2) * np.sin(PH), MU], -1).reshape(-1, 3)
    w = (wmu[:, None] * np.full(96, 2 * np.pi / 96)[None, :]).reshape(-1)
    j = mie.surface_current(k, 1.0, pts)
    F = np.einsum("p,pk,pd->dk", w, j, np.exp(-1j * k * pts @ DIRS.T))
    assert np.abs(farfield.rcs(k, F, DIRS) / farfield.mie_rcs(k, 1.0, DIRS) - 1).max() < 1e-9


def test_rwg_far_field_converges_to_mie():
    """The RWG form of the far field (7-point rule per cell) applied to the
    RWG fluxes of the Mie current: the RCS error against Mie falls at second
    order in h (icosphere levels 2 and 3)."""
    k = 1.0
    errs = []
    for L in (2, 3):
        xyz, tri = synth.icosphere(L)
        top = Topology(xyz, tri)
        j = mie.rwg_flux(top, k)
        s = farfield.rcs(k, farfield.far_field(top, k, j, DIRS)[0], DIRS)
        errs.append(np.abs(s / farfield.mie_rcs(k, 1.0, DIRS) - 1).max())
    assert errs[1] < 0.02 and 3.0 < errs[0] / errs[1] < 5.0, errs


# ------------------------------------------------ low-frequency (split) path
K_1E_25_HZ = 2.0 * np.pi * 1e-25 / 299792458.0


def test_rayleigh_rcs_is_the_low_frequency_limit_of_mie():
    """The dipole closed form against the Mie amplitude functions: relative
    difference O((ka)^2) over the E- and H-plane and oblique directions."""
    for x in (1e-2, 1e-3):
        r = farfield.mie_rcs(x, 1.0, DIRS) / farfield.rayleigh_rcs(x, 1.0, DIRS) - 1
        assert np.abs(r).max() < 4 * x * x


def test_planewave_split_sums_to_the_excitation():
    """e = Sigma s + e1: the split excitation reproduces the plain one where
    both are exact in FP64, its static part lies in the range of Sigma (so
    Lam^T e = Lam^T e1), and e1 is O(k): e1/k converges as k -> 0."""
    from oracle import rhs
    from tests._meshes import topo
    top = topo("ico1")
    kh, pol = synth.plane_waves(2, 3)
    for k in (0.5, 1e-3):
        s, e1 = rhs.planewave_split(top, k, kh, pol)
        e = rhs.planewave(top, k, kh, pol)
        full = (top.Sigma @ s.T).T + e1
        assert np.linalg.norm(full - e) <= 1e-13 * np.linalg.norm(e)
        assert np.linalg.norm(top.Lambda.T @ (e1 - e).T) <= 1e-13 * np.linalg.norm(e)
    _, a = rhs.planewave_split(top, 1e-6, kh, pol)
    _, b = rhs.planewave_split(top, 1e-9, kh, pol)
    assert np.linalg.norm(a / 1e-6 - b / 1e-9) < 1e-5 * np.linalg.norm(b / 1e-9)


def test_split_rhs_recovery_and_far_field_match_the_plain_ones():
    """At a moderate k the split right-hand side, recovery and far field equal
    the plain ones (where the plain ones lose nothing)."""
    from oracle import rhs
    from tests._meshes import precond, topo
    k = 0.5
    pre = precond("ico1", k)
    top = topo("ico1")
    s, e1 = rhs.planewave_split(top, k, *synth.default_plane_wave())
    e = rhs.planewave(top, k, *synth.default_plane_wave())[0]
    b1 = pre.rhs_split(s[0], e1[0])
    b0 = pre.rhs(e)
    assert np.linalg.norm(b1 - b0) <= 1e-12 * np.linalg.norm(b0)
    i = np.linalg.solve(pre.system_split(), b0)
    jl, js = pre.recover_split(i)
    assert np.linalg.norm(jl + js - pre.recover(i)) <= 1e-14 * np.linalg.norm(pre.recover(i))
    F1 = farfield.far_field_split(top, k, jl, js, DIRS)
    F0 = farfield.far_field(top, k, jl + js, DIRS)
    assert np.abs(F1 - F0).max() <= 1e-12 * np.abs(F0).max()


def _lf_rcs_error(name, k):
    from oracle import rfcmp, rhs
    from tests._meshes import blocks, topo
    top = topo(name)
    TA, V = blocks(name, k)
    pre = rfcmp.Preconditioner(top, TA, V, k)
    pre.power_scalings(synth.complex_start(top.N, 11), 30, tol=1e-2)
    s, e1 = rhs.planewave_split(top, k, *synth.default_plane_wave())
    i, _, res = rfcmp.cg(pre.apply, pre.rhs_split(s[0], e1[0]), 1e-10, 500)
    assert res <= 1e-10
    jl, js = pre.recover_split(i)
    th = np.linspace(0.0, np.pi, 19)
    d = np.concatenate([_dirs(th, 0 * th), _dirs(th, 0 * th + np.pi / 2)])
    sig = farfield.rcs(k, farfield.far_field_split(top, k, jl, js, d), d)[0]
    ref = farfield.rayleigh_rcs(k, 1.0, d)
    return np.abs(sig - ref).max() / ref.max()


def test_rcs_down_to_1e_25_hz():
    """Fig. Sphere_RCS: with the split excitation, right-hand side, recovery
    and far field, the RCS of the sphere (icosphere level 2) keeps its
    discretisation error against the Rayleigh limit unchanged from ka = 1e-4
    down to the paper's 1e-25 Hz (k = 2.1e-33); the plain path there returns
    noise 1e70 times the RCS."""
    e4 = _lf_rcs_error("ico2", 1e-4)
    e25 = _lf_rcs_error("ico2", K_1E_25_HZ)
    assert e4 < 0.08
    assert abs(e25 - e4) < 1e-6 * e4
