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
