"""Far field and bistatic radar cross section (Sec. 4, Fig. Sphere_RCS).

Test infrastructure only (tests, smoke and the bench's CPU leg use it).

With e^{-i w t}, the normalised current j = eta J and the scattered field
E^s = i k int G j - (1/(i k)) grad int G div' j (the operator T of Sec. 2),
the far zone (|r| -> infinity along r_hat, G -> exp(i k r)/(4 pi r)
exp(-i k r_hat . r')) keeps only the transverse part:

  E^s(r) = -i k exp(i k r)/(4 pi r) r_hat x (r_hat x F),
  F(r_hat) = int j(r') exp(-i k r_hat . r') dS',

so for a unit incident amplitude the bistatic RCS is

  sigma = lim 4 pi r^2 |E^s|^2 = k^2/(4 pi) |F - r_hat (r_hat . F)|^2.

On cell c the RWG current is j(r) = sum_i j_m sigma_{c,i} (r - r_i)/(2 A_c)
(r_i the vertex opposite local edge i), integrated with the same 7-point
rule as the excitation.

The Mie reference uses the amplitude functions of Bohren and Huffman
(Ch. 4): S1 = sum_n E'_n (a_n pi_n + b_n tau_n), S2 = sum_n E'_n (a_n tau_n +
b_n pi_n), E'_n = (2n+1)/(n(n+1)), with the perfect-conductor coefficients of
oracle.mie, and sigma = 4 pi / k^2 (|S2|^2 cos^2 phi + |S1|^2 sin^2 phi) for
the x-polarised wave along +z.
"""

import numpy as np
from scipy.special import spherical_jn, spherical_yn

from .mie import _nmax, _pi_tau
from .quadrature import tri7_points

__all__ = ["far_field", "far_field_split", "rcs", "mie_rcs", "rayleigh_rcs"]


def far_field(top, k, j, dirs):
    """F(r_hat) [nrhs, D, 3] of RWG coefficients j [nrhs, N] (or [N]) for unit
    directions dirs [D, 3]."""
    j = np.atleast_2d(np.asarray(j, dtype=np.complex128))
    dirs = np.atleast_2d(np.asarray(dirs, dtype=np.float64))
    pts, w = tri7_points(top.xyz, top.tri)                    # [C,7,3], [7]
    phase = np.exp(-1j * k * np.einsum("cqk,dk->cqd", pts, dirs))   # [C,7,D]
    out = np.zeros((len(j), len(dirs), 3), dtype=np.complex128)
    for r in range(len(j)):
        Jq = np.zeros(pts.shape, dtype=np.complex128)          # sum_i j sigma (r_q - r_i)/2 = A_c j(r_q)
        for i in range(3):
            coef = j[r, top.cell_edges[:, i]] * top.cell_sign[:, i] / 2.0
            arm = pts - top.xyz[top.tri[:, i]][:, None, :]
            Jq += coef[:, None, None] * arm
        out[r] = np.einsum("q,cqk,cqd->dk", w, Jq, phase)
    return out


def far_field_split(top, k, j_loop, j_star, dirs):
    """F of j = j_loop + j_star with the parts kept apart: a divergence-free
    (loop) current carries no net current, int j_loop dS = 0 (j = div(j x_i)
    componentwise on the closed surface), so its far field is
    int j_loop (exp(-i k r_hat . r') - 1) dS', whose phase factor is formed as
    -2 sin^2(t/2) - i sin t without cancellation; the star part uses the plain
    phase.  At very low k both terms are O(k) while j_star is O(k) relative
    to j_loop, so neither may go through a sum of the two currents."""
    jl = np.atleast_2d(np.asarray(j_loop, dtype=np.complex128))
    js = np.atleast_2d(np.asarray(j_star, dtype=np.complex128))
    dirs = np.atleast_2d(np.asarray(dirs, dtype=np.float64))
    pts, w = tri7_points(top.xyz, top.tri)
    t = k * np.einsum("cqk,dk->cqd", pts, dirs)
    ph_m1 = -2.0 * np.sin(0.5 * t) ** 2 - 1j * np.sin(t)       # exp(-i t) - 1
    ph = np.exp(-1j * t)
    out = np.zeros((len(jl), len(dirs), 3), dtype=np.complex128)
    for r in range(len(jl)):
        for jj, phase in ((jl[r], ph_m1), (js[r], ph)):
            Jq = np.zeros(pts.shape, dtype=np.complex128)
            for i in range(3):
                coef = jj[top.cell_edges[:, i]] * top.cell_sign[:, i] / 2.0
                arm = pts - top.xyz[top.tri[:, i]][:, None, :]
                Jq += coef[:, None, None] * arm
            out[r] += np.einsum("q,cqk,cqd->dk", w, Jq, phase)
    return out


def rayleigh_rcs(k, a, dirs):
    """Low-frequency limit of the bistatic RCS of a PEC sphere of radius a
    for E^i = x exp(i k z): the field of the induced electric dipole
    (4 pi a^3 E^i) and magnetic dipole (-2 pi a^3 H^i),
    sigma = 4 pi a^2 (ka)^4 ((cos th - 1/2)^2 cos^2 ph + (1 - cos(th)/2)^2 sin^2 ph),
    with a relative error O((ka)^2); backscatter 9 pi a^2 (ka)^4."""
    dirs = np.atleast_2d(np.asarray(dirs, dtype=np.float64))
    ct = np.clip(dirs[:, 2], -1.0, 1.0)
    phi = np.arctan2(dirs[:, 1], dirs[:, 0])
    x = k * a
    return 4.0 * np.pi * a * a * x ** 4 * ((ct - 0.5) ** 2 * np.cos(phi) ** 2 + (1.0 - 0.5 * ct) ** 2 * np.sin(phi) ** 2)


def rcs(k, F, dirs):
    """Bistatic RCS [..., D] from far-field vectors F [..., D, 3]."""
    dirs = np.atleast_2d(np.asarray(dirs, dtype=np.float64))
    Fp = F - dirs * np.sum(dirs * F, axis=-1, keepdims=True)
    return k * k / (4.0 * np.pi) * np.sum(np.abs(Fp) ** 2, axis=-1)


def mie_rcs(k, a, dirs):
    """Mie bistatic RCS of a PEC sphere of radius a for E^i = x exp(i k z),
    at unit directions dirs [D, 3]."""
    dirs = np.atleast_2d(np.asarray(dirs, dtype=np.float64))
    theta = np.arccos(np.clip(dirs[:, 2], -1.0, 1.0))
    phi = np.arctan2(dirs[:, 1], dirs[:, 0])
    x = k * a
    nmax = _nmax(x)
    n = np.arange(1, nmax + 1)
    psi = x * spherical_jn(n, x)
    dpsi = spherical_jn(n, x) + x * spherical_jn(n, x, derivative=True)
    h = spherical_jn(n, x) + 1j * spherical_yn(n, x)
    hp = spherical_jn(n, x, derivative=True) + 1j * spherical_yn(n, x, derivative=True)
    an = dpsi / (h + x * hp)
    bn = psi / (x * h)
    pi, tau = _pi_tau(nmax, np.cos(theta))                    # [nmax, D]
    En = ((2 * n + 1) / (n * (n + 1)))[:, None]
    S1 = np.sum(En * (an[:, None] * pi + bn[:, None] * tau), axis=0)
    S2 = np.sum(En * (an[:, None] * tau + bn[:, None] * pi), axis=0)
    return 4.0 * np.pi / (k * k) * (np.abs(S2) ** 2 * np.cos(phi) ** 2 + np.abs(S1) ** 2 * np.sin(phi) ** 2)
