"""Mie series for a perfectly conducting sphere (pin only; not part of the
paper's method, which the paper checks against Mie in its sphere figures).

Incident field E^i = x exp(i k z), e^{-i w t}.  Vector spherical harmonics,
Riccati-Bessel functions and the expansion follow the textbook treatment of
Bohren and Huffman (Absorption and Scattering of Light by Small Particles,
Wiley 1983, Ch. 4), with the perfect-conductor limit of the coefficients:

  E^i = sum_n E_n (M1_o1n - i N1_e1n),   eta H^i = -sum_n E_n (M1_e1n + i N1_o1n)
  E^s = sum_n E_n (i a_n N3_e1n - b_n M3_o1n),  eta H^s = sum_n E_n (i b_n N3_o1n + a_n M3_e1n)
  E_n = i^n (2n+1)/(n(n+1)),  a_n = psi_n'(x)/xi_n'(x),  b_n = psi_n(x)/xi_n(x),  x = k a

(psi_n = rho j_n, xi_n = rho h_n^(1)).  The normalised surface current is
j = eta J = r_hat x eta H on r = a.
"""

import numpy as np
from scipy.special import spherical_jn, spherical_yn

__all__ = ["fields", "surface_current", "rwg_flux"]


def _pi_tau(nmax, mu):
    """pi_n = P_n^1/sin(theta), tau_n = dP_n^1/dtheta (n = 1..nmax) by recurrence."""
    mu = np.asarray(mu, dtype=np.float64)
    pi = np.zeros((nmax + 1,) + mu.shape)
    tau = np.zeros_like(pi)
    pi[1] = 1.0
    tau[1] = mu
    for n in range(2, nmax + 1):
        pi[n] = (2 * n - 1) / (n - 1) * mu * pi[n - 1] - n / (n - 1) * pi[n - 2]
        tau[n] = n * mu * pi[n] - (n + 1) * pi[n - 1]
    return pi[1:], tau[1:]


def _radial(kind, n, rho):
    """z_n(rho) and [rho z_n(rho)]'/rho for j_n (kind 1) or h_n^(1) (kind 3)."""
    j = spherical_jn(n, rho)
    jp = spherical_jn(n, rho, derivative=True)
    if kind == 1:
        return j, j / rho + jp
    y = spherical_yn(n, rho)
    yp = spherical_yn(n, rho, derivative=True)
    h, hp = j + 1j * y, jp + 1j * yp
    return h, h / rho + hp


def _nmax(x):
    return int(np.ceil(x + 4.0 * x ** (1.0 / 3.0) + 10))


def _vsh(kind, n, rho, theta, phi, pi, tau):
    """Spherical components (r, theta, phi) of M_e1n, M_o1n, N_e1n, N_o1n.

    Shapes: n [nmax, 1], angles [P]; results [nmax, 3, P]."""
    z, dz = _radial(kind, n, rho)
    cp, sp = np.cos(phi), np.sin(phi)
    st = np.sin(theta)
    nn1 = n * (n + 1)
    zero = np.zeros_like(pi * z)
    Me = np.stack([zero, -sp * pi * z, -cp * tau * z], axis=1)
    Mo = np.stack([zero, cp * pi * z, -sp * tau * z], axis=1)
    Ne = np.stack([cp * nn1 * st * pi * z / rho, cp * tau * dz, -sp * pi * dz], axis=1)
    No = np.stack([sp * nn1 * st * pi * z / rho, sp * tau * dz, cp * pi * dz], axis=1)
    return Me, Mo, Ne, No


def _to_cart(v, theta, phi):
    st, ct, sp, cp = np.sin(theta), np.cos(theta), np.sin(phi), np.cos(phi)
    r_hat = np.stack([st * cp, st * sp, ct])
    t_hat = np.stack([ct * cp, ct * sp, -st])
    p_hat = np.stack([-sp, cp, np.zeros_like(sp)])
    return (v[0] * r_hat + v[1] * t_hat + v[2] * p_hat).T


def fields(k, a, pts, part="total"):
    """(E, eta H) at points pts [P,3] (Cartesian, complex [P,3]).

    part: 'incident', 'scattered' or 'total'.  Valid for |r| > 0; the
    scattered part only outside the sphere."""
    pts = np.asarray(pts, dtype=np.float64)
    r = np.linalg.norm(pts, axis=1)
    theta = np.arccos(np.clip(pts[:, 2] / r, -1.0, 1.0))
    phi = np.arctan2(pts[:, 1], pts[:, 0])
    x = k * a
    nmax = _nmax(max(x, k * r.max()))
    n = np.arange(1, nmax + 1)[:, None]
    En = (1j ** n) * (2 * n + 1) / (n * (n + 1))
    pi, tau = _pi_tau(nmax, np.cos(theta))
    rho = k * r[None, :]
    E = np.zeros((3, len(r)), dtype=complex)
    H = np.zeros((3, len(r)), dtype=complex)
    if part in ("incident", "total"):
        Me, Mo, Ne, No = _vsh(1, n, rho, theta, phi, pi, tau)
        E += np.sum(En[:, None, :] * (Mo - 1j * Ne), axis=0)
        H += -np.sum(En[:, None, :] * (Me + 1j * No), axis=0)
    if part in ("scattered", "total"):
        nv = n[:, 0]
        psi = x * spherical_jn(nv, x)
        dpsi = spherical_jn(nv, x) + x * spherical_jn(nv, x, derivative=True)
        h = spherical_jn(nv, x) + 1j * spherical_yn(nv, x)
        hp = spherical_jn(nv, x, derivative=True) + 1j * spherical_yn(nv, x, derivative=True)
        xi = x * h
        dxi = h + x * hp
        an = (dpsi / dxi)[:, None, None]
        bn = (psi / xi)[:, None, None]
        Me, Mo, Ne, No = _vsh(3, n, rho, theta, phi, pi, tau)
        E += np.sum(En[:, None, :] * (1j * an * Ne - bn * Mo), axis=0)
        H += np.sum(En[:, None, :] * (1j * bn * No + an * Me), axis=0)
    return _to_cart(E, theta, phi), _to_cart(H, theta, phi)


def surface_current(k, a, pts):
    """j = eta J = n x eta H on the sphere r = a at points pts [P,3]."""
    pts = np.asarray(pts, dtype=np.float64)
    rhat = pts / np.linalg.norm(pts, axis=1, keepdims=True)
    _, H = fields(k, a, a * rhat, "total")
    return np.cross(rhat, H)


def rwg_flux(top, k, a=1.0, order=5):
    """RWG coefficients of the Mie current: the flux of j across each edge,
    from c+ into c-, along the chord mapped radially onto the sphere
    (Gauss-Legendre of the given order)."""
    g, w = np.polynomial.legendre.leggauss(order)
    t = 0.5 * (g + 1.0)
    w = 0.5 * w
    A = top.xyz[top.edges[:, 0]]
    B = top.xyz[top.edges[:, 1]]
    L = np.linalg.norm(B - A, axis=1)
    pts = A[:, None, :] + t[None, :, None] * (B - A)[:, None, :]        # [N,q,3]
    sph = a * pts / np.linalg.norm(pts, axis=2, keepdims=True)
    j = surface_current(k, a, sph.reshape(-1, 3)).reshape(sph.shape)
    tangent = (B - A) / L[:, None]
    nrm = sph / a
    m = np.cross(tangent[:, None, :], nrm)          # in-surface normal, out of c+ (CCW c+ on the left)
    m /= np.linalg.norm(m, axis=2, keepdims=True)
    return np.sum(w[None, :] * np.einsum("nqd,nqd->nq", j, m), axis=1) * L
