"""Plane-wave excitations and seeded complex start vectors."""

import numpy as np

__all__ = ["plane_waves", "default_plane_wave", "complex_start"]


def default_plane_wave():
    """Incidence along +z, polarisation along x: (khat [1,3], pol [1,3])."""
    return np.array([[0.0, 0.0, 1.0]]), np.array([[1.0, 0.0, 0.0]])


def plane_waves(nrhs, seed):
    """``nrhs`` unit-amplitude plane waves.

    Directions are normalised 3-D standard normals; the polarisation is
    cos(psi) theta_hat + sin(psi) phi_hat with psi ~ U[0, 2pi), where theta_hat
    and phi_hat are the spherical unit vectors at the incidence direction.
    """
    rng = np.random.default_rng(seed)
    k = rng.normal(size=(nrhs, 3))
    k /= np.linalg.norm(k, axis=1, keepdims=True)
    psi = rng.uniform(0.0, 2.0 * np.pi, size=nrhs)
    theta = np.arccos(np.clip(k[:, 2], -1.0, 1.0))
    phi = np.arctan2(k[:, 1], k[:, 0])
    th = np.stack([np.cos(theta) * np.cos(phi), np.cos(theta) * np.sin(phi), -np.sin(theta)], axis=1)
    ph = np.stack([-np.sin(phi), np.cos(phi), np.zeros_like(phi)], axis=1)
    pol = np.cos(psi)[:, None] * th + np.sin(psi)[:, None] * ph
    # re-orthogonalise against rounding
    pol -= np.sum(pol * k, axis=1, keepdims=True) * k
    pol /= np.linalg.norm(pol, axis=1, keepdims=True)
    return np.ascontiguousarray(k), np.ascontiguousarray(pol)


def complex_start(n, seed):
    """Complex Gaussian vector (re + i im, each N(0,1)), complex128 [n]."""
    rng = np.random.default_rng(seed)
    return rng.normal(size=n) + 1j * rng.normal(size=n)
