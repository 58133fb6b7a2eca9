"""Spectral study of the RF-CMP system (Sec. 4: Figs. SphereF and SphereH on the
sphere, Fig. CubeTorus on the multiply connected body): the condition number
of A against the wavenumber, down to the static limit, and against the mesh
size.

Each point is one CG solve of the system A i = b through the library
(``rfcmp_solve_system``) with a seeded complex Gaussian b: the run's Lanczos
tridiagonal gives the extreme eigenvalues of A on the Krylov space of b
(``rfcmp_info.cond_estimate``), a lower bound on cond(A) that a generic b
brings close to it.  (A b formed from a plane wave would not do at low
frequency: it is dominated by one of the two blocks.)  The scalings alpha,
beta, gamma come from the power iteration, as in the paper.
"""

import numpy as np

from . import Mesh, Operator, _torch

# wavenumber of 1e-25 Hz, the lowest frequency of the paper's sphere study:
# k = 2 pi f / c
K_1E_25_HZ = 2.0 * np.pi * 1e-25 / 299792458.0


def _gaussian(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def condition_estimate(mesh, k, seed=0, tol=1e-10, maxit=2000, **opts):
    """cond(A) estimate of the RF-CMP system of one mesh and wavenumber.
    Returns a dict: k, N, cond (the Lanczos estimate), iters, rel_residual,
    status and the scalings alpha, beta, gamma."""
    torch = _torch()
    start = torch.from_numpy(_gaussian(mesh.N, seed + 1)).cuda()
    op = Operator(mesh, k, power_start=start, **opts)
    try:
        b = torch.from_numpy(_gaussian(mesh.N, seed)[None, :].copy()).cuda()
        _, status, info = op.solve_system(b, tol=tol, maxit=maxit)
        alpha, beta, gamma, _ = op.scalings()
    finally:
        op.close()
    return {"k": float(k), "N": mesh.N, "cond": info[0]["cond_estimate"], "iters": info[0]["iters"],
            "rel_residual": info[0]["rel_residual"], "status": status, "alpha": alpha, "beta": beta,
            "gamma": gamma}


def condition_study(meshes, ks, seed=0, tol=1e-10, **opts):
    """cond(A) estimates over meshes x wavenumbers.  meshes: {name: (xyz,
    tri)}; returns one dict per point (condition_estimate's, plus "mesh")."""
    rows = []
    for name, (xyz, tri) in meshes.items():
        m = Mesh(xyz, tri)
        try:
            for k in ks:
                r = condition_estimate(m, k, seed=seed, tol=tol, **opts)
                r["mesh"] = name
                rows.append(r)
        finally:
            m.close()
    return rows
