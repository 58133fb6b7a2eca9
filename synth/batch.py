"""The seeded uneven batch: objects of mixed shape and size, each swept over a
log-spaced set of wavenumbers with a few random plane waves per wavenumber."""

import numpy as np

from .meshes import cube, ellipsoid, icosphere
from .waves import plane_waves

__all__ = ["uneven_objects", "sweep_wavenumbers", "sweep_waves"]


def uneven_objects(n_objects=32, seed=5):
    """``n_objects`` closed meshes, each of a kind drawn uniformly from
    {icosphere of level U{2..4}, radius 1; cube with n U{8..32} squares per
    face edge, side 2; ellipsoid = icosphere of level U{2..4} scaled by axes
    U(0.5, 1.5) each}.  Returns a list of dicts: kind, a parameter string,
    xyz, tri."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_objects):
        kind = ("icosphere", "cube", "ellipsoid")[int(rng.integers(0, 3))]
        if kind == "icosphere":
            level = int(rng.integers(2, 5))
            xyz, tri = icosphere(level)
            par = f"level {level}"
        elif kind == "cube":
            n = int(rng.integers(8, 33))
            xyz, tri = cube(n)
            par = f"n {n}"
        else:
            level = int(rng.integers(2, 5))
            axes = rng.uniform(0.5, 1.5, size=3)
            xyz, tri = ellipsoid(level, axes)
            par = f"level {level}, axes " + ", ".join(f"{a:.3f}" for a in axes)
        out.append({"kind": kind, "param": par, "xyz": xyz, "tri": tri})
    return out


def sweep_wavenumbers(n=8, lo=1e-3, hi=5.0):
    """The wavenumbers of the sweep: ``n`` values log-spaced from lo to hi."""
    return np.geomspace(lo, hi, n)


def sweep_waves(obj_index, k_index, nrhs=4, seed=5):
    """The plane waves (khat, pol) of one (object, wavenumber) item."""
    return plane_waves(nrhs, 1000 * seed + 16 * obj_index + k_index)
