"""Closed, outward-oriented triangle meshes (vertices float64 [V,3], cells int32 [C,3]).

Every generator is deterministic; those with random perturbations take a seed
and use ``numpy.random.default_rng(seed)``.  Cells are listed counter-clockwise
seen from outside (the orientation the RWG sign convention of the solver
relies on).
"""

import numpy as np

__all__ = ["icosphere", "graded_sphere", "torus", "cube", "ellipsoid", "mesh_summary"]


def _orient_outward(xyz, tri):
    """Flip cells so that each normal points away from the mesh centroid.

    Only used for star-shaped convex-ish generators (icosahedron faces).
    """
    centre = xyz.mean(axis=0)
    out = tri.copy()
    for i, (a, b, c) in enumerate(tri):
        n = np.cross(xyz[b] - xyz[a], xyz[c] - xyz[a])
        if np.dot(n, (xyz[a] + xyz[b] + xyz[c]) / 3.0 - centre) < 0:
            out[i] = (a, c, b)
    return out


def _icosahedron():
    phi = (1.0 + np.sqrt(5.0)) / 2.0
    pts = []
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            pts.append((0.0, s1, s2 * phi))
            pts.append((s1, s2 * phi, 0.0))
            pts.append((s2 * phi, 0.0, s1))
    xyz = np.array(pts)
    # faces = triples of mutually adjacent vertices (edge length 2)
    d = np.linalg.norm(xyz[:, None, :] - xyz[None, :, :], axis=-1)
    adj = np.abs(d - 2.0) < 1e-9
    faces = []
    for a in range(12):
        for b in range(a + 1, 12):
            if not adj[a, b]:
                continue
            for c in range(b + 1, 12):
                if adj[a, c] and adj[b, c]:
                    faces.append((a, b, c))
    tri = np.array(faces, dtype=np.int64)
    xyz /= np.linalg.norm(xyz, axis=1, keepdims=True)
    return xyz, _orient_outward(xyz, tri)


def icosphere(level, radius=1.0):
    """Icosahedron refined ``level`` times by midpoint 4-splits, every new
    vertex projected onto the sphere of the given radius.

    V = 10*4**level + 2, C = 20*4**level.
    """
    xyz, tri = _icosahedron()
    verts = [tuple(v) for v in xyz]
    for _ in range(level):
        cache = {}
        new_tri = []

        def midpoint(a, b):
            key = (a, b) if a < b else (b, a)
            idx = cache.get(key)
            if idx is None:
                m = (np.array(verts[a]) + np.array(verts[b])) / 2.0
                m /= np.linalg.norm(m)
                idx = len(verts)
                verts.append(tuple(m))
                cache[key] = idx
            return idx

        for a, b, c in tri:
            ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
            new_tri += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        tri = np.array(new_tri, dtype=np.int64)
    xyz = np.array(verts) * radius
    return np.ascontiguousarray(xyz, dtype=np.float64), np.ascontiguousarray(tri, dtype=np.int32)


def graded_sphere(level, t):
    """Icosphere of the given level with every vertex p moved on the unit
    sphere to (p + t z)/|p + t z|, 0 <= t < 1.  The map keeps the mesh closed
    and its cells well shaped, and concentrates them towards +z: cell areas
    spread by about ((1 + t)/(1 - t))^2 between the poles (t = 0.8: 39x at
    level 2).  A strongly graded but smooth mesh."""
    if not 0.0 <= t < 1.0:
        raise ValueError("t must lie in [0, 1)")
    xyz, tri = icosphere(level)
    p = xyz + np.array([0.0, 0.0, t])
    p /= np.linalg.norm(p, axis=1, keepdims=True)
    return np.ascontiguousarray(p, dtype=np.float64), tri


def _signed_volume(xyz, tri):
    a, b, c = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    return np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0


def _mean_edge_length(xyz, tri):
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    e = np.unique(np.sort(e, axis=1), axis=0)
    return float(np.linalg.norm(xyz[e[:, 0]] - xyz[e[:, 1]], axis=1).mean())


def torus(n_major=96, n_minor=48, R=1.0, r=0.3, jitter=0.01, seed=3):
    """Parametric torus (genus 1): an n_major x n_minor quad grid, each quad
    (i,j)-(i+1,j)-(i+1,j+1)-(i,j+1) split along its (i,j)-(i+1,j+1) diagonal,
    then every vertex moved by an i.i.d. 3-D Gaussian of standard deviation
    ``jitter * h`` (h = mean edge length before the jitter).
    """
    u = 2.0 * np.pi * np.arange(n_major) / n_major
    v = 2.0 * np.pi * np.arange(n_minor) / n_minor
    U, Vv = np.meshgrid(u, v, indexing="ij")
    xyz = np.stack([(R + r * np.cos(Vv)) * np.cos(U),
                    (R + r * np.cos(Vv)) * np.sin(U),
                    r * np.sin(Vv)], axis=-1).reshape(-1, 3)

    def vid(i, j):
        return (i % n_major) * n_minor + (j % n_minor)

    tri = []
    for i in range(n_major):
        for j in range(n_minor):
            a, b, c, d = vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)
            tri.append((a, b, c))
            tri.append((a, c, d))
    tri = np.array(tri, dtype=np.int64)
    if _signed_volume(xyz, tri) < 0:
        tri = tri[:, [0, 2, 1]]
    if jitter > 0:
        h = _mean_edge_length(xyz, tri)
        rng = np.random.default_rng(seed)
        xyz = xyz + rng.normal(0.0, jitter * h, size=xyz.shape)
    return np.ascontiguousarray(xyz, dtype=np.float64), np.ascontiguousarray(tri, dtype=np.int32)


def cube(n, side=2.0):
    """Surface of a cube of the given side centred at the origin, each face an
    n x n grid of squares split along a fixed diagonal.

    V = 6n^2 + 2, C = 12n^2.
    """
    h = side / 2.0
    index = {}
    verts = []
    tri = []

    def vertex(p):
        key = tuple(int(round(x * n / h)) for x in p)  # exact lattice key
        idx = index.get(key)
        if idx is None:
            idx = len(verts)
            verts.append(tuple(p))
            index[key] = idx
        return idx

    grid = np.linspace(-h, h, n + 1)
    for axis in range(3):
        for sgn in (-1.0, 1.0):
            a1, a2 = (axis + 1) % 3, (axis + 2) % 3
            for i in range(n):
                for j in range(n):
                    corners = []
                    for di, dj in ((0, 0), (1, 0), (1, 1), (0, 1)):
                        p = [0.0, 0.0, 0.0]
                        p[axis] = sgn * h
                        p[a1] = grid[i + di]
                        p[a2] = grid[j + dj]
                        corners.append(vertex(p))
                    a, b, c, d = corners
                    t1, t2 = (a, b, c), (a, c, d)
                    # outward orientation for this face
                    pa, pb, pc = (np.array(verts[t]) for t in t1)
                    nrm = np.cross(pb - pa, pc - pa)
                    if nrm[axis] * sgn < 0:
                        t1, t2 = (a, c, b), (a, d, c)
                    tri += [t1, t2]
    xyz = np.array(verts, dtype=np.float64)
    return np.ascontiguousarray(xyz), np.ascontiguousarray(np.array(tri, dtype=np.int32))


def ellipsoid(level, axes):
    """Icosphere of the given level with its coordinates scaled by ``axes``."""
    xyz, tri = icosphere(level)
    return np.ascontiguousarray(xyz * np.asarray(axes, dtype=np.float64)[None, :]), tri


def mesh_summary(xyz, tri):
    """(V, C, N, genus) from Euler's formula for a closed mesh."""
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    n_edges = len(np.unique(np.sort(e, axis=1), axis=0))
    V, C = len(xyz), len(tri)
    chi = V - n_edges + C
    return V, C, n_edges, (2 - chi) // 2
