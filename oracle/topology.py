"""RWG connectivity and the loop/star matrices (Sec. 2 of the paper).

Conventions (the paper defers them to the literature; this is the reading used
throughout, and the GPU library follows the same written convention):

* Cells are CCW seen from outside; local edge i of a cell joins its vertices
  i+1 and i+2 (mod 3), so vertex i is the free vertex of local edge i.
* Edges (= RWG functions, one per edge of the closed mesh) are numbered in the
  order a scan over the cells (and over local edges 0, 1, 2 of each) first
  meets them: by the lower-indexed of their two cells, then the local index
  there.
* c+ of an edge is the cell that walks it from its min to its max vertex in
  its CCW order; c- is the other one.  The RWG of eq. (RWGdef) is
  (r - r+)/(2A+) on c+ and (r- - r)/(2A-) on c-, with r+/r- the free vertices.
* Sigma[n, c+] = +1, Sigma[n, c-] = -1: the divergence of f_n on a cell c is
  Sigma[n, c] / A_c.
* Lambda[n, tail] = +1, Lambda[n, head] = -1 with tail -> head the direction
  c+ walks the edge (tail = min vertex): column v of Lambda holds the RWG
  coefficients of n x grad(lambda_v) (the flux of n x grad(psi) across the edge,
  out of c+, is psi(tail) - psi(head)).
* NoC(v) = number of cells at vertex v; genus g = (2 - V + N - C) / 2.
"""

import numpy as np

__all__ = ["Topology", "MeshError"]


class MeshError(ValueError):
    pass


class Topology:
    """Connectivity of a closed, oriented, 2-manifold triangle mesh."""

    def __init__(self, xyz, tri):
        xyz = np.asarray(xyz, dtype=np.float64)
        tri = np.asarray(tri, dtype=np.int64)
        self.xyz, self.tri = xyz, tri
        self.V, self.C = len(xyz), len(tri)

        directed = {}
        for c in range(self.C):
            for i in range(3):
                a, b = tri[c, (i + 1) % 3], tri[c, (i + 2) % 3]
                if (a, b) in directed:
                    raise MeshError("edge walked twice in the same direction (orientation or non-manifold)")
                directed[(a, b)] = (c, i)
        # edges in the order a scan over the cells first meets them: by the
        # lower-indexed of their two cells, then the local index there (any
        # order is a valid numbering; this one keeps the edges of nearby
        # cells together)
        def first_seen(key):
            lo, hi = key
            return min(directed[k] for k in ((lo, hi), (hi, lo)) if k in directed)
        keys = sorted({(min(a, b), max(a, b)) for (a, b) in directed}, key=first_seen)
        self.N = len(keys)
        self.edges = np.array(keys, dtype=np.int64).reshape(-1, 2)
        self.cplus = np.empty(self.N, dtype=np.int64)
        self.cminus = np.empty(self.N, dtype=np.int64)
        self.lplus = np.empty(self.N, dtype=np.int64)   # local index in c+
        self.lminus = np.empty(self.N, dtype=np.int64)  # local index in c-
        self.cell_edges = np.empty((self.C, 3), dtype=np.int64)
        self.cell_sign = np.empty((self.C, 3), dtype=np.float64)
        for n, (lo, hi) in enumerate(keys):
            if (lo, hi) not in directed or (hi, lo) not in directed:
                raise MeshError("open or non-manifold edge")
            cp, ip = directed[(lo, hi)]
            cm, im = directed[(hi, lo)]
            self.cplus[n], self.lplus[n] = cp, ip
            self.cminus[n], self.lminus[n] = cm, im
            self.cell_edges[cp, ip], self.cell_sign[cp, ip] = n, +1.0
            self.cell_edges[cm, im], self.cell_sign[cm, im] = n, -1.0
        self.free_plus = tri[self.cplus, self.lplus]
        self.free_minus = tri[self.cminus, self.lminus]

        P = xyz[tri]
        cr = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
        nrm = np.linalg.norm(cr, axis=1)
        if np.any(nrm <= 0):
            raise MeshError("degenerate cell")
        self.area = 0.5 * nrm
        self.normal = cr / nrm[:, None]
        self.centroid = P.mean(axis=1)
        self.noc = np.bincount(tri.ravel(), minlength=self.V)
        chi = self.V - self.N + self.C
        self.genus = (2 - chi) // 2

        # star and loop matrices, dense (small meshes only)
        self.Sigma = np.zeros((self.N, self.C))
        self.Sigma[np.arange(self.N), self.cplus] = 1.0
        self.Sigma[np.arange(self.N), self.cminus] = -1.0
        self.Lambda = np.zeros((self.N, self.V))
        self.Lambda[np.arange(self.N), self.edges[:, 0]] = 1.0
        self.Lambda[np.arange(self.N), self.edges[:, 1]] = -1.0

    def free_vertex_xyz(self, c, i):
        """Free vertex of local edge i of cell c."""
        return self.xyz[self.tri[c, i]]

    def longest_edge(self):
        P = self.xyz[self.tri]
        e = np.stack([np.linalg.norm(P[:, (i + 2) % 3] - P[:, (i + 1) % 3], axis=1) for i in range(3)], axis=1)
        return e.max(axis=1)

    def edge_lengths(self):
        return np.linalg.norm(self.xyz[self.edges[:, 0]] - self.xyz[self.edges[:, 1]], axis=1)
