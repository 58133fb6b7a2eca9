"""Triangle quadrature used by the quadrature spec (the paper names no rule).

The 7-point, degree-5 symmetric rule of Radon (1948), also listed as
Stroud T2:5-1 and as Dunavant's degree-5 rule: the centroid plus two orbits of
three points, barycentric coordinates and weights in closed form with sqrt(15).
Weights are normalised to sum to one, so that the integral over a triangle of
area A is A * sum_q w_q f(x_q).
"""

import numpy as np

__all__ = ["tri7_barycentric", "tri7_points"]


def tri7_barycentric():
    """(bary [7,3], weights [7]) of the degree-5 rule, weights summing to 1."""
    s = np.sqrt(15.0)
    a1, b1 = (6.0 - s) / 21.0, (9.0 + 2.0 * s) / 21.0
    a2, b2 = (6.0 + s) / 21.0, (9.0 - 2.0 * s) / 21.0
    w0 = 9.0 / 40.0
    w1 = (155.0 - s) / 1200.0
    w2 = (155.0 + s) / 1200.0
    bary = np.array([
        [1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0],
        [a1, a1, b1], [a1, b1, a1], [b1, a1, a1],
        [a2, a2, b2], [a2, b2, a2], [b2, a2, a2],
    ])
    w = np.array([w0, w1, w1, w1, w2, w2, w2])
    return bary, w


def tri7_points(xyz, tri):
    """Quadrature points of every cell: float64 [C,7,3], and weights [7]."""
    bary, w = tri7_barycentric()
    P = xyz[tri]  # [C,3,3]
    pts = np.einsum("qk,ckd->cqd", bary, P)
    return pts, w
