"""Closed-form potentials of a flat triangle, used for singularity extraction.

The paper fixes the kernel G_k(R) = exp(ikR)/(4 pi R) (Sec. 2) but not how the
singular integrals are evaluated.  The quadrature spec splits
G = 1/(4 pi R) + (exp(ikR) - 1)/(4 pi R) on near pairs and integrates the
1/R part over the source triangle in closed form, with the published formulas
for uniform and linear sources on a polygon (Wilton, Rao, Glisson, Schaubert,
Al-Bundak, Butler, IEEE TAP 32(3), 1984; Graglia, IEEE TAP 41(10), 1993):

  S(r)    = int_T 1/|r - r'| dS'
          = sum_i [ t_i f_i - |d| (atan(t_i l_i+/(R0_i^2 + |d| R_i+))
                                  - atan(t_i l_i-/(R0_i^2 + |d| R_i-))) ]
  W(r)    = int_T (rho' - rho)/|r - r'| dS'
          = 1/2 sum_i u_i [ R0_i^2 f_i + l_i+ R_i+ - l_i- R_i- ]
  int_T (r' - r)/|r - r'| dS' = W(r) - d n S(r)

with, for edge i from vertex a to vertex b (CCW about the unit normal n):
d = n.(r - a) the height of r over the plane, rho = r - d n, l_hat the edge
direction, u_i = l_hat x n the outward in-plane edge normal,
t_i = (a - rho).u_i, l_i- = (a - rho).l_hat, l_i+ = (b - rho).l_hat,
R_i-/R_i+ = |r - a|/|r - b|, R0_i^2 = t_i^2 + d^2 and
f_i = ln((R_i+ + l_i+)/(R_i- + l_i-)) = ln((R_i- - l_i-)/(R_i+ - l_i+)).
"""

import numpy as np

__all__ = ["potentials"]


def potentials(P, r):
    """Closed-form S(r) and int_T (r'-r)/R dS' for one triangle.

    P: [3,3] vertices (CCW about the normal), r: [..., 3] observation points.
    Returns (S [...], Vvec [..., 3]).
    """
    P = np.asarray(P, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    nrm = np.cross(P[1] - P[0], P[2] - P[0])
    n = nrm / np.linalg.norm(nrm)
    d = (r - P[0]) @ n
    rho = r - d[..., None] * n
    ad = np.abs(d)
    S = np.zeros(r.shape[:-1])
    W = np.zeros(r.shape)
    for i in range(3):
        a, b = P[i], P[(i + 1) % 3]
        L = np.linalg.norm(b - a)
        lh = (b - a) / L
        u = np.cross(lh, n)
        t = (a - rho) @ u
        lm = (a - rho) @ lh
        lp = (b - rho) @ lh
        Rm = np.linalg.norm(r - a, axis=-1)
        Rp = np.linalg.norm(r - b, axis=-1)
        R02 = t * t + d * d
        # the two equivalent forms of f; use the one without cancellation
        with np.errstate(divide="ignore", invalid="ignore"):
            f_pos = np.log((Rp + lp) / (Rm + lm))
            f_neg = np.log((Rm - lm) / (Rp - lp))
        f = np.where(lp + lm >= 0.0, f_pos, f_neg)
        # on the edge line itself (R0 = 0) the f-terms carry a zero factor
        tiny = R02 <= (1e-30 * L * L)
        f = np.where(tiny, 0.0, f)
        with np.errstate(divide="ignore", invalid="ignore"):
            at = np.arctan(t * lp / (R02 + ad * Rp)) - np.arctan(t * lm / (R02 + ad * Rm))
        at = np.where(ad > 0.0, at, 0.0)
        S += t * f - ad * at
        W += 0.5 * (R02 * f + lp * Rp - lm * Rm)[..., None] * u
    Vvec = W - (d * S)[..., None] * n
    return S, Vvec
