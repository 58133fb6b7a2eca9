"""Excitations (Sec. 2 of the paper, the entries of e): plane wave and
voltage gap (the second source of the Fokker example, Sec. 4).

e_m = (n x f_m, n x E^i) = int f_m . E^i dS for tangential f_m, with
E^i(r) = pol exp(i k khat . r) (unit amplitude, e^{-i omega t} convention).
On cell c the RWG piece is sigma (r - r_m^c)/(2 A_c), so with the 7-point rule

  e_m = sum_{c in m} sigma/2 sum_q w_q (r_q - r_m^c) . pol exp(i k khat . r_q).
"""

import numpy as np

from .quadrature import tri7_points

__all__ = ["planewave", "planewave_split", "voltage_gap"]


def planewave(top, k, khat, pol):
    """e [nrhs, N] complex128 for plane waves khat [nrhs,3], pol [nrhs,3]."""
    khat = np.atleast_2d(np.asarray(khat, dtype=np.float64))
    pol = np.atleast_2d(np.asarray(pol, dtype=np.float64))
    pts, w = tri7_points(top.xyz, top.tri)
    e = np.zeros((len(khat), top.N), dtype=np.complex128)
    for l in range(len(khat)):
        phase = np.exp(1j * k * (pts @ khat[l]))            # [C,7]
        for c in range(top.C):
            for i in range(3):
                m = top.cell_edges[c, i]
                arm = pts[c] - top.xyz[top.tri[c, i]]          # [7,3]
                e[l, m] += top.cell_sign[c, i] / 2.0 * np.sum(w * (arm @ pol[l]) * phase[c])
    return e


def planewave_split(top, k, khat, pol):
    """The plane-wave excitation as e = Sigma s + e1, without cancellation at
    any k (the loop part of e is O(k) relative to e and is lost in a single
    FP64 vector below k ~ 1e-16).

    Split E^i = pol + pol (exp(i k khat . r) - 1).  The static term is the
    gradient of pol . r, so int f_m . pol = -int div(f_m) (pol . r) = -sum_c
    sigma_mc (pol . x_c), x_c the centroid: e_static = Sigma s with
    s_c = -pol . x_c, in the range of Sigma exactly (divergence theorem on the
    RWG function, whose normal component vanishes on the cell boundary except
    across its edge, where it is continuous).  The rest, e1, is integrated with
    the 7-point rule and exp(i t) - 1 = -2 sin^2(t/2) + i sin t.
    Returns s [nrhs, C] and e1 [nrhs, N], complex128."""
    khat = np.atleast_2d(np.asarray(khat, dtype=np.float64))
    pol = np.atleast_2d(np.asarray(pol, dtype=np.float64))
    pts, w = tri7_points(top.xyz, top.tri)
    s = np.zeros((len(khat), top.C), dtype=np.complex128)
    e1 = np.zeros((len(khat), top.N), dtype=np.complex128)
    for l in range(len(khat)):
        s[l] = -(top.centroid @ pol[l])
        t = k * (pts @ khat[l])                                # [C,7]
        em1 = -2.0 * np.sin(0.5 * t) ** 2 + 1j * np.sin(t)     # exp(i t) - 1
        for c in range(top.C):
            for i in range(3):
                m = top.cell_edges[c, i]
                arm = pts[c] - top.xyz[top.tri[c, i]]
                e1[l, m] += top.cell_sign[c, i] / 2.0 * np.sum(w * (arm @ pol[l]) * em1[c])
    return s, e1


def voltage_gap(top, edges, volts):
    """Delta-gap excitation, e [nrhs, N] complex128.  edges [nrhs, G] (or [G])
    RWG indices, volts complex of the same shape.

    The source field of a gap of voltage V across edge m is E^i = V delta(s)
    n_m, with s the in-plane distance from the edge and n_m its in-plane unit
    normal pointing from c+ into c- (the direction in which f_m carries
    current).  Then e_n = int f_n . E^i dS = V times the flux of f_n across
    edge m: 1 for n = m (the RWG normalisation) and 0 for every other n (their
    normal components vanish on edge m).  Gaps on the same edge add."""
    edges = np.atleast_2d(np.asarray(edges, dtype=np.int64))
    volts = np.atleast_2d(np.asarray(volts, dtype=np.complex128))
    if edges.shape != volts.shape:
        raise ValueError("edges and volts must have the same shape")
    if edges.size and (edges.min() < 0 or edges.max() >= top.N):
        raise ValueError("edge index out of range")
    e = np.zeros((len(edges), top.N), dtype=np.complex128)
    for r in range(len(edges)):
        for m, v in zip(edges[r], volts[r]):
            e[r, m] += v
    return e
