"""Cached small meshes and oracle results shared by the CPU tests."""
import functools

import numpy as np

import synth
from oracle import assembly, rfcmp, rhs, topology


@functools.lru_cache(maxsize=None)
def mesh(name):
    if name.startswith("ico"):
        return synth.icosphere(int(name[3:]))
    if name == "torus_small":
        return synth.torus(12, 8, jitter=0.01, seed=3)
    if name.startswith("cube"):
        return synth.cube(int(name[4:]))
    if name == "ellipsoid1":
        return synth.ellipsoid(1, (1.3, 0.8, 0.6))
    raise KeyError(name)


@functools.lru_cache(maxsize=None)
def topo(name):
    return topology.Topology(*mesh(name))


@functools.lru_cache(maxsize=None)
def blocks(name, k):
    return assembly.assemble(topo(name), k)


@functools.lru_cache(maxsize=None)
def precond(name, k, outer_star="sigma", scal="power"):
    top = topo(name)
    TA, V = blocks(name, k)
    pre = rfcmp.Preconditioner(top, TA, V, k, outer_star=outer_star)
    if scal == "power":
        pre.power_scalings(synth.complex_start(top.N, 11), 30)
    else:
        pre.k_scalings()
    return pre


@functools.lru_cache(maxsize=None)
def excitation(name, k):
    kh, pol = synth.default_plane_wave()
    return rhs.planewave(topo(name), k, kh, pol)[0]


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))
