"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every function include/rfcmp.h declares, and its topology, near-pair list and
mesh validation agree with the oracle exactly."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from oracle import assembly
from oracle.topology import Topology

from ._meshes import mesh


def _header_functions(root):
    src = open(os.path.join(root, "include", "rfcmp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rfcmp_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol(root):
    import paper_1803_08333_amd as rf
    declared = _header_functions(root)
    assert len(declared) >= 20
    raw = ctypes.CDLL(rf.LIB_PATH)
    for name in declared:
        assert hasattr(raw, name), name
        assert name in rf.EXPORTED, name
    assert set(rf.EXPORTED) == set(declared)


@pytest.mark.parametrize("name", ["ico0", "ico2", "torus_small", "cube2", "ellipsoid1"])
def test_topology_matches_oracle(name):
    import paper_1803_08333_amd as rf
    xyz, tri = mesh(name)
    top = Topology(xyz, tri)
    m = rf.Mesh(xyz, tri)
    assert (m.N, m.V, m.C, m.genus) == (top.N, top.V, top.C, top.genus)
    ev, ec, el = m.edges()
    assert np.array_equal(ev, top.edges)
    assert np.array_equal(ec, np.stack([top.cplus, top.cminus], 1))
    assert np.array_equal(el, np.stack([top.lplus, top.lminus], 1))


@pytest.mark.parametrize("name,factor", [("ico2", 2.0), ("cube2", 2.0), ("cube2", 1.0), ("torus_small", 3.0)])
def test_near_pairs_match_oracle(name, factor):
    """Includes the structured cube, where exact distance ties sit on the
    threshold (resolved as near by the 1e-9 slack on both sides)."""
    import paper_1803_08333_amd as rf
    xyz, tri = mesh(name)
    top = Topology(xyz, tri)
    ref = np.argwhere(np.triu(assembly.near_mask(top, factor)))
    got = rf.Mesh(xyz, tri).near_pairs(factor)
    assert np.array_equal(got, ref)


def _status(xyz, tri):
    import paper_1803_08333_amd as rf
    try:
        rf.Mesh(xyz, tri)
    except rf.RfcmpError as e:
        return e.status
    return 0


def test_mesh_validation_codes():
    xyz, tri = synth.icosphere(1)
    assert _status(xyz, tri) == 0
    assert _status(xyz, tri[:-1]) == -2                          # open
    bad = tri.copy()
    bad[0] = bad[0][[0, 2, 1]]
    assert _status(xyz, bad) == -4                                # orientation
    bad = tri.copy()
    bad[0, 0] = bad[0, 1]
    assert _status(xyz, bad) == -3                                # repeated vertex
    bad = tri.copy()
    bad[0, 0] = len(xyz)
    assert _status(xyz, bad) == -3                                # out of range
    deg = xyz.copy()
    t0 = tri[0]
    deg[t0[2]] = 0.5 * (deg[t0[0]] + deg[t0[1]])
    assert _status(deg, tri) == -6                                # zero area
    # two disjoint spheres
    x2 = np.concatenate([xyz, xyz + 5.0])
    t2 = np.concatenate([tri, tri + len(xyz)])
    assert _status(x2, t2) == -5
    # two spheres glued at one vertex (pinch: one vertex, two fans)
    # second sphere: reflect so that its vertex 0 lands on the first one's vertex 0
    xb = -xyz + 2 * xyz[0]
    x3 = np.concatenate([xyz, xb[1:]])
    tb = np.where(tri == 0, 0, tri + len(xyz) - 1)[:, [0, 2, 1]]  # reflection flips orientation
    assert _status(x3, np.concatenate([tri, tb])) == -3
    assert _status(xyz, np.zeros((0, 3), np.int32)) == -1


def test_options_defaults():
    import paper_1803_08333_amd as rf
    o = rf.options()
    assert (o.near_factor, o.outer_star, o.scaling, o.power_iters, o.precision, o.power_tol, o.streams) == \
        (2.0, 0, 0, 30, 0, 1e-2, 4)
    assert (o.projector, o.graphs, o.aca_tol, o.block_cg) == (0, 0, 0.0, -1)


def test_rhs_gap_argument_errors():
    """rfcmp_rhs_gap rejects bad arguments before any device work (no GPU
    needed): an edge out of range, nrhs = 0, missing edge or voltage arrays."""
    import paper_1803_08333_amd as rf
    m = rf.Mesh(*synth.icosphere(1))
    e = ctypes.c_void_p(16)                      # never dereferenced: every call below fails validation
    v = np.ones(2, dtype=np.complex128)
    for edges, ng, nr in (([0, m.N], 2, 1), ([-1, 0], 2, 1), ([0, 1], 2, 0)):
        ed = np.asarray(edges, dtype=np.int32)
        st = rf.lib.rfcmp_rhs_gap(m.handle, ed.ctypes.data_as(rf._PI32), v.ctypes.data_as(ctypes.c_void_p),
                                  ng, nr, e, None)
        msg = rf.lib.rfcmp_last_error()
        assert st < 0 and (b"nrhs" in msg or b"range" in msg), msg
    assert rf.lib.rfcmp_rhs_gap(m.handle, None, None, 1, 1, e, None) < 0
    with pytest.raises(ValueError):
        m.rhs_gap([1, 2], [1.0])
    m.close()


def test_create_many_argument_errors():
    """rfcmp_op_create_many rejects bad arguments before any device work and
    leaves every output NULL."""
    import paper_1803_08333_amd as rf
    m = rf.Mesh(*synth.icosphere(1))
    out = (ctypes.c_void_p * 2)(1, 1)
    ks = np.array([1.0, 0.0])
    o = rf.options(scaling=1)
    st = rf.lib.rfcmp_op_create_many(m.handle, ks.ctypes.data_as(rf._PD), 0, ctypes.byref(o), None, None, out)
    assert st < 0
    st = rf.lib.rfcmp_op_create_many(m.handle, ks.ctypes.data_as(rf._PD), 2, ctypes.byref(o), None, None, out)
    assert st < 0 and not out[0] and not out[1], rf.lib.rfcmp_last_error()
    ks = np.array([1.0, 2.0])
    for streams in (0, 5, -1):
        o = rf.options(scaling=1, streams=streams)
        st = rf.lib.rfcmp_op_create_many(m.handle, ks.ctypes.data_as(rf._PD), 2, ctypes.byref(o), None, None, out)
        assert st == -1 and b"streams" in rf.lib.rfcmp_last_error() and not out[0] and not out[1]
    # compressed blocks: a tolerance in [0, 1), and precision 0 only
    for kw in ({"block_cg": 2}, {"block_cg": -2}):
        o = rf.options(scaling=1, **kw)
        st = rf.lib.rfcmp_op_create_many(m.handle, ks.ctypes.data_as(rf._PD), 2, ctypes.byref(o), None, None, out)
        assert st == -1 and b"block_cg" in rf.lib.rfcmp_last_error() and not out[0] and not out[1]
    for kw in ({"aca_tol": -1e-4}, {"aca_tol": 1.0}, {"aca_tol": float("nan")}, {"aca_tol": 1e-4, "precision": 1}):
        o = rf.options(scaling=1, **kw)
        st = rf.lib.rfcmp_op_create_many(m.handle, ks.ctypes.data_as(rf._PD), 2, ctypes.byref(o), None, None, out)
        assert st == -1 and b"aca_tol" in rf.lib.rfcmp_last_error() and not out[0] and not out[1]
    m.close()


def test_batch_solve_argument_errors():
    """rfcmp_batch_solve rejects bad arguments before any device work (no GPU
    needed): no operators, NULL arrays, a bad tolerance, a NULL or aliased
    entry, nrhs = 0, the same handle twice.  The handles are never
    dereferenced by these checks."""
    import paper_1803_08333_amd as rf
    P = ctypes.c_void_p

    def call(ops, es, js, nr, tol=1e-6, maxit=10, n=None):
        n = len(ops) if n is None else n
        arr = lambda xs: (P * max(len(xs), 1))(*xs)
        st = rf.lib.rfcmp_batch_solve(arr(ops), n, arr(es), arr(js), (ctypes.c_int32 * max(len(nr), 1))(*nr),
                                      tol, maxit, None, None)
        return st, rf.lib.rfcmp_last_error()

    assert call([], [], [], [], n=0)[0] == -1
    assert rf.lib.rfcmp_batch_solve(None, 1, None, None, None, 1e-6, 10, None, None) == -1
    assert call([16], [32], [48], [1], tol=0.0)[0] == -1
    assert call([16], [32], [48], [1], tol=float("nan"))[0] == -1
    assert call([16], [32], [48], [1], maxit=0)[0] == -1
    st, msg = call([16, 0], [32, 64], [48, 80], [1, 1])
    assert st == -1 and b"operator 1" in msg, msg
    st, msg = call([16, 24], [32, 64], [48, 64], [1, 1])
    assert st == -1 and b"operator 1" in msg, msg
    st, msg = call([16, 24], [32, 64], [48, 80], [1, 0])
    assert st == -1 and b"nrhs" in msg, msg
    st, msg = call([16, 24, 16], [32, 64, 96], [48, 80, 112], [1, 1, 1])
    assert st == -1 and b"twice" in msg, msg
    with pytest.raises(ValueError):
        rf.batch_solve([], [])


def test_set_allocator_arguments():
    """rfcmp_set_allocator: both functions or neither (else RFCMP_E_ARG);
    registering and resetting are host calls that touch no device."""
    import paper_1803_08333_amd as rf
    lib = rf.lib
    none_a, none_f = ctypes.cast(None, rf.ALLOC_FN), ctypes.cast(None, rf.FREE_FN)
    a = rf.ALLOC_FN(lambda n, s, c: None)
    f = rf.FREE_FN(lambda p, n, s, c: None)
    assert lib.rfcmp_set_allocator(a, none_f, None) == -1
    assert b"both" in lib.rfcmp_last_error()
    assert lib.rfcmp_set_allocator(none_a, f, None) == -1
    assert lib.rfcmp_set_allocator(a, f, None) == 0
    assert lib.rfcmp_set_allocator(none_a, none_f, None) == 0
    with pytest.raises(ValueError):
        rf.set_allocator(lambda n: 0, None)
    rf.use_torch_allocator()             # the import default, restored
    assert rf._alloc_state["fns"] is not None


def test_noalloc_limit_matches_header(root):
    import paper_1803_08333_amd as rf
    src = open(os.path.join(root, "include", "rfcmp.h")).read()
    m = re.search(r"#define RFCMP_RHS_NOALLOC_MAX (\d+)", src)
    assert m and int(m.group(1)) == rf.RHS_NOALLOC_MAX
