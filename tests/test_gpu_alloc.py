"""Device memory through the registered allocator (rfcmp_set_allocator).

The binding registers torch's caching allocator at import, so the library's
buffers (blocks, projector matrices, workspaces, scratch) are torch memory.
An allocator that has nothing left (returns NULL) must turn the call that
needed memory into RFCMP_E_OOM, with its outputs untouched, and leave the
mesh usable once memory is back.
"""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    import paper_1803_08333_amd as rf
    assert torch.cuda.is_available()
    return torch, rf


def test_buffers_come_from_torch():
    """An operator's blocks (T_A 8 N ldA bytes, V 8 C ldV bytes at least)
    show in torch's allocated memory, and closing the operator and the mesh
    gives them back."""
    torch, rf = _gpu()
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    m = rf.Mesh(*synth.icosphere(3))
    op = rf.Operator(m, 1.0, scaling=1)
    grown = torch.cuda.memory_allocated() - before
    assert grown >= 8 * m.N * m.N + 8 * m.C * m.C, grown
    op.close()
    m.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before


def test_allocator_without_memory_gives_oom():
    """With an allocator that returns NULL, rfcmp_op_create fails with
    RFCMP_E_OOM and leaves *out NULL; rfcmp_solve on an existing operator
    fails the same way once it needs a larger workspace, and leaves j as it
    was.  After torch's allocator is back the same mesh builds an operator
    equal to one built on a fresh mesh."""
    torch, rf = _gpu()
    xyz, tri = synth.icosphere(2)
    m = rf.Mesh(xyz, tri)
    op1 = rf.Operator(m, 0.5, scaling=1)
    e1 = op1.rhs_planewave(*synth.default_plane_wave())
    op1.solve(e1, tol=1e-6)                      # workspace for one right-hand side
    e = op1.rhs_planewave(*synth.plane_waves(9, 2))   # nine right-hand sides: needs a larger workspace
    calls = []

    def refuse(nbytes):
        calls.append(nbytes)
        return None

    rf.set_allocator(refuse, lambda p, n: None)
    try:
        h = ctypes.c_void_p(12345)
        opts = rf.options(scaling=1)
        st = rf.lib.rfcmp_op_create(m.handle, 0.7, ctypes.byref(opts), None,
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), ctypes.byref(h))
        assert st == -7, (st, rf.lib.rfcmp_last_error())
        assert h.value is None
        assert calls
        j = torch.full_like(e, 3.0 + 1.0j)
        info = (rf.Info * 9)()
        st = rf.lib.rfcmp_solve(op1.handle, ctypes.c_void_p(e.data_ptr()), ctypes.c_void_p(j.data_ptr()), 9,
                                1e-6, 100, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), info)
        assert st == -7, (st, rf.lib.rfcmp_last_error())
        assert torch.all(j == 3.0 + 1.0j)
    finally:
        rf.use_torch_allocator()
    op2 = rf.Operator(m, 0.7, scaling=1)
    fresh = rf.Operator(rf.Mesh(xyz, tri), 0.7, scaling=1)
    for a, b in zip(op2.export(), fresh.export()):
        assert torch.equal(a, b)
    j, st, _ = op1.solve(e, tol=1e-6)
    assert st == 0


def test_counting_allocator_balances():
    """Every block the library takes from a registered allocator is handed
    back to it, with the size it asked for."""
    torch, rf = _gpu()
    live = {}

    def alloc(nbytes):
        p = torch.cuda.caching_allocator_alloc(nbytes)
        live[p] = nbytes
        return p

    def free(p, nbytes):
        assert live.pop(p) == nbytes
        torch.cuda.caching_allocator_delete(p)

    rf.set_allocator(alloc, free)
    try:
        m = rf.Mesh(*synth.torus(12, 8))
        start = torch.from_numpy(synth.complex_start(m.N, 11)).cuda()
        op = rf.Operator(m, 0.5, power_start=start, precision=1)
        e = op.rhs_planewave(*synth.plane_waves(6, 3))
        _, st, _ = op.solve(e, tol=1e-6)
        assert st == 0 and live
        op.close()
        m.close()
        assert not live, live
    finally:
        rf.use_torch_allocator()
