"""rfcmp_rhs_planewave_noalloc: the allocation-free plane-wave excitation.

Called through the C ABI, it must reproduce rfcmp_rhs_planewave exactly (the
same kernel on the same inputs: bit for bit), on two calls in a row, the
second with fewer plane waves than the first (the staging array keeps the
first call's contents), and it must take no memory from the library's
allocator: with an allocator that refuses every request registered, the
allocating entry point fails with RFCMP_E_OOM while this one succeeds.
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


def _call(rf, torch, fn, op, kh, pol, e):
    kh = np.ascontiguousarray(kh, dtype=np.float64)
    pol = np.ascontiguousarray(pol, dtype=np.float64)
    PD = ctypes.POINTER(ctypes.c_double)
    return fn(op.handle, kh.ctypes.data_as(PD), pol.ctypes.data_as(PD), len(kh), ctypes.c_void_p(e.data_ptr()),
              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def test_noalloc_matches_allocating_entry_point():
    torch, rf = _gpu()
    m = rf.Mesh(*synth.cube(5))                  # N = 450: ragged against 256-thread blocks
    op = rf.Operator(m, 1.3, scaling=1)
    refused = []

    def refuse(nbytes):
        refused.append(nbytes)
        return None

    for nrhs, seed in ((40, 8), (7, 9)):
        kh, pol = synth.plane_waves(nrhs, seed)
        ref = torch.empty((nrhs, m.N), dtype=torch.complex128, device="cuda")
        assert _call(rf, torch, rf.lib.rfcmp_rhs_planewave, op, kh, pol, ref) == 0
        got = torch.full((nrhs, m.N), np.nan + 0j, dtype=torch.complex128, device="cuda")
        rf.set_allocator(refuse, lambda p, n: None)
        try:
            st = _call(rf, torch, rf.lib.rfcmp_rhs_planewave_noalloc, op, kh, pol, got)
            assert st == 0, rf.lib.rfcmp_last_error()
            assert not refused
            # the allocating entry point needs its staging buffer
            other = torch.empty_like(ref)
            assert _call(rf, torch, rf.lib.rfcmp_rhs_planewave, op, kh, pol, other) == -7
            assert refused
            refused.clear()
        finally:
            rf.use_torch_allocator()
        torch.cuda.synchronize()
        assert torch.equal(got, ref), nrhs
    op.close()
    m.close()


def test_noalloc_rejects_too_many_plane_waves():
    torch, rf = _gpu()
    m = rf.Mesh(*synth.icosphere(1))
    op = rf.Operator(m, 0.5, scaling=1)
    n = rf.RHS_NOALLOC_MAX
    kh = np.tile([[0.0, 0.0, 1.0]], (n + 1, 1))
    pol = np.tile([[1.0, 0.0, 0.0]], (n + 1, 1))
    e = torch.empty((n + 1, m.N), dtype=torch.complex128, device="cuda")
    assert _call(rf, torch, rf.lib.rfcmp_rhs_planewave_noalloc, op, kh, pol, e) == -1
    assert b"nrhs" in rf.lib.rfcmp_last_error()
    op.close()
    m.close()
