"""Python binding of librfcmp (RF-CMP EFIE solver on MI355X / gfx950).

Argument marshalling only: every step of the computation runs in the HIP
library.  Device buffers are torch tensors on the current CUDA (HIP) device
and work is enqueued on torch's current stream.  The functions keep the C
names of include/rfcmp.h; ``Mesh`` and ``Operator`` wrap the handles.

The library must be built first (``python paper_1803_08333_amd/build.py``);
importing this module without it raises, there is no fallback path.

Device memory: importing the module registers torch's caching allocator with
the library (rfcmp_set_allocator), so every device buffer the library owns
comes from torch and shows in torch.cuda.memory_allocated().  Handles still
open at interpreter exit are closed by an exit hook, while torch is alive.

torch is imported before the library is loaded.  torch brings its own HIP
runtime; when the library (linked against the system ROCm) is loaded first,
its first HIP call in a process that later initialises torch finds no
device, whereas with torch's runtime loaded first both see the GPU.
"""

import atexit
import ctypes
import os
import threading
import weakref

import numpy as np
import torch  # noqa: F401  (load order of the HIP runtimes, see above)

__all__ = [
    "LIB_PATH", "RfcmpError", "Options", "Info", "Mesh", "Operator", "lib",
    "PROJ_SIGMA", "PROJ_LH", "PROJ_GSIGMA", "PROJ_LPINV", "PROJ_GLL_INV", "PROJ_SIGMA_T", "PROJ_LAMBDA_T",
    "EXPORTED", "batch_solve", "set_allocator", "use_torch_allocator", "RHS_NOALLOC_MAX",
    "PROJECTOR_AUTO", "PROJECTOR_SPARSE", "PROJECTOR_DENSE",
]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "librfcmp.so")

PROJ_SIGMA, PROJ_LH, PROJ_GSIGMA, PROJ_LPINV, PROJ_GLL_INV, PROJ_SIGMA_T, PROJ_LAMBDA_T = range(7)
RHS_NOALLOC_MAX = 4096   # RFCMP_RHS_NOALLOC_MAX
PROJECTOR_AUTO, PROJECTOR_SPARSE, PROJECTOR_DENSE = 0, 1, 2   # rfcmp_options.projector

_STATUS = {
    0: "OK", 1: "W_NOT_CONVERGED", -1: "E_ARG", -2: "E_MESH_OPEN", -3: "E_MESH_NONMANIFOLD",
    -4: "E_MESH_ORIENT", -5: "E_MESH_DISCONNECTED", -6: "E_MESH_DEGENERATE", -7: "E_OOM",
    -8: "E_HIP", -9: "E_BREAKDOWN", -10: "E_STATE",
}


class RfcmpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"rfcmp {_STATUS.get(status, status)} ({status}): {msg}")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("near_factor", ctypes.c_double), ("outer_star", ctypes.c_int32),
                ("scaling", ctypes.c_int32), ("power_iters", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("power_tol", ctypes.c_double),
                ("streams", ctypes.c_int32), ("projector", ctypes.c_int32), ("graphs", ctypes.c_int32),
                ("aca_tol", ctypes.c_double), ("block_cg", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("rel_residual", ctypes.c_double), ("ms_solve", ctypes.c_double),
                ("cond_estimate", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_D = ctypes.c_double
_PI64 = ctypes.POINTER(ctypes.c_int64)
_PI32 = ctypes.POINTER(ctypes.c_int32)
_PD = ctypes.POINTER(ctypes.c_double)

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)

# name -> (restype, argtypes)
EXPORTED = {
    "rfcmp_set_allocator": (_I32, [ALLOC_FN, FREE_FN, _P]),
    "rfcmp_last_error": (ctypes.c_char_p, []),
    "rfcmp_version": (ctypes.c_char_p, []),
    "rfcmp_mesh_create": (_I32, [_PD, _I64, _PI32, _I64, ctypes.POINTER(_P)]),
    "rfcmp_mesh_sizes": (_I32, [_P, _PI64, _PI64, _PI64, _PI32]),
    "rfcmp_mesh_edges": (_I32, [_P, _PI32, _PI32, _PI32]),
    "rfcmp_mesh_near_pairs": (_I32, [_P, _D, _PI64, _PI32]),
    "rfcmp_mesh_factor_info": (_I32, [_P, _I32, _PI64, _PI32, _PI32, _PI64, _PD]),
    "rfcmp_mesh_destroy": (None, [_P]),
    "rfcmp_options_default": (_I32, [ctypes.POINTER(Options)]),
    "rfcmp_op_create": (_I32, [_P, _D, ctypes.POINTER(Options), _P, _P, ctypes.POINTER(_P)]),
    "rfcmp_op_create_many": (_I32, [_P, _PD, _I32, ctypes.POINTER(Options), _P, _P, ctypes.POINTER(_P)]),
    "rfcmp_op_scalings": (_I32, [_P, _PD, _PD, _PD, _PD]),
    "rfcmp_op_set_scalings": (_I32, [_P, _D, _D, _D]),
    "rfcmp_op_power_steps": (_I32, [_P, _PI32]),
    "rfcmp_op_export": (_I32, [_P, _P, _P, _P]),
    "rfcmp_op_compression": (_I32, [_P, _PI64, _PI64, _PI32, _PI32, _PD]),
    "rfcmp_op_destroy": (None, [_P]),
    "rfcmp_rhs_planewave": (_I32, [_P, _PD, _PD, _I32, _P, _P]),
    "rfcmp_rhs_planewave_noalloc": (_I32, [_P, _PD, _PD, _I32, _P, _P]),
    "rfcmp_rhs_planewave_split": (_I32, [_P, _PD, _PD, _I32, _P, _P, _P]),
    "rfcmp_solve_split": (_I32, [_P, _P, _P, _P, _P, _I32, _D, _I32, _P, ctypes.POINTER(Info)]),
    "rfcmp_farfield_split": (_I32, [_P, _P, _P, _I32, _PD, _I32, _P, _P, _P]),
    "rfcmp_rhs_gap": (_I32, [_P, _PI32, _P, _I32, _I32, _P, _P]),
    "rfcmp_farfield": (_I32, [_P, _P, _I32, _PD, _I32, _P, _P, _P]),
    "rfcmp_precond_rhs": (_I32, [_P, _P, _P, _I32, _P]),
    "rfcmp_apply": (_I32, [_P, _P, _P, _I32, _P]),
    "rfcmp_recover": (_I32, [_P, _P, _P, _I32, _P]),
    "rfcmp_project": (_I32, [_P, _I32, _P, _P, _I32, _P]),
    "rfcmp_matvec": (_I32, [_P, _I32, _I32, _P, _P, _I32, _P]),
    "rfcmp_solve": (_I32, [_P, _P, _P, _I32, _D, _I32, _P, ctypes.POINTER(Info)]),
    "rfcmp_solve_system": (_I32, [_P, _P, _P, _I32, _D, _I32, _P, ctypes.POINTER(Info)]),
    "rfcmp_batch_solve": (_I32, [ctypes.POINTER(_P), _I32, ctypes.POINTER(_P), ctypes.POINTER(_P), _PI32, _D, _I32,
                                 _P, ctypes.POINTER(Info)]),
    "rfcmp_profile_enable": (_I32, [_I32]),
    "rfcmp_profile_read": (_I32, [ctypes.c_char_p, _PD, _PI64]),
    "rfcmp_profile_select": (_I32, [ctypes.c_char_p]),
    "rfcmp_release_cached_memory": (_I32, [_PI64]),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python paper_1803_08333_amd/build.py`")
    h = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in EXPORTED.items():
        fn = getattr(h, name)
        fn.restype = res
        fn.argtypes = args
    return h


lib = _load()


def _check(status):
    if status < 0:
        raise RfcmpError(status, lib.rfcmp_last_error().decode())
    return status


def _torch():
    import torch
    return torch


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _dptr(t, dtype=None, numel=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA (HIP) tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"expected {numel} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


# ------------------------------------------------------------ device memory
_live = weakref.WeakSet()          # open Mesh / Operator objects
_alloc_state = {"fns": None, "closing": False}
_alloc_lock = threading.Lock()


def set_allocator(alloc=None, free=None):
    """rfcmp_set_allocator with Python callables: alloc(nbytes) -> device
    address (int) or None/0 when out of memory, free(address, nbytes).  Both
    None restores the library's own cache.  The callables run on whichever
    thread the library allocates from and must not raise; an exception is
    treated as out of memory (alloc) or ignored (free)."""
    if (alloc is None) != (free is None):
        raise ValueError("give both functions or neither")
    if alloc is None:
        _check(lib.rfcmp_set_allocator(ctypes.cast(None, ALLOC_FN), ctypes.cast(None, FREE_FN), None))
        _alloc_state["fns"] = None
        return

    def _a(nbytes, stream, ctx):
        if _alloc_state["closing"]:
            return None
        try:
            return alloc(int(nbytes)) or None
        except Exception:
            return None

    def _f(p, nbytes, stream, ctx):
        if _alloc_state["closing"] or not p:
            return
        try:
            free(int(p), int(nbytes))
        except Exception:
            pass

    fns = (ALLOC_FN(_a), FREE_FN(_f))
    with _alloc_lock:
        _check(lib.rfcmp_set_allocator(fns[0], fns[1], None))
        # every block goes back through the free function that was current
        # when it was made: keep all registered thunks alive
        _alloc_state.setdefault("kept", []).append(fns)
        _alloc_state["fns"] = fns


def use_torch_allocator():
    """Register torch's caching allocator (the import default)."""
    torch = _torch()

    def alloc(nbytes):
        return torch.cuda.caching_allocator_alloc(nbytes)

    def free(p, nbytes):
        torch.cuda.caching_allocator_delete(p)

    set_allocator(alloc, free)


def _close_all_at_exit():
    # operators before meshes (an operator needs its mesh); then stop calling
    # back into Python
    for obj in sorted(list(_live), key=lambda o: 0 if isinstance(o, Operator) else 1):
        try:
            obj.close()
        except Exception:
            pass
    _alloc_state["closing"] = True


def profile_enable(on=True):
    """rfcmp_profile_enable: start (or stop) HIP-event timing of tagged kernels."""
    _check(lib.rfcmp_profile_enable(int(bool(on))))


def release_cached_memory():
    """rfcmp_release_cached_memory: return kept device memory; bytes freed."""
    n = ctypes.c_int64(0)
    _check(lib.rfcmp_release_cached_memory(ctypes.byref(n)))
    return n.value


def profile_select(tags=None):
    """rfcmp_profile_select: time only the given kernel tags (None: all)."""
    _check(lib.rfcmp_profile_select(None if not tags else ",".join(tags).encode()))


def profile_read(tag):
    """rfcmp_profile_read: (total ms, launches) of one kernel tag."""
    t, n = _D(), _I64()
    _check(lib.rfcmp_profile_read(tag.encode(), ctypes.byref(t), ctypes.byref(n)))
    return t.value, n.value


def options(**kw):
    o = Options()
    _check(lib.rfcmp_options_default(ctypes.byref(o)))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Mesh:
    """rfcmp_mesh_create: topology of a closed triangle mesh (host work)."""

    def __init__(self, xyz, tri):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        tri = np.ascontiguousarray(tri, dtype=np.int32)
        h = _P()
        _check(lib.rfcmp_mesh_create(xyz.ctypes.data_as(_PD), len(xyz), tri.ctypes.data_as(_PI32), len(tri),
                                     ctypes.byref(h)))
        self.handle = h
        _live.add(self)
        N, V, C, g = _I64(), _I64(), _I64(), _I32()
        _check(lib.rfcmp_mesh_sizes(h, ctypes.byref(N), ctypes.byref(V), ctypes.byref(C), ctypes.byref(g)))
        self.N, self.V, self.C, self.genus = N.value, V.value, C.value, g.value

    def edges(self):
        """(edge_vtx, edge_cell, edge_local), each int32 [N, 2]."""
        out = [np.zeros((self.N, 2), dtype=np.int32) for _ in range(3)]
        _check(lib.rfcmp_mesh_edges(self.handle, *[a.ctypes.data_as(_PI32) for a in out]))
        return tuple(out)

    def near_pairs(self, near_factor=2.0):
        cnt = _I64()
        _check(lib.rfcmp_mesh_near_pairs(self.handle, near_factor, ctypes.byref(cnt), None))
        p = np.zeros((cnt.value, 2), dtype=np.int32)
        _check(lib.rfcmp_mesh_near_pairs(self.handle, near_factor, ctypes.byref(cnt), p.ctypes.data_as(_PI32)))
        return p

    def rhs_gap(self, edges, volts):
        """rfcmp_rhs_gap: voltage-gap excitation e [nrhs, N] (complex128) of
        gaps across the RWG edges edges [nrhs, G] (or [G]) with voltages volts
        of the same shape."""
        torch = _torch()
        edges = np.ascontiguousarray(np.atleast_2d(edges), dtype=np.int32)
        volts = np.ascontiguousarray(np.atleast_2d(volts), dtype=np.complex128)
        if edges.shape != volts.shape:
            raise ValueError("edges and volts must have the same shape")
        e = torch.empty((edges.shape[0], self.N), dtype=torch.complex128, device="cuda")
        _check(lib.rfcmp_rhs_gap(self.handle, edges.ctypes.data_as(_PI32), volts.ctypes.data_as(_P),
                                 edges.shape[1], edges.shape[0], _dptr(e), _stream()))
        return e

    def factor_info(self, which):
        """rfcmp_mesh_factor_info: dict of the sparse projector factor `which`
        (0 = L, 1 = G_ll, 2 = G_tp)."""
        n, st = _I64(), _I64()
        sn, lv = _I32(), _I32()
        sec = _D()
        _check(lib.rfcmp_mesh_factor_info(self.handle, which, ctypes.byref(n), ctypes.byref(sn), ctypes.byref(lv),
                                          ctypes.byref(st), ctypes.byref(sec)))
        return {"n": n.value, "supernodes": sn.value, "levels": lv.value, "stored_doubles": st.value,
                "host_seconds": sec.value}

    def close(self):
        if self.handle:
            lib.rfcmp_mesh_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Operator:
    """rfcmp_op_create: assembled T_A, V and scalings for one wavenumber."""

    def __init__(self, mesh, k, power_start=None, **opts):
        torch = _torch()
        self.mesh = mesh
        self.k = float(k)
        self.opts = options(**opts)
        ps = None
        if power_start is not None:
            ps = _dptr(power_start, torch.complex128, mesh.N)
        h = _P()
        _check(lib.rfcmp_op_create(mesh.handle, self.k, ctypes.byref(self.opts), ps, _stream(), ctypes.byref(h)))
        self.handle = h
        _live.add(self)

    @classmethod
    def create_many(cls, mesh, ks, power_start=None, **opts):
        """rfcmp_op_create_many: the operators of several wavenumbers on one
        mesh, their assemblies queued ahead of the first scalings."""
        torch = _torch()
        ks = np.ascontiguousarray(np.atleast_1d(ks), dtype=np.float64)
        o = options(**opts)
        ps = None if power_start is None else _dptr(power_start, torch.complex128, mesh.N)
        hs = (_P * len(ks))()
        _check(lib.rfcmp_op_create_many(mesh.handle, ks.ctypes.data_as(_PD), len(ks), ctypes.byref(o), ps,
                                        _stream(), hs))
        out = []
        for k, h in zip(ks, hs):
            op = cls.__new__(cls)
            op.mesh, op.k, op.opts, op.handle = mesh, float(k), options(**opts), _P(h)
            _live.add(op)
            out.append(op)
        return out

    def scalings(self):
        a, b, g = _D(), _D(), _D()
        lam = (_D * 3)()
        _check(lib.rfcmp_op_scalings(self.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(g), lam))
        return a.value, b.value, g.value, tuple(lam)

    def power_steps(self):
        """rfcmp_op_power_steps: power-iteration steps run at creation."""
        n = _I32()
        _check(lib.rfcmp_op_power_steps(self.handle, ctypes.byref(n)))
        return n.value

    def set_scalings(self, alpha, beta, gamma):
        _check(lib.rfcmp_op_set_scalings(self.handle, alpha, beta, gamma))

    def export(self):
        torch = _torch()
        N, C = self.mesh.N, self.mesh.C
        TA = torch.empty((N, N), dtype=torch.complex64, device="cuda")
        V = torch.empty((C, C), dtype=torch.complex64, device="cuda")
        _check(lib.rfcmp_op_export(self.handle, _dptr(TA), _dptr(V), _stream()))
        return TA, V

    def compression(self):
        """rfcmp_op_compression: storage of the compressed blocks (dict)."""
        de, le = (_I64 * 2)(), (_I64 * 2)()
        nb, mx = _I32(), _I32()
        mean = _D()
        _check(lib.rfcmp_op_compression(self.handle, de, le, ctypes.byref(nb), ctypes.byref(mx), ctypes.byref(mean)))
        return {"dense_entries": [de[0], de[1]], "lowrank_entries": [le[0], le[1]], "lowrank_blocks": nb.value,
                "max_rank": mx.value, "mean_rank": mean.value}

    def rhs_planewave(self, khat, pol):
        torch = _torch()
        khat = np.ascontiguousarray(np.atleast_2d(khat), dtype=np.float64)
        pol = np.ascontiguousarray(np.atleast_2d(pol), dtype=np.float64)
        e = torch.empty((len(khat), self.mesh.N), dtype=torch.complex128, device="cuda")
        _check(lib.rfcmp_rhs_planewave(self.handle, khat.ctypes.data_as(_PD), pol.ctypes.data_as(_PD), len(khat),
                                       _dptr(e), _stream()))
        return e

    def rhs_planewave_split(self, khat, pol):
        """rfcmp_rhs_planewave_split: (s [nrhs, C], e1 [nrhs, N]) with
        e = Sigma s + e1, complex128."""
        torch = _torch()
        khat = np.ascontiguousarray(np.atleast_2d(khat), dtype=np.float64)
        pol = np.ascontiguousarray(np.atleast_2d(pol), dtype=np.float64)
        s = torch.empty((len(khat), self.mesh.C), dtype=torch.complex128, device="cuda")
        e1 = torch.empty((len(khat), self.mesh.N), dtype=torch.complex128, device="cuda")
        _check(lib.rfcmp_rhs_planewave_split(self.handle, khat.ctypes.data_as(_PD), pol.ctypes.data_as(_PD),
                                             len(khat), _dptr(s), _dptr(e1), _stream()))
        return s, e1

    def solve_split(self, s, e1, tol=1e-6, maxit=1000):
        """rfcmp_solve_split: (j_loop, j_star, status, [info dict per rhs])."""
        torch = _torch()
        s, e1 = s.contiguous(), e1.contiguous()
        nr = e1.shape[0] if e1.dim() == 2 else 1
        jl, js = torch.empty_like(e1), torch.empty_like(e1)
        info = (Info * nr)()
        st = _check(lib.rfcmp_solve_split(self.handle, _dptr(s, torch.complex128, nr * self.mesh.C),
                                          _dptr(e1, torch.complex128, nr * self.mesh.N), _dptr(jl), _dptr(js), nr,
                                          tol, maxit, _stream(), info))
        return jl, js, st, [i.as_dict() for i in info]

    def far_field_split(self, j_loop, j_star, dirs):
        """rfcmp_farfield_split: F [nrhs, ndir, 3] and RCS [nrhs, ndir] of the
        current j_loop + j_star given as its two parts."""
        torch = _torch()
        jl, js = j_loop.contiguous(), j_star.contiguous()
        nr = jl.shape[0] if jl.dim() == 2 else 1
        dirs = np.ascontiguousarray(np.atleast_2d(dirs), dtype=np.float64)
        F = torch.empty((nr, len(dirs), 3), dtype=torch.complex128, device=jl.device)
        rcs = torch.empty((nr, len(dirs)), dtype=torch.float64, device=jl.device)
        _check(lib.rfcmp_farfield_split(self.handle, _dptr(jl, torch.complex128, nr * self.mesh.N),
                                        _dptr(js, torch.complex128, nr * self.mesh.N), nr, dirs.ctypes.data_as(_PD),
                                        len(dirs), _dptr(F), _dptr(rcs), _stream()))
        return F, rcs

    def rhs_planewave_noalloc(self, khat, pol, e):
        """rfcmp_rhs_planewave_noalloc into the caller's tensor e (complex128
        [nrhs, N]); the library allocates nothing."""
        torch = _torch()
        khat = np.ascontiguousarray(np.atleast_2d(khat), dtype=np.float64)
        pol = np.ascontiguousarray(np.atleast_2d(pol), dtype=np.float64)
        _check(lib.rfcmp_rhs_planewave_noalloc(self.handle, khat.ctypes.data_as(_PD), pol.ctypes.data_as(_PD),
                                               len(khat), _dptr(e, torch.complex128, len(khat) * self.mesh.N),
                                               _stream()))
        return e

    def _unary(self, fn, x, nout=None, *pre):
        torch = _torch()
        x = x.contiguous()
        nr = x.shape[0] if x.dim() == 2 else 1
        n_in = x.shape[-1]
        y = torch.empty((nr, nout or n_in) if x.dim() == 2 else (nout or n_in,), dtype=torch.complex128,
                        device=x.device)
        _check(fn(self.handle, *pre, _dptr(x, torch.complex128), _dptr(y), nr, _stream()))
        return y

    def far_field(self, j, dirs):
        """rfcmp_farfield: far-field vectors F [nrhs, ndir, 3] (complex128) and
        bistatic RCS [nrhs, ndir] of RWG currents j at unit directions dirs."""
        torch = _torch()
        j = j.contiguous()
        nr = j.shape[0] if j.dim() == 2 else 1
        dirs = np.ascontiguousarray(np.atleast_2d(dirs), dtype=np.float64)
        F = torch.empty((nr, len(dirs), 3), dtype=torch.complex128, device=j.device)
        rcs = torch.empty((nr, len(dirs)), dtype=torch.float64, device=j.device)
        _check(lib.rfcmp_farfield(self.handle, _dptr(j, torch.complex128, nr * self.mesh.N), nr,
                                  dirs.ctypes.data_as(_PD), len(dirs),
                                  _dptr(F), _dptr(rcs), _stream()))
        return F, rcs

    def precond_rhs(self, e):
        return self._unary(lib.rfcmp_precond_rhs, e)

    def apply(self, x):
        return self._unary(lib.rfcmp_apply, x)

    def recover(self, i):
        return self._unary(lib.rfcmp_recover, i)

    def project(self, which, x):
        m = self.mesh
        nout = {PROJ_SIGMA: m.N, PROJ_LH: m.N, PROJ_GSIGMA: m.N, PROJ_LPINV: m.C, PROJ_GLL_INV: m.V,
                PROJ_SIGMA_T: m.C, PROJ_LAMBDA_T: m.V}[which]
        return self._unary(lib.rfcmp_project, x, nout, ctypes.c_int32(which))

    def matvec(self, which, x, conj=False):
        return self._unary(lib.rfcmp_matvec, x, None, ctypes.c_int32(which), ctypes.c_int32(int(conj)))

    def solve(self, e, tol=1e-6, maxit=1000):
        """Returns (j, status, [info dict per rhs])."""
        torch = _torch()
        e = e.contiguous()
        nr = e.shape[0] if e.dim() == 2 else 1
        j = torch.empty_like(e)
        info = (Info * nr)()
        st = _check(lib.rfcmp_solve(self.handle, _dptr(e, torch.complex128), _dptr(j), nr, tol, maxit, _stream(),
                                    info))
        return j, st, [i.as_dict() for i in info]

    def solve_system(self, b, tol=1e-6, maxit=1000):
        """CG on A i = b itself (rfcmp_solve_system).  Returns (i, status,
        [info dict per rhs])."""
        torch = _torch()
        b = b.contiguous()
        nr = b.shape[0] if b.dim() == 2 else 1
        i = torch.empty_like(b)
        info = (Info * nr)()
        st = _check(lib.rfcmp_solve_system(self.handle, _dptr(b, torch.complex128), _dptr(i), nr, tol, maxit,
                                           _stream(), info))
        return i, st, [x.as_dict() for x in info]

    def close(self):
        if self.handle:
            lib.rfcmp_op_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_solve(ops, es, tol=1e-6, maxit=1000):
    """rfcmp_batch_solve: the solves of several operators (distinct
    ``Operator`` objects, meshes may be shared) run concurrently; es[q] holds
    operator q's right-hand sides (c128 [nrhs][N] or [N]).  Returns
    (js, status, [list of info dicts per operator])."""
    torch = _torch()
    n = len(ops)
    if n == 0 or len(es) != n:
        raise ValueError("need one right-hand-side tensor per operator")
    es = [e.contiguous() for e in es]
    js = [torch.empty_like(e) for e in es]
    nr = [e.shape[0] if e.dim() == 2 else 1 for e in es]
    hs = (_P * n)(*[op.handle for op in ops])
    ep = (_P * n)(*[_dptr(e, torch.complex128, r * op.mesh.N).value for e, r, op in zip(es, nr, ops)])
    jp = (_P * n)(*[_dptr(x).value for x in js])
    info = (Info * sum(nr))()
    st = _check(lib.rfcmp_batch_solve(hs, n, ep, jp, (_I32 * n)(*nr), tol, maxit, _stream(), info))
    out, k = [], 0
    for r in nr:
        out.append([info[k + i].as_dict() for i in range(r)])
        k += r
    return js, st, out


use_torch_allocator()
atexit.register(_close_all_at_exit)
