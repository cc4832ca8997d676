"""ctypes binding of libpetgem (include/petgem.h).

Argument marshalling only: every step of the solve runs in the HIP library.
PyTorch provides the device memory (``torch.cuda`` tensors are passed by
their data pointers) and the stream (the caller's current stream). Loading
fails loudly when the library has not been built; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpetgem.so")

OK, INVALID_ARG, DEGENERATE_ELEMENT, MESH_TOPOLOGY = 0, -1, -2, -3
RECEIVER_OUTSIDE, SOURCE_SINGULAR, NOT_CONVERGED, NONFINITE = -4, -5, -6, -7
HIP_ERROR, OUT_OF_MEMORY = -8, -9
GMRES, COCG, BCOCG, SQMR = 0, 1, 2, 3
JACOBI, SSOR = 0, 1
FP64, MIXED = 0, 1

_NAMES = {0: "OK", -1: "INVALID_ARG", -2: "DEGENERATE_ELEMENT", -3: "MESH_TOPOLOGY",
          -4: "RECEIVER_OUTSIDE", -5: "SOURCE_SINGULAR", -6: "NOT_CONVERGED", -7: "NONFINITE",
          -8: "HIP_ERROR", -9: "OUT_OF_MEMORY"}


class PetgemError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class Mesh(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_tets", C.c_int32),
                ("xyz", C.POINTER(C.c_double)), ("tets", C.POINTER(C.c_int32))]


class Source(C.Structure):
    _fields_ = [("freq_hz", C.c_double), ("pos", C.c_double * 3), ("dir", C.c_double * 3),
                ("moment", C.c_double)]


class Opts(C.Structure):
    _fields_ = [("method", C.c_int32), ("precision", C.c_int32), ("restart", C.c_int32),
                ("max_iter", C.c_int32), ("rtol", C.c_double), ("inner_rtol", C.c_double),
                ("use_graph", C.c_int32), ("profile", C.c_int32), ("verbose", C.c_int32),
                ("spmm_shape", C.c_int32), ("precond", C.c_int32), ("omega", C.c_double)]


class Background(C.Structure):
    _fields_ = [("layered", C.c_int32), ("z0", C.c_double), ("sigma_above", C.c_double),
                ("sigma_below", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("ir_steps", C.c_int32), ("used_fallback", C.c_int32),
                ("status", C.c_int32), ("rel_residual", C.c_double),
                ("x0_rel_residual", C.c_double), ("t_rhs_ms", C.c_double),
                ("t_solve_ms", C.c_double), ("spmv_ms", C.c_double),
                ("spmv_launches", C.c_int32), ("spmv_shape", C.c_int32), ("b_norm", C.c_double),
                ("block_iters", C.c_int32), ("reserved", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None

_SIGS = {
    "petgem_default_opts": (None, [C.POINTER(Opts)]),
    "petgem_assemble": (C.c_int, [C.POINTER(Mesh), C.POINTER(C.c_double), C.c_double, C.c_void_p,
                                  C.POINTER(C.c_void_p)]),
    "petgem_reassemble": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_void_p]),
    "petgem_set_background": (C.c_int, [C.c_void_p, C.POINTER(Background)]),
    "petgem_rhs": (C.c_int, [C.c_void_p, C.POINTER(Source), C.c_int32, C.c_void_p, C.c_void_p]),
    "petgem_rhs_noalloc": (C.c_int, [C.c_void_p, C.POINTER(Source), C.c_int32, C.c_void_p, C.c_void_p]),
    "petgem_solve": (C.c_int, [C.c_void_p, C.POINTER(Source), C.c_int32, C.POINTER(Opts),
                               C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(Stats)]),
    "petgem_solve_many": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(Source), C.c_int32,
                                    C.POINTER(Opts), C.POINTER(C.c_void_p), C.c_void_p,
                                    C.POINTER(C.c_void_p), C.POINTER(Stats)]),
    "petgem_receivers": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_void_p,
                                   C.c_void_p, C.c_void_p]),
    "petgem_receivers_h": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_void_p,
                                     C.c_void_p, C.c_void_p]),
    "petgem_num_dofs": (C.c_int32, [C.c_void_p]),
    "petgem_nnz": (C.c_int64, [C.c_void_p]),
    "petgem_solution_nsrc": (C.c_int32, [C.c_void_p]),
    "petgem_solution_x": (C.c_void_p, [C.c_void_p]),
    "petgem_solution_copy": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "petgem_get_dof_edges": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "petgem_get_csr": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                 C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_void_p]),
    "petgem_spmv": (C.c_int, [C.c_void_p, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p]),
    "petgem_setup_seconds": (C.c_double, [C.c_void_p]),
    "petgem_ssor_colors": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int32), C.c_void_p]),
    "petgem_ssor_apply": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p]),
    "petgem_sync_probe": (C.c_int, [C.c_int32, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_float), C.c_void_p]),
    "petgem_spmm_candidates": (C.c_int32, [C.c_int32, C.c_int32, C.POINTER(C.c_int32), C.c_int32]),
    "petgem_tuning": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_float)]),
    "petgem_mesh_pattern": (C.c_int, [C.POINTER(Mesh), C.POINTER(C.c_int32), C.POINTER(C.c_int64),
                                      C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int32)]),
    "petgem_locate": (C.c_int, [C.POINTER(Mesh), C.POINTER(C.c_double), C.c_int32, C.c_double,
                                C.POINTER(C.c_int32)]),
    "petgem_free_system": (None, [C.c_void_p]),
    "petgem_free_solution": (None, [C.c_void_p]),
    "petgem_last_error": (C.c_char_p, []),
    "petgem_net_create": (C.c_int, [C.c_int32, C.c_uint64, C.POINTER(C.c_void_p)]),
    "petgem_net_num_params": (C.c_int64, [C.c_void_p]),
    "petgem_net_get_params": (C.c_int, [C.c_void_p, C.POINTER(C.c_float)]),
    "petgem_net_set_params": (C.c_int, [C.c_void_p, C.POINTER(C.c_float)]),
    "petgem_net_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "petgem_net_loss_grad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                       C.POINTER(C.c_double), C.POINTER(C.c_float)]),
    "petgem_net_train_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_float,
                                        C.c_void_p, C.POINTER(C.c_double)]),
    "petgem_voxelize": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(Source), C.c_int32, C.c_void_p,
                                  C.c_void_p]),
    "petgem_vox_targets": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_void_p, C.c_void_p]),
    "petgem_learned_x0": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(Source), C.c_int32, C.c_double,
                                    C.c_void_p, C.POINTER(C.c_double), C.c_void_p]),
    "petgem_learned_x0_many": (C.c_int, [C.POINTER(C.c_void_p), C.c_void_p, C.POINTER(Source), C.c_int32,
                                         C.c_double, C.POINTER(C.c_void_p), C.POINTER(C.c_double), C.c_void_p]),
    "petgem_net_free": (None, [C.c_void_p]),
}


def lib():
    """Load libpetgem.so (built in-tree); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1808_00186_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int, allow=()):
    if rc != OK and rc not in allow:
        raise PetgemError(rc, lib().petgem_last_error().decode())
    return rc


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t) -> C.c_void_p:
    if t is None:
        return C.c_void_p(None)
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous CUDA tensor")
    return C.c_void_p(t.data_ptr())


def make_sources(dipoles) -> "C.Array":
    """Sources from objects with .pos, .dir, .freq, .moment (e.g. synth.Dipole)."""
    arr = (Source * len(dipoles))()
    for i, d in enumerate(dipoles):
        arr[i].freq_hz = d.freq
        arr[i].pos[:] = list(d.pos)
        arr[i].dir[:] = list(d.dir)
        arr[i].moment = d.moment
    return arr


def default_opts(**kw) -> Opts:
    o = Opts()
    lib().petgem_default_opts(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


class Solution:
    def __init__(self, system: "System", handle: C.c_void_p, n_src: int):
        self.system = system
        self.handle = handle
        self.n_src = n_src

    def x(self, stream=None):
        """Solution DOFs as a complex128 CUDA tensor [n_src][n_dof] (a copy)."""
        import torch
        out = torch.empty((self.n_src, self.system.n_dof), dtype=torch.complex128, device="cuda")
        _check(lib().petgem_solution_copy(self.handle, _ptr(out), _stream(stream)))
        return out

    def receivers(self, rx: np.ndarray, secondary: bool = False, stream=None):
        """Total field (and optionally the secondary field) at receivers:
        complex128 CUDA tensors [n_src][n_rx][3]."""
        import torch
        rx = np.ascontiguousarray(rx, dtype=np.float64)
        E = torch.empty((self.n_src, len(rx), 3), dtype=torch.complex128, device="cuda")
        Es = torch.empty_like(E) if secondary else None
        _check(lib().petgem_receivers(self.handle, rx.ctypes.data_as(C.POINTER(C.c_double)),
                                      len(rx), _ptr(E), _ptr(Es), _stream(stream)))
        return (E, Es) if secondary else E

    def receivers_h(self, rx: np.ndarray, secondary: bool = False, stream=None):
        """Total magnetic field H = curl E / (i w mu0) (and optionally its
        secondary part) at receivers: complex128 CUDA tensors [n_src][n_rx][3]."""
        import torch
        rx = np.ascontiguousarray(rx, dtype=np.float64)
        H = torch.empty((self.n_src, len(rx), 3), dtype=torch.complex128, device="cuda")
        Hs = torch.empty_like(H) if secondary else None
        _check(lib().petgem_receivers_h(self.handle, rx.ctypes.data_as(C.POINTER(C.c_double)),
                                        len(rx), _ptr(H), _ptr(Hs), _stream(stream)))
        return (H, Hs) if secondary else H

    def free(self):
        if self.handle:
            lib().petgem_free_solution(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class System:
    """An assembled system on the current GPU (petgem_assemble)."""

    def __init__(self, xyz: np.ndarray, tets: np.ndarray, sigma: np.ndarray, sigma_bg: float,
                 stream=None):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        tets = np.ascontiguousarray(tets, dtype=np.int32)
        sigma = np.ascontiguousarray(sigma, dtype=np.float64)
        m = Mesh(len(xyz), len(tets), xyz.ctypes.data_as(C.POINTER(C.c_double)),
                 tets.ctypes.data_as(C.POINTER(C.c_int32)))
        h = C.c_void_p()
        _check(lib().petgem_assemble(C.byref(m), sigma.ctypes.data_as(C.POINTER(C.c_double)),
                                     sigma_bg, _stream(stream), C.byref(h)))
        self.handle = h
        self.n_dof = lib().petgem_num_dofs(h)
        self.nnz = lib().petgem_nnz(h)
        self.n_tets = len(tets)
        self.sigma_bg = sigma_bg
        self.setup_seconds = lib().petgem_setup_seconds(h)

    @classmethod
    def from_model(cls, model, stream=None):
        S = cls(model.xyz, model.tets, model.sigma, model.sigma_bg, stream)
        layers = getattr(model, "layers", None)
        if layers is not None:
            S.set_background(layers)
        return S

    def set_background(self, layers=None):
        """The primary field's background: None = the whole space sigma_bg,
        or (z0, sigma_above, sigma_below) = two half-spaces."""
        bg = Background(0, 0.0, 1.0, 1.0) if layers is None else Background(1, *map(float, layers))
        _check(lib().petgem_set_background(self.handle, C.byref(bg)))

    def reassemble(self, sigma_dev, sigma_bg: float, stream=None):
        _check(lib().petgem_reassemble(self.handle, _ptr(sigma_dev), sigma_bg, _stream(stream)))
        self.sigma_bg = sigma_bg

    def rhs(self, dipoles, stream=None):
        import torch
        src = make_sources(dipoles)
        b = torch.empty((len(dipoles), self.n_dof), dtype=torch.complex128, device="cuda")
        _check(lib().petgem_rhs(self.handle, src, len(dipoles), _ptr(b), _stream(stream)))
        return b

    def rhs_noalloc(self, dipoles, b=None, stream=None):
        """petgem_rhs_noalloc: the right-hand sides without any device
        allocation inside the library (b: an optional caller tensor
        complex128 [n_src][n_dof])."""
        import torch
        src = make_sources(dipoles)
        if b is None:
            b = torch.empty((len(dipoles), self.n_dof), dtype=torch.complex128, device="cuda")
        _check(lib().petgem_rhs_noalloc(self.handle, src, len(dipoles), _ptr(b), _stream(stream)))
        return b

    def solve(self, dipoles, opts: Optional[Opts] = None, x0=None, stream=None,
              solution: Optional[Solution] = None, allow_not_converged: bool = False):
        """Returns (Solution, [stats dict per source], return code)."""
        src = make_sources(dipoles)
        st = (Stats * len(dipoles))()
        h = C.c_void_p(solution.handle.value if solution is not None else None)
        o = opts if opts is not None else default_opts()
        allow = (NOT_CONVERGED, NONFINITE) if allow_not_converged else ()
        rc = _check(lib().petgem_solve(self.handle, src, len(dipoles), C.byref(o), _ptr(x0),
                                       _stream(stream), C.byref(h), st), allow)
        sol = solution if solution is not None else Solution(self, h, len(dipoles))
        return sol, [s.as_dict() for s in st], rc

    def csr(self):
        """Host copies (row_ptr, col, K, Ms) of the assembled matrices."""
        n, nnz = self.n_dof, self.nnz
        rp = np.empty(n + 1, np.int32)
        col = np.empty(nnz, np.int32)
        K = np.empty(nnz, np.float64)
        Ms = np.empty(nnz, np.float64)
        _check(lib().petgem_get_csr(self.handle, rp.ctypes.data_as(C.POINTER(C.c_int32)),
                                    col.ctypes.data_as(C.POINTER(C.c_int32)),
                                    K.ctypes.data_as(C.POINTER(C.c_double)),
                                    Ms.ctypes.data_as(C.POINTER(C.c_double)), _stream()))
        return rp, col, K, Ms

    def dof_edges(self) -> np.ndarray:
        out = np.empty((self.n_dof, 2), np.int32)
        _check(lib().petgem_get_dof_edges(self.handle, out.ctypes.data_as(C.POINTER(C.c_int32))))
        return out

    def spmv(self, freq: float, x, stream=None):
        import torch
        y = torch.empty_like(x)
        _check(lib().petgem_spmv(self.handle, freq, _ptr(x), _ptr(y), _stream(stream)))
        return y

    def ssor_colors(self, stream=None) -> np.ndarray:
        """Colour of every DOF of the multicolour SSOR (library DOF order)."""
        out = np.empty(self.n_dof, np.int32)
        _check_count(lib().petgem_ssor_colors(self.handle, out.ctypes.data_as(C.POINTER(C.c_int32)),
                                              _stream(stream)))
        return out

    def ssor_apply(self, freq: float, omega: float, r, stream=None):
        """z = M^-1 r of the multicolour SSOR for one complex64 CUDA vector."""
        import torch
        z = torch.empty_like(r)
        _check(lib().petgem_ssor_apply(self.handle, freq, omega, _ptr(r), _ptr(z), _stream(stream)))
        return z

    def tuning(self) -> dict:
        g = C.c_int32()
        ms = (C.c_float * 3)()
        _check(lib().petgem_tuning(self.handle, C.byref(g), ms))
        return {"spmv_group": g.value, "spmv_ms_g4_g8_g16": [round(v, 5) for v in ms]}

    def free(self):
        if self.handle:
            lib().petgem_free_system(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


NET_SIDE = 32
NET_VOX = NET_SIDE ** 3
NET_IN, NET_OUT, NET_OUT_USED = 16, 16, 6
NET_LAYERS = ((16, 16), (16, 32), (32, 64), (64, 64), (96, 32), (48, 16), (16, 16))


class Net:
    """The learned-initial-guess network (petgem_net_*). Tensors are CUDA
    tensors: inputs bfloat16 [B][32^3][16], outputs float32 [B][32^3][16],
    targets float32 [B][32^3][6]."""

    def __init__(self, batch_max: int = 16, seed: int = 0):
        h = C.c_void_p()
        _check(lib().petgem_net_create(batch_max, seed, C.byref(h)))
        self.handle = h
        self.batch_max = batch_max
        self.n_params = lib().petgem_net_num_params(h)

    def params(self) -> np.ndarray:
        out = np.empty(self.n_params, np.float32)
        _check(lib().petgem_net_get_params(self.handle, out.ctypes.data_as(C.POINTER(C.c_float))))
        return out

    def set_params(self, p: np.ndarray):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == self.n_params
        _check(lib().petgem_net_set_params(self.handle, p.ctypes.data_as(C.POINTER(C.c_float))))

    def forward(self, x, stream=None):
        import torch
        y = torch.empty((x.shape[0], NET_VOX, NET_OUT), dtype=torch.float32, device="cuda")
        _check(lib().petgem_net_forward(self.handle, _ptr(x), x.shape[0], _ptr(y), _stream(stream)))
        return y

    def loss_grad(self, x, t, stream=None):
        loss = C.c_double()
        g = np.empty(self.n_params, np.float32)
        _check(lib().petgem_net_loss_grad(self.handle, _ptr(x), _ptr(t), x.shape[0], _stream(stream),
                                          C.byref(loss), g.ctypes.data_as(C.POINTER(C.c_float))))
        return loss.value, g

    def train_step(self, x, t, lr: float, stream=None) -> float:
        loss = C.c_double()
        _check(lib().petgem_net_train_step(self.handle, _ptr(x), _ptr(t), x.shape[0], lr,
                                           _stream(stream), C.byref(loss)))
        return loss.value

    def free(self):
        if self.handle:
            lib().petgem_net_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def voxelize(system: "System", dipoles, sigma_dev=None, stream=None):
    import torch
    src = make_sources(dipoles)
    x = torch.empty((len(dipoles), NET_VOX, NET_IN), dtype=torch.bfloat16, device="cuda")
    _check(lib().petgem_voxelize(system.handle, _ptr(sigma_dev), src, len(dipoles), _ptr(x),
                                 _stream(stream)))
    return x


def vox_targets(solution: "Solution", scale, stream=None):
    import torch
    sc = np.ascontiguousarray(scale, dtype=np.float64)
    t = torch.empty((solution.n_src, NET_VOX, NET_OUT_USED), dtype=torch.float32, device="cuda")
    _check(lib().petgem_vox_targets(solution.handle, sc.ctypes.data_as(C.POINTER(C.c_double)),
                                    _ptr(t), _stream(stream)))
    return t


def learned_x0(system: "System", net: Net, dipoles, g: float, stream=None):
    """(x0 complex128 CUDA tensor [B][n_dof], |b| per source)."""
    import torch
    src = make_sources(dipoles)
    x0 = torch.empty((len(dipoles), system.n_dof), dtype=torch.complex128, device="cuda")
    bn = np.empty(len(dipoles), np.float64)
    _check(lib().petgem_learned_x0(system.handle, net.handle, src, len(dipoles), g, _ptr(x0),
                                   bn.ctypes.data_as(C.POINTER(C.c_double)), _stream(stream)))
    return x0, bn


def learned_x0_many(systems, net: Net, dipoles, g: float, stream=None):
    """One guess per system (dipoles[k] on systems[k]) from one network batch:
    ([x0 complex128 CUDA tensor [n_dof_k]], |b| per system)."""
    import torch
    n = len(systems)
    if len(dipoles) != n:
        raise ValueError("one dipole per system")
    src = make_sources(dipoles)
    x0 = [torch.empty(S.n_dof, dtype=torch.complex128, device="cuda") for S in systems]
    hs = (C.c_void_p * n)(*[S.handle.value for S in systems])
    ps = (C.c_void_p * n)(*[_ptr(t).value for t in x0])
    bn = np.empty(n, np.float64)
    _check(lib().petgem_learned_x0_many(hs, net.handle, src, n, g, ps,
                                        bn.ctypes.data_as(C.POINTER(C.c_double)), _stream(stream)))
    return x0, bn


def _mesh(xyz, tets):
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    tets = np.ascontiguousarray(tets, dtype=np.int32)
    return Mesh(len(xyz), len(tets), xyz.ctypes.data_as(C.POINTER(C.c_double)),
                tets.ctypes.data_as(C.POINTER(C.c_int32))), (xyz, tets)


def mesh_pattern(xyz, tets):
    """Host-only: (dof_edges [n][2], row_ptr, col) of the library's numbering."""
    m, keep = _mesh(xyz, tets)
    n = C.c_int32()
    nnz = C.c_int64()
    _check(lib().petgem_mesh_pattern(C.byref(m), C.byref(n), C.byref(nnz), None, None, None))
    de = np.empty((n.value, 2), np.int32)
    rp = np.empty(n.value + 1, np.int32)
    col = np.empty(nnz.value, np.int32)
    P = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))
    _check(lib().petgem_mesh_pattern(C.byref(m), C.byref(n), C.byref(nnz), P(de), P(rp), P(col)))
    return de, rp, col


def sync_probe(rounds: int, mode: int, stream=None):
    """(us per round, blocks) of a graph-replayed kernel boundary (mode 0)
    or a grid barrier in one cooperative kernel (mode 1)."""
    b = C.c_int32()
    us = C.c_float()
    _check(lib().petgem_sync_probe(rounds, mode, C.byref(b), C.byref(us), _stream(stream)))
    return us.value, b.value


def spmm_candidates(n_cols: int, sliced: bool) -> List[int]:
    """The complex64 SpMM shapes the autotuner times for n_cols columns
    (``spmm_shape`` codes); host only."""
    L = lib()
    n = _check_count(L.petgem_spmm_candidates(n_cols, int(sliced), None, 0))
    out = (C.c_int32 * max(n, 1))()
    _check_count(L.petgem_spmm_candidates(n_cols, int(sliced), out, n))
    return list(out[:n])


def _check_count(n: int) -> int:
    if n < 0:
        raise PetgemError(n, lib().petgem_last_error().decode())
    return n


def locate(xyz, tets, pts, tol=1e-12):
    """Host-only point location (lowest containing element id, -1 outside)."""
    m, keep = _mesh(xyz, tets)
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    out = np.empty(len(pts), np.int32)
    _check(lib().petgem_locate(C.byref(m), pts.ctypes.data_as(C.POINTER(C.c_double)), len(pts),
                               tol, out.ctypes.data_as(C.POINTER(C.c_int32))))
    return out


def solve_many(systems: Sequence[System], dipoles, opts: Optional[Opts] = None, stream=None,
               allow_not_converged: bool = False, x0=None):
    """One source per system, all systems in shared launches (petgem_solve_many).
    x0: None, or one complex128 CUDA tensor [n_dof] (or None) per system."""
    n = len(systems)
    hs = (C.c_void_p * n)(*[s.handle.value for s in systems])
    src = make_sources(dipoles)
    sols = (C.c_void_p * n)()
    st = (Stats * n)()
    o = opts if opts is not None else default_opts(method=COCG, precision=MIXED)
    allow = (NOT_CONVERGED, NONFINITE) if allow_not_converged else ()
    x0p = None
    if x0 is not None:
        if len(x0) != n:
            raise ValueError("one initial guess (or None) per system")
        for k, t in enumerate(x0):
            if t is not None and (t.numel() != systems[k].n_dof or not t.is_cuda):
                raise ValueError(f"initial guess {k}: a CUDA tensor of {systems[k].n_dof} values")
        x0p = (C.c_void_p * n)(*[None if t is None else _ptr(t).value for t in x0])
    rc = _check(lib().petgem_solve_many(hs, src, n, C.byref(o), x0p, _stream(stream), sols, st), allow)
    out = [Solution(systems[k], C.c_void_p(sols[k]), 1) for k in range(n)]
    return out, [s.as_dict() for s in st], rc
