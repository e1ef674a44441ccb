"""Python binding of libp2m: the C-ABI calls under the same names, on torch
device tensors.  Argument marshalling only -- every step runs in the HIP
library; nothing here computes on the host.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional, Tuple

import torch

from . import _lib
from ._lib import (P2M_BF16, P2M_DETERMINISTIC, P2M_F32, P2M_F64, P2M_LINEAR, P2M_PERIODIC, P2M_STRICT, P2M_WEIGHTS_F32, MAX_SUPPORT, P2MDiag, P2MError,
                   P2MMesh, check, load)

__all__ = [
    "Mesh",
    "Weights",
    "p2m_build_weights",
    "p2m_project",
    "m2p_interpolate",
    "m2p_interpolate_backward",
    "m2p_interpolate_backward_binned",
    "p2m_project_backward",
    "p2m_build_weights_backward",
    "p2m_set_option",
    "p2m_get_option",
    "p2m_project_fused",
    "p2m_backward_fused",
    "p2m_project_fused_noalloc",
    "Batch",
    "p2m_build_weights_batched",
    "m2p_interpolate_batched",
    "m2p_interpolate_backward_batched",
    "P2MError",
    "P2M_WEIGHTS_F32",
    "P2M_STRICT",
    "P2M_LINEAR",
    "P2M_PERIODIC",
    "P2M_DETERMINISTIC",
    "p2m_advect",
    "MeshQCSF",
    "kinematic_step",
]


@dataclass(frozen=True)
class Mesh:
    """Uniform fixed mesh: nodes (x0 + i*H, y0 + j*H), 0<=i<=nx, 0<=j<=ny."""

    nx: int
    ny: int
    H: float
    x0: float = 0.0
    y0: float = 0.0

    @property
    def n_nodes(self) -> int:
        return (self.nx + 1) * (self.ny + 1)

    def c(self) -> P2MMesh:
        return P2MMesh(int(self.nx), int(self.ny), float(self.H), float(self.x0), float(self.y0))

    @classmethod
    def of(cls, m) -> "Mesh":
        return m if isinstance(m, Mesh) else cls(int(m.nx), int(m.ny), float(m.H), float(m.x0), float(m.y0))


def _stream(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> ctypes.c_void_p:
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _need(t: torch.Tensor, name: str, dtype=None, shape=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


def _dtype_code(particle_dtype: torch.dtype) -> int:
    if particle_dtype == torch.float64:
        return P2M_F64
    if particle_dtype == torch.float32:
        return P2M_F32
    if particle_dtype == torch.bfloat16:
        return P2M_BF16
    raise ValueError(f"unsupported value dtype {particle_dtype}")


def _mesh_dtype(code: int) -> torch.dtype:
    return torch.float64 if code == P2M_F64 else torch.float32


class Weights:
    """Owner of a p2m_weights handle (the P2M operator of one particle set)."""

    def __init__(self):
        self._h = ctypes.c_void_p(0)
        self.mesh: Optional[Mesh] = None   # None for a batched handle
        self.n_nodes = 0
        self.N = 0
        self.flags = 0
        self.device = None

    @property
    def handle(self) -> ctypes.c_void_p:
        if not self._h.value:
            raise ValueError("weights were never built")
        return self._h

    def diag(self, check_status: bool = True) -> dict:
        d = P2MDiag()
        st = ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
        rc = load().p2m_weights_diag(self.handle, ctypes.byref(d), st)
        if check_status:
            check(rc)
        return d.as_dict()

    def export(self):
        """ELL weights as CPU tensors: idx [K, n_nodes], w [K, n_nodes], cnt, tri [n_nodes, 3]."""
        dev = self.device
        nn = self.n_nodes
        idx = torch.empty((MAX_SUPPORT, nn), dtype=torch.int32, device=dev)
        w = torch.empty((MAX_SUPPORT, nn), dtype=torch.float64, device=dev)
        cnt = torch.empty((nn,), dtype=torch.int32, device=dev)
        tri = torch.empty((nn, 3), dtype=torch.int32, device=dev)
        check(load().p2m_weights_export(self.handle, _ptr(idx), _ptr(w), _ptr(cnt), _ptr(tri), _stream(idx)))
        torch.cuda.synchronize(dev)
        return idx.cpu(), w.cpu(), cnt.cpu(), tri.cpu()

    def close(self):
        if self._h.value:
            load().p2m_weights_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def p2m_set_option(name: str, value: float):
    check(load().p2m_set_option(name.encode(), float(value)))


def p2m_get_option(name: str) -> float:
    out = ctypes.c_double()
    check(load().p2m_get_option(name.encode(), ctypes.byref(out)))
    return out.value


def p2m_build_weights(mesh, h: float, pos: torch.Tensor, flags: int = 0,
                      weights: Optional[Weights] = None, check_diag: bool = True) -> Weights:
    """Build psi_mu(r_i) for all mesh nodes (C call of the same name).

    ``weights`` reuses an existing handle (no allocation when it is large
    enough).  ``check_diag`` synchronises and raises on data errors.
    """
    mesh = Mesh.of(mesh)
    _need(pos, "pos", torch.float64)
    if pos.dim() != 2 or pos.shape[1] != 2:
        raise ValueError("pos must have shape [N, 2]")
    w = weights if weights is not None else Weights()
    lib = load()
    cm = mesh.c()
    with torch.cuda.device(pos.device):
        rc = lib.p2m_build_weights(ctypes.byref(cm), float(h), _ptr(pos), pos.shape[0], int(flags),
                                   ctypes.byref(w._h), _stream(pos))
    check(rc)
    w.mesh, w.n_nodes, w.N, w.flags, w.device = mesh, mesh.n_nodes, pos.shape[0], int(flags), pos.device
    if check_diag:
        w.diag(check_status=True)
    return w


def p2m_project(w: Weights, vals: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Eq. (p2m): mesh values [n_nodes, C] from particle values [N, C]."""
    _need(vals, "vals")
    if vals.dim() != 2 or vals.shape[0] != w.N:
        raise ValueError(f"vals must have shape [{w.N}, C]")
    code = _dtype_code(vals.dtype)
    C = vals.shape[1]
    if out is None:
        out = torch.empty((w.n_nodes, C), dtype=_mesh_dtype(code), device=vals.device)
    _need(out, "out", _mesh_dtype(code), (w.n_nodes, C))
    with torch.cuda.device(vals.device):
        check(load().p2m_project(w.handle, _ptr(vals), C, code, _ptr(out), _stream(vals)))
    return out


class MeshQCSF:
    """Owner of a p2m_mesh_qcsf handle: the edge coefficients of one mesh's
    quadratically consistent functions, computed once on ``device``
    (``periodic``: in the periodic box, p2m_mesh_qcsf_create_periodic)."""

    def __init__(self, mesh, device="cuda:0", periodic: bool = False):
        self.mesh = Mesh.of(mesh)
        self.device = torch.device(device)
        self.periodic = bool(periodic)
        self._h = ctypes.c_void_p(0)
        cm = self.mesh.c()
        with torch.cuda.device(self.device):
            st = ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
            fn = load().p2m_mesh_qcsf_create_periodic if periodic else load().p2m_mesh_qcsf_create
            check(fn(ctypes.byref(cm), ctypes.byref(self._h), st))

    def __del__(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            try:
                load().p2m_mesh_qcsf_destroy(self._h)
            except Exception:  # noqa: BLE001 - interpreter shutdown
                pass
            self._h = ctypes.c_void_p(0)

    def interpolate(self, mesh_vals: torch.Tensor, pos: torch.Tensor, out: Optional[torch.Tensor] = None,
                    bf16_out: bool = False) -> torch.Tensor:
        """Eq. (m2p) with the mesh's quadratically consistent functions (C call
        m2p_interpolate_qcsf): particle values [N, C]."""
        mesh = self.mesh
        _need(mesh_vals, "mesh_vals")
        _need(pos, "pos", torch.float64)
        if mesh_vals.dim() != 2 or mesh_vals.shape[0] != mesh.n_nodes:
            raise ValueError(f"mesh_vals must have shape [{mesh.n_nodes}, C]")
        C = mesh_vals.shape[1]
        if mesh_vals.dtype == torch.float64:
            code, odt = P2M_F64, torch.float64
        elif mesh_vals.dtype == torch.float32:
            code, odt = (P2M_BF16, torch.bfloat16) if bf16_out else (P2M_F32, torch.float32)
        else:
            raise ValueError("mesh_vals must be float64 or float32")
        N = pos.shape[0]
        if out is None:
            out = torch.empty((N, C), dtype=odt, device=pos.device)
        _need(out, "out", odt, (N, C))
        with torch.cuda.device(pos.device):
            check(load().m2p_interpolate_qcsf(self._h, _ptr(mesh_vals), C, code, _ptr(pos), N, _ptr(out),
                                              _stream(pos)))
        return out


def p2m_advect(mesh, pos: torch.Tensor, amp: float, dt: float, periodic: bool = False) -> torch.Tensor:
    """One midpoint step of the particles in the cellular flow of the mesh box
    (C call of the same name; ``periodic``: p2m_advect_periodic, the periodic
    flow with positions wrapped into the box); ``pos`` is updated in place
    and returned."""
    mesh = Mesh.of(mesh)
    _need(pos, "pos", torch.float64)
    if pos.dim() != 2 or pos.shape[1] != 2:
        raise ValueError("pos must have shape [N, 2]")
    cm = mesh.c()
    with torch.cuda.device(pos.device):
        fn = load().p2m_advect_periodic if periodic else load().p2m_advect
        check(fn(ctypes.byref(cm), _ptr(pos), pos.shape[0], float(amp), float(dt), _stream(pos)))
    return pos


def kinematic_step(mesh, h: float, pos: torch.Tensor, mesh_vals: torch.Tensor, amp: float, dt: float,
                   flags: int = 0, weights: Optional[Weights] = None) -> Tuple[torch.Tensor, Weights]:
    """One step of the kinematic projection loop, every step on the GPU:
    particle values from the mesh (M2P), the particles moved one step
    (p2m_advect), their functions rebuilt, and projected back (P2M).
    ``pos`` is updated in place; returns (new mesh values, weights).  With
    P2M_PERIODIC in ``flags`` the particles move in the periodic flow."""
    vals = m2p_interpolate(mesh, mesh_vals, pos)
    p2m_advect(mesh, pos, amp, dt, periodic=bool(flags & P2M_PERIODIC))
    w = p2m_build_weights(mesh, h, pos, flags, weights=weights, check_diag=False)
    return p2m_project(w, vals), w


def m2p_interpolate(mesh, mesh_vals: torch.Tensor, pos: torch.Tensor, out: Optional[torch.Tensor] = None,
                    bf16_out: bool = False) -> torch.Tensor:
    """Eq. (m2p) with linear FE mesh functions: particle values [N, C]."""
    mesh = Mesh.of(mesh)
    _need(mesh_vals, "mesh_vals")
    _need(pos, "pos", torch.float64)
    if mesh_vals.dim() != 2 or mesh_vals.shape[0] != mesh.n_nodes:
        raise ValueError(f"mesh_vals must have shape [{mesh.n_nodes}, C]")
    C = mesh_vals.shape[1]
    if mesh_vals.dtype == torch.float64:
        code, odt = P2M_F64, torch.float64
    elif mesh_vals.dtype == torch.float32:
        code, odt = (P2M_BF16, torch.bfloat16) if bf16_out else (P2M_F32, torch.float32)
    else:
        raise ValueError("mesh_vals must be float64 or float32")
    N = pos.shape[0]
    if out is None:
        out = torch.empty((N, C), dtype=odt, device=pos.device)
    _need(out, "out", odt, (N, C))
    cm = mesh.c()
    with torch.cuda.device(pos.device):
        check(load().m2p_interpolate(ctypes.byref(cm), _ptr(mesh_vals), C, code, _ptr(pos), N, _ptr(out),
                                     _stream(pos)))
    return out


def m2p_interpolate_backward(mesh, mesh_vals: Optional[torch.Tensor], pos: torch.Tensor, grad_vals: torch.Tensor,
                             want_mesh: bool = True, grad_pos: Optional[torch.Tensor] = None):
    """Adjoint of m2p_interpolate: (grad_mesh or None, grad_pos or None).

    grad_pos, when given, is accumulated into (+=)."""
    mesh = Mesh.of(mesh)
    _need(pos, "pos", torch.float64)
    _need(grad_vals, "grad_vals")
    C = grad_vals.shape[1]
    code = P2M_F64 if grad_vals.dtype == torch.float64 else P2M_F32
    mdt = _mesh_dtype(code)
    gm = torch.empty((mesh.n_nodes, C), dtype=mdt, device=pos.device) if want_mesh else None
    if grad_pos is not None:
        _need(grad_pos, "grad_pos", torch.float64, tuple(pos.shape))
        _need(mesh_vals, "mesh_vals", mdt, (mesh.n_nodes, C))
    cm = mesh.c()
    with torch.cuda.device(pos.device):
        check(load().m2p_interpolate_backward(ctypes.byref(cm), _ptr(mesh_vals), C, code, _ptr(pos), pos.shape[0],
                                              _ptr(grad_vals), _ptr(gm), _ptr(grad_pos), _stream(pos)))
    return gm, grad_pos


def m2p_interpolate_backward_binned(w: Weights, mesh_vals: Optional[torch.Tensor], pos: torch.Tensor,
                                    grad_vals: torch.Tensor, want_mesh: bool = True,
                                    grad_pos: Optional[torch.Tensor] = None, grad_mesh: Optional[torch.Tensor] = None):
    """Adjoint of m2p_interpolate at the particles ``w`` was built from
    (``pos``), grad_mesh gathered per node through w's binning (no atomics):
    (grad_mesh or None, grad_pos or None); grad_pos, when given, is
    accumulated into."""
    _need(pos, "pos", torch.float64, (w.N, 2))
    _need(grad_vals, "grad_vals")
    C = grad_vals.shape[1]
    code = P2M_F64 if grad_vals.dtype == torch.float64 else P2M_F32
    mdt = _mesh_dtype(code)
    gm = grad_mesh
    if want_mesh and gm is None:
        gm = torch.empty((w.n_nodes, C), dtype=mdt, device=pos.device)
    if gm is not None:
        _need(gm, "grad_mesh", mdt, (w.n_nodes, C))
    if grad_pos is not None:
        _need(grad_pos, "grad_pos", torch.float64, tuple(pos.shape))
        _need(mesh_vals, "mesh_vals", mdt, (w.n_nodes, C))
    with torch.cuda.device(pos.device):
        check(load().m2p_interpolate_backward_binned(w.handle, _ptr(mesh_vals), C, code, _ptr(pos), _ptr(grad_vals),
                                                     _ptr(gm), _ptr(grad_pos), _stream(pos)))
    return gm, grad_pos


def p2m_project_backward(w: Weights, grad_mesh: torch.Tensor, vals: Optional[torch.Tensor] = None,
                         want_vals: bool = True, want_w: bool = False):
    """Adjoint of p2m_project for fixed weights: (grad_vals or None, grad_w or None).

    grad_w has the ELL layout [MAX_SUPPORT, n_nodes] (FP64)."""
    _need(grad_mesh, "grad_mesh")
    C = grad_mesh.shape[1]
    if vals is not None:
        code = _dtype_code(vals.dtype)
    else:
        code = P2M_F64 if grad_mesh.dtype == torch.float64 else P2M_F32
    gdt = _mesh_dtype(code)
    _need(grad_mesh, "grad_mesh", gdt, (w.n_nodes, C))
    gv = torch.empty((w.N, C), dtype=gdt, device=grad_mesh.device) if want_vals else None
    gw = torch.empty((MAX_SUPPORT, w.n_nodes), dtype=torch.float64, device=grad_mesh.device) if want_w else None
    if want_w:
        if vals is None:
            raise ValueError("vals are needed for grad_w")
        _need(vals, "vals", None, (w.N, C))
    with torch.cuda.device(grad_mesh.device):
        check(load().p2m_project_backward(w.handle, _ptr(grad_mesh), C, code, _ptr(vals), _ptr(gv), _ptr(gw),
                                          _stream(grad_mesh)))
    return gv, gw


def p2m_build_weights_backward(w: Weights, pos: torch.Tensor, grad_w: torch.Tensor,
                               grad_pos: Optional[torch.Tensor] = None) -> torch.Tensor:
    """d L / d pos through the weights (accumulates into grad_pos)."""
    _need(pos, "pos", torch.float64, (w.N, 2))
    _need(grad_w, "grad_w", torch.float64, (MAX_SUPPORT, w.n_nodes))
    if grad_pos is None:
        grad_pos = torch.zeros_like(pos)
    _need(grad_pos, "grad_pos", torch.float64, (w.N, 2))
    with torch.cuda.device(pos.device):
        check(load().p2m_build_weights_backward(w.handle, _ptr(pos), _ptr(grad_w), _ptr(grad_pos), _stream(pos)))
    return grad_pos


def fused_diag() -> dict:
    """Diagnostics of the last recompute build on the current device."""
    h = load().p2m_fused_handle()
    if not h:
        raise ValueError("no recompute build on this device yet")
    d = P2MDiag()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    load().p2m_weights_diag(ctypes.c_void_p(h), ctypes.byref(d), st)
    return d.as_dict()


def p2m_project_fused(mesh, h: float, pos: torch.Tensor, vals: torch.Tensor,
                      out: Optional[torch.Tensor] = None, check_diag: bool = False) -> torch.Tensor:
    """Eq. (p2m) with the weights rebuilt inside the call (no handle kept).
    ``check_diag`` synchronises and raises on data errors of that build."""
    mesh = Mesh.of(mesh)
    _need(pos, "pos", torch.float64)
    _need(vals, "vals")
    if vals.dim() != 2 or vals.shape[0] != pos.shape[0]:
        raise ValueError(f"vals must have shape [{pos.shape[0]}, C]")
    code = _dtype_code(vals.dtype)
    C = vals.shape[1]
    if out is None:
        out = torch.empty((mesh.n_nodes, C), dtype=_mesh_dtype(code), device=vals.device)
    _need(out, "out", _mesh_dtype(code), (mesh.n_nodes, C))
    cm = mesh.c()
    with torch.cuda.device(pos.device):
        check(load().p2m_project_fused(ctypes.byref(cm), float(h), _ptr(pos), pos.shape[0], _ptr(vals), C, code,
                                       _ptr(out), _stream(pos)))
        if check_diag:
            d = fused_diag()
            if d["status"] != 0:
                check(d["status"])
    return out


def p2m_project_fused_noalloc(mesh, h: float, pos: torch.Tensor, vals: torch.Tensor,
                              out: torch.Tensor) -> torch.Tensor:
    """p2m_project_fused in the library's static per-device workspace: the
    call allocates no device memory (the caller passes ``out``)."""
    mesh = Mesh.of(mesh)
    _need(pos, "pos", torch.float64)
    _need(vals, "vals")
    if vals.dim() != 2 or vals.shape[0] != pos.shape[0]:
        raise ValueError(f"vals must have shape [{pos.shape[0]}, C]")
    code = _dtype_code(vals.dtype)
    C = vals.shape[1]
    _need(out, "out", _mesh_dtype(code), (mesh.n_nodes, C))
    cm = mesh.c()
    with torch.cuda.device(pos.device):
        check(load().p2m_project_fused_noalloc(ctypes.byref(cm), float(h), _ptr(pos), pos.shape[0], _ptr(vals), C,
                                               code, _ptr(out), _stream(pos)))
    return out


def p2m_backward_fused(mesh, h: float, pos: torch.Tensor, vals: torch.Tensor, grad_mesh: torch.Tensor,
                       want_vals: bool = True, grad_pos: Optional[torch.Tensor] = None):
    """Adjoint of p2m_project_fused (weights rebuilt from pos): (grad_vals or
    None, grad_pos or None); grad_pos, when given, is accumulated into."""
    mesh = Mesh.of(mesh)
    _need(pos, "pos", torch.float64)
    _need(vals, "vals", None, (pos.shape[0], grad_mesh.shape[1]))
    code = _dtype_code(vals.dtype)
    gdt = _mesh_dtype(code)
    C = grad_mesh.shape[1]
    _need(grad_mesh, "grad_mesh", gdt, (mesh.n_nodes, C))
    gv = torch.empty((pos.shape[0], C), dtype=gdt, device=pos.device) if want_vals else None
    if grad_pos is not None:
        _need(grad_pos, "grad_pos", torch.float64, tuple(pos.shape))
    cm = mesh.c()
    with torch.cuda.device(pos.device):
        check(load().p2m_backward_fused(ctypes.byref(cm), float(h), _ptr(pos), pos.shape[0], _ptr(vals), C, code,
                                        _ptr(grad_mesh), _ptr(gv), _ptr(grad_pos), _stream(pos)))
    return gv, grad_pos


class Batch:
    """Owner of a p2m_batch handle: S particle sets, each with its own mesh
    and spacing h; set s owns particles offsets[s]:offsets[s+1] and mesh
    nodes node_offsets[s]:node_offsets[s+1] of the concatenated arrays."""

    def __init__(self, meshes, hs, offsets):
        meshes = [Mesh.of(m) for m in meshes]
        S = len(meshes)
        if len(hs) != S or len(offsets) != S + 1:
            raise ValueError("need S meshes, S spacings and S+1 offsets")
        cm = (P2MMesh * S)(*[m.c() for m in meshes])
        ch = (ctypes.c_double * S)(*[float(h) for h in hs])
        co = (ctypes.c_int64 * (S + 1))(*[int(o) for o in offsets])
        self._h = ctypes.c_void_p(0)
        check(load().p2m_batch_create(cm, ch, S, co, ctypes.byref(self._h)))
        nn, npart = ctypes.c_int64(), ctypes.c_int64()
        no = (ctypes.c_int64 * (S + 1))()
        check(load().p2m_batch_shape(self._h, ctypes.byref(nn), ctypes.byref(npart), no))
        self.meshes = meshes
        self.hs = [float(h) for h in hs]
        self.offsets = [int(o) for o in offsets]
        self.node_offsets = [int(v) for v in no]
        self.S = S
        self.n_nodes = int(nn.value)
        self.N = int(npart.value)

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    def close(self):
        if self._h.value:
            load().p2m_batch_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def p2m_build_weights_batched(b: Batch, pos: torch.Tensor, flags: int = 0, weights: Optional[Weights] = None,
                              check_diag: bool = True) -> Weights:
    """Weights of every set of a batch in one pass (C call of the same name)."""
    _need(pos, "pos", torch.float64, (b.N, 2))
    w = weights if weights is not None else Weights()
    with torch.cuda.device(pos.device):
        rc = load().p2m_build_weights_batched(b.handle, _ptr(pos), int(flags), ctypes.byref(w._h), _stream(pos))
    check(rc)
    w.mesh, w.n_nodes, w.N, w.flags, w.device = None, b.n_nodes, b.N, int(flags), pos.device
    if check_diag:
        w.diag(check_status=True)
    return w


def m2p_interpolate_batched(b: Batch, mesh_vals: torch.Tensor, pos: torch.Tensor,
                            out: Optional[torch.Tensor] = None, bf16_out: bool = False) -> torch.Tensor:
    """m2p_interpolate over every set of a batch in one launch."""
    _need(mesh_vals, "mesh_vals")
    _need(pos, "pos", torch.float64, (b.N, 2))
    if mesh_vals.dim() != 2 or mesh_vals.shape[0] != b.n_nodes:
        raise ValueError(f"mesh_vals must have shape [{b.n_nodes}, C]")
    C = mesh_vals.shape[1]
    if mesh_vals.dtype == torch.float64:
        code, odt = P2M_F64, torch.float64
    elif mesh_vals.dtype == torch.float32:
        code, odt = (P2M_BF16, torch.bfloat16) if bf16_out else (P2M_F32, torch.float32)
    else:
        raise ValueError("mesh_vals must be float64 or float32")
    if out is None:
        out = torch.empty((b.N, C), dtype=odt, device=pos.device)
    _need(out, "out", odt, (b.N, C))
    with torch.cuda.device(pos.device):
        check(load().m2p_interpolate_batched(b.handle, _ptr(mesh_vals), C, code, _ptr(pos), _ptr(out),
                                             _stream(pos)))
    return out


def m2p_interpolate_backward_batched(b: Batch, mesh_vals: Optional[torch.Tensor], pos: torch.Tensor,
                                     grad_vals: torch.Tensor, want_mesh: bool = True,
                                     grad_pos: Optional[torch.Tensor] = None):
    """Adjoint of m2p_interpolate_batched: (grad_mesh or None, grad_pos or None)."""
    _need(pos, "pos", torch.float64, (b.N, 2))
    _need(grad_vals, "grad_vals")
    C = grad_vals.shape[1]
    code = P2M_F64 if grad_vals.dtype == torch.float64 else P2M_F32
    mdt = _mesh_dtype(code)
    gm = torch.empty((b.n_nodes, C), dtype=mdt, device=pos.device) if want_mesh else None
    if grad_pos is not None:
        _need(grad_pos, "grad_pos", torch.float64, tuple(pos.shape))
        _need(mesh_vals, "mesh_vals", mdt, (b.n_nodes, C))
    with torch.cuda.device(pos.device):
        check(load().m2p_interpolate_backward_batched(b.handle, _ptr(mesh_vals), C, code, _ptr(pos),
                                                      _ptr(grad_vals), _ptr(gm), _ptr(grad_pos), _stream(pos)))
    return gm, grad_pos
