"""Python binding of liblsdf.so (ctypes).  Argument marshalling only: every
step of the computation runs in the library's HIP kernels; PyTorch provides
device memory and streams.  Names follow the C ABI (include/lsdf.h) without
the ``lsdf_`` prefix.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblsdf.so")

LSDF_OK = 0
LSDF_E_INVALID_ARG = -1
LSDF_E_SHAPE = -2
LSDF_E_UNSUPPORTED = -3
LSDF_E_DEVICE = -4
LSDF_F32, LSDF_BF16, LSDF_F16 = 0, 1, 2
LSDF_MAX_LINKS = 16
LSDF_MAX_DOF = 15
LSDF_MAX_COMPONENTS = 16

DTYPE_CODES = {torch.float32: LSDF_F32}


class LsdfError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"lsdf error {code}: {message}")
        self.code = code


class lsdf_grid(ct.Structure):
    _fields_ = [("lo", ct.c_float * 3), ("hi", ct.c_float * 3), ("n", ct.c_int32 * 3),
                ("dtype", ct.c_int32), ("elem_offset", ct.c_int64)]


class lsdf_dh(ct.Structure):
    _fields_ = [("a", ct.c_float), ("alpha", ct.c_float), ("d", ct.c_float), ("theta_offset", ct.c_float)]


_lib = None


def load_library():
    """Loads liblsdf.so; raises if it has not been built (there is no CPU
    fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2309_12543_amd.build` (hipcc, gfx950)")
    lib = ct.CDLL(LIB_PATH)
    vp, i32, i64, u32, sz = ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_uint32, ct.c_size_t
    lib.lsdf_version.restype = ct.c_int
    lib.lsdf_version.argtypes = []
    lib.lsdf_last_error.restype = ct.c_char_p
    lib.lsdf_last_error.argtypes = []
    lib.lsdf_fk_batch.restype = ct.c_int
    lib.lsdf_fk_batch.argtypes = [ct.POINTER(lsdf_dh), i32, ct.POINTER(ct.c_float), vp, i32, vp, vp]
    lib.lsdf_query_workspace_size.restype = ct.c_int
    lib.lsdf_query_workspace_size.argtypes = [i32, i32, i64, ct.POINTER(sz)]
    lib.lsdf_query_min_distance.restype = ct.c_int
    lib.lsdf_query_min_distance.argtypes = [vp, i32, i32, ct.POINTER(lsdf_grid), vp, vp, i64, vp, vp, vp,
                                            u32, vp, sz, vp]
    lib.lsdf_build_link_sdf.restype = ct.c_int
    lib.lsdf_build_link_sdf.argtypes = [vp, i32, vp, i32, ct.POINTER(ct.c_int32), i32, ct.POINTER(lsdf_grid),
                                        vp, vp]
    _lib = lib
    return lib


def _check(rc: int):
    if rc != LSDF_OK:
        raise LsdfError(rc, load_library().lsdf_last_error().decode())


def version() -> int:
    return int(load_library().lsdf_version())


def last_error() -> str:
    return load_library().lsdf_last_error().decode()


def _stream_handle(stream, device):
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return ct.c_void_p(stream.cuda_stream)


def _require(t: torch.Tensor, name: str, dtype, shape=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


# ---------------------------------------------------------------------------
# grids
# ---------------------------------------------------------------------------

class GridSet:
    """Descriptors of L link grids packed into one device buffer."""

    def __init__(self, lo, hi, n, buf: torch.Tensor | None = None, device=None):
        lo = np.asarray(lo, dtype=np.float32).reshape(-1, 3)
        hi = np.asarray(hi, dtype=np.float32).reshape(-1, 3)
        n = np.asarray(n, dtype=np.int64).reshape(-1, 3)
        if not (lo.shape == hi.shape == n.shape):
            raise ValueError("lo, hi and n must all be [L][3]")
        self.L = lo.shape[0]
        if not 1 <= self.L <= LSDF_MAX_LINKS:
            raise ValueError(f"1 <= L <= {LSDF_MAX_LINKS} required")
        sizes = n.prod(axis=1)
        self.offsets = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
        self.total = int(sizes.sum())
        self.lo, self.hi, self.n = lo, hi, n.astype(np.int32)
        self.desc = (lsdf_grid * self.L)()
        for i in range(self.L):
            d = self.desc[i]
            for a in range(3):
                d.lo[a] = float(lo[i, a])
                d.hi[a] = float(hi[i, a])
                d.n[a] = int(n[i, a])
            d.dtype = LSDF_F32
            d.elem_offset = int(self.offsets[i])
        if buf is None:
            buf = torch.empty(self.total, dtype=torch.float32, device=device or "cuda")
        _require(buf, "grid buffer", torch.float32)
        if buf.numel() < self.total:
            raise ValueError(f"grid buffer holds {buf.numel()} elements, descriptors need {self.total}")
        self.buf = buf

    def grid(self, i: int) -> torch.Tensor:
        """View of link i's grid as [nz][ny][nx]."""
        o, (nx, ny, nz) = int(self.offsets[i]), self.n[i]
        return self.buf[o:o + int(nx) * int(ny) * int(nz)].view(int(nz), int(ny), int(nx))

    def set_grid(self, i: int, values):
        self.grid(i).copy_(torch.as_tensor(np.ascontiguousarray(values), dtype=torch.float32))


# ---------------------------------------------------------------------------
# calls
# ---------------------------------------------------------------------------

def fk_batch(dh, q: torch.Tensor, base_T=None, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Link poses [C][dof+1][3][4] for joint angles q [C][dof] (lsdf_fk_batch)."""
    lib = load_library()
    dh = np.asarray(dh, dtype=np.float64).reshape(-1, 4)
    dof = dh.shape[0]
    if q.dim() != 2 or q.shape[1] != dof:
        raise ValueError(f"q must be [C][{dof}]")
    _require(q, "q", torch.float32)
    C = q.shape[0]
    if out is None:
        out = torch.empty((C, dof + 1, 3, 4), dtype=torch.float32, device=q.device)
    _require(out, "out", torch.float32, (C, dof + 1, 3, 4))
    rows = (lsdf_dh * dof)(*[lsdf_dh(*map(float, r)) for r in dh])
    base_p = None
    if base_T is not None:
        b = np.ascontiguousarray(np.asarray(base_T, dtype=np.float32).reshape(12))
        base_p = b.ctypes.data_as(ct.POINTER(ct.c_float))
    _check(lib.lsdf_fk_batch(rows, dof, base_p, q.data_ptr(), C, out.data_ptr(), _stream_handle(stream, q.device)))
    return out


def query_workspace_size(C: int, L: int, M: int) -> int:
    n = ct.c_size_t(0)
    _check(load_library().lsdf_query_workspace_size(C, L, M, ct.byref(n)))
    return int(n.value)


_workspaces: dict = {}


def query_workspace(C: int, L: int, M: int, device) -> torch.Tensor:
    """A zero-filled workspace, cached per device and kept for reuse (every
    call leaves it zero-filled again)."""
    need = query_workspace_size(C, L, M)
    dev = torch.device(device)
    key = (dev.type, dev.index if dev.index is not None else torch.cuda.current_device())
    ws = _workspaces.get(key)
    if ws is None or ws.numel() < need:
        ws = torch.zeros(max(need, 1 << 16), dtype=torch.uint8, device=dev)
        _workspaces[key] = ws
    return ws


def query_min_distance(link_T: torch.Tensor, grids: GridSet, points: torch.Tensor, *,
                       link_dist: bool = False, workspace: torch.Tensor | None = None,
                       out=None, stream=None):
    """Per configuration: (clearance [C] float32, argmin link [C] int32, and
    per-link minima [C][L] when ``link_dist``) (lsdf_query_min_distance)."""
    lib = load_library()
    if link_T.dim() != 4 or tuple(link_T.shape[2:]) != (3, 4):
        raise ValueError("link_T must be [C][L][3][4]")
    _require(link_T, "link_T", torch.float32)
    C, L = int(link_T.shape[0]), int(link_T.shape[1])
    if L != grids.L:
        raise ValueError(f"link_T has {L} links, grids has {grids.L}")
    if points.dim() != 2 or points.shape[1] != 3:
        raise ValueError("points must be [M][3]")
    _require(points, "points", torch.float32)
    M = int(points.shape[0])
    dev = link_T.device
    if grids.buf.device != dev or points.device != dev:
        raise ValueError("link_T, grids and points must be on one device")
    if out is None:
        dist = torch.empty(C, dtype=torch.float32, device=dev)
        link = torch.empty(C, dtype=torch.int32, device=dev)
        ld = torch.empty((C, L), dtype=torch.float32, device=dev) if link_dist else None
    else:
        dist, link, ld = out
    _require(dist, "out_dist", torch.float32, (C,))
    _require(link, "out_link", torch.int32, (C,))
    if ld is not None:
        _require(ld, "out_link_dist", torch.float32, (C, L))
    if workspace is None:
        workspace = query_workspace(C, L, M, dev)
    _require(workspace, "workspace", torch.uint8)
    _check(lib.lsdf_query_min_distance(
        link_T.data_ptr(), C, L, grids.desc, grids.buf.data_ptr(),
        points.data_ptr() if M > 0 else None, M, dist.data_ptr(), link.data_ptr(),
        ld.data_ptr() if ld is not None else None, 0, workspace.data_ptr(), workspace.numel(),
        _stream_handle(stream, dev)))
    return (dist, link, ld) if link_dist else (dist, link)


def build_link_sdf(verts: torch.Tensor, tris: torch.Tensor, comp_first, grids: GridSet, index: int, stream=None):
    """Fills link ``index`` of ``grids`` with the signed distance to the mesh
    (lsdf_build_link_sdf)."""
    lib = load_library()
    _require(verts, "verts", torch.float32)
    _require(tris, "tris", torch.int32)
    if verts.dim() != 2 or verts.shape[1] != 3 or tris.dim() != 2 or tris.shape[1] != 3:
        raise ValueError("verts must be [nv][3] and tris [nt][3]")
    nv, nt = int(verts.shape[0]), int(tris.shape[0])
    cf_p, ncomp = None, 0
    if comp_first is not None:
        cf = np.ascontiguousarray(np.asarray(comp_first, dtype=np.int32))
        ncomp = cf.shape[0] - 1
        cf_p = cf.ctypes.data_as(ct.POINTER(ct.c_int32))
    desc = ct.pointer(grids.desc[index])
    _check(lib.lsdf_build_link_sdf(verts.data_ptr(), nv, tris.data_ptr(), nt, cf_p, ncomp, desc,
                                   grids.buf.data_ptr(), _stream_handle(stream, verts.device)))


def build_robot_grids(meshes, lo, hi, n, device="cuda", stream=None) -> GridSet:
    """GridSet with every link's SDF built on the GPU from its mesh."""
    gs = GridSet(lo, hi, n, device=device)
    for i, m in enumerate(meshes):
        v = torch.as_tensor(np.asarray(m.verts, dtype=np.float32), device=device)
        t = torch.as_tensor(np.asarray(m.tris, dtype=np.int32), device=device)
        build_link_sdf(v, t, m.comp_first, gs, i, stream=stream)
    return gs
