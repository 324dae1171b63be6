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
LSDF_QUERY_NOALLOC_SCRATCH = 8 << 20
LSDF_MAX_DOF = 15
LSDF_MAX_COMPONENTS = 16
LSDF_MLP_HIDDEN = 128
LSDF_MLP_PARAMS = 33665

DTYPE_CODES = {torch.float32: LSDF_F32, torch.bfloat16: LSDF_BF16, torch.float16: LSDF_F16}


class LsdfError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"lsdf error {code}: {message}")
        self.code = code


class lsdf_grid(ct.Structure):
    _fields_ = [("lo", ct.c_float * 3), ("hi", ct.c_float * 3), ("n", ct.c_int32 * 3),
                ("dtype", ct.c_int32), ("elem_offset", ct.c_int64)]


class lsdf_mlp_domain(ct.Structure):
    _fields_ = [("centre", ct.c_float * 3), ("half", ct.c_float * 3), ("core_half", ct.c_float * 3),
                ("bound", ct.c_float)]


LSDF_SCHED_DEFAULT, LSDF_SCHED_XCD_SLICES, LSDF_SCHED_INTERLEAVED = 0, 1, 2


class lsdf_query_tuning(ct.Structure):
    _fields_ = [("chunk_points", ct.c_int32), ("blocks_per_cu", ct.c_int32), ("schedule", ct.c_int32),
                ("reserved", ct.c_int32)]

    def __repr__(self):
        return (f"lsdf_query_tuning(chunk_points={self.chunk_points}, blocks_per_cu={self.blocks_per_cu}, "
                f"schedule={self.schedule})")

    def as_tuple(self):
        return (self.chunk_points, self.blocks_per_cu, self.schedule)


class lsdf_env(ct.Structure):
    _fields_ = [("lo", ct.c_float * 3), ("voxel", ct.c_float), ("n", ct.c_int32 * 3)]


def make_env(lo, voxel, n) -> lsdf_env:
    e = lsdf_env()
    for a in range(3):
        e.lo[a] = float(lo[a])
        e.n[a] = int(n[a])
    e.voxel = float(voxel)
    return e


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
    lib.lsdf_query_workspace_size.argtypes = [i32, i32, i64, ct.c_uint32, ct.POINTER(sz)]
    lib.lsdf_query_min_distance.restype = ct.c_int
    lib.lsdf_query_min_distance.argtypes = [vp, i32, i32, ct.POINTER(lsdf_grid), vp, vp, i64, vp, vp, vp,
                                            u32, vp, sz, vp]
    lib.lsdf_query_min_distance_noalloc.restype = ct.c_int
    lib.lsdf_query_min_distance_noalloc.argtypes = [vp, i32, i32, ct.POINTER(lsdf_grid), vp, vp, i64, vp, vp, vp,
                                                    u32, vp]
    lib.lsdf_set_kernel_events.restype = ct.c_int
    lib.lsdf_set_kernel_events.argtypes = [vp, vp]
    tun = ct.POINTER(lsdf_query_tuning)
    lib.lsdf_query_batched_workspace_size.restype = ct.c_int
    lib.lsdf_query_batched_workspace_size.argtypes = [i32, i32, i32, i64, ct.POINTER(sz)]
    lib.lsdf_query_min_distance_batched.restype = ct.c_int
    lib.lsdf_query_min_distance_batched.argtypes = [i32, vp, vp, vp, i32, i32, ct.POINTER(lsdf_grid), vp, vp, i64,
                                                    vp, vp, vp, tun, u32, vp, sz, vp]
    lib.lsdf_query_from_joints.restype = ct.c_int
    lib.lsdf_query_from_joints.argtypes = [ct.POINTER(lsdf_dh), i32, ct.POINTER(ct.c_float), vp, i32, vp, vp, i32,
                                           ct.POINTER(lsdf_grid), vp, vp, i64, vp, vp, vp, vp, tun, u32, vp, sz, vp]
    lib.lsdf_query_autotune.restype = ct.c_int
    lib.lsdf_query_autotune.argtypes = [i32, vp, vp, vp, i32, i32, ct.POINTER(lsdf_grid), vp, vp, i64, vp, vp,
                                        tun, i32, i32, vp, sz, vp, tun, ct.POINTER(ct.c_float)]
    env = ct.POINTER(lsdf_env)
    lib.lsdf_robot_sdf_size.restype = ct.c_int
    lib.lsdf_robot_sdf_size.argtypes = [i32, env, ct.POINTER(sz)]
    lib.lsdf_robot_sdf_build_workspace_size.restype = ct.c_int
    lib.lsdf_robot_sdf_build_workspace_size.argtypes = [i32, i32, ct.POINTER(sz)]
    lib.lsdf_robot_sdf_build.restype = ct.c_int
    lib.lsdf_robot_sdf_build.argtypes = [vp, i32, i32, ct.POINTER(lsdf_grid), vp, env, vp, vp, sz, vp]
    lib.lsdf_robot_sdf_query_workspace_size.restype = ct.c_int
    lib.lsdf_robot_sdf_query_workspace_size.argtypes = [env, i64, ct.POINTER(sz)]
    lib.lsdf_robot_sdf_query.restype = ct.c_int
    lib.lsdf_robot_sdf_query.argtypes = [vp, i32, env, vp, i64, vp, vp, sz, vp]
    lib.lsdf_frnn_nparam.restype = ct.c_int
    lib.lsdf_frnn_nparam.argtypes = [i32, ct.POINTER(i64)]
    lib.lsdf_frnn_train_workspace_size.restype = ct.c_int
    lib.lsdf_frnn_train_workspace_size.argtypes = [i32, i32, ct.POINTER(sz)]
    lib.lsdf_frnn_train_step.restype = ct.c_int
    lib.lsdf_frnn_train_step.argtypes = [vp, vp, vp, i64, ct.c_float, ct.c_float, ct.c_float, ct.c_float, i32, vp,
                                         i32, vp, vp, vp, sz, vp]
    lib.lsdf_frnn_max_error.restype = ct.c_int
    lib.lsdf_frnn_max_error.argtypes = [vp, i32, vp, i64, vp, vp]
    lib.lsdf_robot_sdf_build_frnn.restype = ct.c_int
    lib.lsdf_robot_sdf_build_frnn.argtypes = [vp, i32, i32, ct.POINTER(lsdf_grid), vp, env, vp, i32, vp, vp, sz, vp]
    lib.lsdf_build_link_sdf.restype = ct.c_int
    lib.lsdf_build_link_sdf.argtypes = [vp, i32, vp, i32, ct.POINTER(ct.c_int32), i32, ct.POINTER(lsdf_grid),
                                        vp, vp]
    fp = ct.POINTER(ct.c_float)
    dom = ct.POINTER(lsdf_mlp_domain)
    lib.lsdf_mlp_eval.restype = ct.c_int
    lib.lsdf_mlp_eval.argtypes = [vp, dom, vp, i64, vp, vp]
    lib.lsdf_query_min_distance_mlp.restype = ct.c_int
    lib.lsdf_query_min_distance_mlp.argtypes = [vp, i32, i32, ct.POINTER(lsdf_grid), vp, vp, dom, ct.c_float, vp, i64,
                                                vp, vp, vp, u32, vp, sz, vp]
    lib.lsdf_mlp_train_workspace_size.restype = ct.c_int
    lib.lsdf_mlp_train_workspace_size.argtypes = [i32, i32, ct.POINTER(sz)]
    lib.lsdf_mlp_loss_grad.restype = ct.c_int
    lib.lsdf_mlp_loss_grad.argtypes = [vp, dom, i32, vp, vp, i64, vp, i32, vp, vp, vp, sz, vp]
    lib.lsdf_mlp_train_step.restype = ct.c_int
    lib.lsdf_mlp_train_step.argtypes = [vp, vp, vp, i64, ct.c_float, ct.c_float, ct.c_float, ct.c_float, dom, i32,
                                        vp, vp, i64, vp, i32, vp, vp, vp, sz, vp]
    lib.lsdf_gather_roof.restype = ct.c_int
    lib.lsdf_gather_roof.argtypes = [vp, i32, i32, i64, vp, vp]
    lib.lsdf_sdf_labels.restype = ct.c_int
    lib.lsdf_sdf_labels.argtypes = [vp, i32, vp, i32, ct.POINTER(ct.c_int32), i32, ct.POINTER(lsdf_grid), vp, vp,
                                    i64, vp, vp]
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

    def __init__(self, lo, hi, n, buf: torch.Tensor | None = None, device=None, dtype=torch.float32):
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
            d.dtype = DTYPE_CODES[dtype]
            d.elem_offset = int(self.offsets[i])
        self.dtype = dtype
        if buf is None:
            buf = torch.empty(self.total, dtype=dtype, device=device or "cuda")
        _require(buf, "grid buffer", dtype)
        if buf.numel() < self.total:
            raise ValueError(f"grid buffer holds {buf.numel()} elements, descriptors need {self.total}")
        self.buf = buf

    def grid(self, i: int) -> torch.Tensor:
        """View of link i's grid as [nz][ny][nx]."""
        o, (nx, ny, nz) = int(self.offsets[i]), self.n[i]
        return self.buf[o:o + int(nx) * int(ny) * int(nz)].view(int(nz), int(ny), int(nx))

    def set_grid(self, i: int, values):
        """Stores float values, rounded to the grid's storage type (nearest even)."""
        v = torch.as_tensor(np.ascontiguousarray(values, dtype=np.float32), dtype=torch.float32)
        self.grid(i).copy_(v.to(self.dtype))


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


def set_kernel_events(before=None, after=None):
    """The next query on this thread records torch.cuda.Event ``before`` /
    ``after`` around its main kernel (lsdf_set_kernel_events).  The events
    must already exist (record them once first)."""
    h = lambda e: None if e is None else ct.c_void_p(e.cuda_event)
    _check(load_library().lsdf_set_kernel_events(h(before), h(after)))


def query_workspace_size(C: int, L: int, M: int) -> int:
    n = ct.c_size_t(0)
    _check(load_library().lsdf_query_workspace_size(C, L, M, 0, ct.byref(n)))
    return int(n.value)


def query_batched_workspace_size(K: int, C: int, L: int, M: int) -> int:
    n = ct.c_size_t(0)
    _check(load_library().lsdf_query_batched_workspace_size(K, C, L, M, ct.byref(n)))
    return int(n.value)


_workspaces: dict = {}


def _cached_workspace(need: int, device) -> torch.Tensor:
    dev = torch.device(device)
    key = (dev.type, dev.index if dev.index is not None else torch.cuda.current_device())
    ws = _workspaces.get(key)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1 << 16), dtype=torch.uint8, device=dev)
        _workspaces[key] = ws
    return ws


def query_workspace(C: int, L: int, M: int, device, K: int = 1) -> torch.Tensor:
    """A query workspace, cached per device and reused by every call that
    passes none (calls on one device share it, so they must not overlap in
    time: same stream is fine)."""
    return _cached_workspace(query_batched_workspace_size(K, C, L, M), device)


def _query_shapes(link_T, grids, points):
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
    return C, L, M, dev


def _query_outputs(out, C, L, dev, link_dist):
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
    return dist, link, ld


def make_tuning(chunk_points: int = 0, blocks_per_cu: int = 0, schedule: int = 0) -> lsdf_query_tuning:
    return lsdf_query_tuning(int(chunk_points), int(blocks_per_cu), int(schedule), 0)


def query_min_distance(link_T: torch.Tensor, grids: GridSet, points: torch.Tensor, *,
                       link_dist: bool = False, workspace: torch.Tensor | None = None,
                       out=None, stream=None):
    """Per configuration: (clearance [C] float32, argmin link [C] int32, and
    per-link minima [C][L] when ``link_dist``) (lsdf_query_min_distance)."""
    lib = load_library()
    C, L, M, dev = _query_shapes(link_T, grids, points)
    dist, link, ld = _query_outputs(out, C, L, dev, link_dist)
    if workspace is None:
        workspace = query_workspace(C, L, M, dev)
    _require(workspace, "workspace", torch.uint8)
    _check(lib.lsdf_query_min_distance(
        link_T.data_ptr(), C, L, grids.desc, grids.buf.data_ptr(),
        points.data_ptr() if M > 0 else None, M, dist.data_ptr(), link.data_ptr(),
        ld.data_ptr() if ld is not None else None, 0, workspace.data_ptr(), workspace.numel(),
        _stream_handle(stream, dev)))
    return (dist, link, ld) if link_dist else (dist, link)


def query_min_distance_noalloc(link_T: torch.Tensor, grids: GridSet, points: torch.Tensor, *,
                               link_dist: bool = False, out=None, stream=None):
    """query_min_distance with the library's own device workspace
    (lsdf_query_min_distance_noalloc): the call allocates nothing when
    ``out`` is given.  Calls that overlap in time on one GPU race."""
    lib = load_library()
    C, L, M, dev = _query_shapes(link_T, grids, points)
    dist, link, ld = _query_outputs(out, C, L, dev, link_dist)
    _check(lib.lsdf_query_min_distance_noalloc(
        link_T.data_ptr(), C, L, grids.desc, grids.buf.data_ptr(),
        points.data_ptr() if M > 0 else None, M, dist.data_ptr(), link.data_ptr(),
        ld.data_ptr() if ld is not None else None, 0, _stream_handle(stream, dev)))
    return (dist, link, ld) if link_dist else (dist, link)


def _offsets(c_off: torch.Tensor, m_off: torch.Tensor, dev):
    _require(c_off, "c_offsets", torch.int32)
    _require(m_off, "m_offsets", torch.int64)
    if c_off.dim() != 1 or m_off.dim() != 1 or c_off.numel() != m_off.numel() or c_off.numel() < 2:
        raise ValueError("c_offsets and m_offsets must be [K+1] with K >= 1")
    if c_off.device != dev or m_off.device != dev:
        raise ValueError("offsets must be on the query's device")
    return int(c_off.numel()) - 1


def query_min_distance_batched(link_T: torch.Tensor, grids: GridSet, points: torch.Tensor, c_offsets: torch.Tensor,
                               m_offsets: torch.Tensor, *, link_dist: bool = False, tuning=None,
                               workspace: torch.Tensor | None = None, out=None, stream=None):
    """K trajectories in one call (lsdf_query_min_distance_batched):
    trajectory k pairs poses link_T[c_offsets[k]:c_offsets[k+1]] with
    points[m_offsets[k]:m_offsets[k+1]].  The offsets are device tensors
    (int32 and int64, [K+1]) and are never read on the host."""
    lib = load_library()
    C, L, M, dev = _query_shapes(link_T, grids, points)
    K = _offsets(c_offsets, m_offsets, dev)
    dist, link, ld = _query_outputs(out, C, L, dev, link_dist)
    if workspace is None:
        workspace = query_workspace(C, L, M, dev, K=K)
    _require(workspace, "workspace", torch.uint8)
    tun = ct.byref(tuning) if tuning is not None else None
    _check(lib.lsdf_query_min_distance_batched(
        K, c_offsets.data_ptr(), m_offsets.data_ptr(), link_T.data_ptr(), C, L, grids.desc, grids.buf.data_ptr(),
        points.data_ptr() if M > 0 else None, M, dist.data_ptr(), link.data_ptr(),
        ld.data_ptr() if ld is not None else None, tun, 0, workspace.data_ptr(), workspace.numel(),
        _stream_handle(stream, dev)))
    return (dist, link, ld) if link_dist else (dist, link)


def _dh_rows(dh):
    dh = np.asarray(dh, dtype=np.float64).reshape(-1, 4)
    return (lsdf_dh * dh.shape[0])(*[lsdf_dh(*map(float, r)) for r in dh]), dh.shape[0]


def _base_ptr(base_T):
    if base_T is None:
        return None, None
    b = np.ascontiguousarray(np.asarray(base_T, dtype=np.float32).reshape(12))
    return b, b.ctypes.data_as(ct.POINTER(ct.c_float))


def query_from_joints(dh, q: torch.Tensor, grids: GridSet, points: torch.Tensor, *, base_T=None,
                      c_offsets: torch.Tensor | None = None, m_offsets: torch.Tensor | None = None,
                      link_T: torch.Tensor | None = None, link_dist: bool = False, tuning=None,
                      workspace: torch.Tensor | None = None, out=None, stream=None):
    """Kinematics and clearance in one call (lsdf_query_from_joints): joint
    angles q [C][dof] in, (dist [C], link [C][, link_dist [C][L]]) out; the
    poses go to ``link_T`` [C][dof+1][3][4] when given.  With c_offsets /
    m_offsets (device, [K+1]) it is the batched query."""
    lib = load_library()
    rows, dof = _dh_rows(dh)
    if q.dim() != 2 or q.shape[1] != dof:
        raise ValueError(f"q must be [C][{dof}]")
    _require(q, "q", torch.float32)
    C, L, dev = int(q.shape[0]), dof + 1, q.device
    if grids.L != L:
        raise ValueError(f"grids has {grids.L} links, the arm has {L} frames")
    if points.dim() != 2 or points.shape[1] != 3:
        raise ValueError("points must be [M][3]")
    _require(points, "points", torch.float32)
    M = int(points.shape[0])
    if grids.buf.device != dev or points.device != dev:
        raise ValueError("q, grids and points must be on one device")
    if (c_offsets is None) != (m_offsets is None):
        raise ValueError("give both offset arrays or neither")
    K = 1 if c_offsets is None else _offsets(c_offsets, m_offsets, dev)
    if link_T is not None:
        _require(link_T, "link_T", torch.float32, (C, L, 3, 4))
    dist, link, ld = _query_outputs(out, C, L, dev, link_dist)
    if workspace is None:
        workspace = query_workspace(C, L, M, dev, K=K)
    _require(workspace, "workspace", torch.uint8)
    b, base_p = _base_ptr(base_T)
    tun = ct.byref(tuning) if tuning is not None else None
    _check(lib.lsdf_query_from_joints(
        rows, dof, base_p, q.data_ptr(), K, c_offsets.data_ptr() if c_offsets is not None else None,
        m_offsets.data_ptr() if m_offsets is not None else None, C, grids.desc, grids.buf.data_ptr(),
        points.data_ptr() if M > 0 else None, M, link_T.data_ptr() if link_T is not None else None,
        dist.data_ptr(), link.data_ptr(), ld.data_ptr() if ld is not None else None, tun, 0,
        workspace.data_ptr(), workspace.numel(), _stream_handle(stream, dev)))
    return (dist, link, ld) if link_dist else (dist, link)


class PreparedQueryFromJoints:
    """lsdf_query_from_joints with every argument checked and marshalled
    once, for a loop that makes the same call over and over on the same
    buffers (new joint angles or points written into them in place between
    calls, as a control cycle does).  Calling the object makes the C call and
    nothing else, so the host cost of a step is one ctypes call.  The
    tensors given here must stay allocated and keep their shapes; the stream
    is fixed here too (the current one when none is given).  Arguments as in
    query_from_joints; the outputs are ``dist``, ``link`` and ``link_dist``."""

    def __init__(self, dh, q: torch.Tensor, grids: GridSet, points: torch.Tensor, *, base_T=None,
                 c_offsets: torch.Tensor | None = None, m_offsets: torch.Tensor | None = None,
                 link_T: torch.Tensor | None = None, link_dist: bool = False, tuning=None,
                 workspace: torch.Tensor | None = None, out=None, stream=None):
        lib = load_library()
        rows, dof = _dh_rows(dh)
        if q.dim() != 2 or q.shape[1] != dof:
            raise ValueError(f"q must be [C][{dof}]")
        _require(q, "q", torch.float32)
        C, L, dev = int(q.shape[0]), dof + 1, q.device
        if grids.L != L:
            raise ValueError(f"grids has {grids.L} links, the arm has {L} frames")
        if points.dim() != 2 or points.shape[1] != 3:
            raise ValueError("points must be [M][3]")
        _require(points, "points", torch.float32)
        M = int(points.shape[0])
        if grids.buf.device != dev or points.device != dev:
            raise ValueError("q, grids and points must be on one device")
        if (c_offsets is None) != (m_offsets is None):
            raise ValueError("give both offset arrays or neither")
        K = 1 if c_offsets is None else _offsets(c_offsets, m_offsets, dev)
        if link_T is not None:
            _require(link_T, "link_T", torch.float32, (C, L, 3, 4))
        self.dist, self.link, self.link_dist = _query_outputs(out, C, L, dev, link_dist)
        if workspace is None:
            workspace = torch.empty(query_batched_workspace_size(K, C, L, M), dtype=torch.uint8, device=dev)
        _require(workspace, "workspace", torch.uint8)
        b, base_p = _base_ptr(base_T)
        self._tuning = tuning
        vp, i32 = ct.c_void_p, ct.c_int32
        self._keep = (rows, b, q, grids, points, c_offsets, m_offsets, link_T, workspace, tuning)
        self._fn = lib.lsdf_query_from_joints
        self._args = (
            rows, i32(dof), base_p, vp(q.data_ptr()), i32(K),
            vp(c_offsets.data_ptr()) if c_offsets is not None else None,
            vp(m_offsets.data_ptr()) if m_offsets is not None else None, i32(C), grids.desc,
            vp(grids.buf.data_ptr()), vp(points.data_ptr()) if M > 0 else None, ct.c_int64(M),
            vp(link_T.data_ptr()) if link_T is not None else None, vp(self.dist.data_ptr()),
            vp(self.link.data_ptr()), vp(self.link_dist.data_ptr()) if self.link_dist is not None else None,
            ct.byref(tuning) if tuning is not None else None, ct.c_uint32(0), vp(workspace.data_ptr()),
            ct.c_size_t(workspace.numel()), _stream_handle(stream, dev))

    def __call__(self):
        rc = self._fn(*self._args)
        if rc != LSDF_OK:
            _check(rc)


def query_autotune(link_T: torch.Tensor, grids: GridSet, points: torch.Tensor, c_offsets: torch.Tensor,
                   m_offsets: torch.Tensor, *, candidates=None, reps: int = 5, workspace=None, stream=None):
    """Times the batched query under each candidate tiling
    (lsdf_query_autotune) and returns (best lsdf_query_tuning, its ms,
    (dist, link) of the problem)."""
    lib = load_library()
    C, L, M, dev = _query_shapes(link_T, grids, points)
    K = _offsets(c_offsets, m_offsets, dev)
    dist, link, _ = _query_outputs(None, C, L, dev, False)
    if workspace is None:
        workspace = query_workspace(C, L, M, dev, K=K)
    arr, n = None, 0
    if candidates is not None:
        cands = [c if isinstance(c, lsdf_query_tuning) else make_tuning(*c) for c in candidates]
        n = len(cands)
        arr = (lsdf_query_tuning * n)(*cands)
    best = lsdf_query_tuning()
    ms = ct.c_float(0.0)
    _check(lib.lsdf_query_autotune(
        K, c_offsets.data_ptr(), m_offsets.data_ptr(), link_T.data_ptr(), C, L, grids.desc, grids.buf.data_ptr(),
        points.data_ptr() if M > 0 else None, M, dist.data_ptr(), link.data_ptr(), arr, n, reps,
        workspace.data_ptr(), workspace.numel(), _stream_handle(stream, dev), ct.byref(best), ct.byref(ms)))
    return best, float(ms.value), (dist, link)


def robot_sdf_build(link_T: torch.Tensor, grids: GridSet, env: lsdf_env, out: torch.Tensor | None = None,
                    stream=None) -> torch.Tensor:
    """The paper's Robot SDFs [C][n_z][n_y][n_x] float32 (lsdf_robot_sdf_build)."""
    lib = load_library()
    if link_T.dim() != 4 or tuple(link_T.shape[2:]) != (3, 4):
        raise ValueError("link_T must be [C][L][3][4]")
    _require(link_T, "link_T", torch.float32)
    C, L, dev = int(link_T.shape[0]), int(link_T.shape[1]), link_T.device
    if L != grids.L:
        raise ValueError(f"link_T has {L} links, grids has {grids.L}")
    shape = (C, int(env.n[2]), int(env.n[1]), int(env.n[0]))
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=dev)
    _require(out, "robot_sdf", torch.float32, shape)
    n = ct.c_size_t(0)
    _check(lib.lsdf_robot_sdf_build_workspace_size(C, L, ct.byref(n)))
    ws = _cached_workspace(int(n.value), dev)
    _check(lib.lsdf_robot_sdf_build(link_T.data_ptr(), C, L, grids.desc, grids.buf.data_ptr(), ct.byref(env),
                                    out.data_ptr(), ws.data_ptr(), ws.numel(), _stream_handle(stream, dev)))
    return out


def robot_sdf_query(robot_sdf: torch.Tensor, env: lsdf_env, points: torch.Tensor, out: torch.Tensor | None = None,
                    stream=None, workspace: torch.Tensor | None = None) -> torch.Tensor:
    """Per configuration, the minimum of its Robot SDF over the voxels the
    points occupy (lsdf_robot_sdf_query).  ``workspace`` (uint8, optional)
    is the call's workspace; afterwards it holds the distinct occupied voxels
    as the header describes."""
    lib = load_library()
    _require(robot_sdf, "robot_sdf", torch.float32)
    C, dev = int(robot_sdf.shape[0]), robot_sdf.device
    if tuple(robot_sdf.shape[1:]) != (int(env.n[2]), int(env.n[1]), int(env.n[0])):
        raise ValueError("robot_sdf does not match the environment")
    if points.dim() != 2 or points.shape[1] != 3:
        raise ValueError("points must be [M][3]")
    _require(points, "points", torch.float32)
    M = int(points.shape[0])
    if out is None:
        out = torch.empty(C, dtype=torch.float32, device=dev)
    _require(out, "out_dist", torch.float32, (C,))
    n = ct.c_size_t(0)
    _check(lib.lsdf_robot_sdf_query_workspace_size(ct.byref(env), M, ct.byref(n)))
    if workspace is None:
        ws = _cached_workspace(int(n.value), dev)
    else:
        _require(workspace, "workspace", torch.uint8)
        ws = workspace
    _check(lib.lsdf_robot_sdf_query(robot_sdf.data_ptr(), C, ct.byref(env), points.data_ptr() if M > 0 else None, M,
                                    out.data_ptr(), ws.data_ptr(), ws.numel(), _stream_handle(stream, dev)))
    return out


def frnn_nparam(m: int) -> int:
    n = ct.c_int64(0)
    _check(load_library().lsdf_frnn_nparam(int(m), ct.byref(n)))
    return int(n.value)


def frnn_train_step(params: torch.Tensor, m: int, R: torch.Tensor, *, adam=None, t: int = 1, lr: float = 1e-4,
                    beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, grad: torch.Tensor | None = None,
                    loss: torch.Tensor | None = None, workspace: torch.Tensor | None = None, stream=None):
    """One step of the grid-transformation network (lsdf_frnn_train_step):
    R [B][3][3] rotations; adam = (m, v) moment tensors or None (gradient
    only).  Returns (loss [1], grad [n])."""
    lib = load_library()
    n = frnn_nparam(m)
    _require(params, "params", torch.float32, (n,))
    R = R.reshape(-1, 9)
    _require(R, "R", torch.float32)
    B, dev = int(R.shape[0]), params.device
    grad = torch.empty(n, dtype=torch.float32, device=dev) if grad is None else grad
    loss = torch.empty(1, dtype=torch.float32, device=dev) if loss is None else loss
    if workspace is None:
        need = ct.c_size_t(0)
        _check(lib.lsdf_frnn_train_workspace_size(int(m), B, ct.byref(need)))
        workspace = _cached_workspace(int(need.value), dev)
    am, av = (None, None) if adam is None else adam
    if am is not None:
        _require(am, "adam_m", torch.float32, (n,))
        _require(av, "adam_v", torch.float32, (n,))
    _check(lib.lsdf_frnn_train_step(params.data_ptr(), am.data_ptr() if am is not None else None,
                                    av.data_ptr() if av is not None else None, int(t), float(lr), float(beta1),
                                    float(beta2), float(eps), int(m), R.data_ptr(), B, loss.data_ptr(),
                                    grad.data_ptr(), workspace.data_ptr(), workspace.numel(),
                                    _stream_handle(stream, dev)))
    return loss, grad


def frnn_max_error(params: torch.Tensor, m: int, R: torch.Tensor, out: torch.Tensor | None = None,
                   stream=None) -> torch.Tensor:
    """max |f(R) - R^T P| over the rotations R [N][3][3] (lsdf_frnn_max_error)."""
    lib = load_library()
    _require(params, "params", torch.float32, (frnn_nparam(m),))
    R = R.reshape(-1, 9)
    _require(R, "R", torch.float32)
    out = torch.empty(1, dtype=torch.float32, device=params.device) if out is None else out
    _check(lib.lsdf_frnn_max_error(params.data_ptr(), int(m), R.data_ptr() if R.shape[0] else None,
                                   int(R.shape[0]), out.data_ptr(), _stream_handle(stream, params.device)))
    return out


def robot_sdf_build_frnn(link_T: torch.Tensor, grids: GridSet, env: lsdf_env, frnn_params: torch.Tensor, m: int,
                         out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Robot SDFs with the network's transformation (lsdf_robot_sdf_build_frnn)."""
    lib = load_library()
    if link_T.dim() != 4 or tuple(link_T.shape[2:]) != (3, 4):
        raise ValueError("link_T must be [C][L][3][4]")
    _require(link_T, "link_T", torch.float32)
    _require(frnn_params, "frnn_params", torch.float32, (frnn_nparam(m),))
    C, L, dev = int(link_T.shape[0]), int(link_T.shape[1]), link_T.device
    if L != grids.L:
        raise ValueError(f"link_T has {L} links, grids has {grids.L}")
    shape = (C, int(env.n[2]), int(env.n[1]), int(env.n[0]))
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=dev)
    _require(out, "robot_sdf", torch.float32, shape)
    n = ct.c_size_t(0)
    _check(lib.lsdf_robot_sdf_build_workspace_size(C, L, ct.byref(n)))
    ws = _cached_workspace(int(n.value), dev)
    _check(lib.lsdf_robot_sdf_build_frnn(link_T.data_ptr(), C, L, grids.desc, grids.buf.data_ptr(), ct.byref(env),
                                         frnn_params.data_ptr(), int(m), out.data_ptr(), ws.data_ptr(), ws.numel(),
                                         _stream_handle(stream, dev)))
    return out


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


def build_robot_grids(meshes, lo, hi, n, device="cuda", stream=None, dtype=torch.float32) -> GridSet:
    """GridSet with every link's SDF built on the GPU from its mesh."""
    gs = GridSet(lo, hi, n, device=device, dtype=dtype)
    for i, m in enumerate(meshes):
        v = torch.as_tensor(np.asarray(m.verts, dtype=np.float32), device=device)
        t = torch.as_tensor(np.asarray(m.tris, dtype=np.int32), device=device)
        build_link_sdf(v, t, m.comp_first, gs, i, stream=stream)
    return gs


# ---------------------------------------------------------------------------
# learned per-link SDF surrogate
# ---------------------------------------------------------------------------

def make_domains(centre, half, core_half, bound=float("inf")):
    """ctypes array of lsdf_mlp_domain from [L][3] centres, half extents of
    the network domains and half extents of the core boxes, and the remainder
    bounds (a scalar or [L]; +inf: the network's share unbounded)."""
    centre = np.asarray(centre, dtype=np.float32).reshape(-1, 3)
    half = np.asarray(half, dtype=np.float32).reshape(-1, 3)
    core = np.asarray(core_half, dtype=np.float32).reshape(-1, 3)
    if half.shape != centre.shape or core.shape != centre.shape:
        raise ValueError("centre, half and core_half must all be [L][3]")
    bd = np.broadcast_to(np.asarray(bound, dtype=np.float32), (centre.shape[0],))
    arr = (lsdf_mlp_domain * centre.shape[0])()
    for i in range(centre.shape[0]):
        for a in range(3):
            arr[i].centre[a] = float(centre[i, a])
            arr[i].half[a] = float(half[i, a])
            arr[i].core_half[a] = float(core[i, a])
        arr[i].bound = float(bd[i])
    return arr


def mlp_eval(params: torch.Tensor, domain, points: torch.Tensor, out=None, stream=None) -> torch.Tensor:
    """The surrogate's estimates (bounded network share + core distance) of
    one link at link-frame points [N][3] (lsdf_mlp_eval); domain = (centre,
    half, core_half[, bound]) or a one-element lsdf_mlp_domain array."""
    lib = load_library()
    _require(params, "params", torch.float32, (LSDF_MLP_PARAMS,))
    if points.dim() != 2 or points.shape[1] != 3:
        raise ValueError("points must be [N][3]")
    _require(points, "points", torch.float32)
    N = int(points.shape[0])
    if out is None:
        out = torch.empty(N, dtype=torch.float32, device=points.device)
    _require(out, "out", torch.float32, (N,))
    d = domain if isinstance(domain, ct.Array) else make_domains(*domain)
    _check(lib.lsdf_mlp_eval(params.data_ptr(), d, points.data_ptr() if N else None, N, out.data_ptr(),
                             _stream_handle(stream, points.device)))
    return out


def query_min_distance_mlp(link_T: torch.Tensor, grids: GridSet, mlp_params: torch.Tensor, domains,
                           points: torch.Tensor, *, margin: float = 0.05, link_dist: bool = False,
                           workspace: torch.Tensor | None = None, out=None, stream=None):
    """Clearance with the learned surrogate and exact-grid fallback below
    ``margin`` (lsdf_query_min_distance_mlp)."""
    lib = load_library()
    if link_T.dim() != 4 or tuple(link_T.shape[2:]) != (3, 4):
        raise ValueError("link_T must be [C][L][3][4]")
    _require(link_T, "link_T", torch.float32)
    C, L = int(link_T.shape[0]), int(link_T.shape[1])
    if L != grids.L:
        raise ValueError(f"link_T has {L} links, grids has {grids.L}")
    _require(mlp_params, "mlp_params", torch.float32, (L, LSDF_MLP_PARAMS))
    d = domains if isinstance(domains, ct.Array) else make_domains(*domains)
    if len(d) != L:
        raise ValueError("one domain per link required")
    if points.dim() != 2 or points.shape[1] != 3:
        raise ValueError("points must be [M][3]")
    _require(points, "points", torch.float32)
    M = int(points.shape[0])
    dev = link_T.device
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
    _check(lib.lsdf_query_min_distance_mlp(
        link_T.data_ptr(), C, L, grids.desc, grids.buf.data_ptr(), mlp_params.data_ptr(), d, float(margin),
        points.data_ptr() if M > 0 else None, M, dist.data_ptr(), link.data_ptr(),
        ld.data_ptr() if ld is not None else None, 0, workspace.data_ptr(), workspace.numel(),
        _stream_handle(stream, dev)))
    return (dist, link, ld) if link_dist else (dist, link)


def mlp_train_workspace_size(L: int, B: int) -> int:
    n = ct.c_size_t(0)
    _check(load_library().lsdf_mlp_train_workspace_size(L, B, ct.byref(n)))
    return int(n.value)


def _train_args(params, domains, samples, labels, batch_index, B):
    if params.dim() != 2 or params.shape[1] != LSDF_MLP_PARAMS:
        raise ValueError("params must be [L][33665]")
    L = int(params.shape[0])
    if samples.dim() != 3 or samples.shape[0] != L or samples.shape[2] != 3:
        raise ValueError("samples must be [L][N][3]")
    N = int(samples.shape[1])
    _require(samples, "samples", torch.float32)
    _require(labels, "labels", torch.float32, (L, N))
    if batch_index is not None:
        _require(batch_index, "batch_index", torch.int32, (L, B))
    d = domains if isinstance(domains, ct.Array) else make_domains(*domains)
    if len(d) != L:
        raise ValueError("one domain per link required")
    return L, N, d


def mlp_loss_grad(params, domains, samples, labels, B, batch_index=None, workspace=None, stream=None):
    """(loss [L], gradient [L][33665]) of the mean absolute error over B
    samples per link (lsdf_mlp_loss_grad)."""
    lib = load_library()
    _require(params, "params", torch.float32)
    L, N, d = _train_args(params, domains, samples, labels, batch_index, B)
    dev = params.device
    loss = torch.empty(L, dtype=torch.float32, device=dev)
    grad = torch.empty_like(params)
    if workspace is None:
        workspace = torch.empty(mlp_train_workspace_size(L, B), dtype=torch.uint8, device=dev)
    _check(lib.lsdf_mlp_loss_grad(params.data_ptr(), d, L, samples.data_ptr(), labels.data_ptr(), N,
                                  batch_index.data_ptr() if batch_index is not None else None, B, loss.data_ptr(),
                                  grad.data_ptr(), workspace.data_ptr(), workspace.numel(), _stream_handle(stream, dev)))
    return loss, grad


def mlp_train_step(params, adam_m, adam_v, t, lr, domains, samples, labels, B, batch_index=None, *,
                   beta1=0.9, beta2=0.999, eps=1e-8, loss=None, grad=None, workspace=None, stream=None):
    """One Adam step on every link's network (lsdf_mlp_train_step); updates
    params, adam_m and adam_v in place."""
    lib = load_library()
    for name, tns in (("params", params), ("adam_m", adam_m), ("adam_v", adam_v)):
        _require(tns, name, torch.float32, tuple(params.shape))
    L, N, d = _train_args(params, domains, samples, labels, batch_index, B)
    dev = params.device
    if workspace is None:
        workspace = torch.empty(mlp_train_workspace_size(L, B), dtype=torch.uint8, device=dev)
    _check(lib.lsdf_mlp_train_step(params.data_ptr(), adam_m.data_ptr(), adam_v.data_ptr(), int(t), float(lr),
                                   float(beta1), float(beta2), float(eps), d, L, samples.data_ptr(), labels.data_ptr(),
                                   N, batch_index.data_ptr() if batch_index is not None else None, B,
                                   loss.data_ptr() if loss is not None else None,
                                   grad.data_ptr() if grad is not None else None, workspace.data_ptr(),
                                   workspace.numel(), _stream_handle(stream, dev)))


def sdf_labels(verts: torch.Tensor, tris: torch.Tensor, comp_first, grids: GridSet, index: int,
               points: torch.Tensor, out=None, stream=None) -> torch.Tensor:
    """Training labels of link ``index`` at link-frame points: grid value in
    the box, exact mesh distance outside (lsdf_sdf_labels)."""
    lib = load_library()
    _require(verts, "verts", torch.float32)
    _require(tris, "tris", torch.int32)
    _require(points, "points", torch.float32)
    if points.dim() != 2 or points.shape[1] != 3:
        raise ValueError("points must be [N][3]")
    N = int(points.shape[0])
    if out is None:
        out = torch.empty(N, dtype=torch.float32, device=points.device)
    _require(out, "out", torch.float32, (N,))
    cf_p, ncomp = None, 0
    if comp_first is not None:
        cf = np.ascontiguousarray(np.asarray(comp_first, dtype=np.int32))
        ncomp = cf.shape[0] - 1
        cf_p = cf.ctypes.data_as(ct.POINTER(ct.c_int32))
    _check(lib.lsdf_sdf_labels(verts.data_ptr(), int(verts.shape[0]), tris.data_ptr(), int(tris.shape[0]), cf_p, ncomp,
                               ct.pointer(grids.desc[index]), grids.buf.data_ptr(),
                               points.data_ptr() if N else None, N, out.data_ptr(), _stream_handle(stream, points.device)))
    return out


def gather_roof(grid: torch.Tensor, n: int, iters: int, threads: int, out: torch.Tensor | None = None,
                stream=None) -> torch.Tensor:
    """Per-thread sums of `iters` random 8-corner cell gathers from an n^3
    FP32 grid (lsdf_gather_roof, a measurement aid)."""
    lib = load_library()
    _require(grid, "grid", torch.float32, (n * n * n,))
    if out is None:
        out = torch.empty(threads, dtype=torch.float32, device=grid.device)
    _require(out, "out", torch.float32, (threads,))
    _check(lib.lsdf_gather_roof(grid.data_ptr(), n, iters, threads, out.data_ptr(), _stream_handle(stream, grid.device)))
    return out

