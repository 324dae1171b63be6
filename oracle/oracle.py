"""ctypes front end of the C oracle (lsdf_oracle.c) plus numpy glue.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg; never by the product library.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lsdf_oracle.c")
LIB = os.path.join(HERE, "liblsdf_oracle.so")

_lib = None

_dp = ct.POINTER(ct.c_double)
_fp = ct.POINTER(ct.c_float)
_ip = ct.POINTER(ct.c_int32)
_lp = ct.POINTER(ct.c_int64)


def build_oracle(force: bool = True) -> str:
    """Compile the oracle with gcc: no fast-math, no FMA contraction."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-std=gnu11", "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        build_oracle()
    lib = ct.CDLL(LIB)
    lib.orc_set_threads.restype = None
    lib.orc_set_threads.argtypes = [ct.c_int32]
    lib.orc_max_threads.restype = ct.c_int32
    lib.orc_max_threads.argtypes = []
    lib.orc_point_triangle_distance.restype = ct.c_double
    lib.orc_point_triangle_distance.argtypes = [_dp, _dp, _dp, _dp]
    lib.orc_winding_number.restype = ct.c_double
    lib.orc_winding_number.argtypes = [_dp, _dp, _ip, ct.c_int32, ct.c_int32]
    lib.orc_mesh_sdf.restype = ct.c_double
    lib.orc_mesh_sdf.argtypes = [_dp, _dp, _ip, _ip, ct.c_int32]
    lib.orc_mesh_sdf_many.restype = None
    lib.orc_mesh_sdf_many.argtypes = [_dp, ct.c_int64, _dp, _ip, _ip, ct.c_int32, _dp]
    lib.orc_build_grid.restype = None
    lib.orc_build_grid.argtypes = [_dp, _ip, _ip, ct.c_int32, _dp, _dp, _ip, _dp]
    lib.orc_fk.restype = None
    lib.orc_fk.argtypes = [_dp, ct.c_int32, _dp, _dp, ct.c_int32, _dp]
    lib.orc_trilinear_f64.restype = ct.c_double
    lib.orc_trilinear_f64.argtypes = [_dp, _ip, _dp]
    lib.orc_query_f64.restype = None
    lib.orc_query_f64.argtypes = [_dp, ct.c_int32, ct.c_int32, _dp, _dp, _ip, _dp, _lp, _dp,
                                  ct.c_int64, _dp]
    lib.orc_query_f64_each.restype = None
    lib.orc_query_f64_each.argtypes = [_dp, ct.c_int32, ct.c_int32, _dp, _dp, _ip, _dp, _lp, _dp, ct.c_int64,
                                       _dp, _dp]
    lib.orc_query_f32.restype = None
    lib.orc_query_f32.argtypes = [_fp, ct.c_int32, ct.c_int32, _fp, _fp, _ip, _fp, _lp, _fp,
                                  ct.c_int64, _fp]
    lib.orc_exact_min.restype = None
    lib.orc_exact_min.argtypes = [_dp, ct.c_int32, ct.c_int32, ct.POINTER(_dp), ct.POINTER(_ip),
                                  ct.POINTER(_ip), _ip, _dp, ct.c_int64, _dp]
    lib.orc_reduce_f64.restype = None
    lib.orc_reduce_f64.argtypes = [_dp, ct.c_int32, ct.c_int32, _dp, _ip]
    lib.orc_reduce_f32.restype = None
    lib.orc_reduce_f32.argtypes = [_fp, ct.c_int32, ct.c_int32, _fp, _ip]
    lib.orc_mlp_nparam.restype = ct.c_int64
    lib.orc_mlp_nparam.argtypes = []
    lib.orc_mlp_forward.restype = None
    lib.orc_mlp_forward.argtypes = [_dp, _dp, ct.c_int64, ct.c_int32, _dp]
    lib.orc_mlp_value.restype = None
    lib.orc_mlp_value.argtypes = [_dp, _dp, ct.c_int64, _dp, _dp, _dp, ct.c_double, ct.c_int32, _dp]
    lib.orc_mlp_loss_grad.restype = ct.c_double
    lib.orc_mlp_loss_grad.argtypes = [_dp, _dp, _dp, _dp, ct.c_int64, ct.c_double, ct.c_int32, _dp]
    lib.orc_adam_step.restype = None
    lib.orc_adam_step.argtypes = [_dp, _dp, _dp, _dp, ct.c_int64, ct.c_int64, ct.c_double, ct.c_double,
                                  ct.c_double, ct.c_double]
    lib.orc_judge_min.restype = None
    lib.orc_judge_min.argtypes = [_dp, ct.c_int32, ct.c_int32, _dp, _dp, _ip, _dp, _lp, ct.POINTER(_dp),
                                  ct.POINTER(_ip), ct.POINTER(_ip), _ip, _dp, _dp, _dp, _dp, _dp, ct.c_int64, _dp]
    lib.orc_query_mlp.restype = None
    lib.orc_query_mlp.argtypes = [_fp, ct.c_int32, ct.c_int32, _fp, _fp, _ip, _fp, _lp, _fp, ct.c_int64, _dp, _dp,
                                  _dp, _dp, _dp, ct.c_double, ct.c_int32, _dp, _dp, _dp]
    lib.orc_query_f32_each.restype = None
    lib.orc_query_f32_each.argtypes = [_fp, ct.c_int32, ct.c_int32, _fp, _fp, _ip, _fp, _lp, _fp, ct.c_int64, _fp,
                                       _fp]
    lib.orc_frnn_nparam.restype = ct.c_int64
    lib.orc_frnn_nparam.argtypes = [ct.c_int32]
    lib.orc_frnn_target.restype = None
    lib.orc_frnn_target.argtypes = [ct.c_int32, _dp, ct.c_int64, _dp]
    lib.orc_frnn_forward.restype = None
    lib.orc_frnn_forward.argtypes = [_dp, ct.c_int32, _dp, ct.c_int64, _dp]
    lib.orc_frnn_loss_grad.restype = ct.c_double
    lib.orc_frnn_loss_grad.argtypes = [_dp, ct.c_int32, _dp, ct.c_int64, _dp]
    lib.orc_align.restype = None
    lib.orc_align.argtypes = [_dp, _dp, ct.c_double, ct.c_int32, _lp, _dp]
    lib.orc_robot_sdf_f64.restype = None
    lib.orc_robot_sdf_f64.argtypes = [_dp, ct.c_int32, ct.c_int32, _dp, _dp, _ip, _dp, _lp, _ip, _dp, ct.c_double,
                                      _ip, _dp]
    lib.orc_voxel_index.restype = ct.c_int64
    lib.orc_voxel_index.argtypes = [_dp, _dp, ct.c_double, _ip]
    lib.orc_robot_sdf_query.restype = None
    lib.orc_robot_sdf_query.argtypes = [_dp, ct.c_int32, _dp, ct.c_double, _ip, _dp, ct.c_int64, _dp]
    _lib = lib
    return lib


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a, typ):
    return a.ctypes.data_as(typ)


# ---------------------------------------------------------------------------
# mesh distance
# ---------------------------------------------------------------------------

def point_triangle_distance(p, a, b, c) -> float:
    lib = load()
    arrs = [_c(x, np.float64) for x in (p, a, b, c)]
    return float(lib.orc_point_triangle_distance(*[_ptr(x, _dp) for x in arrs]))


def winding_number(p, verts, tris, t0=0, t1=None) -> float:
    lib = load()
    p, V, T = _c(p, np.float64), _c(verts, np.float64), _c(tris, np.int32)
    t1 = T.shape[0] if t1 is None else t1
    return float(lib.orc_winding_number(_ptr(p, _dp), _ptr(V, _dp), _ptr(T, _ip), t0, t1))


def set_threads(n: int) -> None:
    """Number of threads of the oracle's OpenMP loops."""
    load().orc_set_threads(int(n))


def max_threads() -> int:
    """Threads the oracle's OpenMP loops use."""
    return int(load().orc_max_threads())


def mesh_sdf(points, verts, tris, comp_first=None) -> np.ndarray:
    """Signed distance of each point [N][3] to a union of closed parts."""
    lib = load()
    P = _c(np.atleast_2d(points), np.float64)
    V, T = _c(verts, np.float64), _c(tris, np.int32)
    cf = _c([0, T.shape[0]] if comp_first is None else comp_first, np.int32)
    out = np.empty(P.shape[0], dtype=np.float64)
    lib.orc_mesh_sdf_many(_ptr(P, _dp), P.shape[0], _ptr(V, _dp), _ptr(T, _ip), _ptr(cf, _ip),
                          cf.shape[0] - 1, _ptr(out, _dp))
    return out


def build_grid(mesh, lo, hi, n) -> np.ndarray:
    """float64 grid [nz][ny][nx] of the link's signed distance at the nodes."""
    lib = load()
    V, T, cf = _c(mesh.verts, np.float64), _c(mesh.tris, np.int32), _c(mesh.comp_first, np.int32)
    lo, hi, n = _c(lo, np.float64), _c(hi, np.float64), _c(n, np.int32)
    out = np.empty(int(n[2]) * int(n[1]) * int(n[0]), dtype=np.float64)
    lib.orc_build_grid(_ptr(V, _dp), _ptr(T, _ip), _ptr(cf, _ip), cf.shape[0] - 1, _ptr(lo, _dp),
                       _ptr(hi, _dp), _ptr(n, _ip), _ptr(out, _dp))
    return out.reshape(int(n[2]), int(n[1]), int(n[0]))


def grid_bound(h) -> float:
    """Largest interpolation error of a 1-Lipschitz field on a cell with
    spacing h: half the cell diagonal (the |r_r|/2 term of Sec. III-B)."""
    h = np.asarray(h, dtype=np.float64)
    return 0.5 * float(np.sqrt((h * h).sum()))


# ---------------------------------------------------------------------------
# kinematics and queries
# ---------------------------------------------------------------------------

def fk(dh, q, base=None) -> np.ndarray:
    """float64 [C][dof+1][3][4] link-to-world poses."""
    lib = load()
    dh = _c(dh, np.float64)
    q = _c(np.atleast_2d(q), np.float64)
    C, dof = q.shape
    base_p = None
    if base is not None:
        base = _c(base, np.float64)
        base_p = _ptr(base, _dp)
    T = np.empty((C, dof + 1, 3, 4), dtype=np.float64)
    lib.orc_fk(_ptr(dh, _dp), dof, base_p, _ptr(q, _dp), C, _ptr(T, _dp))
    return T


def _pack(grids, dtype):
    offs = np.zeros(len(grids), dtype=np.int64)
    tot = 0
    for i, g in enumerate(grids):
        offs[i] = tot
        tot += g.size
    buf = np.concatenate([np.ravel(g).astype(dtype) for g in grids]) if grids else np.zeros(0, dtype)
    return _c(buf, dtype), offs


def query_f64(T, lo, hi, n, grids, points) -> np.ndarray:
    """Per-link minima [C][L] in double (trilinear as a weighted sum)."""
    lib = load()
    T = _c(T, np.float64)
    C, L = T.shape[0], T.shape[1]
    lo, hi, n = _c(lo, np.float64), _c(hi, np.float64), _c(n, np.int32)
    buf, offs = _pack(grids, np.float64)
    P = _c(points, np.float64).reshape(-1, 3)
    out = np.empty((C, L), dtype=np.float64)
    lib.orc_query_f64(_ptr(T, _dp), C, L, _ptr(lo, _dp), _ptr(hi, _dp), _ptr(n, _ip),
                      _ptr(buf, _dp), _ptr(offs, _lp), _ptr(P, _dp), P.shape[0], _ptr(out, _dp))
    return out


def query_f64_each(T, lo, hi, n, grids, points):
    """Every pair of the double query: grid coordinates u [C][L][M][3] (in
    or out of the box) and the trilinear value at u clamped into the box
    [C][L][M] (finite for every pair)."""
    lib = load()
    T = _c(T, np.float64)
    C, L = T.shape[0], T.shape[1]
    lo, hi, n = _c(lo, np.float64), _c(hi, np.float64), _c(n, np.int32)
    buf, offs = _pack(grids, np.float64)
    P = _c(points, np.float64).reshape(-1, 3)
    M = P.shape[0]
    u = np.empty((C, L, M, 3), dtype=np.float64)
    v = np.empty((C, L, M), dtype=np.float64)
    lib.orc_query_f64_each(_ptr(T, _dp), C, L, _ptr(lo, _dp), _ptr(hi, _dp), _ptr(n, _ip), _ptr(buf, _dp),
                           _ptr(offs, _lp), _ptr(P, _dp), M, _ptr(u, _dp), _ptr(v, _dp))
    return u, v


def query_f32(T, lo, hi, n, grids, points) -> np.ndarray:
    """Per-link minima [C][L] in the fixed single-precision operation order."""
    lib = load()
    T = _c(T, np.float32)
    C, L = T.shape[0], T.shape[1]
    lo, hi, n = _c(lo, np.float32), _c(hi, np.float32), _c(n, np.int32)
    buf, offs = _pack(grids, np.float32)
    P = _c(points, np.float32).reshape(-1, 3)
    out = np.empty((C, L), dtype=np.float32)
    lib.orc_query_f32(_ptr(T, _fp), C, L, _ptr(lo, _fp), _ptr(hi, _fp), _ptr(n, _ip),
                      _ptr(buf, _fp), _ptr(offs, _lp), _ptr(P, _fp), P.shape[0], _ptr(out, _fp))
    return out


def query_batched(query, T, lo, hi, n, grids, points, c_off, m_off) -> np.ndarray:
    """Per-link minima [C][L] of a batch of trajectories: trajectory k's
    configurations [c_off[k], c_off[k+1]) against its points [m_off[k],
    m_off[k+1]), one plain query per trajectory (query = query_f32 or
    query_f64).  Offsets are clamped as the library does: c into [0, C] and
    non-decreasing from c_off[k], m likewise into [0, M]; a configuration
    covered by several trajectories takes the minimum over them, and one
    covered by none stays +inf."""
    T = np.asarray(T)
    P = np.asarray(points).reshape(-1, 3)
    C, L, M = T.shape[0], T.shape[1], P.shape[0]
    out = np.full((C, L), np.inf)
    for k in range(len(c_off) - 1):
        c0 = min(max(int(c_off[k]), 0), C)
        c1 = min(max(int(c_off[k + 1]), c0), C)
        m0 = min(max(int(m_off[k]), 0), M)
        m1 = min(max(int(m_off[k + 1]), m0), M)
        if c1 > c0 and m1 > m0:
            part = query(T[c0:c1], lo, hi, n, grids, P[m0:m1])
            out[c0:c1] = np.minimum(out[c0:c1], part)
    return out


# ---------------------------------------------------------------------------
# the paper's Robot-SDF pipeline (Sec. III-A, Eq. 1-4)
# ---------------------------------------------------------------------------

def align(t, env_lo, r, m):
    """Eq. 1-3: block corner k (int64 [3]) and residual shift dt ([3])."""
    lib = load()
    t, lo = _c(t, np.float64), _c(env_lo, np.float64)
    k = np.zeros(3, np.int64)
    dt = np.zeros(3, np.float64)
    lib.orc_align(_ptr(t, _dp), _ptr(lo, _dp), float(r), int(m), _ptr(k, _lp), _ptr(dt, _dp))
    return k, dt


def robot_sdf_f64(T, lo, hi, n, grids, m, env_lo, r, env_n) -> np.ndarray:
    """Robot SDFs [C][N_z][N_y][N_x] in double (Eq. 1-4, per-voxel minimum
    over links); m [L] = block half-widths in voxels."""
    lib = load()
    T = _c(T, np.float64)
    C, L = T.shape[0], T.shape[1]
    lo, hi, n = _c(lo, np.float64), _c(hi, np.float64), _c(n, np.int32)
    buf, offs = _pack(grids, np.float64)
    m = _c(m, np.int32)
    elo, en = _c(env_lo, np.float64), _c(env_n, np.int32)
    out = np.empty((C, int(en[2]), int(en[1]), int(en[0])), dtype=np.float64)
    lib.orc_robot_sdf_f64(_ptr(T, _dp), C, L, _ptr(lo, _dp), _ptr(hi, _dp), _ptr(n, _ip), _ptr(buf, _dp),
                          _ptr(offs, _lp), _ptr(m, _ip), _ptr(elo, _dp), float(r), _ptr(en, _ip), _ptr(out, _dp))
    return out


def voxel_index(x, env_lo, r, env_n) -> int:
    lib = load()
    x, lo, en = _c(x, np.float64), _c(env_lo, np.float64), _c(env_n, np.int32)
    return int(lib.orc_voxel_index(_ptr(x, _dp), _ptr(lo, _dp), float(r), _ptr(en, _ip)))


def robot_sdf_query(rs, env_lo, r, env_n, points) -> np.ndarray:
    """Runtime of the pipeline: per configuration, the minimum of its Robot
    SDF over the voxels the points occupy."""
    lib = load()
    rs = _c(rs, np.float64)
    C = rs.shape[0]
    lo, en = _c(env_lo, np.float64), _c(env_n, np.int32)
    P = _c(points, np.float64).reshape(-1, 3)
    out = np.empty(C, dtype=np.float64)
    lib.orc_robot_sdf_query(_ptr(rs, _dp), C, _ptr(lo, _dp), float(r), _ptr(en, _ip), _ptr(P, _dp), P.shape[0],
                            _ptr(out, _dp))
    return out


def voxel_centres(env_lo, r, env_n, flat_index) -> np.ndarray:
    """float32 centres lo + (v + 1/2) r of the given flat voxel indices
    (computed in double, rounded once)."""
    en = np.asarray(env_n, dtype=np.int64)
    idx = np.asarray(flat_index, dtype=np.int64)
    v = np.stack([idx % en[0], (idx // en[0]) % en[1], idx // (en[0] * en[1])], axis=-1).astype(np.float64)
    return (np.asarray(env_lo, np.float64) + (v + 0.5) * float(r)).astype(np.float32)


def query_f32_each(T, lo, hi, n, grids, points) -> np.ndarray:
    """Every pair's value [C][L][M] in the single-precision twin's order
    (+inf outside the box)."""
    lib = load()
    T = _c(T, np.float32)
    C, L = T.shape[0], T.shape[1]
    lo, hi, n = _c(lo, np.float32), _c(hi, np.float32), _c(n, np.int32)
    buf, offs = _pack(grids, np.float32)
    P = _c(points, np.float32).reshape(-1, 3)
    out = np.empty((C, L), dtype=np.float32)
    each = np.empty((C, L, P.shape[0]), dtype=np.float32)
    lib.orc_query_f32_each(_ptr(T, _fp), C, L, _ptr(lo, _fp), _ptr(hi, _fp), _ptr(n, _ip), _ptr(buf, _fp),
                           _ptr(offs, _lp), _ptr(P, _fp), P.shape[0], _ptr(out, _fp), _ptr(each, _fp))
    return each


# ---------------------------------------------------------------------------
# the paper's tiny network for the grid transformation (Sec. III-B-1)
# ---------------------------------------------------------------------------

FRNN_HIDDEN = 32


def frnn_nparam(m: int) -> int:
    return int(load().orc_frnn_nparam(int(m)))


def frnn_target(m: int, R) -> np.ndarray:
    """Exact R^T P_j for rotations R [N][3][3]: [N][3 V] (o = 3 j + a)."""
    lib = load()
    R = _c(np.asarray(R).reshape(-1, 9), np.float64)
    V = (2 * m) ** 3
    out = np.empty((R.shape[0], 3 * V), dtype=np.float64)
    lib.orc_frnn_target(int(m), _ptr(R, _dp), R.shape[0], _ptr(out, _dp))
    return out


def frnn_forward(params, m: int, R) -> np.ndarray:
    lib = load()
    P = _c(params, np.float64)
    R = _c(np.asarray(R).reshape(-1, 9), np.float64)
    V = (2 * m) ** 3
    out = np.empty((R.shape[0], 3 * V), dtype=np.float64)
    lib.orc_frnn_forward(_ptr(P, _dp), int(m), _ptr(R, _dp), R.shape[0], _ptr(out, _dp))
    return out


def frnn_loss_grad(params, m: int, R):
    """(mean absolute error against R^T P, gradient [nparam])."""
    lib = load()
    P = _c(params, np.float64)
    R = _c(np.asarray(R).reshape(-1, 9), np.float64)
    g = np.empty(P.shape[0], dtype=np.float64)
    loss = lib.orc_frnn_loss_grad(_ptr(P, _dp), int(m), _ptr(R, _dp), R.shape[0], _ptr(g, _dp))
    return float(loss), g


def exact_min(T, meshes, points) -> np.ndarray:
    """Grid-free per-link minima [C][L]: exact mesh SDF at every point."""
    lib = load()
    T = _c(T, np.float64)
    C, L = T.shape[0], T.shape[1]
    Vs = [_c(m.verts, np.float64) for m in meshes]
    Ts = [_c(m.tris, np.int32) for m in meshes]
    Cs = [_c(m.comp_first, np.int32) for m in meshes]
    nc = _c([m.comp_first.shape[0] - 1 for m in meshes], np.int32)
    Vp = (_dp * L)(*[_ptr(v, _dp) for v in Vs])
    Tp = (_ip * L)(*[_ptr(t, _ip) for t in Ts])
    Cp = (_ip * L)(*[_ptr(c, _ip) for c in Cs])
    P = _c(points, np.float64).reshape(-1, 3)
    out = np.empty((C, L), dtype=np.float64)
    lib.orc_exact_min(_ptr(T, _dp), C, L, Vp, Tp, Cp, _ptr(nc, _ip), _ptr(P, _dp), P.shape[0],
                      _ptr(out, _dp))
    return out


def judge_min(T, lo, hi, n, grids, meshes, dom_c, dom_h, points) -> np.ndarray:
    """Per-link minima [C][L] of the judge field of the learned surrogate:
    grid value inside each link's box, exact mesh distance outside it, over
    the points inside each link's network domain."""
    lib = load()
    T = _c(T, np.float64)
    C, L = T.shape[0], T.shape[1]
    lo, hi, n = _c(lo, np.float64), _c(hi, np.float64), _c(n, np.int32)
    buf, offs = _pack(grids, np.float64)
    Vs = [_c(m.verts, np.float64) for m in meshes]
    Ts = [_c(m.tris, np.int32) for m in meshes]
    Cs = [_c(m.comp_first, np.int32) for m in meshes]
    nc = _c([m.comp_first.shape[0] - 1 for m in meshes], np.int32)
    alo = _c([m.verts.min(axis=0) for m in meshes], np.float64)
    ahi = _c([m.verts.max(axis=0) for m in meshes], np.float64)
    dc, dh = _c(dom_c, np.float64), _c(dom_h, np.float64)
    Vp = (_dp * L)(*[_ptr(v, _dp) for v in Vs])
    Tp = (_ip * L)(*[_ptr(t, _ip) for t in Ts])
    Cp = (_ip * L)(*[_ptr(c, _ip) for c in Cs])
    P = _c(points, np.float64).reshape(-1, 3)
    out = np.empty((C, L), dtype=np.float64)
    lib.orc_judge_min(_ptr(T, _dp), C, L, _ptr(lo, _dp), _ptr(hi, _dp), _ptr(n, _ip), _ptr(buf, _dp),
                      _ptr(offs, _lp), Vp, Tp, Cp, _ptr(nc, _ip), _ptr(alo, _dp), _ptr(ahi, _dp), _ptr(dc, _dp),
                      _ptr(dh, _dp), _ptr(P, _dp), P.shape[0], _ptr(out, _dp))
    return out


def query_mlp(T, lo, hi, n, grids, points, params, dom_c, dom_h, margin, bf16=True, each=False, core_k=None,
              bounds=None):
    """Per-link minima [C][L] of the learned clearance with its margin
    fallback: the surrogate's estimate per in-domain pair (the network plus
    the distance to the core box of half extents core_k [L][3] centred on the
    domain; core_k None: the network alone; with bounds [L], the network's
    share is bounds[i] tanh(m / bounds[i])), replaced by the single-
    precision twin's grid value when it is below the margin and the point is
    in the grid box.  With each=True also returns the per-pair estimates
    (evaluated for every pair, in the domain or not) and twin grid values
    (+inf outside the box), [C][L][M]."""
    lib = load()
    T = _c(T, np.float32)
    C, L = T.shape[0], T.shape[1]
    lo, hi, n = _c(lo, np.float32), _c(hi, np.float32), _c(n, np.int32)
    buf, offs = _pack(grids, np.float32)
    P = _c(points, np.float32).reshape(-1, 3)
    M = P.shape[0]
    prm = _c(params, np.float64).reshape(L, -1)
    dc, dh = _c(dom_c, np.float64).reshape(L, 3), _c(dom_h, np.float64).reshape(L, 3)
    out = np.empty((C, L), dtype=np.float64)
    em = np.empty((C, L, M), dtype=np.float64) if each else None
    eg = np.empty((C, L, M), dtype=np.float64) if each else None
    null = ct.POINTER(ct.c_double)()
    ck = None if core_k is None else _c(core_k, np.float64).reshape(L, 3)
    bd = None if bounds is None else _c(np.broadcast_to(np.asarray(bounds, dtype=np.float64), (L,)), np.float64)
    lib.orc_query_mlp(_ptr(T, _fp), C, L, _ptr(lo, _fp), _ptr(hi, _fp), _ptr(n, _ip), _ptr(buf, _fp),
                      _ptr(offs, _lp), _ptr(P, _fp), M, _ptr(prm, _dp), _ptr(dc, _dp), _ptr(dh, _dp),
                      null if ck is None else _ptr(ck, _dp), null if bd is None else _ptr(bd, _dp), float(margin), int(bool(bf16)), _ptr(out, _dp),
                      _ptr(em, _dp) if each else null, _ptr(eg, _dp) if each else null)
    return (out, em, eg) if each else out


def reduce(cl):
    """Per configuration: (min over links, lowest argmin link or -1)."""
    lib = load()
    C, L = cl.shape
    link = np.empty(C, dtype=np.int32)
    if cl.dtype == np.float32:
        cl = _c(cl, np.float32)
        d = np.empty(C, dtype=np.float32)
        lib.orc_reduce_f32(_ptr(cl, _fp), C, L, _ptr(d, _fp), _ptr(link, _ip))
    else:
        cl = _c(cl, np.float64)
        d = np.empty(C, dtype=np.float64)
        lib.orc_reduce_f64(_ptr(cl, _dp), C, L, _ptr(d, _dp), _ptr(link, _ip))
    return d, link


def trilinear_f64(grid, u) -> float:
    lib = load()
    g = _c(grid, np.float64)
    n = _c([g.shape[2], g.shape[1], g.shape[0]], np.int32)
    u = _c(u, np.float64)
    return float(lib.orc_trilinear_f64(_ptr(g, _dp), _ptr(n, _ip), _ptr(u, _dp)))


def workload_grids(w, dtype=np.float64):
    """Oracle grids for every link of a synthetic workload."""
    return [build_grid(m, w.grid_lo[i].astype(np.float64), w.grid_hi[i].astype(np.float64),
                       w.grid_n[i]).astype(dtype)
            for i, m in enumerate(w.robot.links)]


# ---------------------------------------------------------------------------
# learned per-link SDF (MLP 3 -> 128 -> 128 -> 128 -> 1, SiLU)
# ---------------------------------------------------------------------------

MLP_HIDDEN = 128


def mlp_nparam() -> int:
    return int(load().orc_mlp_nparam())


def mlp_forward(params, X, bf16: bool = False) -> np.ndarray:
    """Network output at normalised inputs X [N][3]; bf16=True rounds weights
    and activations to bfloat16 where the GPU kernels do."""
    lib = load()
    P = _c(params, np.float64)
    X = _c(np.atleast_2d(X), np.float64)
    out = np.empty(X.shape[0], dtype=np.float64)
    lib.orc_mlp_forward(_ptr(P, _dp), _ptr(X, _dp), X.shape[0], int(bf16), _ptr(out, _dp))
    return out


def mlp_value(params, points, dom_c, dom_h, core_k=None, bf16: bool = False, bound=np.inf) -> np.ndarray:
    """The surrogate's estimate at link-frame points [N][3] of one link: the
    network m at (l - dom_c) / dom_h, bounded (bound tanh(m / bound); bound
    = inf: m), plus the distance from l to the core box |l - dom_c| <= core_k
    (core_k None: no core term)."""
    lib = load()
    P = _c(params, np.float64)
    X = _c(np.atleast_2d(points), np.float64)
    dc, dh = _c(dom_c, np.float64).reshape(3), _c(dom_h, np.float64).reshape(3)
    ck = None if core_k is None else _c(core_k, np.float64).reshape(3)
    out = np.empty(X.shape[0], dtype=np.float64)
    lib.orc_mlp_value(_ptr(P, _dp), _ptr(X, _dp), X.shape[0], _ptr(dc, _dp), _ptr(dh, _dp),
                      ct.POINTER(ct.c_double)() if ck is None else _ptr(ck, _dp), float(bound), int(bf16),
                      _ptr(out, _dp))
    return out


def mlp_loss_grad(params, X, Y, bf16: bool = False, offset=None, bound=np.inf):
    """(mean absolute error, gradient [nparam]) of the estimate
    bounded(network(X)) + offset (per sample; None: none) against Y, where
    bounded(m) = bound tanh(m / bound) (bound = inf: m)."""
    lib = load()
    P = _c(params, np.float64)
    X = _c(np.atleast_2d(X), np.float64)
    Y = _c(Y, np.float64)
    D = None if offset is None else _c(offset, np.float64)
    g = np.empty(P.shape[0], dtype=np.float64)
    loss = lib.orc_mlp_loss_grad(_ptr(P, _dp), _ptr(X, _dp), ct.POINTER(ct.c_double)() if D is None else _ptr(D, _dp),
                                 _ptr(Y, _dp), X.shape[0], float(bound), int(bf16), _ptr(g, _dp))
    return float(loss), g


def adam_step(params, m, v, grad, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam update of float64 arrays params, m, v."""
    lib = load()
    for a in (params, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _c(grad, np.float64)
    lib.orc_adam_step(_ptr(params, _dp), _ptr(m, _dp), _ptr(v, _dp), _ptr(g, _dp), params.shape[0], int(t),
                      float(lr), float(beta1), float(beta2), float(eps))


def mlp_unpack(params):
    """Views of the parameter vector: W1[128][3], b1, W2[128][128], b2, W3, b3, w4, b4."""
    H = MLP_HIDDEN
    P = np.asarray(params)
    o = 0
    out = []
    for shape in ((H, 3), (H,), (H, H), (H,), (H, H), (H,), (H,), (1,)):
        n = int(np.prod(shape))
        out.append(P[o:o + n].reshape(shape))
        o += n
    return out


__all__ = ["FRNN_HIDDEN", "frnn_forward", "frnn_loss_grad", "frnn_nparam", "frnn_target", "align", "robot_sdf_f64", "robot_sdf_query", "voxel_centres", "voxel_index", "build_grid", "exact_min", "fk", "grid_bound", "mesh_sdf", "point_triangle_distance",
           "query_batched", "query_f32", "query_f32_each", "query_f64", "query_f64_each", "query_mlp", "reduce", "trilinear_f64", "winding_number", "workload_grids",
           "MLP_HIDDEN", "adam_step", "judge_min", "mlp_forward", "mlp_loss_grad", "mlp_value", "mlp_nparam", "mlp_unpack",
           "max_threads", "set_threads"]
