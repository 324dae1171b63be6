"""Host-side checks of liblsdf.so that need no GPU: the library loads, exports
every entry point include/lsdf.h declares, and rejects bad arguments with the
documented status codes before anything reaches the device."""
import ctypes as ct
import os
import re
import shutil

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lsdf.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2309_12543_amd import lsdf
    if not os.path.exists(lsdf.LIB_PATH):
        if shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"):
            pytest.skip("liblsdf.so is not built and hipcc is unavailable")
        from paper_2309_12543_amd import build
        build.build()
    return lsdf.load_library()


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lsdf_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol(lib):
    syms = declared_symbols()
    assert "lsdf_query_min_distance" in syms and "lsdf_fk_batch" in syms and "lsdf_build_link_sdf" in syms
    for s in syms:
        assert hasattr(lib, s), f"{s} declared in lsdf.h but not exported"


def test_version_and_error_string(lib):
    assert lib.lsdf_version() >= 0x000100
    assert isinstance(lib.lsdf_last_error(), bytes)


def grid_array(L=2, n=8, dtype=0):
    from paper_2309_12543_amd.lsdf import lsdf_grid
    arr = (lsdf_grid * L)()
    for i in range(L):
        for a in range(3):
            arr[i].lo[a] = -0.5
            arr[i].hi[a] = 0.5
            arr[i].n[a] = n
        arr[i].dtype = dtype
        arr[i].elem_offset = i * n ** 3
    return arr


FAKE = ct.c_void_p(0x100000)      # never dereferenced: every case fails validation first


def call_query(lib, C=4, L=2, grids="default", M=10, flags=0, ws=0x100000, ws_bytes=1 << 20, points=FAKE):
    g = grid_array(L) if grids == "default" else grids
    return lib.lsdf_query_min_distance(FAKE, C, L, g, FAKE, points, M, FAKE, FAKE, None, flags,
                                       ct.c_void_p(ws) if ws else None, ws_bytes, None)


def test_query_argument_errors(lib):
    from paper_2309_12543_amd import lsdf as B
    assert call_query(lib, flags=1) == B.LSDF_E_UNSUPPORTED
    assert call_query(lib, L=0) == B.LSDF_E_SHAPE
    assert call_query(lib, L=17, grids=grid_array(16)) == B.LSDF_E_SHAPE
    assert call_query(lib, C=-1) == B.LSDF_E_SHAPE
    assert call_query(lib, M=-5) == B.LSDF_E_SHAPE
    assert call_query(lib, grids=None) == B.LSDF_E_INVALID_ARG
    assert call_query(lib, ws=0) == B.LSDF_E_INVALID_ARG
    assert call_query(lib, ws=0x100004) == B.LSDF_E_INVALID_ARG          # not 256-byte aligned
    assert call_query(lib, ws_bytes=16) == B.LSDF_E_SHAPE
    assert call_query(lib, points=None) == B.LSDF_E_INVALID_ARG
    assert b"points" in lib.lsdf_last_error()
    bad = grid_array(2)
    bad[1].n[2] = 1
    assert call_query(lib, grids=bad) == B.LSDF_E_SHAPE
    bad = grid_array(2)
    bad[0].hi[0] = -0.5
    assert call_query(lib, grids=bad) == B.LSDF_E_INVALID_ARG
    bad = grid_array(2)
    bad[0].lo[1] = float("nan")
    assert call_query(lib, grids=bad) == B.LSDF_E_INVALID_ARG
    assert call_query(lib, grids=grid_array(2, dtype=7)) == B.LSDF_E_UNSUPPORTED
    # C = 0 is a successful no-op
    assert call_query(lib, C=0) == B.LSDF_OK


def test_noalloc_query_rejects_before_touching_the_device(lib):
    """The entry point without a workspace checks its arguments and the size
    of the problem against the scratch the library holds before any device
    call, so these run without a GPU."""
    from paper_2309_12543_amd import lsdf as B

    def call(C=500, L=7, M=20000, flags=0):
        return lib.lsdf_query_min_distance_noalloc(FAKE, C, L, grid_array(L), FAKE, FAKE, M, FAKE, FAKE, None,
                                                   flags, None)
    assert call(flags=1) == B.LSDF_E_UNSUPPORTED
    assert call(L=0) == B.LSDF_E_SHAPE
    assert call(C=-1) == B.LSDF_E_SHAPE
    assert call(C=0) == B.LSDF_OK
    n = ct.c_size_t(0)
    M_big = 4_000_000
    assert lib.lsdf_query_workspace_size(500, 7, M_big, 0, ct.byref(n)) == 0
    assert n.value > B.LSDF_QUERY_NOALLOC_SCRATCH
    assert call(M=M_big) == B.LSDF_E_SHAPE
    assert b"needs" in lib.lsdf_last_error()
    assert lib.lsdf_query_workspace_size(500, 7, 3_000_000, 0, ct.byref(n)) == 0
    assert n.value <= B.LSDF_QUERY_NOALLOC_SCRATCH        # the example the header gives fits


def test_workspace_size(lib):
    n = ct.c_size_t(0)
    assert lib.lsdf_query_workspace_size(500, 7, 20000, 0, ct.byref(n)) == 0
    assert n.value >= 500 * 7 * 4 and n.value % 256 == 0
    assert lib.lsdf_query_workspace_size(500, 0, 20000, 0, ct.byref(n)) != 0
    assert lib.lsdf_query_workspace_size(500, 7, 20000, 0, None) != 0
    assert lib.lsdf_query_workspace_size(500, 7, 20000, 1, ct.byref(n)) == -3      # LSDF_E_UNSUPPORTED


def test_fk_argument_errors(lib):
    from paper_2309_12543_amd import lsdf as B
    rows = (B.lsdf_dh * 6)()
    assert lib.lsdf_fk_batch(None, 6, None, FAKE, 10, FAKE, None) == B.LSDF_E_INVALID_ARG
    assert lib.lsdf_fk_batch(rows, 0, None, FAKE, 10, FAKE, None) == B.LSDF_E_SHAPE
    assert lib.lsdf_fk_batch(rows, 16, None, FAKE, 10, FAKE, None) == B.LSDF_E_SHAPE
    assert lib.lsdf_fk_batch(rows, 6, None, None, 10, FAKE, None) == B.LSDF_E_INVALID_ARG
    assert lib.lsdf_fk_batch(rows, 6, None, FAKE, -1, FAKE, None) == B.LSDF_E_SHAPE
    rows[2].a = float("inf")
    assert lib.lsdf_fk_batch(rows, 6, None, FAKE, 10, FAKE, None) == B.LSDF_E_INVALID_ARG
    rows[2].a = 0.0
    assert lib.lsdf_fk_batch(rows, 6, None, FAKE, 0, FAKE, None) == B.LSDF_OK


def test_build_argument_errors(lib):
    from paper_2309_12543_amd import lsdf as B
    g = grid_array(1)
    cf = (ct.c_int32 * 3)(0, 5, 12)
    assert lib.lsdf_build_link_sdf(FAKE, 8, FAKE, 12, cf, 2, None, FAKE, None) == B.LSDF_E_INVALID_ARG
    assert lib.lsdf_build_link_sdf(FAKE, 0, FAKE, 12, cf, 2, g, FAKE, None) == B.LSDF_E_SHAPE
    assert lib.lsdf_build_link_sdf(None, 8, FAKE, 12, cf, 2, g, FAKE, None) == B.LSDF_E_INVALID_ARG
    bad = (ct.c_int32 * 3)(0, 5, 11)                       # does not end at nt
    assert lib.lsdf_build_link_sdf(FAKE, 8, FAKE, 12, bad, 2, g, FAKE, None) == B.LSDF_E_SHAPE
    bad = (ct.c_int32 * 3)(0, 0, 12)                       # empty part
    assert lib.lsdf_build_link_sdf(FAKE, 8, FAKE, 12, bad, 2, g, FAKE, None) == B.LSDF_E_SHAPE
    assert lib.lsdf_build_link_sdf(FAKE, 8, FAKE, 12, cf, 17, g, FAKE, None) == B.LSDF_E_SHAPE


def test_mlp_argument_errors(lib):
    from paper_2309_12543_amd import lsdf as B
    n = ct.c_size_t(0)
    assert lib.lsdf_mlp_train_workspace_size(7, 4096, ct.byref(n)) == 0 and n.value > 7 * 4096 * 128 * 4
    assert lib.lsdf_mlp_train_workspace_size(7, 1000, ct.byref(n)) == B.LSDF_E_SHAPE     # not a multiple of 512
    assert lib.lsdf_mlp_train_workspace_size(0, 4096, ct.byref(n)) == B.LSDF_E_SHAPE
    dom = B.make_domains([[0, 0, 0], [0, 0, 0]], [[1, 1, 1], [1, 1, 1]], [[0.2, 0.1, 0], [0, 0, 0]])
    bad = B.make_domains([[0, 0, 0]], [[1, 0, 1]], [[0, 0, 0]])
    bad_core = B.make_domains([[0, 0, 0]], [[1, 1, 1]], [[0, -0.1, 0]])
    nan_core = B.make_domains([[0, 0, 0]], [[1, 1, 1]], [[0, float("nan"), 0]])
    with pytest.raises(ValueError):
        B.make_domains([[0, 0, 0]], [[1, 1, 1]], [[0, 0, 0], [0, 0, 0]])         # shapes differ
    # lsdf_mlp_eval: domain NULL, half <= 0, core_half < 0 or NaN, N < 0, N = 0 no-op
    assert lib.lsdf_mlp_eval(FAKE, None, FAKE, 10, FAKE, None) == B.LSDF_E_INVALID_ARG
    assert lib.lsdf_mlp_eval(FAKE, bad, FAKE, 10, FAKE, None) == B.LSDF_E_INVALID_ARG
    assert lib.lsdf_mlp_eval(FAKE, bad_core, FAKE, 10, FAKE, None) == B.LSDF_E_INVALID_ARG
    assert lib.lsdf_mlp_eval(FAKE, nan_core, FAKE, 10, FAKE, None) == B.LSDF_E_INVALID_ARG
    for bad_bound in (0.0, -0.1, float("nan")):   # the remainder bound: > 0 or +inf
        d = B.make_domains([[0, 0, 0]], [[1, 1, 1]], [[0, 0, 0]], bad_bound)
        assert lib.lsdf_mlp_eval(FAKE, d, FAKE, 10, FAKE, None) == B.LSDF_E_INVALID_ARG, bad_bound
    for ok_bound in (0.05, float("inf")):
        d = B.make_domains([[0, 0, 0]], [[1, 1, 1]], [[0, 0, 0]], ok_bound)
        assert lib.lsdf_mlp_eval(FAKE, d, FAKE, 0, FAKE, None) == B.LSDF_OK, ok_bound
    assert lib.lsdf_mlp_eval(FAKE, dom, FAKE, -1, FAKE, None) == B.LSDF_E_SHAPE
    assert lib.lsdf_mlp_eval(FAKE, dom, FAKE, 0, FAKE, None) == B.LSDF_OK
    # training: B not a multiple of 512, NULL moments, t = 0, workspace too small or misaligned
    args = lambda Bt=512, t=1, m=FAKE, ws=FAKE, wsb=1 << 30: (
        FAKE, m, FAKE, t, 1e-3, 0.9, 0.999, 1e-8, dom, 2, FAKE, FAKE, 1024, None, Bt, None, None, ws, wsb, None)
    assert lib.lsdf_mlp_train_step(*args(Bt=500)) == B.LSDF_E_SHAPE
    assert lib.lsdf_mlp_train_step(*args(m=None)) == B.LSDF_E_INVALID_ARG
    assert lib.lsdf_mlp_train_step(*args(t=0)) == B.LSDF_E_INVALID_ARG
    assert lib.lsdf_mlp_train_step(*args(wsb=16)) == B.LSDF_E_SHAPE
    assert lib.lsdf_mlp_train_step(*args(ws=ct.c_void_p(0x100010))) == B.LSDF_E_INVALID_ARG
    assert lib.lsdf_mlp_loss_grad(FAKE, dom, 2, FAKE, FAKE, 1024, None, 512, None, None, FAKE, 1 << 30, None) \
        == B.LSDF_E_INVALID_ARG                                                      # grad_out NULL
    # learned query: margin NaN, NULL domains, flags
    g = grid_array(2)
    q = lambda margin=0.05, doms=dom, flags=0: lib.lsdf_query_min_distance_mlp(
        FAKE, 4, 2, g, FAKE, FAKE, doms, margin, FAKE, 10, FAKE, FAKE, None, flags, FAKE, 1 << 20, None)
    assert q(margin=float("nan")) == B.LSDF_E_INVALID_ARG
    assert q(doms=None) == B.LSDF_E_INVALID_ARG
    assert q(flags=2) == B.LSDF_E_UNSUPPORTED
    # labels: empty mesh, NULL descriptor
    assert lib.lsdf_sdf_labels(FAKE, 0, FAKE, 12, None, 0, g, FAKE, FAKE, 10, FAKE, None) == B.LSDF_E_SHAPE
    assert lib.lsdf_sdf_labels(FAKE, 8, FAKE, 12, None, 0, None, FAKE, FAKE, 10, FAKE, None) == B.LSDF_E_INVALID_ARG


def test_batched_query_argument_errors(lib):
    from paper_2309_12543_amd import lsdf as B
    g = grid_array(2)

    def q(K=3, c_off=FAKE, m_off=FAKE, C=4, M=10, tuning=None, ws=0x100000, ws_bytes=1 << 20, flags=0):
        return lib.lsdf_query_min_distance_batched(K, c_off, m_off, FAKE, C, 2, g, FAKE, FAKE, M, FAKE, FAKE, None,
                                                   tuning, flags, ct.c_void_p(ws) if ws else None, ws_bytes, None)
    assert q(K=0) == B.LSDF_E_SHAPE
    assert q(K=65537) == B.LSDF_E_SHAPE
    assert q(c_off=None) == B.LSDF_E_INVALID_ARG
    assert q(m_off=None) == B.LSDF_E_INVALID_ARG
    assert q(flags=4) == B.LSDF_E_UNSUPPORTED
    assert q(M=(1 << 34) + 1) == B.LSDF_E_SHAPE
    for bad in [(12, 0), (4, 0), (8200, 0), (0, 17), (0, -1), (0, 0, 3), (0, 0, -1)]:
        assert q(tuning=ct.byref(B.make_tuning(*bad))) == B.LSDF_E_INVALID_ARG, bad
    assert b"schedule" in lib.lsdf_last_error()
    t = B.make_tuning(32, 8, 1)
    t.reserved = 1
    assert q(tuning=ct.byref(t)) == B.LSDF_E_INVALID_ARG
    # the plan of K trajectories lives in the workspace: K = 3 fits where K = 60000 does not
    n = ct.c_size_t(0)
    assert lib.lsdf_query_batched_workspace_size(3, 4, 2, 10, ct.byref(n)) == 0
    assert q(K=60000, ws_bytes=n.value) == B.LSDF_E_SHAPE
    assert q(ws=0x100008) == B.LSDF_E_INVALID_ARG
    # C = 0 is a successful no-op
    assert q(C=0) == B.LSDF_OK


def test_batched_workspace_size(lib):
    n1, nk = ct.c_size_t(0), ct.c_size_t(0)
    assert lib.lsdf_query_workspace_size(500, 7, 20000, 0, ct.byref(n1)) == 0
    assert lib.lsdf_query_batched_workspace_size(1, 500, 7, 20000, ct.byref(nk)) == 0
    assert n1.value == nk.value
    assert lib.lsdf_query_batched_workspace_size(64, 500, 7, 20000, ct.byref(nk)) == 0
    assert nk.value > n1.value and nk.value % 256 == 0
    assert lib.lsdf_query_batched_workspace_size(0, 500, 7, 20000, ct.byref(nk)) != 0


def test_autotune_argument_errors(lib):
    from paper_2309_12543_amd import lsdf as B
    g = grid_array(2)
    best = B.lsdf_query_tuning()

    def a(cands=None, n=0, reps=3, best_p=True, c_off=FAKE):
        return lib.lsdf_query_autotune(2, c_off, FAKE, FAKE, 4, 2, g, FAKE, FAKE, 10, FAKE, FAKE, cands, n, reps,
                                       FAKE, 1 << 20, None, ct.byref(best) if best_p else None, None)
    assert a(best_p=False) == B.LSDF_E_INVALID_ARG
    assert a(reps=0) == B.LSDF_E_INVALID_ARG
    assert a(c_off=None) == B.LSDF_E_INVALID_ARG
    arr = (B.lsdf_query_tuning * 2)(B.make_tuning(32, 8), B.make_tuning(9, 8))
    assert a(cands=arr, n=2) == B.LSDF_E_INVALID_ARG          # 9 is not a multiple of 8
    assert a(cands=arr, n=0) == B.LSDF_E_INVALID_ARG


def test_set_kernel_events_arguments(lib):
    from paper_2309_12543_amd import lsdf as B
    assert lib.lsdf_set_kernel_events(FAKE, None) == B.LSDF_E_INVALID_ARG
    assert lib.lsdf_set_kernel_events(None, FAKE) == B.LSDF_E_INVALID_ARG
    assert lib.lsdf_set_kernel_events(None, None) == B.LSDF_OK


def test_query_from_joints_argument_errors(lib):
    from paper_2309_12543_amd import lsdf as B
    rows = (B.lsdf_dh * 6)()
    g = grid_array(7)

    def f(dh=rows, dof=6, q=FAKE, K=1, co=None, mo=None, C=4, M=10):
        return lib.lsdf_query_from_joints(dh, dof, None, q, K, co, mo, C, g, FAKE, FAKE, M, None, FAKE, FAKE, None,
                                          None, 0, FAKE, 1 << 20, None)
    assert f(dh=None) == B.LSDF_E_INVALID_ARG
    assert f(dof=0) == B.LSDF_E_SHAPE
    assert f(dof=16) == B.LSDF_E_SHAPE
    assert f(co=FAKE) == B.LSDF_E_INVALID_ARG          # one offset array without the other
    assert f(K=2) == B.LSDF_E_SHAPE                    # K > 1 needs offset arrays
    assert f(q=None) == B.LSDF_E_INVALID_ARG
    assert f(C=0) == B.LSDF_OK


def test_robot_sdf_argument_errors(lib):
    from paper_2309_12543_amd import lsdf as B
    env = B.make_env((-2, -2, -2), 1 / 32, (128, 128, 128))
    n = ct.c_size_t(0)
    assert lib.lsdf_robot_sdf_size(500, ct.byref(env), ct.byref(n)) == 0 and n.value == 500 * 128 ** 3 * 4
    bad = B.make_env((-2, -2, -2), 0.0, (128, 128, 128))
    assert lib.lsdf_robot_sdf_size(5, ct.byref(bad), ct.byref(n)) == B.LSDF_E_INVALID_ARG
    bad = B.make_env((-2, float("nan"), -2), 0.1, (8, 8, 8))
    assert lib.lsdf_robot_sdf_size(5, ct.byref(bad), ct.byref(n)) == B.LSDF_E_INVALID_ARG
    bad = B.make_env((-2, -2, -2), 0.1, (8, 0, 8))
    assert lib.lsdf_robot_sdf_size(5, ct.byref(bad), ct.byref(n)) == B.LSDF_E_SHAPE
    assert lib.lsdf_robot_sdf_size(5, None, ct.byref(n)) == B.LSDF_E_INVALID_ARG
    g = grid_array(2)
    assert lib.lsdf_robot_sdf_build_workspace_size(4, 2, ct.byref(n)) == 0
    assert lib.lsdf_robot_sdf_build(FAKE, 4, 2, g, FAKE, ct.byref(env), FAKE, FAKE, 16, None) == B.LSDF_E_SHAPE
    assert lib.lsdf_robot_sdf_build(FAKE, 4, 2, None, FAKE, ct.byref(env), FAKE, FAKE, n.value, None) \
        == B.LSDF_E_INVALID_ARG
    assert lib.lsdf_robot_sdf_build(FAKE, 4, 17, g, FAKE, ct.byref(env), FAKE, FAKE, n.value, None) == B.LSDF_E_SHAPE
    assert lib.lsdf_robot_sdf_build(FAKE, 0, 2, g, FAKE, ct.byref(env), FAKE, FAKE, n.value, None) == B.LSDF_OK
    assert lib.lsdf_robot_sdf_query_workspace_size(ct.byref(env), 1000, ct.byref(n)) == 0
    assert lib.lsdf_robot_sdf_query(FAKE, 4, ct.byref(env), FAKE, 1000, FAKE, FAKE, 16, None) == B.LSDF_E_SHAPE
    assert lib.lsdf_robot_sdf_query(FAKE, 4, ct.byref(env), None, 1000, FAKE, FAKE, n.value, None) \
        == B.LSDF_E_INVALID_ARG
    assert lib.lsdf_robot_sdf_query(FAKE, 0, ct.byref(env), FAKE, 1000, FAKE, FAKE, n.value, None) == B.LSDF_OK


def test_frnn_argument_errors(lib):
    from paper_2309_12543_amd import lsdf as B
    n = ct.c_int64(0)
    assert lib.lsdf_frnn_nparam(2, ct.byref(n)) == 0 and n.value == 32 * 9 + 32 + 3 * 64 * 32 + 3 * 64
    assert lib.lsdf_frnn_nparam(0, ct.byref(n)) == B.LSDF_E_SHAPE
    assert lib.lsdf_frnn_nparam(65, ct.byref(n)) == B.LSDF_E_SHAPE
    sz = ct.c_size_t(0)
    assert lib.lsdf_frnn_train_workspace_size(2, 65, ct.byref(sz)) == B.LSDF_E_SHAPE
    assert lib.lsdf_frnn_train_workspace_size(2, 64, ct.byref(sz)) == 0

    def step(mo=FAKE, vo=FAKE, t=1, lr=1e-3, B_=8, wsb=1 << 24):
        return lib.lsdf_frnn_train_step(FAKE, mo, vo, t, lr, 0.9, 0.999, 1e-8, 2, FAKE, B_, None, FAKE, FAKE, wsb,
                                        None)
    assert step(mo=None) == B.LSDF_E_INVALID_ARG          # one moment without the other
    assert step(t=0) == B.LSDF_E_INVALID_ARG
    assert step(lr=float("nan")) == B.LSDF_E_INVALID_ARG
    assert step(B_=0) == B.LSDF_E_SHAPE
    assert step(wsb=16) == B.LSDF_E_SHAPE
    assert lib.lsdf_frnn_max_error(FAKE, 0, FAKE, 10, FAKE, None) == B.LSDF_E_SHAPE
    assert lib.lsdf_frnn_max_error(None, 2, FAKE, 10, FAKE, None) == B.LSDF_E_INVALID_ARG
    env = B.make_env((-2, -2, -2), 1 / 32, (128, 128, 128))
    g = grid_array(2)
    assert lib.lsdf_robot_sdf_build_frnn(FAKE, 4, 2, g, FAKE, ct.byref(env), FAKE, 0, FAKE, FAKE, 1 << 20, None) \
        == B.LSDF_E_SHAPE
    # grid boxes of half-width 0.5 m need m >= ceil(0.866 / r) + 2 = 30 at r = 1/32: m = 10 is too small
    assert lib.lsdf_robot_sdf_build_frnn(FAKE, 4, 2, g, FAKE, ct.byref(env), FAKE, 10, FAKE, FAKE, 1 << 20, None) \
        == B.LSDF_E_SHAPE
    assert b"does not hold" in lib.lsdf_last_error()


def test_gather_roof_rejects_bad_arguments(lib):
    vp = ct.c_void_p
    dummy = vp(4096)
    lib.lsdf_gather_roof.restype = ct.c_int
    lib.lsdf_gather_roof.argtypes = [vp, ct.c_int32, ct.c_int32, ct.c_int64, vp, vp]
    for n, it, th, g, o in [(1, 1, 1, dummy, dummy), (1025, 1, 1, dummy, dummy), (8, 0, 1, dummy, dummy),
                            (8, 1, 0, dummy, dummy), (8, 1, 1, None, dummy), (8, 1, 1, dummy, None)]:
        assert lib.lsdf_gather_roof(g, n, it, th, o, None) != 0
