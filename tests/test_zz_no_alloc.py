"""The clearance query that allocates nothing (lsdf_query_min_distance_noalloc,
whose workspace is device memory the library holds) against the query that
takes a caller's workspace, through the C ABI: the same bits on two calls in
a row, the second smaller than the first, so that it runs on scratch the
first call left behind."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-noalloc]", *a, flush=True)


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_12543_amd import lsdf
    lsdf.load_library()
    return lsdf


def _inputs(B, name):
    w = synth.make_workload(name)
    gs = B.build_robot_grids(w.robot.links, w.grid_lo, w.grid_hi, w.grid_n, device="cuda")
    T = B.fk_batch(w.robot.dh, torch.as_tensor(w.q, dtype=torch.float32, device="cuda"), base_T=w.robot.base_T)
    pts = torch.as_tensor(w.points, dtype=torch.float32, device="cuda")
    return w, gs, T, pts


def _outputs(C, L):
    return (torch.empty(C, dtype=torch.float32, device="cuda"), torch.empty(C, dtype=torch.int32, device="cuda"),
            torch.empty((C, L), dtype=torch.float32, device="cuda"))


def _same_bits(a, b):
    return all(torch.equal(x.view(torch.int32), y.view(torch.int32)) for x, y in zip(a, b))


def test_noalloc_query_matches_workspace_query_twice(B):
    runs = []
    for name in ("paper", "tiny"):
        w, gs, T, pts = _inputs(B, name)
        ref = B.query_min_distance(T, gs, pts, link_dist=True)
        runs.append((name, w, gs, T, pts, ref, _outputs(w.C, w.L)))
    torch.cuda.synchronize()
    # two calls in a row on one stream, outputs given: nothing is allocated
    for name, w, gs, T, pts, ref, out in runs:
        say(f"noalloc query {name}: C={w.C} M={w.M} L={w.L}")
        B.query_min_distance_noalloc(T, gs, pts, link_dist=True, out=out)
    torch.cuda.synchronize()
    for name, w, gs, T, pts, ref, out in runs:
        assert _same_bits(out, ref), name
        assert torch.isfinite(out[0]).any()
    # and again in the other order: the small problem first, then the large
    for name, w, gs, T, pts, ref, out in reversed(runs):
        for t in out:
            t.fill_(-7)
        B.query_min_distance_noalloc(T, gs, pts, link_dist=True, out=out)
    torch.cuda.synchronize()
    for name, w, gs, T, pts, ref, out in runs:
        assert _same_bits(out, ref), name


def test_noalloc_query_edge_cases(B):
    w, gs, T, pts = _inputs(B, "tiny")
    # empty cloud: (+inf, -1)
    d, l, ld = B.query_min_distance_noalloc(T, gs, pts[:0], link_dist=True)
    torch.cuda.synchronize()
    assert torch.isinf(d).all() and (l == -1).all() and torch.isinf(ld).all()
    # one configuration and a ragged cloud, against the workspace query
    ref = B.query_min_distance(T[:1].contiguous(), gs, pts[:777].contiguous(), link_dist=True)
    got = B.query_min_distance_noalloc(T[:1].contiguous(), gs, pts[:777].contiguous(), link_dist=True)
    torch.cuda.synchronize()
    assert _same_bits(got, ref)
    # a problem larger than the scratch is refused before anything runs
    big = torch.zeros((3_500_000, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(B.LsdfError) as e:
        B.query_min_distance_noalloc(T, gs, big)
    assert e.value.code == B.LSDF_E_SHAPE
