"""GPU parity of the learned per-link SDF path against the oracle, through
the C ABI: network evaluation and L1-loss gradients against the oracle's
bfloat16 twin (same rounding points, double accumulation) and its pure
double network, the Adam step against the oracle's, labels against the
oracle's grid and mesh distances, and the learned clearance query against
the oracle's rule (orc_query_mlp): constant networks bit for bit, a finite
margin pair by pair and per link at tiny and full size, and the network
alone (no pair falling back) against the twin network."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

# bfloat16 activations: a flip of one rounding between the GPU and the twin
# (their FP32 / double sums differ in the last bits) moves an activation by
# one bfloat16 ulp (2^-8 relative); over two hidden layers of 128 units that
# stays well below 2e-3 of the output scale for these weights.
TOL_EVAL = 2e-3


def say(*a):
    print("[gpu-mlp]", *a, flush=True)


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_12543_amd import lsdf
    lsdf.load_library()
    return lsdf


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def params_f32(L, seed, scale=2.0):
    return (synth.mlp_init(L, synth.BASE_SEED + 5 + seed) * scale).astype(np.float32)


def domains_of(w):
    """Network domains and core boxes of a workload's links, as the GPU is
    given them (float32): (centre, half, core_half)."""
    cen, half = synth.mlp_domain(w.grid_lo.astype(np.float64), w.grid_hi.astype(np.float64))
    core = synth.mlp_core(w.grid_lo, w.grid_hi)
    return cen.astype(np.float32), half.astype(np.float32), core.astype(np.float32)


def normalise(points, cen, half):
    """The kernel's normalisation, (x - centre) * (1 / half), in float32."""
    inv = (1.0 / half.astype(np.float64)).astype(np.float32)
    return ((points.astype(np.float32) - cen.astype(np.float32)) * inv).astype(np.float64)


@pytest.mark.parametrize("bound", [np.inf, 0.2])
def test_mlp_eval_matches_twin(B, orc, tiny, bound):
    """Estimates (the network's share, unbounded or bounded by 0.2, plus the
    core distance) over the whole domain against the oracle's bfloat16 twin
    and its double network, each plus the oracle's core distance in double."""
    cen, half, core = domains_of(tiny)
    P = params_f32(1, 0)[0]
    rng = np.random.default_rng(40)
    pts = rng.uniform(cen[2] - half[2], cen[2] + half[2], size=(3001, 3)).astype(np.float32)
    say("mlp_eval N=3001")
    got = B.mlp_eval(dev(P), (cen[2:3], half[2:3], core[2:3], bound), dev(pts)).cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    p64 = pts.astype(np.float64)
    twin = orc.mlp_value(P.astype(np.float64), p64, cen[2], half[2], core[2], bf16=True, bound=bound)
    full = orc.mlp_value(P.astype(np.float64), p64, cen[2], half[2], core[2], bf16=False, bound=bound)
    E = orc.mlp_value(np.zeros_like(P, dtype=np.float64), p64, cen[2], half[2], core[2])
    assert (E > 0.3).mean() > 0.5                                   # the core term is exercised
    # a GPU-twin difference inside the network scales with the unbounded
    # output, and a bounded share moves by at most as much
    raw = orc.mlp_value(P.astype(np.float64), p64, cen[2], half[2], core[2], bf16=True)
    scale = max(1.0, np.abs(raw - E).max())
    e_twin, e_full = np.abs(got - twin).max(), np.abs(got - full).max()
    say(f"max |gpu - bf16 twin| = {e_twin:.3g}, max |gpu - double net| = {e_full:.3g}, network output scale "
        f"{scale:.3g}, core distance up to {E.max():.3f} m")
    assert e_twin <= TOL_EVAL * scale
    assert e_full <= 5e-2 * scale
    if np.isfinite(bound):
        assert np.all(np.abs(got - E) <= bound * (1 + 1e-6))         # the share never exceeds its bound
        assert (np.abs(twin - E) > 0.5 * bound).mean() > 0.1        # and the bound is reached
    # the core term alone: a zero network gives the FP32 core distance
    z = B.mlp_eval(dev(np.zeros_like(P)), (cen[2:3], half[2:3], core[2:3], bound),
                   dev(pts)).cpu().numpy().astype(np.float64)
    assert np.abs(z - E).max() <= 4e-7 * max(1.0, E.max())


@pytest.mark.parametrize("bound", [np.inf, 0.3])
def test_mlp_loss_grad_matches_twin(B, orc, tiny, bound):
    cen, half, core = domains_of(tiny)
    L, N, Bt = 2, 1536, 1024
    P = params_f32(L, 1)
    rng = np.random.default_rng(41)
    samples = np.stack([rng.uniform(cen[i] - half[i], cen[i] + half[i], size=(N, 3)) for i in range(L)]).astype(np.float32)
    X = [normalise(samples[i], cen[i], half[i]) for i in range(L)]
    # the core distance of every sample (the oracle's, zero network)
    E = [orc.mlp_value(np.zeros(P.shape[1]), samples[i].astype(np.float64), cen[i], half[i], core[i])
         for i in range(L)]
    # labels 0.3 away from the estimates, so that sign(m - y) is the same everywhere
    share = [orc.mlp_forward(P[i].astype(np.float64), X[i], bf16=True) for i in range(L)]
    if np.isfinite(bound):
        share = [bound * np.tanh(v / bound) for v in share]
    labels = np.stack([share[i] + E[i] + rng.choice([-0.3, 0.3], size=N) for i in range(L)]).astype(np.float32)
    bidx = np.stack([rng.permutation(N)[:Bt] for _ in range(L)]).astype(np.int32)
    say(f"mlp_loss_grad L={L} N={N} B={Bt}")
    loss, grad = B.mlp_loss_grad(dev(P), (cen[:L], half[:L], core[:L], bound), dev(samples), dev(labels), Bt,
                                 dev(bidx, torch.int32))
    loss, grad = loss.cpu().numpy().astype(np.float64), grad.cpu().numpy().astype(np.float64)
    for i in range(L):
        Xi, Yi, Ei = X[i][bidx[i]], labels[i][bidx[i]].astype(np.float64), E[i][bidx[i]]
        l_twin, g_twin = orc.mlp_loss_grad(P[i].astype(np.float64), Xi, Yi, bf16=True, offset=Ei, bound=bound)
        l_full, g_full = orc.mlp_loss_grad(P[i].astype(np.float64), Xi, Yi, bf16=False, offset=Ei, bound=bound)
        cos_t = g_twin @ grad[i] / np.linalg.norm(g_twin) / np.linalg.norm(grad[i])
        cos_f = g_full @ grad[i] / np.linalg.norm(g_full) / np.linalg.norm(grad[i])
        rel_t = np.abs(grad[i] - g_twin).max() / np.abs(g_twin).max()
        say(f"link {i}: loss {loss[i]:.6f} vs twin {l_twin:.6f}; grad cosine twin {cos_t:.6f} full {cos_f:.6f}; "
            f"max-norm rel vs twin {rel_t:.3g}")
        assert loss[i] == pytest.approx(l_twin, rel=1e-4)
        assert cos_t >= 0.9999 and rel_t <= 1e-2
        assert cos_f >= 0.999


def test_mlp_train_step_is_adam(B, orc, tiny):
    cen, half, core = domains_of(tiny)
    L, N, Bt = 2, 1024, 512
    P = params_f32(L, 2)
    rng = np.random.default_rng(42)
    samples = np.stack([rng.uniform(cen[i] - half[i], cen[i] + half[i], size=(N, 3)) for i in range(L)]).astype(np.float32)
    labels = rng.normal(size=(L, N)).astype(np.float32)
    p = dev(P)
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    grad = torch.empty_like(p)
    lr = 1e-3
    say("mlp_train_step t=1, 2")
    for t in (1, 2):
        before = p.cpu().numpy().astype(np.float64)
        m64, v64 = m.cpu().numpy().astype(np.float64), v.cpu().numpy().astype(np.float64)
        B.mlp_train_step(p, m, v, t, lr, (cen[:L], half[:L], core[:L]), dev(samples), dev(labels), Bt, grad=grad)
        torch.cuda.synchronize()
        g = grad.cpu().numpy().astype(np.float64)
        want = before.copy()
        for i in range(L):
            orc.adam_step(want[i], m64[i], v64[i], g[i], t, lr)
        got = p.cpu().numpy().astype(np.float64)
        assert np.abs(got - want).max() <= 1e-6 * max(1.0, np.abs(want).max()) + 1e-7
        assert np.abs(m.cpu().numpy() - m64).max() <= 1e-6 * max(1e-30, np.abs(m64).max())


def test_sdf_labels_match_oracle(B, orc, tiny, tiny_grids):
    i = 3
    mesh = tiny.robot.links[i]
    pts = synth.mlp_samples(mesh, tiny.grid_lo[i], tiny.grid_hi[i], 4000, 43).astype(np.float32)
    gs = B.GridSet(tiny.grid_lo, tiny.grid_hi, tiny.grid_n, device="cuda")
    for k, g in enumerate(tiny_grids):
        gs.set_grid(k, g.astype(np.float32))
    say("sdf_labels N=4000")
    lab = B.sdf_labels(dev(mesh.verts), dev(mesh.tris, torch.int32), mesh.comp_first, gs, i, dev(pts)).cpu().numpy()
    # inside the box: the query arithmetic with an identity pose, bit for bit
    ident = np.concatenate([np.eye(3), np.zeros((3, 1))], 1)[None, None].astype(np.float32)
    inbox = np.zeros(len(pts), bool)
    ref = np.empty(len(pts))
    for j in range(len(pts)):
        cl = orc.query_f32(ident, tiny.grid_lo[i:i + 1], tiny.grid_hi[i:i + 1], tiny.grid_n[i:i + 1],
                           [tiny_grids[i].astype(np.float32)], pts[j:j + 1])
        inbox[j] = np.isfinite(cl[0, 0])
        ref[j] = cl[0, 0]
    out = ~inbox
    ref[out] = orc.mesh_sdf(pts[out].astype(np.float64), mesh.verts, mesh.tris, mesh.comp_first)
    assert inbox.sum() > 500 and out.sum() > 500
    assert np.array_equal(lab[inbox].view(np.uint32), ref[inbox].astype(np.float32).view(np.uint32))
    assert np.abs(lab[out] - ref[out]).max() < 2e-6


def _poses(orc, w, sel):
    return orc.fk(w.robot.dh, w.q[sel], w.robot.base_T).astype(np.float32)


def _domain_bands(T32, cen, half, pts, eps=1e-5):
    """[C][L][M] membership of each pair in its link's network domain, decided
    in double from the FP32 poses with a band of +-eps (normalised units)
    around the boundary: (surely inside, possibly inside).  The kernel and the
    oracle form the normalised point in different precisions, so a pair in
    the band may fall on either side."""
    T = T32.astype(np.float64)
    loc = np.einsum("jb,clba->clja", pts.astype(np.float64), T[..., :3]) \
        - np.einsum("clb,clba->cla", T[..., 3], T[..., :3])[:, :, None, :]
    r = np.abs((loc - cen.astype(np.float64)[None, :, None, :]) / half.astype(np.float64)[None, :, None, :]).max(-1)
    return r <= 1.0 - eps, r <= 1.0 + eps


def _grid_set(B, w, grids):
    gs = B.GridSet(w.grid_lo, w.grid_hi, w.grid_n, device="cuda")
    for k, g in enumerate(grids):
        gs.set_grid(k, g.astype(np.float32))
    return gs


@pytest.mark.parametrize("k,margin", [(0.01, 0.05), (0.05, 0.05), (0.2, 0.05), (10.0, float("inf"))])
def test_query_mlp_constant_network_matches_oracle(B, orc, tiny, tiny_grids, k, margin):
    """A network whose output is the constant k (every weight zero, b4 = k)
    gives the same value on the GPU and in the oracle, so the learned query's
    per-link minima must equal the oracle's (orc_query_mlp) bit for bit: below
    the margin an in-box pair takes the grid value and a pair outside the box
    keeps k; at the margin (strict test) and above it every in-domain pair
    keeps k.  With margin +inf and k above every grid value the result is the
    plain query's wherever that is finite.  The workspace starts full of 0xFF:
    the query clears its keys itself."""
    sel = np.arange(0, tiny.C, 5)
    T32 = _poses(orc, tiny, sel)
    cen, half, _ = domains_of(tiny)
    core = half            # the core box fills the domain: every in-domain estimate is k exactly
    pts = tiny.points.astype(np.float32)
    g32 = [g.astype(np.float32) for g in tiny_grids]
    gs = _grid_set(B, tiny, tiny_grids)
    P = np.zeros((tiny.L, B.LSDF_MLP_PARAMS), np.float32)
    P[:, -1] = k
    C = len(sel)
    ws = torch.full((B.query_workspace_size(C, tiny.L, tiny.M),), 0xFF, dtype=torch.uint8, device="cuda")
    say(f"query_mlp constant network k={k} margin={margin} C={C} M={tiny.M}")
    d, l, ld = B.query_min_distance_mlp(dev(T32), gs, dev(P), (cen, half, core), dev(pts), margin=margin,
                                        link_dist=True, workspace=ws)
    ld = ld.cpu().numpy().astype(np.float64)
    want = orc.query_mlp(T32, tiny.grid_lo, tiny.grid_hi, tiny.grid_n, g32, pts, P.astype(np.float64), cen, half,
                         margin, core_k=core)
    # (c, i) whose result a pair in the domain's boundary band could change
    sure, maybe = _domain_bands(T32, cen, half, pts)
    inbox = np.isfinite(orc.query_f32_each(T32, tiny.grid_lo, tiny.grid_hi, tiny.grid_n, g32, pts))
    keeps_k = ~inbox if k < margin else np.ones_like(inbox)
    amb = (sure & keeps_k).any(-1) != (maybe & keeps_k).any(-1)
    ok = ~amb
    say(f"  {ok.sum()} of {ok.size} link minima compared bit for bit ({amb.sum()} with a boundary pair deciding)")
    assert amb.sum() <= 2
    assert np.array_equal(ld[ok].astype(np.float32).view(np.uint32), want[ok].astype(np.float32).view(np.uint32))
    assert np.array_equal(ld[ok], want[ok])
    if k < margin < np.inf:
        assert (inbox.any(-1) & (want < k)).any() and (want == np.float32(k)).any()   # both kinds of pair decide
    dn, ln = d.cpu().numpy().astype(np.float64), l.cpu().numpy()
    want_l = np.where(np.isfinite(ld.min(axis=1)), ld.argmin(axis=1), -1)
    assert np.array_equal(dn, ld.min(axis=1)) and np.array_equal(ln, want_l)
    if np.isinf(margin):
        plain = B.query_min_distance(dev(T32), gs, dev(pts), link_dist=True)[2].cpu().numpy()
        fin = np.isfinite(plain)
        assert fin.sum() > 50
        assert np.array_equal(ld[fin].astype(np.float32).view(np.uint32), plain[fin].view(np.uint32))


def _core_each(orc, w, T32, pts, cen, half, core):
    """[C][L][M] core distance of every pair, the oracle's (a zero network's
    estimates)."""
    zero = np.zeros((T32.shape[1], orc.mlp_nparam()))
    lo, hi, n = w.grid_lo[:T32.shape[1]], w.grid_hi[:T32.shape[1]], w.grid_n[:T32.shape[1]]
    _, E, _ = orc.query_mlp(T32, lo, hi, n, [np.zeros(tuple(k[::-1]), np.float32) for k in n], pts, zero, cen, half,
                            -np.inf, each=True, core_k=core)
    return E


def _shift_to_margin(orc, w, T32, pts, P, cen, half, core, margin, q=0.4, s=1.0):
    """Scale each link's output weights w4 by s and shift its output bias so
    that the margin sits at quantile q of the twin network's outputs (the
    estimates less the core distance) over the pairs in that link's domain:
    pairs near the link (small core distance) then fall on both sides of the
    margin, and so do some farther ones.  Returns the FP32
    parameters (what the GPU is given; the oracle reads the same values) and
    the per-pair tolerance function of the estimates em and core distances E:
    a GPU-twin difference comes from bfloat16 rounding flips inside the
    network, so it scales with the network output's distance from its bias
    (the core distance differs only by FP32 rounding)."""
    P = P.copy()
    P[:, -129:-1] *= np.float32(s)
    _, em, _ = orc.query_mlp(T32, w.grid_lo, w.grid_hi, w.grid_n, [np.zeros(tuple(n[::-1]), np.float32)
                                                                    for n in w.grid_n],
                             pts, P.astype(np.float64), cen, half, -np.inf, each=True, core_k=core)
    net = em - _core_each(orc, w, T32, pts, cen, half, core)
    sure, _ = _domain_bands(T32, cen, half, pts)
    for i in range(w.L):
        P[i, -1] += np.float32(margin - np.quantile(net[:, i][sure[:, i]], q))
    P = P.astype(np.float32)
    b4 = P[:, -1].astype(np.float64)

    def tol(em, E):
        return TOL_EVAL * np.maximum(s, np.abs(em - E - b4.reshape((1, -1) + (1,) * (em.ndim - 2)))) + 1e-6
    return P, tol


def _bounded_tol(tol_raw, net, bound):
    """Per-pair tolerance of a bounded share B tanh(net / B) from the
    tolerance tol_raw of the network's output net: the share moves by at
    most its largest slope over [net - tol_raw, net + tol_raw] times
    tol_raw, plus the FP32 evaluation of tanh."""
    if not np.isfinite(bound):
        return tol_raw
    near0 = np.sign(net) * np.maximum(np.abs(net) - tol_raw, 0.0)
    return tol_raw * (1.0 - np.tanh(near0 / bound) ** 2) + 1e-6


def _pair_intervals(em, eg, sure, maybe, margin, tol):
    """Per pair, the interval [lo, hi] of values the learned query may give:
    the oracle decides with the twin network's m, the GPU with its own m
    (within tol of the twin's), so a decision is fixed only where m is more
    than tol from the margin and the pair is clear of the domain's boundary
    band.  A pair that takes the grid value gives the twin's grid bits."""
    below = em < margin - tol
    near = np.abs(em - margin) <= tol
    inbox = np.isfinite(eg)
    lo = np.where(below & inbox, eg, em - tol)
    hi = np.where(below & inbox, eg, em + tol)
    lo = np.where(near & inbox, np.minimum(eg, em - tol), lo)
    hi = np.where(near & inbox, np.maximum(eg, em + tol), hi)
    lo = np.where(maybe, lo, np.inf)
    hi = np.where(sure, hi, np.inf)
    return lo, hi


def test_query_mlp_finite_margin_pairs_match_oracle(B, orc, tiny, tiny_grids):
    """Margin 5 cm with a random network whose outputs are shifted to put the
    margin inside their range, pair by pair: each GPU call takes one point,
    so its per-link values are the values of single pairs.  Every pair whose
    decision is fixed (network value more than TOL_EVAL from the margin,
    clear of the domain boundary) must follow the oracle's rule: below the
    margin and in the box, the twin's grid value bit for bit; below the
    margin outside the box, the network value; above the margin, the network
    value.  The network is not a distance field, so a wrong decision moves a
    value far beyond the tolerance."""
    sel = np.arange(0, tiny.C, 5)
    T32 = _poses(orc, tiny, sel)
    cen, half, core = domains_of(tiny)
    g32 = [g.astype(np.float32) for g in tiny_grids]
    # the 100 points in the most grid boxes over these poses, and 60 others
    nbox = np.isfinite(orc.query_f32_each(T32, tiny.grid_lo, tiny.grid_hi, tiny.grid_n, g32,
                                          tiny.points.astype(np.float32))).sum(axis=(0, 1))
    order = np.argsort(-nbox, kind="stable")
    pts = tiny.points[np.concatenate([order[:100], order[-60:]])].astype(np.float32)
    gs = _grid_set(B, tiny, tiny_grids)
    margin = 0.05
    P, tolf = _shift_to_margin(orc, tiny, T32, pts, params_f32(7, 7), cen, half, core, margin, q=0.8, s=2.0)
    _, em, eg = orc.query_mlp(T32, tiny.grid_lo, tiny.grid_hi, tiny.grid_n, g32, pts, P.astype(np.float64), cen, half,
                              margin, each=True, core_k=core)
    E = _core_each(orc, tiny, T32, pts, cen, half, core)
    sure, maybe = _domain_bands(T32, cen, half, pts)
    C, L, M = em.shape
    Tg, Pg = dev(T32), dev(P)
    ws = B.query_workspace(C, L, 1, "cuda")
    say(f"query_mlp margin={margin}: {M} single-point calls, C={C}")
    got = np.empty((C, L, M))
    for j in range(M):
        got[:, :, j] = B.query_min_distance_mlp(Tg, gs, Pg, (cen, half, core), dev(pts[j:j + 1]), margin=margin,
                                                link_dist=True, workspace=ws)[2].cpu().numpy()
    tol = tolf(em, E)
    fixed = sure & (np.abs(em - margin) > tol)
    inbox = np.isfinite(eg)
    grid_pairs = fixed & (em < margin) & inbox
    far_pairs = fixed & (em < margin) & ~inbox
    net_pairs = fixed & (em >= margin)
    say(f"  pairs: {grid_pairs.sum()} take the grid, {far_pairs.sum()} below the margin outside the box keep m, "
        f"{net_pairs.sum()} above the margin; {(sure & ~fixed).sum()} within the tolerance of the margin")
    assert grid_pairs.sum() > 100 and far_pairs.sum() > 100 and net_pairs.sum() > 100
    assert np.array_equal(got[grid_pairs].astype(np.float32).view(np.uint32),
                          eg[grid_pairs].astype(np.float32).view(np.uint32))
    assert np.all(np.abs(got[far_pairs] - em[far_pairs]) <= tol[far_pairs])
    assert np.all(np.abs(got[net_pairs] - em[net_pairs]) <= tol[net_pairs])
    assert np.all(np.isinf(got[~maybe]))                     # outside the domain: no value
    # the rule has teeth: the grid value is far from m for most grid pairs
    assert (np.abs(eg[grid_pairs] - em[grid_pairs]) > tol[grid_pairs]).mean() > 0.9
    lo, hi = _pair_intervals(em, eg, sure, maybe, margin, tol)
    assert np.all((got >= lo) & (got <= hi))


def _check_minima(ld, lo, hi, where):
    """Per-link minima against the intervals of their pairs: the minimum of
    the learned values lies between the minima of the lower and upper ends;
    where the two coincide (a grid pair decides) it is that value exactly."""
    mlo, mhi = lo.min(-1), hi.min(-1)
    exact = mlo == mhi
    assert np.all((ld >= mlo) & (ld <= mhi)), (where, np.argwhere(~((ld >= mlo) & (ld <= mhi)))[:5])
    assert np.array_equal(ld[exact], mlo[exact])
    return int(exact.sum())


@pytest.mark.parametrize("bound", [np.inf, 0.03])
def test_query_mlp_finite_margin_minima_match_oracle(B, orc, tiny, tiny_grids, bound):
    """Margin 5 cm, every point of the tiny workload in one call, with a
    random network whose output is scaled to vary a few centimetres around
    the margin: some per-link minima are decided by a grid value (then they
    are that value exactly), others by a network value, and every one must
    lie within the oracle's per-pair intervals.  The oracle evaluates every
    pair; with a finite bound the GPU skips the tiles that cannot hold a
    minimum, so equal minima show that the skipping is exact."""
    sel = np.arange(0, tiny.C, 5)
    T32 = _poses(orc, tiny, sel)
    cen, half, core = domains_of(tiny)
    pts = tiny.points.astype(np.float32)
    g32 = [g.astype(np.float32) for g in tiny_grids]
    gs = _grid_set(B, tiny, tiny_grids)
    margin = 0.05
    P, tolf = _shift_to_margin(orc, tiny, T32, pts[:300], params_f32(7, 8), cen, half, core, margin, q=0.5, s=0.05)
    bounds = None if np.isinf(bound) else np.full(tiny.L, bound)
    _, em_raw, _ = orc.query_mlp(T32, tiny.grid_lo, tiny.grid_hi, tiny.grid_n, g32, pts, P.astype(np.float64), cen,
                                 half, margin, each=True, core_k=core)
    _, em, eg = orc.query_mlp(T32, tiny.grid_lo, tiny.grid_hi, tiny.grid_n, g32, pts, P.astype(np.float64), cen, half,
                              margin, each=True, core_k=core, bounds=bounds)
    E = _core_each(orc, tiny, T32, pts, cen, half, core)
    sure, maybe = _domain_bands(T32, cen, half, pts)
    say(f"query_mlp margin={margin} bound={bound} C={len(sel)} M={tiny.M}")
    ld = B.query_min_distance_mlp(dev(T32), gs, dev(P), (cen, half, core, bound), dev(pts), margin=margin,
                                  link_dist=True)[2].cpu().numpy().astype(np.float64)
    tol = _bounded_tol(tolf(em_raw, E), em_raw - E, bound)
    lo, hi = _pair_intervals(em, eg, sure, maybe, margin, tol)
    n_exact = _check_minima(ld, lo, hi, "tiny")
    n_net = int((np.isfinite(hi.min(-1)) & (lo.min(-1) < hi.min(-1))).sum())
    say(f"  {n_exact} of {ld.size} minima decided by a grid pair (exact), {n_net} by network values")
    assert n_exact > 0 and n_net > 0
    if np.isfinite(bound):
        # the pairs the GPU may skip: E - B above the smallest E + B of the
        # pairs that cannot fall back (the first kernel's bound), in double
        nf = sure & (E - bound >= margin)
        U = np.where(nf, E + bound, np.inf).min(-1, keepdims=True)
        skippable = sure & (E - bound > np.maximum(U, margin))
        say(f"  {skippable.sum() / sure.sum():.2f} of the in-domain pairs lie beyond the skipping bound")
        assert skippable.sum() > 0.3 * sure.sum()


@pytest.mark.parametrize("bound", [np.inf, 0.1])
def test_query_mlp_finite_margin_learned_scale_sampled(B, orc, bound):
    """The learned workload at full size (500 waypoints x 100,000 points x 7
    links) at margin 5 cm in the benchmark's launch configuration, with a
    random network scaled to vary a few centimetres around the margin,
    unbounded and bounded (the GPU then skips the tiles that cannot hold a
    minimum): sampled per-link minima against the oracle's per-pair intervals
    over all 100,000 points of that link."""
    w = synth.make_workload("learned")
    cen, half, core = domains_of(w)
    g32 = [g.astype(np.float32) for g in orc.workload_grids(w)]
    gs = _grid_set(B, w, g32)                    # the oracle's grids on both sides
    T32 = orc.fk(w.robot.dh, w.q, w.robot.base_T).astype(np.float32)
    pts = w.points.astype(np.float32)
    margin = 0.05
    s = 0.05
    P, tolf = _shift_to_margin(orc, w, T32[::100], pts[::50], params_f32(7, 9), cen, half, core, margin, q=0.5, s=s)
    say(f"query_mlp learned scale C={w.C} M={w.M} margin={margin} bound={bound}")
    ld = B.query_min_distance_mlp(dev(T32), gs, dev(P), (cen, half, core, bound), dev(pts), margin=margin,
                                  link_dist=True)[2].cpu().numpy().astype(np.float64)
    n_exact = 0
    for c, i in [(0, 1), (123, 4), (250, 0), (377, 6), (499, 3)]:
        Tci = T32[c:c + 1, i:i + 1]
        args = (Tci, w.grid_lo[i:i + 1], w.grid_hi[i:i + 1], w.grid_n[i:i + 1], [g32[i]], pts)
        bnd = None if np.isinf(bound) else [bound]
        _, em, eg = orc.query_mlp(*args, P[i:i + 1].astype(np.float64), cen[i:i + 1], half[i:i + 1], margin,
                                  each=True, core_k=core[i:i + 1], bounds=bnd)
        _, em_raw, _ = orc.query_mlp(*args, P[i:i + 1].astype(np.float64), cen[i:i + 1], half[i:i + 1], margin,
                                     each=True, core_k=core[i:i + 1])
        _, E, _ = orc.query_mlp(*args, np.zeros((1, P.shape[1])), cen[i:i + 1], half[i:i + 1], -np.inf, each=True,
                                core_k=core[i:i + 1])
        sure, maybe = _domain_bands(Tci, cen[i:i + 1], half[i:i + 1], pts)
        tol = _bounded_tol(TOL_EVAL * np.maximum(s, np.abs(em_raw - E - np.float64(P[i, -1]))) + 1e-6, em_raw - E,
                           bound)
        lo, hi = _pair_intervals(em, eg, sure, maybe, margin, tol)
        below = (em < margin) & sure
        say(f"  c={c} link={i}: {sure.sum()} in-domain pairs, {(below & np.isfinite(eg)).sum()} take the grid, "
            f"{(below & ~np.isfinite(eg)).sum()} below the margin outside the box; gpu {ld[c, i]:.6g}, "
            f"interval [{lo.min():.6g}, {hi.min():.6g}]")
        n_exact += _check_minima(ld[c:c + 1, i:i + 1], lo, hi, (c, i))
    assert n_exact >= 1


def test_query_mlp_no_fallback_matches_twin(B, orc, tiny, tiny_grids):
    """With margin -inf every in-domain pair takes the estimate: the per-link
    minima must match the twin's estimates (network + core distance) over the
    same pairs."""
    cen, half, core = domains_of(tiny)
    gs = B.GridSet(tiny.grid_lo, tiny.grid_hi, tiny.grid_n, device="cuda")
    for k, g in enumerate(tiny_grids):
        gs.set_grid(k, g.astype(np.float32))
    C, M = 3, 301
    T32 = orc.fk(tiny.robot.dh, tiny.q[:C], tiny.robot.base_T).astype(np.float32)
    pts = tiny.points[:M].astype(np.float32)
    P = params_f32(7, 4)
    say(f"query_mlp margin=-inf C={C} M={M}")
    d, l, ld = B.query_min_distance_mlp(dev(T32), gs, dev(P), (cen, half, core), dev(pts), margin=float("-inf"),
                                        link_dist=True)
    ld = ld.cpu().numpy().astype(np.float64)
    for c in range(C):
        for i in range(7):
            R, t = T32[c, i, :, :3].astype(np.float64), T32[c, i, :, 3].astype(np.float64)
            loc = (pts.astype(np.float64) - t) @ R
            X = (loc - cen[i]) / half[i]
            ind = np.all(np.abs(X) <= 1.0, axis=1)
            want = orc.mlp_value(P[i].astype(np.float64), loc[ind], cen[i], half[i], core[i], bf16=True).min() \
                if ind.any() else np.inf
            assert abs(ld[c, i] - want) <= TOL_EVAL * max(1.0, abs(want)), (c, i, ld[c, i], want)


def test_query_mlp_learned_scale_sampled(B, orc):
    """The learned workload at full size (500 waypoints x 100,000 points x 7
    links) in the launch configuration the benchmark times, margin -inf (every
    in-domain pair takes the network value): sampled per-link minima against
    the twin network over all of that link's in-domain points."""
    w = synth.make_workload("learned")
    cen, half, core = domains_of(w)
    gs = B.build_robot_grids(w.robot.links, w.grid_lo, w.grid_hi, w.grid_n, device="cuda")
    T32 = orc.fk(w.robot.dh, w.q, w.robot.base_T).astype(np.float32)
    pts = w.points.astype(np.float32)
    P = params_f32(7, 6)
    say(f"query_mlp learned scale C={w.C} M={w.M} margin=-inf")
    d, l, ld = B.query_min_distance_mlp(dev(T32), gs, dev(P), (cen, half, core), dev(pts), margin=float("-inf"),
                                        link_dist=True)
    ld = ld.cpu().numpy().astype(np.float64)
    assert np.isfinite(ld).mean() > 0.5
    for c, i in [(0, 1), (123, 4), (377, 6), (499, 3)]:
        R, t = T32[c, i, :, :3].astype(np.float64), T32[c, i, :, 3].astype(np.float64)
        loc = (pts.astype(np.float64) - t) @ R
        X = (loc - cen[i]) / half[i]
        ind = np.all(np.abs(X) <= 1.0, axis=1)
        want = orc.mlp_value(P[i].astype(np.float64), loc[ind], cen[i], half[i], core[i], bf16=True).min() \
            if ind.any() else np.inf
        say(f"  c={c} link={i}: {ind.sum()} in-domain points, gpu {ld[c, i]:.6g} twin {want:.6g}")
        assert abs(ld[c, i] - want) <= TOL_EVAL * max(1.0, abs(want)), (c, i, ld[c, i], want)
    # per-waypoint results are the minima over links (lowest link on ties)
    dn, ln = d.cpu().numpy().astype(np.float64), l.cpu().numpy()
    want_l = np.where(np.isfinite(ld.min(axis=1)), ld.argmin(axis=1), -1)
    assert np.array_equal(dn, ld.min(axis=1)) and np.array_equal(ln, want_l)


@pytest.mark.parametrize("M", [1, 31, 33, 257, 300])
def test_query_mlp_bounded_ragged_sizes(B, orc, tiny, tiny_grids, M):
    """The bounded query (skipping on) at cloud sizes that leave partial
    tiles and chunks (1, 31, 33, 257 and 300 points) and 3 configurations:
    per-link minima against the oracle's per-pair intervals (every pair
    evaluated there)."""
    T32 = orc.fk(tiny.robot.dh, tiny.q[:3], tiny.robot.base_T).astype(np.float32)
    cen, half, core = domains_of(tiny)
    pts = tiny.points[::3][:M].astype(np.float32)
    g32 = [g.astype(np.float32) for g in tiny_grids]
    gs = _grid_set(B, tiny, tiny_grids)
    margin, bound, s = 0.05, 0.04, 0.05
    P, tolf = _shift_to_margin(orc, tiny, T32, tiny.points[:300].astype(np.float32), params_f32(7, 11), cen, half, core,
                               margin, q=0.5, s=s)
    _, em_raw, _ = orc.query_mlp(T32, tiny.grid_lo, tiny.grid_hi, tiny.grid_n, g32, pts, P.astype(np.float64), cen,
                                 half, margin, each=True, core_k=core)
    _, em, eg = orc.query_mlp(T32, tiny.grid_lo, tiny.grid_hi, tiny.grid_n, g32, pts, P.astype(np.float64), cen, half,
                              margin, each=True, core_k=core, bounds=np.full(tiny.L, bound))
    E = _core_each(orc, tiny, T32, pts, cen, half, core)
    sure, maybe = _domain_bands(T32, cen, half, pts)
    say(f"query_mlp bounded M={M} C=3")
    ld = B.query_min_distance_mlp(dev(T32), gs, dev(P), (cen, half, core, bound), dev(pts), margin=margin,
                                  link_dist=True)[2].cpu().numpy().astype(np.float64)
    tol = _bounded_tol(tolf(em_raw, E), em_raw - E, bound)
    lo, hi = _pair_intervals(em, eg, sure, maybe, margin, tol)
    _check_minima(ld, lo, hi, f"M={M}")
    assert np.array_equal(np.isfinite(ld), np.isfinite(lo.min(-1)) | np.isfinite(hi.min(-1)))
