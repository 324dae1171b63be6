"""Host-side driver of the learned per-link SDF surrogate.

The arithmetic (labels, forward, backward, Adam, evaluation) runs in
liblsdf.so; this module only sequences the calls: it computes labels for
given sample positions, shuffles sample indices per epoch and steps the
optimiser.  The paper trains its own small network with an L1 loss and Adam
at learning rate 1e-4 (Sec. IV-B); the same loss and optimiser are used here.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import lsdf


# Training recipe of the per-link networks (fit()): L1 loss and Adam (as the
# paper trains its own network, Sec. IV-B), batches of 8192 samples per link.
# A first phase of 1200 epochs over the samples, the learning rate decayed by
# a cosine from 4e-3 to 4e-5; then two rounds that each add the 1/16 of the
# samples the network fits worst (among those at least 3 cm from the
# surface, where its answers are used) four more times and train 800 epochs
# over the enlarged set, at 1.5e-3 and then 1e-3 decayed a hundredfold.
BATCH = 8192
EPOCHS = 1200
LR = 4e-3
LR_FINAL = 4e-5
MINE_ROUNDS = ((1.5e-3, 800), (1e-3, 800))
MINE_FRACTION = 1 / 16
MINE_REPEAT = 4
MINE_MIN_LABEL = 0.03
# The remainder bound of each link's network: 1.25 times the largest
# |label - E| over its training samples (E the distance to the core box),
# rounded up to whole centimetres.
BOUND_FACTOR = 1.25
BOUND_QUANTUM = 0.01


def labels_for_samples(meshes, grids: lsdf.GridSet, samples: torch.Tensor) -> torch.Tensor:
    """Labels [L][N]: grid value inside each link's box, exact mesh distance
    outside (lsdf_sdf_labels), for link-frame samples [L][N][3]."""
    L, N = int(samples.shape[0]), int(samples.shape[1])
    out = torch.empty((L, N), dtype=torch.float32, device=samples.device)
    for i, m in enumerate(meshes):
        v = torch.as_tensor(np.asarray(m.verts, dtype=np.float32), device=samples.device)
        t = torch.as_tensor(np.asarray(m.tris, dtype=np.int32), device=samples.device)
        lsdf.sdf_labels(v, t, m.comp_first, grids, i, samples[i], out=out[i])
    return out


def train(params: torch.Tensor, domains, samples: torch.Tensor, labels: torch.Tensor, *, epochs: int,
          batch: int = 4096, lr: float = 1e-4, lr_final: float | None = None, seed: int = 0,
          log_every: int = 0, log=print):
    """Adam on every link's network at once; params [L][33665] is updated in
    place.  domains: (centre, half, core_half) arrays [L][3] or an
    lsdf_mlp_domain array.  The learning rate follows a cosine from ``lr`` to
    ``lr_final`` (constant when lr_final is None).  Returns the per-epoch mean
    loss [L]."""
    L, N = int(samples.shape[0]), int(samples.shape[1])
    dev = params.device
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    ws = torch.empty(lsdf.mlp_train_workspace_size(L, batch), dtype=torch.uint8, device=dev)
    loss = torch.empty(L, dtype=torch.float32, device=dev)
    doms = domains if not isinstance(domains, tuple) else lsdf.make_domains(*domains)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    steps_per_epoch = N // batch
    total = epochs * steps_per_epoch
    history = []
    t = 0
    for ep in range(epochs):
        perm = torch.stack([torch.randperm(N, generator=gen, device=dev) for _ in range(L)]).to(torch.int32)
        acc = torch.zeros(L, dtype=torch.float32, device=dev)
        for k in range(steps_per_epoch):
            t += 1
            rate = lr if lr_final is None else lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * t / total))
            idx = perm[:, k * batch:(k + 1) * batch].contiguous()
            lsdf.mlp_train_step(params, m, v, t, rate, doms, samples, labels, batch, idx, loss=loss, workspace=ws)
            acc += loss
        history.append((acc / max(1, steps_per_epoch)).cpu().numpy())
        if log_every and (ep + 1) % log_every == 0:
            log(f"[train] epoch {ep + 1}/{epochs}: mean L1 per link (mm) "
                + " ".join(f"{1e3 * x:.2f}" for x in history[-1]))
    return np.array(history)


def _domain_arrays(domains, L):
    """(centre, half, core_half, bound) as float32 arrays [L][3], [L][3],
    [L][3], [L] from a 3- or 4-tuple (no bound: +inf)."""
    cen, half, core = (np.asarray(a, dtype=np.float32).reshape(L, 3) for a in domains[:3])
    bound = np.broadcast_to(np.asarray(domains[3] if len(domains) > 3 else np.inf, dtype=np.float32), (L,))
    return cen, half, core, np.ascontiguousarray(bound)


def remainder_bounds(domains, samples: torch.Tensor, labels: torch.Tensor) -> np.ndarray:
    """Per link, the remainder bound B of the recipe: BOUND_FACTOR times the
    largest |label - E| over the link's samples, rounded up to BOUND_QUANTUM
    (E from the library's own evaluation: a zero network gives E exactly)."""
    L, N = int(samples.shape[0]), int(samples.shape[1])
    cen, half, core, _ = _domain_arrays(domains, L)
    zero = torch.zeros(lsdf.LSDF_MLP_PARAMS, dtype=torch.float32, device=samples.device)
    E = torch.empty(N, dtype=torch.float32, device=samples.device)
    out = np.empty(L)
    for i in range(L):
        lsdf.mlp_eval(zero, (cen[i], half[i], core[i]), samples[i], out=E)
        r = float((labels[i] - E).abs().max())
        out[i] = math.ceil(BOUND_FACTOR * r / BOUND_QUANTUM) * BOUND_QUANTUM
    return out


def fit(params: torch.Tensor, domains, samples: torch.Tensor, labels: torch.Tensor, *, log_every: int = 0,
        log=print):
    """The library's training recipe (constants above) on every link's
    network at once; domains = (centre, half, core_half[, bound]) arrays
    [L][3] (and [L]); params [L][33665] is updated in place.  Returns the
    per-epoch mean loss [epochs][L] of all phases."""
    L, N = int(samples.shape[0]), int(samples.shape[1])
    cen, half, core, bound = _domain_arrays(domains, L)
    doms = lsdf.make_domains(cen, half, core, bound)
    hist = [train(params, doms, samples, labels, epochs=EPOCHS, batch=BATCH, lr=LR, lr_final=LR_FINAL,
                  log_every=log_every, log=log)]
    k = int(N * MINE_FRACTION)
    est = torch.empty(N, dtype=torch.float32, device=samples.device)
    for r, (lr, epochs) in enumerate(MINE_ROUNDS):
        grown_s, grown_y = [], []
        for i in range(L):
            lsdf.mlp_eval(params[i], (cen[i], half[i], core[i], bound[i]), samples[i], out=est)
            err = torch.where(labels[i] >= MINE_MIN_LABEL, (est - labels[i]).abs(), torch.zeros_like(est))
            worst = torch.topk(err, k).indices
            grown_s.append(torch.cat([samples[i]] + [samples[i][worst]] * MINE_REPEAT))
            grown_y.append(torch.cat([labels[i]] + [labels[i][worst]] * MINE_REPEAT))
        if log_every:
            log(f"[train] round {r + 1}: {k} worst samples per link added {MINE_REPEAT} times")
        hist.append(train(params, doms, torch.stack(grown_s).contiguous(), torch.stack(grown_y).contiguous(),
                          epochs=epochs, batch=BATCH, lr=lr, lr_final=lr / 100, seed=r + 1, log_every=log_every,
                          log=log))
    return np.concatenate(hist)
