"""Training driver for the learned Davidson preconditioner (control flow only).

Every arithmetic step runs in the HIP library: the Davidson that generates the
(residual, target) pairs, the pair extraction, the loss/gradient and Adam; this
module only chooses which rows to keep and moves them.

Recipe (small cells only):
  1. solve the cell to a tight tolerance for the converged eigenvectors;
  2. re-run the Teter Davidson from the same start and extract, after every
     iteration, one row per (G, unconverged band): features, residual and the
     target direction toward the converged eigenvector;
  3. keep the late phase: bands whose residual norm is at most ``max_resid``
     (1e-3 Ha).  Rows from the early phase (random-start residuals) taught the
     network gains that slowed the Davidson down on every cell tried;
  4. Adam on the per-band cosine loss, each step over a random subset of whole
     bands (contiguous band ranges share k-point and iteration, and made the
     result depend on the order of the data), with the input weights of
     ``frozen_inputs`` held at zero.  The residual-amplitude
     input (index 3) is frozen by default: networks that used it converged
     faster on the cell they were trained on but transferred worse.
"""
from __future__ import annotations

import numpy as np

from . import (QM_MLP_NIN, QM_MLP_NHID, QM_MLP_NPARAM, qm_davidson_solve, qm_davidson_step,
               qm_dav_training_pairs, qm_mlp_adam, qm_mlp_loss_grad)


def init_weights(seed=0):
    """W1 ~ N(0, 1/5), b1 = 0, W2 = 0, b2 = 0: the untrained network is the Teter gain."""
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    w = np.zeros(QM_MLP_NPARAM, np.float32)
    n1 = QM_MLP_NHID * QM_MLP_NIN
    w[:n1] = rng.standard_normal(n1) * np.sqrt(1.0 / QM_MLP_NIN)
    return torch.from_numpy(w).cuda()


def collect_pairs(plan, psi_start, nbnd, tol=1e-8, tight=1e-10, max_iter=200, max_rows=None,
                  max_resid=None):
    """Training rows from one Teter Davidson run; returns dict of device tensors.
    With ``max_resid``, only bands whose residual norm is <= max_resid are kept."""
    import torch
    xs = psi_start.clone()
    eig_star, _, _, _ = qm_davidson_solve(plan, -1, xs, nbnd, tol=tight, max_iter=4 * max_iter)
    npw_sum = int(plan.npw.sum())
    per_step_rows = nbnd * npw_sum
    cap = max_rows if max_rows is not None else per_step_rows * 60
    feat = torch.empty((cap, QM_MLP_NIN), dtype=torch.float32, device="cuda")
    resid = torch.empty((cap, 2), dtype=torch.float32, device="cuda")
    target = torch.empty((cap, 2), dtype=torch.float32, device="cuda")
    spans = []          # (first row, last row + 1) of every kept band
    rows = 0
    x = psi_start.clone()
    _, res, nun = qm_davidson_step(plan, -1, x, nbnd, tol=tol, restart=1)
    it = 0
    tmp_ptr = torch.empty(plan.nk * nbnd + 1, dtype=torch.int32, device="cuda")
    while nun > 0 and it < max_iter and rows + per_step_rows <= cap:
        n, nb = qm_dav_training_pairs(plan, xs, eig_star, feat[rows:], resid[rows:], target[rows:],
                                      tmp_ptr)
        ptr = tmp_ptr[:nb + 1].cpu().numpy().astype(np.int64) + rows
        # bands come out in (k, band) order over the unconverged bands of this iteration
        norms = np.concatenate([r[r > tol] for r in res])
        assert norms.size == nb, "training rows do not match the unconverged bands"
        for b in range(nb):
            if max_resid is None or norms[b] <= max_resid:
                spans.append((int(ptr[b]), int(ptr[b + 1])))
        rows += n
        _, res, nun = qm_davidson_step(plan, -1, x, nbnd, tol=tol)
        it += 1
    if max_resid is not None:
        idx = torch.from_numpy(np.concatenate([np.arange(a, b) for a, b in spans])).cuda() \
            if spans else torch.zeros(0, dtype=torch.int64, device="cuda")
        feat, resid, target = feat[idx], resid[idx], target[idx]
    else:
        feat, resid, target = feat[:rows], resid[:rows], target[:rows]
    lens = np.array([b - a for a, b in spans], np.int64)
    band_ptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    return {"feat": feat, "resid": resid, "target": target, "band_ptr": band_ptr,
            "iterations": it}


def concat(a, b):
    """Two row sets as one (bands of b after those of a)."""
    import torch
    off = int(a["band_ptr"][-1])
    return {"feat": torch.cat([a["feat"], b["feat"]]), "resid": torch.cat([a["resid"], b["resid"]]),
            "target": torch.cat([a["target"], b["target"]]),
            "band_ptr": np.concatenate([a["band_ptr"], b["band_ptr"][1:] + off]).astype(np.int32),
            "iterations": a.get("iterations", 0) + b.get("iterations", 0)}


def train(data, steps=1200, batch_bands=256, lr=(3e-3, 3e-4), seed=0, frozen_inputs=(3,), log=None):
    """Adam on the per-band cosine loss; every step draws a random subset of ``batch_bands``
    bands (rows gathered into one batch), the learning rate falls linearly from lr[0] to
    lr[1].  Returns (weights, loss history)."""
    import torch
    w = init_weights(seed)
    frozen = torch.tensor([u * QM_MLP_NIN + f for u in range(QM_MLP_NHID) for f in frozen_inputs],
                          dtype=torch.int64, device="cuda")
    w[frozen] = 0.0
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    g = torch.zeros_like(w)
    bp = data["band_ptr"]
    lens = np.diff(bp)
    nbands = len(bp) - 1
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    hist = []
    for t in range(1, steps + 1):
        sel = np.sort(rng.choice(nbands, size=min(batch_bands, nbands), replace=False))
        rows = torch.from_numpy(np.concatenate([np.arange(bp[b], bp[b + 1]) for b in sel])).cuda()
        ptr = torch.from_numpy(np.concatenate([[0], np.cumsum(lens[sel])]).astype(np.int32)).cuda()
        loss = qm_mlp_loss_grad(w, data["feat"][rows], data["resid"][rows], data["target"][rows],
                                ptr, len(sel), g)
        rate = lr[0] + (lr[1] - lr[0]) * (t - 1) / max(1, steps - 1)
        qm_mlp_adam(w, g, m, v, t, lr=rate)
        w[frozen] = 0.0
        hist.append(loss)
        if log is not None and (t % 100 == 0 or t == 1):
            log(f"step {t} loss {loss:.5f}")
    return w, hist


def full_loss(w, data):
    import torch
    g = torch.zeros_like(w)
    ptr = torch.from_numpy(data["band_ptr"]).cuda()
    return qm_mlp_loss_grad(w, data["feat"], data["resid"], data["target"], ptr,
                            len(data["band_ptr"]) - 1, g)
