"""Training driver for the learned Davidson preconditioner (control flow only).

Every arithmetic step runs in the HIP library: the Davidson that generates the
(residual, target) pairs, the pair extraction, the loss/gradient and Adam.
Recipe (used on the 8-atom cubic cell): solve to a tight tolerance for the
converged eigenvectors, re-run the Teter Davidson from the same start and take
the rows of every iteration as training data, then Adam on the per-band cosine
loss with mini-batches of whole bands.
"""
from __future__ import annotations

import numpy as np

from . import (QM_MLP_NPARAM, qm_davidson_solve, qm_davidson_step, qm_dav_training_pairs,
               qm_mlp_adam, qm_mlp_loss_grad)


def init_weights(seed=0):
    """W1 ~ N(0, 1/5), b1 = 0, W2 = 0, b2 = 0: the untrained network is the Teter gain."""
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    w = np.zeros(QM_MLP_NPARAM, np.float32)
    w[:640] = rng.standard_normal(640) * np.sqrt(1.0 / 5.0)
    return torch.from_numpy(w).cuda()


def collect_pairs(plan, psi_start, nbnd, tol=1e-8, tight=1e-10, max_iter=200, max_rows=None):
    """Training rows from one Teter Davidson run; returns dict of device tensors."""
    import torch
    xs = psi_start.clone()
    eig_star, _, _, _ = qm_davidson_solve(plan, -1, xs, nbnd, tol=tight, max_iter=4 * max_iter)
    npw_sum = int(plan.npw.sum())
    per_step_rows = nbnd * npw_sum
    cap = max_rows if max_rows is not None else per_step_rows * 60
    feat = torch.empty((cap, 5), dtype=torch.float32, device="cuda")
    resid = torch.empty((cap, 2), dtype=torch.float32, device="cuda")
    target = torch.empty((cap, 2), dtype=torch.float32, device="cuda")
    bptr = []
    rows = 0
    x = psi_start.clone()
    _, _, nun = qm_davidson_step(plan, -1, x, nbnd, tol=tol, restart=1)
    it = 0
    tmp_ptr = torch.empty(plan.nk * nbnd + 1, dtype=torch.int32, device="cuda")
    while nun > 0 and it < max_iter and rows + per_step_rows <= cap:
        n, nb = qm_dav_training_pairs(plan, xs, eig_star, feat[rows:], resid[rows:], target[rows:],
                                      tmp_ptr)
        bptr.append(tmp_ptr[:nb].cpu().numpy().astype(np.int64) + rows)
        rows += n
        _, _, nun = qm_davidson_step(plan, -1, x, nbnd, tol=tol)
        it += 1
    band_ptr = np.concatenate(bptr + [np.array([rows])]).astype(np.int32)
    return {"feat": feat[:rows], "resid": resid[:rows], "target": target[:rows],
            "band_ptr": band_ptr, "iterations": it}


def train(data, steps=300, batch_bands=256, lr=3e-3, seed=0, log=None):
    """Adam on the per-band cosine loss over mini-batches of bands; returns (weights, history)."""
    import torch
    w = init_weights(seed)
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    g = torch.zeros_like(w)
    bp = data["band_ptr"]
    nbands = len(bp) - 1
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    hist = []
    for t in range(1, steps + 1):
        b0 = int(rng.integers(0, max(1, nbands - batch_bands + 1)))
        b1 = min(nbands, b0 + batch_bands)
        r0, r1 = int(bp[b0]), int(bp[b1])
        ptr = torch.from_numpy((bp[b0:b1 + 1] - r0).astype(np.int32)).cuda()
        loss = qm_mlp_loss_grad(w, data["feat"][r0:r1], data["resid"][r0:r1],
                                data["target"][r0:r1], ptr, b1 - b0, g)
        qm_mlp_adam(w, g, m, v, t, lr=lr)
        hist.append(loss)
        if log is not None and (t % 50 == 0 or t == 1):
            log(f"step {t} loss {loss:.5f}")
    return w, hist


def full_loss(w, data):
    import torch
    g = torch.zeros_like(w)
    ptr = torch.from_numpy(data["band_ptr"]).cuda()
    return qm_mlp_loss_grad(w, data["feat"], data["resid"], data["target"], ptr,
                            len(data["band_ptr"]) - 1, g)
