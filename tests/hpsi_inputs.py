"""Shared helpers of the GPU tests: plan inputs from a synthetic workload."""
import numpy as np

import workload


def plan_arrays(w):
    miller = np.concatenate(w.miller).astype(np.int32)
    beta = np.concatenate([w.beta(ik).reshape(-1) for ik in range(w.nk)])
    return dict(cell=w.cell, grid=w.grid, k_cart=w.k_cart, npw=w.npw, miller=miller,
                nproj=w.nproj, vloc=w.vloc_r(), beta=beta, dmat=w.dmat())


def make_plan(w, nbnd_max, prec=0, arrays=None):
    import torch
    import paper_2308_07277_amd as qm
    a = arrays if arrays is not None else plan_arrays(w)
    dev = torch.device("cuda:0")
    v = torch.from_numpy(a["vloc"]).to(dev)
    b = torch.from_numpy(a["beta"]).to(dev)
    plan = qm.qm_hpsi_plan_create(a["cell"], a["grid"], a["k_cart"], a["npw"], a["miller"],
                                  nbnd_max, a["nproj"], v, b, a["dmat"], prec)
    del v, b
    return plan, a


def psi_block(w, nbnd, purpose=1):
    """[nk][nbnd][npw_k] concatenated, as one flat complex128 numpy array, plus the per-k list."""
    per = [w.psi(ik, purpose=purpose, nbnd=nbnd) for ik in range(w.nk)]
    return np.concatenate([p.reshape(-1) for p in per]), per


def split_k(flat, w, nbnd):
    out, off = [], 0
    for ik in range(w.nk):
        n = nbnd * int(w.npw[ik])
        out.append(flat[off:off + n].reshape(nbnd, int(w.npw[ik])))
        off += n
    return out


def band_rel_err(a, b):
    return np.linalg.norm(a - b, axis=-1) / np.linalg.norm(b, axis=-1)
