"""Plane-wave matrix elements of the GW polarizability, FP64 reference.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Definition (Sec. 5, 'gw' module, matrix elements of the Epsilon class):
    M_nn'(k, q, G) = <n k+q| e^{i(q+G).r} |n' k>.
With psi_nk(r) = Omega^{-1/2} sum_G c_nk(G) e^{i(k+G).r}, the integral over the cell leaves
    M_nn'(G) = sum_{G'} conj(c_{n,k+q}(G + G')) c_{n',k}(G'),
a correlation of the two coefficient sets: ``mtxel_direct`` writes that sum out.
``mtxel_fft`` follows the paper's route (same passage): both bands to real space
(u(r) = sum_G c(G) e^{iG.r}), the product conj(u_{n,k+q}) u_{n',k}, and the inverse FFT
(with its 1/N_r), read at the requested G.  The two agree when the grid holds the product
without aliasing (it has components up to the sum of the two spheres' radii).
"""
import numpy as np

from .gspace import idxgrid


def mtxel_direct(c_kq, miller_kq, c_k, miller_k, miller_g):
    """M[n, n', g] = sum_{G'} conj(c_kq[n, G_g + G']) c_k[n', G'] (zero where G_g + G' is
    not in the k+q sphere)."""
    c_kq = np.atleast_2d(np.asarray(c_kq, np.complex128))
    c_k = np.atleast_2d(np.asarray(c_k, np.complex128))
    pos = {tuple(m): i for i, m in enumerate(np.asarray(miller_kq).tolist())}
    mk = np.asarray(miller_k)
    out = np.zeros((c_kq.shape[0], c_k.shape[0], len(miller_g)), np.complex128)
    for g, mg in enumerate(np.asarray(miller_g)):
        idx = [pos.get(tuple(mg + m2), -1) for m2 in mk.tolist()]
        sel = np.array([i >= 0 for i in idx])
        if not sel.any():
            continue
        a = c_kq[:, [i for i in idx if i >= 0]]          # [nb1, n_sel]
        out[:, :, g] = a.conj() @ c_k[:, sel].T
    return out


def mtxel_fft(grid, c_kq, miller_kq, c_k, miller_k, miller_g):
    """The same elements through real space: ifftn(conj(u_{n,k+q}) u_{n',k}) at G."""
    grid = tuple(int(x) for x in grid)
    n = int(np.prod(grid))

    def to_r(c, miller):
        idx = idxgrid(miller, grid)
        out = np.zeros((c.shape[0], n), np.complex128)
        out[:, idx] = c
        return np.fft.ifftn(out.reshape((-1,) + grid), axes=(1, 2, 3)) * n     # sum_G c e^{iG.r}

    u_kq = to_r(np.atleast_2d(c_kq), miller_kq)
    u_k = to_r(np.atleast_2d(c_k), miller_k)
    gi = idxgrid(miller_g, grid)
    out = np.empty((u_kq.shape[0], u_k.shape[0], len(gi)), np.complex128)
    for a in range(u_kq.shape[0]):
        prod = u_kq[a].conj()[None] * u_k                     # [nb2, N1, N2, N3]
        f = np.fft.ifftn(prod, axes=(1, 2, 3)).reshape(u_k.shape[0], -1)
        out[a] = f[:, gi]
    return out
