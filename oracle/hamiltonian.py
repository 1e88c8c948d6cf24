"""Kohn-Sham Hamiltonian in the plane-wave basis at one k-point.

Definition (eq. KSHamMat of Sec. 2.2 plus the Kleinman-Bylander separable
non-local term of Sec. 2.3, written as sum_ij |beta_i> D_ij <beta_j|):

  (H c)(G) = 1/2 |k+G|^2 c(G)
           + sum_{G' in S_k} V(G - G') c(G')
           + sum_{ij} beta_i(k+G) D_ij sum_{G' in S_k} conj(beta_j(k+G')) c(G')

with V(dG) = (1/N_r) sum_r V(r) exp(-i dG.r) the grid Fourier coefficient of
the sampled local potential, dG taken modulo the grid.  ``dense_h`` writes this
matrix out element by element; ``apply_h_ref`` evaluates the same product the
way Sec. 4.3 describes (inverse FFT, multiply by V(r), forward FFT, keep the
sphere) with numpy.fft as a library step.  Both are float64/complex128.

Array conventions: miller [npw, 3] ints in the caller's order; psi [nbnd, npw];
beta [nproj, npw] holding <k+G|beta_i>; dmat [nproj, nproj] Hermitian (Ha);
vloc_r [N1, N2, N3] real (Ha), C order, grid point r = sum_i (j_i/N_i) a_i.
"""
import numpy as np

from .lattice import reciprocal
from .gspace import idxgrid


def kinetic(cell, k_cryst, miller):
    """1/2 |k+G|^2 in Ha (Sec. 4.3, kinetic operator in reciprocal space)."""
    q = (np.asarray(miller, np.float64) + np.asarray(k_cryst, np.float64)) @ reciprocal(cell)
    return 0.5 * (q * q).sum(-1)


def vloc_fourier(vloc_r):
    """V(G) on the full grid: (1/N_r) sum_r V(r) e^{-iG.r} (numpy.fft as the step)."""
    v = np.asarray(vloc_r, np.float64)
    return np.fft.fftn(v) / v.size


def local_dense(vloc_r, miller, grid):
    """Matrix V(G_m - G_n) over the sphere, indices taken modulo the grid."""
    vg = vloc_fourier(vloc_r)
    m = np.asarray(miller)
    d = np.mod(m[:, None, :] - m[None, :, :], np.asarray(grid))
    return vg[d[..., 0], d[..., 1], d[..., 2]]


def nonlocal_dense(beta, dmat):
    """sum_ij beta_i(G) D_ij conj(beta_j(G'))  ->  [npw, npw]."""
    b = np.asarray(beta, np.complex128)
    return b.T @ np.asarray(dmat) @ b.conj()


def dense_h(cell, grid, k_cryst, miller, vloc_r, beta=None, dmat=None):
    """Explicit H_GG' (eq. KSHamMat + KB term); for small spheres only."""
    h = local_dense(vloc_r, miller, grid).astype(np.complex128)
    h[np.diag_indices_from(h)] += kinetic(cell, k_cryst, miller)
    if beta is not None and dmat is not None and np.asarray(beta).size:
        h += nonlocal_dense(beta, dmat)
    return h


def apply_local_fft(vloc_r, miller, grid, psi):
    """sum_G' V(G-G') c(G') via g2r -> multiply by V(r) -> r2g (Sec. 4.3 steps 1-3)."""
    psi = np.atleast_2d(np.asarray(psi, np.complex128))
    idx = idxgrid(miller, grid)
    n = int(np.prod(grid))
    out = np.empty_like(psi)
    v = np.asarray(vloc_r, np.float64).reshape(tuple(grid))
    for b in range(psi.shape[0]):
        buf = np.zeros(n, np.complex128)
        buf[idx] = psi[b]
        pr = np.fft.ifftn(buf.reshape(tuple(grid)))          # g2r (includes 1/N)
        out[b] = np.fft.fftn(v * pr).reshape(-1)[idx]         # r2g
    return out


def apply_nonlocal(beta, dmat, psi):
    """beta D beta^dagger psi: P = conj(beta) psi^T, Q = D P, add beta^T Q."""
    b = np.asarray(beta, np.complex128)
    psi = np.atleast_2d(np.asarray(psi, np.complex128))
    p = b.conj() @ psi.T                  # [nproj, nbnd]
    q = np.asarray(dmat) @ p
    return (b.T @ q).T                    # [nbnd, npw]


def apply_h_ref(cell, grid, k_cryst, miller, vloc_r, beta, dmat, psi):
    """H(k)|psi> for a block of bands, psi [nbnd, npw] -> [nbnd, npw]."""
    psi = np.atleast_2d(np.asarray(psi, np.complex128))
    out = kinetic(cell, k_cryst, miller)[None, :] * psi
    out += apply_local_fft(vloc_r, miller, grid, psi)
    if beta is not None and dmat is not None and np.asarray(beta).size:
        out += apply_nonlocal(beta, dmat, psi)
    return out
