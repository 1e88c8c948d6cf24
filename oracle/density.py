"""Electron density, Hartree potential and a Hartree-only SCF cycle, FP64 reference.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* Density (Sec. 2.1, the density of the Kohn-Sham equations): n(r) = sum_i f_i |psi_i(r)|^2,
  the states i running over k-points and bands; with k-point weights w_k (sum 1) the
  occupation of band n at k is w_k f_kn, f_kn = 2 for a doubly occupied band.  A band
  psi(r) = Omega^{-1/2} sum_G c(G) e^{i(k+G).r} with unit-norm coefficients is normalised
  over the cell, so the integral of n over the cell is sum_k w_k sum_n f_kn.
* Hartree potential (Sec. 2.1, V_Hartree, the classical potential of the charge density):
  the periodic solution of Poisson's equation in Hartree atomic units,
  V_H(G) = 4 pi n(G) / |G|^2 for G != 0 and V_H(0) = 0 (the average of the Coulomb potential
  of a periodic, neutral system is a convention; this one puts it at zero), with
  n(G) = (1/N_r) sum_r n(r) e^{-iG.r} the grid Fourier coefficient and G = m.B, m taken in
  the centred range of the grid (numpy.fft.fftfreq's).  E_H = 1/2 integral V_H n.
* Hartree-only SCF (Sec. 2.1, the self-consistency cycle n -> V -> {psi} -> n_out, mixed
  until n_out = n): V = V_ext + V_H[n]; the lowest bands from a dense diagonalisation;
  linear mixing n <- n + alpha (n_out - n); start from the uniform density (V_H = 0).
  The paper's code mixes with Broyden's method; linear mixing is the simplest mixing
  and the one used here, on both the CPU and the GPU side.

Arrays: grid arrays [N1, N2, N3] in C order, grid point r = sum_i (j_i / N_i) a_i.
"""
import numpy as np

from .gspace import idxgrid
from .lattice import reciprocal, volume


def band_density(cell, grid, miller, c):
    """|psi_n(r)|^2 on the grid for coefficient rows c [nb, npw] -> [nb, N1, N2, N3]."""
    c = np.atleast_2d(np.asarray(c, np.complex128))
    grid = tuple(int(x) for x in grid)
    n = int(np.prod(grid))
    idx = idxgrid(miller, grid)
    out = np.empty((c.shape[0],) + grid)
    for b in range(c.shape[0]):
        buf = np.zeros(n, np.complex128)
        buf[idx] = c[b]
        s = np.fft.ifftn(buf.reshape(grid)) * n       # sum_G c(G) e^{iG.r}
        out[b] = np.abs(s) ** 2 / volume(cell)
    return out


def density_ref(cell, grid, millers, weights, occ, psis):
    """n(r) = sum_k w_k sum_n f_kn |psi_kn(r)|^2; millers/psis per k, occ [nk][nb]."""
    rho = np.zeros(tuple(int(x) for x in grid))
    for m, w, f, c in zip(millers, weights, occ, psis):
        bd = band_density(cell, grid, m, c)
        rho += w * np.tensordot(np.asarray(f, np.float64), bd, axes=(0, 0))
    return rho


def grid_g2(cell, grid):
    """|G|^2 of every grid point's G = m.B, m in the centred range of the grid."""
    grid = tuple(int(x) for x in grid)
    m = np.meshgrid(*[np.fft.fftfreq(n) * n for n in grid], indexing="ij")
    g = np.stack(m, -1) @ reciprocal(cell)
    return (g * g).sum(-1)


def hartree_ref(cell, grid, rho):
    """V_H(r) from n(r): 4 pi n(G)/|G|^2 for G != 0, 0 at G = 0."""
    rho = np.asarray(rho, np.float64)
    ng = np.fft.fftn(rho) / rho.size
    g2 = grid_g2(cell, grid)
    vg = np.zeros_like(ng)
    nz = g2 > 0
    vg[nz] = 4.0 * np.pi * ng[nz] / g2[nz]
    v = np.fft.ifftn(vg) * rho.size
    return v.real


def hartree_energy(cell, rho, vh):
    """E_H = 1/2 integral V_H n = 1/2 (Omega / N_r) sum_r V_H(r) n(r)."""
    rho = np.asarray(rho, np.float64)
    return 0.5 * volume(cell) / rho.size * float((np.asarray(vh) * rho).sum())


def density_residual(cell, a, b):
    """L2 norm over the cell of a - b: sqrt((Omega / N_r) sum_r (a - b)^2)."""
    d = np.asarray(a, np.float64) - np.asarray(b, np.float64)
    return float(np.sqrt(volume(cell) / d.size * (d * d).sum()))


def hartree_scf_ref(cell, grid, millers, k_cryst, weights, vext, beta, dmat, nocc, alpha=0.5,
                    tol=1e-9, max_iter=200, eigh_fn=None):
    """Hartree-only SCF with dense diagonalisation (small cells only).

    beta: list per k of [nproj, npw] (or None); nocc doubly occupied bands at every k.
    Returns dict(rho, vh, eig [nk][nocc], psi (list per k), iterations, residual, e_hartree).
    """
    from .hamiltonian import dense_h
    grid = tuple(int(x) for x in grid)
    nel = 2.0 * nocc * float(np.sum(weights))
    rho = np.full(grid, nel / volume(cell))
    res, it = np.inf, 0
    eig, psi = None, None
    occ = [np.full(nocc, 2.0) for _ in millers]
    for it in range(1, max_iter + 1):
        vh = hartree_ref(cell, grid, rho)
        v = np.asarray(vext, np.float64) + vh
        eig, psi = [], []
        for ik, m in enumerate(millers):
            b = None if beta is None else beta[ik]
            h = dense_h(cell, grid, k_cryst[ik], m, v, b, None if b is None else dmat)
            lam, vec = np.linalg.eigh(h) if eigh_fn is None else eigh_fn(h)
            eig.append(lam[:nocc])
            psi.append(vec[:, :nocc].T.copy())
        rho_out = density_ref(cell, grid, millers, weights, occ, psi)
        res = density_residual(cell, rho_out, rho)
        if res <= tol:
            rho = rho_out
            break
        rho = rho + alpha * (rho_out - rho)
    vh = hartree_ref(cell, grid, rho)
    return dict(rho=rho, vh=vh, eig=np.array(eig), psi=psi, iterations=it, residual=res,
                e_hartree=hartree_energy(cell, rho, vh))
