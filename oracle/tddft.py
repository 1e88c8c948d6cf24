"""Real-time propagation of the time-dependent Kohn-Sham equations, FP64 reference.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* Taylor exponential (Sec. 5, 'tddft' module, expoper): exp(-i dt H) psi is approximated by
  the series truncated at order k, sum_{r=0}^{k} (-i dt)^r / r! H^r psi, built term by term:
  t_0 = psi, t_r = (-i dt / r) H t_{r-1}, result = sum_r t_r.
* ETRS propagator (Sec. 5, 'tddft' module, prop: enforced time-reversal symmetry): with
  H[psi] the Hamiltonian built from the density of psi,
      psi_bar = exp(-i dt H[psi_n]) psi_n,
      psi_{n+1} = exp(-i dt H[psi_bar] / 2) exp(-i dt H[psi_n] / 2) psi_n,
  every exponential applied with the Taylor series above.
* Hamiltonian of the time-dependent equations (Sec. 2.4: the Kohn-Sham Hamiltonian with the
  instantaneous density): the Hartree-only model of oracle.density, H[psi] = T + V_ext +
  V_H[n(psi)] + V_NL (no exchange-correlation).
* exact_expm: exp(-i dt H) from the eigendecomposition of the dense matrix (small cells).
"""
import numpy as np

from . import density as od
from . import hamiltonian as ham


def taylor_expm(apply_h, psi, dt, order):
    """sum_{r=0}^{order} (-i dt)^r / r! H^r psi for psi [nb, npw]."""
    psi = np.atleast_2d(np.asarray(psi, np.complex128))
    out = psi.copy()
    term = psi.copy()
    for r in range(1, order + 1):
        term = (-1j * dt / r) * apply_h(term)
        out = out + term
    return out


def exact_expm(hmat, psi, dt):
    """exp(-i dt H) psi with H the dense Hermitian matrix (rows of psi are the bands)."""
    lam, vec = np.linalg.eigh(hmat)
    c = np.asarray(psi, np.complex128) @ vec.conj()          # [nb, n]: <v_j | psi>
    return (c * np.exp(-1j * dt * lam)[None, :]) @ vec.T


def hartree_model_h(cell, grid, millers, k_cryst, weights, occ, vext, beta, dmat):
    """Function psis -> (list of per-k H applications, V total) of the Hartree-only model:
    V = V_ext + V_H[n(psis)] with n = sum_k w_k sum_n f_kn |psi_kn|^2."""
    def build(psis):
        rho = od.density_ref(cell, grid, millers, weights, occ, psis)
        v = np.asarray(vext, np.float64) + od.hartree_ref(cell, grid, rho)
        hs = []
        for ik, m in enumerate(millers):
            b = None if beta is None else beta[ik]
            hs.append(lambda x, ik=ik, m=m, b=b: ham.apply_h_ref(cell, grid, k_cryst[ik], m, v, b,
                                                                 None if b is None else dmat, x))
        return hs, v
    return build


def etrs_step(build_h, psis, dt, order):
    """One ETRS step of every k-point's bands; build_h(psis) -> (per-k H applications, V)."""
    h_n, _ = build_h(psis)
    half = [taylor_expm(h, p, 0.5 * dt, order) for h, p in zip(h_n, psis)]
    bar = [taylor_expm(h, p, dt, order) for h, p in zip(h_n, psis)]
    h_bar, _ = build_h(bar)
    return [taylor_expm(h, p, 0.5 * dt, order) for h, p in zip(h_bar, half)]


def hartree_model_energy(cell, grid, millers, k_cryst, weights, occ, vext, beta, dmat, psis):
    """E = sum_k w_k sum_n f_kn <psi|T + V_ext + V_NL|psi> + E_H[n] of the Hartree-only model."""
    rho = od.density_ref(cell, grid, millers, weights, occ, psis)
    vh = od.hartree_ref(cell, grid, rho)
    e = od.hartree_energy(cell, rho, vh)
    for ik, m in enumerate(millers):
        b = None if beta is None else beta[ik]
        hx = ham.apply_h_ref(cell, grid, k_cryst[ik], m, vext, b, None if b is None else dmat, psis[ik])
        e += weights[ik] * float(np.real(np.einsum("nj,nj,n->", psis[ik].conj(), hx, occ[ik])))
    return e
