"""Pins of oracle/density.py (density, Hartree potential, Hartree-only SCF) against what the
mathematics fixes: normalisation and the electron count, the density of a band written out
as a direct sum of plane waves at sampled points, the Hartree potential of a single density
wave (closed form), the Hartree potential as the Fourier-series definition written out with
explicit loops on a small grid, the Hartree energy in real and reciprocal space, and the
uniform-density fixed point of the SCF cycle."""
import numpy as np
import pytest

import workload
from oracle import density as od
from oracle import hamiltonian as ham
from oracle.lattice import reciprocal, volume


def _fcc():
    cell, atoms = workload.synth.cell_fcc2()
    return cell


def test_band_density_normalised_and_direct_sum():
    w = workload.make_workload("c2")
    ik = 1
    c = w.psi(ik, nbnd=3)
    bd = od.band_density(w.cell, w.grid, w.miller[ik], c)
    n_r = int(np.prod(w.grid))
    # each band integrates to one over the cell
    np.testing.assert_allclose(bd.sum((1, 2, 3)) * volume(w.cell) / n_r, 1.0, rtol=1e-12)
    # direct sum Omega^-1/2 sum_G c(G) e^{i(k+G).r} at a few grid points
    rng = np.random.default_rng(3)
    q = (w.miller[ik] + w.k_cryst[ik]) @ reciprocal(w.cell)          # cartesian k + G
    for _ in range(5):
        j = rng.integers(0, w.grid[0], 3)
        r = (j / np.asarray(w.grid)) @ w.cell
        psi_r = (c * np.exp(1j * (q @ r))[None, :]).sum(1) / np.sqrt(volume(w.cell))
        np.testing.assert_allclose(bd[:, j[0], j[1], j[2]], np.abs(psi_r) ** 2, rtol=1e-10)


def test_density_integrates_to_electron_count():
    w = workload.make_workload("c2")
    wk = np.full(w.nk, 1.0 / w.nk)
    nocc = 16                                    # 32 electrons of the 8-atom cell
    occ = [np.full(nocc, 2.0)] * w.nk
    psis = [w.psi(ik, nbnd=nocc) for ik in range(w.nk)]
    rho = od.density_ref(w.cell, w.grid, w.miller, wk, occ, psis)
    assert rho.min() >= 0.0
    assert rho.sum() * volume(w.cell) / rho.size == pytest.approx(32.0, rel=1e-12)


@pytest.mark.parametrize("m0", [(1, 0, 0), (1, -2, 1), (0, 3, 2)])
def test_hartree_of_a_density_wave(m0):
    """n = n0 + a cos(G0.r) + b sin(G0.r)  ->  V_H = 4 pi / |G0|^2 (a cos + b sin), no constant
    (Poisson: -laplacian V = 4 pi (n - n0) for a periodic V of zero mean)."""
    cell = _fcc()
    grid = (12, 12, 12)
    fr = np.stack(np.meshgrid(*[np.arange(n) / n for n in grid], indexing="ij"), -1)
    r = fr @ cell
    g0 = np.asarray(m0, float) @ reciprocal(cell)
    ph = r @ g0
    rho = 0.3 + 0.05 * np.cos(ph) - 0.02 * np.sin(ph)
    vh = od.hartree_ref(cell, grid, rho)
    expect = 4.0 * np.pi / (g0 @ g0) * (0.05 * np.cos(ph) - 0.02 * np.sin(ph))
    np.testing.assert_allclose(vh, expect, atol=1e-12 * np.abs(expect).max())


def test_hartree_fourier_series_written_out():
    """V_H(r) = sum_{G != 0} 4 pi n(G)/|G|^2 e^{iG.r}, n(G) = (1/N) sum_r n(r) e^{-iG.r},
    evaluated with explicit exponentials over every grid G (m in the centred range) on a
    6 x 6 x 5 grid of the fcc cell, against the FFT route."""
    cell = _fcc()
    grid = (6, 6, 5)
    rng = np.random.default_rng(7)
    rho = rng.uniform(0.1, 1.0, grid)
    jj = np.stack(np.meshgrid(*[np.arange(n) for n in grid], indexing="ij"), -1).reshape(-1, 3)
    frac = jj / np.asarray(grid)
    mm = np.stack(np.meshgrid(*[np.where(np.arange(n) < (n + 1) // 2, np.arange(n), np.arange(n) - n)
                                for n in grid], indexing="ij"), -1).reshape(-1, 3)
    phase = np.exp(-2j * np.pi * (mm @ frac.T))          # [G, r]: e^{-iG.r}, G.r = 2 pi m.frac
    ng = phase @ rho.reshape(-1) / rho.size
    g = mm @ reciprocal(cell)
    g2 = (g * g).sum(1)
    coef = np.where(g2 > 0, 4.0 * np.pi / np.where(g2 > 0, g2, 1.0), 0.0) * ng
    v_direct = (phase.conj().T @ coef).real.reshape(grid)
    np.testing.assert_allclose(od.hartree_ref(cell, grid, rho), v_direct, atol=1e-12)
    # Hartree energy in reciprocal space: (Omega / 2) sum_{G != 0} 4 pi |n(G)|^2 / |G|^2
    e_g = 0.5 * volume(cell) * float((np.abs(ng[g2 > 0]) ** 2 * 4.0 * np.pi / g2[g2 > 0]).sum())
    assert od.hartree_energy(cell, rho, v_direct) == pytest.approx(e_g, rel=1e-12)
    assert e_g > 0.0


def test_scf_uniform_density_fixed_point():
    """V_ext = 0, no projectors, one doubly occupied band at Gamma: the lowest state is the
    constant G = 0 plane wave, its density is uniform, V_H of it is zero, so the cycle stops
    after one step with eigenvalue 0 and n = 2/Omega."""
    w = workload.make_workload("c1")
    out = od.hartree_scf_ref(w.cell, w.grid, w.miller, w.k_cryst, [1.0], np.zeros(w.grid), None, None,
                             nocc=1, tol=1e-12)
    assert out["iterations"] == 1
    assert abs(out["eig"][0][0]) <= 1e-12
    np.testing.assert_allclose(out["rho"], 2.0 / volume(w.cell), rtol=1e-12)
    assert abs(out["e_hartree"]) <= 1e-20


def test_scf_gaussian_model_is_self_consistent():
    """The 2-atom cell with the Gaussian model and one doubly occupied band (the isolated
    lowest band, 0.45 Ha below the next level): the cycle converges, and the converged
    density reproduces itself - the density of the lowest eigenvector of H[V_ext + V_H[n]],
    recomputed here, is n within the tolerance - and the Hartree term raises the occupied
    eigenvalue above its non-self-consistent (V_H = 0) value."""
    w = workload.make_workload("c1")
    beta = [w.beta(0)]
    out = od.hartree_scf_ref(w.cell, w.grid, w.miller, w.k_cryst, [1.0], w.vloc_r(), beta, w.dmat(),
                             nocc=1, alpha=0.7, tol=1e-10)
    print("iterations", out["iterations"], "E_H", out["e_hartree"], "eig", out["eig"])
    assert out["residual"] <= 1e-10 and out["iterations"] < 60
    v = w.vloc_r() + od.hartree_ref(w.cell, w.grid, out["rho"])
    h = ham.dense_h(w.cell, w.grid, w.k_cryst[0], w.miller[0], v, beta[0], w.dmat())
    lam, vec = np.linalg.eigh(h)
    rho2 = od.density_ref(w.cell, w.grid, w.miller, [1.0], [np.full(1, 2.0)], [vec[:, :1].T])
    assert od.density_residual(w.cell, rho2, out["rho"]) <= 1e-9
    np.testing.assert_allclose(lam[:1], out["eig"][0], atol=1e-8)
    h0 = ham.dense_h(w.cell, w.grid, w.k_cryst[0], w.miller[0], w.vloc_r(), beta[0], w.dmat())
    assert lam[0] > np.linalg.eigvalsh(h0)[0]
    assert out["rho"].sum() * volume(w.cell) / out["rho"].size == pytest.approx(2.0, rel=1e-12)
    assert out["e_hartree"] > 0.0
