"""Pins of oracle/tddft.py (Taylor exponential, ETRS step, Hartree-model energy) against the
mathematics: the truncated series of a scalar, the exact exponential of a dense Hermitian
matrix (itself pinned by the free-electron closed form and unitarity), and the stationary
evolution of a self-consistent ground state (eigenstates of the self-consistent H only pick
up phases e^{-i eps dt}, and the density does not move)."""
import math

import numpy as np
import pytest

import workload
from oracle import density as od
from oracle import hamiltonian as ham
from oracle import tddft as otd


def test_taylor_of_a_scalar():
    lam, dt = 0.8, 0.3
    for order in (1, 2, 4, 7):
        got = otd.taylor_expm(lambda x: lam * x, np.ones((1, 1)), dt, order)[0, 0]
        expect = sum((-1j * dt * lam) ** r / math.factorial(r) for r in range(order + 1))
        assert got == pytest.approx(expect, rel=1e-15, abs=1e-15)


def test_exact_expm_free_electrons_and_unitarity():
    """V = 0, no projectors: H is diagonal with 1/2|k+G|^2, so exp(-i dt H) multiplies each
    coefficient by exp(-i dt |k+G|^2 / 2)."""
    w = workload.make_workload("c1")
    kin = ham.kinetic(w.cell, w.k_cryst[0], w.miller[0])
    h = ham.dense_h(w.cell, w.grid, w.k_cryst[0], w.miller[0], np.zeros(w.grid))
    psi = w.psi(0, nbnd=3)
    got = otd.exact_expm(h, psi, 0.7)
    np.testing.assert_allclose(got, psi * np.exp(-0.7j * kin)[None, :], atol=1e-13)
    h = ham.dense_h(w.cell, w.grid, w.k_cryst[0], w.miller[0], w.vloc_r(), w.beta(0), w.dmat())
    out = otd.exact_expm(h, psi, 2.3)
    np.testing.assert_allclose(out.conj() @ out.T, psi.conj() @ psi.T, atol=1e-13)


def test_taylor_converges_to_exact_expm():
    """A high order reaches the exact exponential; order 4 errs by about (dt ||H||)^5 / 5!."""
    w = workload.make_workload("c1")
    beta = w.beta(0)
    h = ham.dense_h(w.cell, w.grid, w.k_cryst[0], w.miller[0], w.vloc_r(), beta, w.dmat())
    hop = lambda x: ham.apply_h_ref(w.cell, w.grid, w.k_cryst[0], w.miller[0], w.vloc_r(), beta, w.dmat(), x)
    psi = w.psi(0, nbnd=4)
    ex = otd.exact_expm(h, psi, 0.05)
    assert np.abs(otd.taylor_expm(hop, psi, 0.05, 30) - ex).max() <= 1e-13
    hn = np.abs(np.linalg.eigvalsh(h)).max()
    e4 = np.abs(otd.taylor_expm(hop, psi, 0.05, 4) - ex).max()
    assert e4 <= (0.05 * hn) ** 5 / math.factorial(5)


def test_etrs_keeps_a_self_consistent_ground_state_stationary():
    """From the converged Hartree-only ground state of the 2-atom cell, ETRS steps with a
    high Taylor order multiply the occupied eigenvector by exp(-i eps dt) and leave the
    density in place; the model energy does not move."""
    w = workload.make_workload("c1")
    beta = [w.beta(0)]
    gs = od.hartree_scf_ref(w.cell, w.grid, w.miller, w.k_cryst, [1.0], w.vloc_r(), beta, w.dmat(),
                            nocc=1, alpha=0.7, tol=1e-12)
    occ = [np.array([2.0])]
    build = otd.hartree_model_h(w.cell, w.grid, w.miller, w.k_cryst, [1.0], occ, w.vloc_r(), beta, w.dmat())
    psi = [gs["psi"][0]]
    e0 = otd.hartree_model_energy(w.cell, w.grid, w.miller, w.k_cryst, [1.0], occ, w.vloc_r(), beta, w.dmat(), psi)
    dt = 0.1
    cur = psi
    for step in range(1, 4):
        cur = otd.etrs_step(build, cur, dt, 16)
        np.testing.assert_allclose(cur[0], psi[0] * np.exp(-1j * gs["eig"][0][0] * dt * step), atol=1e-10)
    e1 = otd.hartree_model_energy(w.cell, w.grid, w.miller, w.k_cryst, [1.0], occ, w.vloc_r(), beta, w.dmat(), cur)
    assert abs(e1 - e0) <= 1e-10


def test_etrs_with_fixed_potential_is_two_half_steps():
    """When H does not depend on psi, ETRS is exp(-i dt H / 2) applied twice."""
    w = workload.make_workload("c1")
    beta = w.beta(0)
    hop = lambda x: ham.apply_h_ref(w.cell, w.grid, w.k_cryst[0], w.miller[0], w.vloc_r(), beta, w.dmat(), x)
    build = lambda psis: ([hop], None)
    psi = [w.psi(0, nbnd=3)]
    got = otd.etrs_step(build, psi, 0.2, 6)[0]
    ref = otd.taylor_expm(hop, otd.taylor_expm(hop, psi[0], 0.1, 6), 0.1, 6)
    np.testing.assert_allclose(got, ref, atol=1e-14)
