"""Density, Hartree potential and the Hartree-only SCF on the GPU against the FP64 oracle
(oracle/density.py).

Bounds: density and Hartree potential element by element within 1e-12 of the grid's largest
value (float64 FFT sums over at most 10^6 terms, rounding ~1e-15 relative); Hartree energy
1e-12 relative.  SCF: both sides converge the same cycle to an L2 density residual of 1e-10,
so their fixed points agree to ~1e-9 in the same norm; the bound is 1e-8, with eigenvalues
within 1e-8 Ha.  For the 8-atom cell (too large for the oracle's dense SCF) the converged GPU
density is checked by the fixed-point property at any size: one oracle step from it (V_H of
the GPU density, dense eigenvectors, density) returns it within 1e-7."""
import numpy as np
import pytest

import workload
from oracle import density as od
from oracle import hamiltonian as ham
from oracle.lattice import volume
from hpsi_inputs import make_plan, psi_block

pytestmark = pytest.mark.gpu


def _t(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("name,nk_limit,nb", [("c1", None, 8), ("c2", None, 32), ("c3", 2, 160)])
def test_density_vs_oracle(name, nk_limit, nb):
    """Random bands with random occupations in [0, 2] and unequal k weights; the 64-atom
    grid is taken with two of its k-points and all 160 bands."""
    import torch
    import paper_2308_07277_amd as qm
    w = workload.make_workload(name, nk_limit=nk_limit)
    plan, a = make_plan(w, nb)
    flat, per = psi_block(w, nb)
    rng = np.random.default_rng(11)
    occ = rng.uniform(0.0, 2.0, (w.nk, nb))
    wk = rng.uniform(0.5, 1.5, w.nk)
    wk /= wk.sum()
    rho = torch.empty(w.grid, dtype=torch.float64, device="cuda")
    qm.qm_density(plan, -1, _t(flat), nb, wk, occ, rho)
    got = rho.cpu().numpy()
    ref = od.density_ref(w.cell, w.grid, w.miller, wk, list(occ), per)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"{name}: density max rel err {err:.2e}, integral {got.sum() * volume(w.cell) / got.size:.12f}"
          f" (oracle {ref.sum() * volume(w.cell) / ref.size:.12f})")
    assert err <= 1e-12
    # deterministic: a second call gives the same bits
    rho2 = torch.empty_like(rho)
    qm.qm_density(plan, -1, _t(flat), nb, wk, occ, rho2)
    assert torch.equal(rho, rho2)
    # a single k-point
    qm.qm_density(plan, w.nk - 1, _t(per[-1].reshape(-1)), nb, [1.0], occ[-1:], rho)
    ref1 = od.density_ref(w.cell, w.grid, [w.miller[-1]], [1.0], [occ[-1]], [per[-1]])
    assert np.abs(rho.cpu().numpy() - ref1).max() <= 1e-12 * np.abs(ref1).max()


@pytest.mark.parametrize("name", ["c1", "c2", "c3"])
def test_hartree_vs_oracle(name):
    import torch
    import paper_2308_07277_amd as qm
    w = workload.make_workload(name, nk_limit=1)
    plan, a = make_plan(w, 1)
    rng = np.random.default_rng(5)
    rho = rng.uniform(0.0, 0.1, w.grid)
    vh = torch.empty(w.grid, dtype=torch.float64, device="cuda")
    e = qm.qm_hartree(plan, _t(rho), vh, energy=True)
    ref = od.hartree_ref(w.cell, w.grid, rho)
    err = np.abs(vh.cpu().numpy() - ref).max() / np.abs(ref).max()
    e_ref = od.hartree_energy(w.cell, rho, ref)
    print(f"{name}: V_H max rel err {err:.2e}, E_H {e:.12e} (oracle {e_ref:.12e})")
    assert err <= 1e-12
    assert e == pytest.approx(e_ref, rel=1e-12)


def test_set_vloc_changes_h():
    """After qm_hpsi_plan_set_vloc the plan applies H with the new potential (oracle, 1e-12)."""
    import torch
    import paper_2308_07277_amd as qm
    w = workload.make_workload("c2", nk_limit=1)
    plan, a = make_plan(w, 8)
    v2 = a["vloc"] + 0.3 * np.cos(2 * np.pi * np.arange(w.grid[0]) / w.grid[0])[:, None, None]
    qm.qm_hpsi_plan_set_vloc(plan, _t(v2))
    psi = w.psi(0, nbnd=8)
    x = _t(psi.reshape(-1))
    y = torch.empty_like(x)
    qm.qm_apply_h(plan, 0, x, y, 8)
    ref = ham.apply_h_ref(w.cell, w.grid, w.k_cryst[0], w.miller[0], v2, a["beta"].reshape(w.nproj, -1),
                          a["dmat"], psi)
    got = y.cpu().numpy().reshape(8, -1)
    assert (np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)).max() <= 1e-12


def _scf(w, nocc, nbnd, tol=1e-10, alpha=0.7):
    import torch
    import paper_2308_07277_amd as qm
    plan, a = make_plan(w, nbnd)
    psi = _t(np.concatenate([w.psi(ik, purpose=2, nbnd=nbnd).reshape(-1) for ik in range(w.nk)]))
    rho = torch.empty(w.grid, dtype=torch.float64, device="cuda")
    vh = torch.empty_like(rho)
    kw = np.full(w.nk, 1.0 / w.nk)
    eig, st, status = qm.qm_scf_hartree(plan, _t(a["vloc"]), kw, nocc, psi, nbnd, rho, vh, alpha=alpha,
                                        tol=tol)
    return plan, a, eig, st, status, rho.cpu().numpy(), vh.cpu().numpy()


def test_scf_hartree_c1_vs_oracle():
    """The 2-atom cell, one doubly occupied band (2 electrons), mixing 0.7, residual 1e-10:
    density, occupied eigenvalue and Hartree energy against the oracle's SCF (dense
    diagonalisation every iteration)."""
    w = workload.make_workload("c1")
    plan, a, eig, st, status, rho, vh = _scf(w, 1, 4)
    print("gpu scf", st, "eig", eig[0][:2])
    assert status == 0 and st["converged"] == 1
    ref = od.hartree_scf_ref(w.cell, w.grid, w.miller, w.k_cryst, [1.0], a["vloc"],
                             [a["beta"].reshape(w.nproj, -1)], a["dmat"], nocc=1, alpha=0.7, tol=1e-10)
    d = od.density_residual(w.cell, rho, ref["rho"])
    print("oracle iterations", ref["iterations"], "density diff", d, "eig diff", abs(eig[0][0] - ref["eig"][0][0]))
    assert d <= 1e-8
    assert abs(eig[0][0] - ref["eig"][0][0]) <= 1e-8
    assert st["e_hartree"] == pytest.approx(ref["e_hartree"], rel=1e-8)
    np.testing.assert_allclose(vh, od.hartree_ref(w.cell, w.grid, rho), atol=1e-12 * np.abs(vh).max())
    assert rho.sum() * volume(w.cell) / rho.size == pytest.approx(2.0, rel=1e-12)


def test_scf_hartree_c2_fixed_point():
    """The 8-atom cell (4 k-points, weights 1/4, four doubly occupied bands = 8 electrons):
    the GPU SCF converges, and one oracle step from its density reproduces it."""
    w = workload.make_workload("c2")
    nocc = 4
    plan, a, eig, st, status, rho, vh = _scf(w, nocc, 8, tol=1e-9)
    print("gpu scf", st)
    assert status == 0 and st["converged"] == 1
    v = a["vloc"] + od.hartree_ref(w.cell, w.grid, rho)
    vecs = []
    off = 0
    for ik in range(w.nk):
        m = w.miller[ik]
        beta = a["beta"][off:off + w.nproj * m.shape[0]].reshape(w.nproj, m.shape[0])
        off += w.nproj * m.shape[0]
        lam, vec = np.linalg.eigh(ham.dense_h(w.cell, w.grid, w.k_cryst[ik], m, v, beta, a["dmat"]))
        assert np.abs(lam[:nocc] - eig[ik][:nocc]).max() <= 1e-7
        vecs.append(vec[:, :nocc].T)
    rho1 = od.density_ref(w.cell, w.grid, w.miller, np.full(w.nk, 0.25), [np.full(nocc, 2.0)] * w.nk, vecs)
    d = od.density_residual(w.cell, rho1, rho)
    print("one oracle step from the GPU density moves it by", d)
    assert d <= 1e-7
