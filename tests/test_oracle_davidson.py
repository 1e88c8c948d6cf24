"""Pins for the oracle Davidson: dense eigenvalues, free electrons, error bounds."""
import numpy as np
import pytest

import workload
from oracle import davidson as dav, hamiltonian as ham


def _setup(name, ik=0, vscale=1.0, nl=True, nbnd=None):
    w = workload.make_workload(name)
    m = w.miller[ik]
    v = w.vloc_r() * vscale
    b, d = (w.beta(ik), w.dmat()) if nl else (None, None)
    kin = ham.kinetic(w.cell, w.k_cryst[ik], m)
    h = lambda x: ham.apply_h_ref(w.cell, w.grid, w.k_cryst[ik], m, v, b, d, x)
    dense = ham.dense_h(w.cell, w.grid, w.k_cryst[ik], m, v, b, d)
    x0 = w.psi(ik, purpose=2, nbnd=nbnd)
    return h, dense, kin, x0


def test_teter_hand_values(golden):
    """K(x) at x = 1/2, 1, 2, 3 against exact fractions evaluated by hand
    (tests/golden/teter_hand.txt), plus the two limits of the Teter-Payne-Allan factor:
    1 - K(x) = 16 x^4/27 + O(x^5) near 0 and x K(x) -> 1/2.  A dropped or wrong coefficient
    in either polynomial changes at least one of the fractions."""
    g = golden("teter_hand.txt")
    x = np.array(g["x"])
    np.testing.assert_allclose(dav.teter(x), np.array(g["num"]) / np.array(g["den"]), rtol=1e-15)
    assert dav.teter(0.0) == 1.0
    for h in (1e-2, 1e-3):
        assert abs((1.0 - dav.teter(h)) / h ** 4 - 16.0 / 27.0) < 2.0 * h
    for big in (1e4, 1e6):
        assert abs(big * dav.teter(big) - 0.5) < 2.0 / big
    xs = np.linspace(0.0, 50.0, 2001)
    assert np.all(np.diff(dav.teter(xs)) < 0.0)


def test_orthonormalise():
    rng = np.random.default_rng(0)
    v = dav.orthonormalise(rng.standard_normal((5, 50)) + 1j * rng.standard_normal((5, 50)))
    t = dav.orthonormalise(rng.standard_normal((4, 50)) + 1j * rng.standard_normal((4, 50)), v)
    np.testing.assert_allclose(t.conj() @ t.T, np.eye(4), atol=1e-14)
    assert np.abs(v.conj() @ t.T).max() < 1e-14


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_davidson_vs_dense(name):
    h, dense, kin, x0 = _setup(name, nbnd=8)
    lam = np.linalg.eigvalsh(dense)[:8]
    hist = []
    out = dav.davidson_ref(h, x0, kin, tol=1e-9, history=hist)
    assert out["converged"]
    assert out["resnorm"].max() <= 1e-9
    # Krylov-Weinstein: each Ritz value lies within ||r|| of an exact eigenvalue,
    # and the Ritz values are upper bounds (Courant-Fischer)
    assert np.abs(out["eig"] - lam).max() < 1e-9
    assert np.all(out["eig"] >= lam - 1e-12)
    # returned vectors are orthonormal
    x = out["x"]
    np.testing.assert_allclose(x.conj() @ x.T, np.eye(8), atol=1e-12)


def test_free_electron_spectrum():
    """V = 0, D = 0: eigenvalues are the sorted 1/2|k+G|^2, with their exact degeneracies."""
    w = workload.make_workload("c2")
    ik = 1
    m = w.miller[ik]
    kin = ham.kinetic(w.cell, w.k_cryst[ik], m)
    h = lambda x: ham.apply_h_ref(w.cell, w.grid, w.k_cryst[ik], m, np.zeros(w.grid), None, None, x)
    nb = 12
    out = dav.davidson_ref(h, w.psi(ik, purpose=2, nbnd=nb), kin, tol=1e-9)
    a = workload.A_SI
    exact = np.sort(0.5 * (2 * np.pi / a) ** 2 * ((m + w.k_cryst[ik]) ** 2).sum(1))[:nb]
    np.testing.assert_allclose(out["eig"], exact, atol=1e-9)


def test_ritz_values_monotone():
    h, dense, kin, x0 = _setup("c1")
    hist = []
    seq = []

    def prec(r, theta, x):
        seq.append(theta.copy())
        return dav.teter_precondition(r, x, kin)
    dav.davidson_ref(h, x0, kin, tol=1e-10, precond=prec, max_basis=10 ** 6)
    # without restarts, Ritz values never increase from one iteration to the next
    # (Cauchy interlacing on a growing subspace); compare the lowest band
    lows = [s[0] for s in seq if s.size and s.size == seq[0].size]
    assert all(b <= a + 1e-12 for a, b in zip(lows, lows[1:]))
