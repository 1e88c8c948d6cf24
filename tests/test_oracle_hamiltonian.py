"""Pins for the oracle Hamiltonian: closed forms, special cases and the dense definition."""
import numpy as np
import pytest

import workload
from oracle import gspace, hamiltonian as ham


def _c1():
    w = workload.make_workload("c1")
    return w, w.miller[0], w.vloc_r(), w.beta(0), w.dmat()


def test_kinetic_closed_form_cubic():
    """For a cubic cell |k+G|^2 = (2 pi / a)^2 |m + k|^2 (crystal coordinates)."""
    w = workload.make_workload("c2")
    a = workload.A_SI
    for ik in range(w.nk):
        m = w.miller[ik]
        expect = 0.5 * (2 * np.pi / a) ** 2 * ((m + w.k_cryst[ik]) ** 2).sum(1)
        np.testing.assert_allclose(ham.kinetic(w.cell, w.k_cryst[ik], m), expect, rtol=1e-14)


def test_constant_potential_shifts():
    w, m, _, _, _ = _c1()
    rng = np.random.default_rng(1)
    psi = rng.standard_normal((3, m.shape[0])) + 1j * rng.standard_normal((3, m.shape[0]))
    v0 = -0.7
    out = ham.apply_h_ref(w.cell, w.grid, w.k_cryst[0], m, np.full(w.grid, v0), None, None, psi)
    kin = ham.kinetic(w.cell, w.k_cryst[0], m)
    np.testing.assert_allclose(out, (kin + v0)[None] * psi, atol=1e-13)


def test_sine_potential_couples_plus_minus_g0():
    """V(r) = 2 sin(G0.r) has V(G0) = -i, V(-G0) = +i: a single plane wave at Ga maps to
    -i at Ga+G0 and +i at Ga-G0 (fixes the sign convention e^{+iG.r} of g2r)."""
    w, m, _, _, _ = _c1()
    grid = np.array(w.grid)
    g0 = np.array([1, 2, 0])
    j = np.stack(np.meshgrid(*[np.arange(n) for n in grid], indexing="ij"), -1)
    phase = 2 * np.pi * (j / grid) @ g0
    v = 2 * np.sin(phase)
    ia = 0                                # G = 0
    c = np.zeros((1, m.shape[0]), complex)
    c[0, ia] = 1.0
    out = ham.apply_local_fft(v, m, w.grid, c)[0]
    expect = np.zeros(m.shape[0], complex)
    for sgn, val in ((+1, -1j), (-1, +1j)):
        hit = np.nonzero((m == m[ia] + sgn * g0).all(1))[0]
        assert hit.size == 1
        expect[hit[0]] = val
    np.testing.assert_allclose(out, expect, atol=1e-13)


def test_nonlocal_closed_form():
    """sum_ij beta_i D_ij <beta_j|c> written with explicit loops and np.vdot."""
    rng = np.random.default_rng(5)
    npw = 40
    beta = rng.standard_normal((3, npw)) + 1j * rng.standard_normal((3, npw))
    d = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
    d = d + d.conj().T
    c = rng.standard_normal(npw) + 1j * rng.standard_normal(npw)
    expect = np.zeros(npw, complex)
    for i in range(3):
        for jj in range(3):
            expect += beta[i] * d[i, jj] * np.vdot(beta[jj], c)
    np.testing.assert_allclose(ham.apply_nonlocal(beta, d, c[None])[0], expect, atol=1e-12)
    hd = ham.nonlocal_dense(beta, d)
    np.testing.assert_allclose(hd @ c, expect, atol=1e-12)
    np.testing.assert_allclose(hd, hd.conj().T, atol=1e-13)


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_dense_equals_fft(name):
    """The FFT route reaches the dense definition to rounding (c1 full; c2 one k-point)."""
    w = workload.make_workload(name, nk_limit=1)
    m = w.miller[0]
    v = w.vloc_r()
    beta, d = w.beta(0), w.dmat()
    h = ham.dense_h(w.cell, w.grid, w.k_cryst[0], m, v, beta, d)
    psi = w.psi(0)[:4]
    ref = psi @ h.T
    out = ham.apply_h_ref(w.cell, w.grid, w.k_cryst[0], m, v, beta, d, psi)
    err = np.linalg.norm(out - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert err.max() < 1e-13
    np.testing.assert_allclose(h, h.conj().T, atol=1e-13 * np.abs(h).max())


def test_hermiticity_c2_k():
    w = workload.make_workload("c2")
    v = w.vloc_r()
    ik = 2
    m = w.miller[ik]
    b, d = w.beta(ik), w.dmat()
    x = w.psi(ik)[:3]
    y = w.psi(ik, purpose=2)[:3]
    hx = ham.apply_h_ref(w.cell, w.grid, w.k_cryst[ik], m, v, b, d, x)
    hy = ham.apply_h_ref(w.cell, w.grid, w.k_cryst[ik], m, v, b, d, y)
    lhs = y.conj() @ hx.T
    rhs = (x.conj() @ hy.T).conj().T
    assert np.abs(lhs - rhs).max() < 1e-13 * np.abs(hx).max() * 10


def test_potential_is_real_and_model_values():
    """Gaussian model: V < 0 everywhere, minimum near -2 Ha at the atom on the grid origin."""
    w = workload.make_workload("c1")
    v = w.vloc_r()
    assert v.max() < 0 and abs(v[0, 0, 0] - (-2.0)) < 1e-2
    assert abs(v.min() - (-2.0)) < 1e-2
