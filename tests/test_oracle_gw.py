"""Pins of oracle/gw.py (plane-wave matrix elements M_nn'(k, q, G)): the correlation sum
against the paper's FFT route, the integral <n k+q| e^{i(q+G).r} |n' k> evaluated by grid
quadrature of the full Bloch functions written out with explicit exponentials (exact for
these band-limited integrands on an alias-free grid), and M_nn'(q = 0, G = 0) = <n|n'>."""
import numpy as np

import workload
from oracle import gw
from oracle.lattice import reciprocal, volume


def _small_g(n=7):
    return np.array([[0, 0, 0], [1, 0, 0], [0, -1, 0], [1, 1, -1], [-2, 0, 1], [0, 0, 2], [1, -1, 1]])[:n]


def test_direct_equals_fft_route():
    w = workload.make_workload("c2")
    a = gw.mtxel_direct(w.psi(1, nbnd=3), w.miller[1], w.psi(0, nbnd=4), w.miller[0], _small_g())
    b = gw.mtxel_fft(w.grid, w.psi(1, nbnd=3), w.miller[1], w.psi(0, nbnd=4), w.miller[0], _small_g())
    np.testing.assert_allclose(a, b, atol=1e-14)


def test_bloch_function_quadrature():
    """k = k-point 0, k+q = k-point 1 of the 8-atom cell (q = their difference)."""
    w = workload.make_workload("c2")
    ck, ckq = w.psi(0, nbnd=2), w.psi(1, nbnd=2)
    B = reciprocal(w.cell)
    kc, kqc = w.k_cryst[0] @ B, w.k_cryst[1] @ B
    grid = np.asarray(w.grid)
    jj = np.stack(np.meshgrid(*[np.arange(n) for n in w.grid], indexing="ij"), -1).reshape(-1, 3)
    r = (jj / grid) @ w.cell
    vol = volume(w.cell)
    psi_k = (ck @ np.exp(1j * ((w.miller[0] @ B + kc) @ r.T))) / np.sqrt(vol)      # [nb, N_r]
    psi_kq = (ckq @ np.exp(1j * ((w.miller[1] @ B + kqc) @ r.T))) / np.sqrt(vol)
    g = _small_g(4)
    ref = gw.mtxel_direct(ckq, w.miller[1], ck, w.miller[0], g)
    for gi, mg in enumerate(g):
        ph = np.exp(1j * (r @ (kqc - kc + mg @ B)))
        quad = vol / len(r) * (psi_kq.conj() * ph[None, :]) @ psi_k.T
        np.testing.assert_allclose(quad, ref[:, :, gi], atol=1e-12)


def test_overlap_at_g_zero():
    w = workload.make_workload("c1")
    q, _ = np.linalg.qr(w.psi(0, nbnd=5).T)
    c = q.T
    m = gw.mtxel_direct(c, w.miller[0], c, w.miller[0], np.zeros((1, 3), int))[:, :, 0]
    np.testing.assert_allclose(m, np.eye(5), atol=1e-14)
