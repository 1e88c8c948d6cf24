"""Brute-force discrete Fourier transform, the sum written out term by term.

F[k] = sum_n f[n] exp(s 2 pi i (k1 n1/N1 + k2 n2/N2 + k3 n3/N3)), s = -1 forward,
+1 inverse (no normalisation).  O(N_r^2); for grids of at most ~10^3 points.
It pins the library FFT that the oracle uses as a step.
"""
import numpy as np


def dft3(f, sign=-1):
    f = np.asarray(f, np.complex128)
    n1, n2, n3 = f.shape
    idx = np.stack(np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3), indexing="ij"),
                   -1).reshape(-1, 3).astype(np.float64)
    frac = idx / np.array([n1, n2, n3], np.float64)
    phase = np.exp(sign * 2j * np.pi * (frac @ idx.T))      # [k, n]: k_a n_a / N_a summed
    return (phase @ f.reshape(-1)).reshape(n1, n2, n3)
