"""G-space: the truncated reciprocal-lattice basis and its FFT grid (Sec. 4.3).

* sphere     G = m.B with |k+G|^2 <= E_cut (cutoff given in Ry, i.e. in bohr^-2),
             the plane-wave truncation of Sec. 2.2 ("energy less than a cutoff").
* grid rule  N_i = smallest 2^a 3^b 5^c 7^d 11^e >= 2 floor(sqrt(E_cut)|a_i|/2pi) + 1.
             The paper does not state it; it reproduces the GSpace example's
             (18, 18, 18) grid of Sec. 4.3.
* ordering   G listed in ascending order of (i3, i2, i1), first axis fastest, where
             i = m mod N; this reproduces the printed g_cryst rows of the GSpace example.
* r2g        unnormalised forward FFT followed by taking the sphere components,
             the identity printed in the GSpace example; g2r is its inverse on the
             sphere: scatter into a zero grid, then the 1/N-normalised inverse FFT.
"""
import math

import numpy as np

from .lattice import reciprocal


def fft_good_size(n):
    """Smallest m >= n whose prime factors are all in {2, 3, 5, 7, 11}."""
    m = max(int(n), 1)
    while True:
        r = m
        for p in (2, 3, 5, 7, 11):
            while r % p == 0:
                r //= p
        if r == 1:
            return m
        m += 1


def grid_rule(cell, ecut_ry):
    cell = np.asarray(cell, np.float64)
    out = []
    for i in range(3):
        mmax = math.floor(math.sqrt(ecut_ry) * np.linalg.norm(cell[i]) / (2 * math.pi))
        out.append(fft_good_size(2 * mmax + 1))
    return tuple(out)


def sphere(cell, ecut_ry, grid, k_cryst=(0.0, 0.0, 0.0), slack=1e-12):
    """Miller indices of the G-sphere in canonical order; int64 [npw, 3]."""
    cell = np.asarray(cell, np.float64)
    b = reciprocal(cell)
    k_cryst = np.asarray(k_cryst, np.float64)
    # |m_i| <= |G||a_i|/2pi + |k_i| bounds every member of the sphere
    lim = [int(math.sqrt(ecut_ry) * np.linalg.norm(cell[i]) / (2 * math.pi) + abs(k_cryst[i])) + 1
           for i in range(3)]
    pts = []
    for m1 in range(-lim[0], lim[0] + 1):
        for m2 in range(-lim[1], lim[1] + 1):
            m3 = np.arange(-lim[2], lim[2] + 1)
            mm = np.stack([np.full_like(m3, m1), np.full_like(m3, m2), m3], 1)
            q = (mm + k_cryst) @ b
            sel = (q * q).sum(1) <= ecut_ry * (1.0 + slack)
            if sel.any():
                pts.append(mm[sel])
    m = np.concatenate(pts).astype(np.int64)
    return canonical_order(m, grid)


def canonical_order(miller, grid):
    g = np.asarray(grid)
    i = np.mod(miller, g)
    key = (i[:, 2] * g[1] + i[:, 1]) * g[0] + i[:, 0]
    return np.asarray(miller)[np.argsort(key, kind="stable")]


def norm2(cell, miller, k_cryst=(0.0, 0.0, 0.0)):
    """|k+G|^2 in bohr^-2."""
    q = (np.asarray(miller, np.float64) + np.asarray(k_cryst, np.float64)) @ reciprocal(cell)
    return (q * q).sum(-1)


def idxgrid(miller, grid):
    """Flat C-order index i1*N2*N3 + i2*N3 + i3 of each G on the grid (i = m mod N)."""
    g = np.asarray(grid)
    i = np.mod(np.asarray(miller), g)
    return (i[:, 0] * g[1] + i[:, 1]) * g[2] + i[:, 2]


def r2g(f_r, miller, grid):
    """Forward transform to the sphere: fftn over the grid, then take the sphere."""
    f = np.asarray(f_r).reshape(tuple(grid))
    return np.fft.fftn(f, axes=(-3, -2, -1)).reshape(-1)[idxgrid(miller, grid)]


def g2r(c_g, miller, grid):
    """Inverse of r2g on the sphere: scatter into a zero grid, then ifftn (1/N)."""
    buf = np.zeros(int(np.prod(grid)), np.complex128)
    buf[idxgrid(miller, grid)] = c_g
    return np.fft.ifftn(buf.reshape(tuple(grid)))
