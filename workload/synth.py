"""Synthetic plane-wave workloads (inputs only; see the package docstring).

Stand-ins for the paper's silicon supercells (Sec. 6 and the GPU scaling
table of Appendix E), whose SG15 pseudopotential files are not available:
the same diamond lattice constant (a = 10.26 bohr), Gamma or small k meshes,
and a model potential made of Gaussians centred on the atoms.

Model (a reading of the workload description, recorded in the design notes):
  * local potential   v(r) = -2 Ha * exp(-|r - tau|^2 / (2 sigma^2)), sigma = 1 bohr,
    summed over atoms and periodic images and sampled on the FFT grid;
  * projectors        unit-normalised real-space Gaussians of s and p symmetry,
    beta_s ~ exp(-r^2/2sigma^2), beta_p,alpha ~ r_alpha exp(-r^2/2sigma^2),
    given in the plane-wave representation <k+G|beta> = Omega^{-1/2} int e^{-i(k+G).r} beta(r - tau) d^3r;
  * D                 = diag(1.5, 0.8, 0.8, 0.8) Ha per atom (separable KB form, Sec. 2.3).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

A_SI = 10.26          # bohr; diamond-structure lattice constant used by every cell here
SIGMA = 1.0           # bohr; Gaussian width of the model potential and projectors
V_DEPTH = -2.0        # Ha
D_DIAG = (1.5, 0.8, 0.8, 0.8)  # Ha; s, px, py, pz


# ----------------------------------------------------------------------------- cells
def cell_fcc2(a: float = A_SI):
    """fcc primitive cell with a 2-atom diamond basis; rows are a_i in bohr."""
    cell = 0.5 * a * np.array([[-1.0, 0.0, 1.0], [0.0, 1.0, 1.0], [-1.0, 1.0, 0.0]])
    atoms = np.array([[0.0, 0.0, 0.0], [0.25 * a, 0.25 * a, 0.25 * a]])
    return cell, atoms


def cell_sc_diamond(n: int = 1, a: float = A_SI):
    """Conventional 8-atom cubic diamond cell repeated n x n x n (8 n^3 atoms)."""
    fcc = np.array([[0, 0, 0], [0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]])
    basis = np.concatenate([fcc, fcc + 0.25])          # fractional, conventional cell
    shifts = np.array([[i, j, l] for i in range(n) for j in range(n) for l in range(n)], float)
    frac = (basis[None, :, :] + shifts[:, None, :]).reshape(-1, 3) / n
    cell = n * a * np.eye(3)
    return cell, frac @ cell


def _recip(cell):
    return 2.0 * math.pi * np.linalg.inv(cell).T


def kmesh_c2():
    """2x2x2 shifted mesh {+-1/4}^3 folded by k == -k: four points, crystal coords."""
    q = 0.25
    return np.array([[q, q, q], [q, q, -q], [q, -q, q], [-q, q, q]])


def kmesh_c3():
    """4x4x1 mesh shifted by (1/2,1/2,0): k_i = (2i-3)/8, k_j = (2j-3)/8, k_z = 0."""
    vals = [(2 * i - 3) / 8.0 for i in range(4)]
    return np.array([[x, y, 0.0] for x in vals for y in vals])


# ----------------------------------------------------------------------------- basis
def miller_sphere(cell, ecut_ry: float, k_cryst, grid):
    """Integer triples m with |k + m.B|^2 <= ecut (bohr^-2), in the caller order used
    throughout the tests and benchmark: ascending (m3 mod N3, m2 mod N2, m1 mod N1)
    with the first axis fastest.  Returns int32 [npw, 3]."""
    b = _recip(cell)
    k_cryst = np.asarray(k_cryst, float)
    kc = k_cryst @ b
    lim = [int(math.floor(math.sqrt(ecut_ry) * np.linalg.norm(cell[i]) / (2 * math.pi)
                          + abs(k_cryst[i]))) + 1 for i in range(3)]
    r = [np.arange(-l, l + 1) for l in lim]
    m = np.stack(np.meshgrid(*r, indexing="ij"), -1).reshape(-1, 3)
    q = m @ b + kc
    keep = (q * q).sum(1) <= ecut_ry * (1.0 + 1e-12)
    m = m[keep]
    g = np.asarray(grid)
    idx = np.mod(m, g)
    order = np.lexsort((idx[:, 0], idx[:, 1], idx[:, 2]))
    m = m[order]
    if np.any(np.abs(m) * 2 >= g[None, :]):
        raise ValueError("FFT grid too small for the sphere")
    return m.astype(np.int32)


# ----------------------------------------------------------------------------- model
def _grid_points_frac(grid):
    n1, n2, n3 = grid
    f = np.stack(np.meshgrid(np.arange(n1) / n1, np.arange(n2) / n2, np.arange(n3) / n3,
                             indexing="ij"), -1)
    return f


def vloc_gaussian(cell, atoms, grid, depth=V_DEPTH, sigma=SIGMA):
    """Periodic sum of Gaussians sampled on the grid; float64 [N1, N2, N3], C order."""
    grid = tuple(int(x) for x in grid)
    inv = np.linalg.inv(cell)
    afrac = atoms @ inv
    nimg = [int(math.ceil(9.0 * sigma / np.linalg.norm(cell[i]) * 1.0)) + 1 for i in range(3)]
    out = np.zeros(grid)
    if np.allclose(cell, np.diag(np.diag(cell))):
        # orthorhombic: the Gaussian factorises into three 1-D periodic sums
        L = np.diag(cell)
        axes = [np.arange(grid[i]) / grid[i] for i in range(3)]
        for tau in afrac:
            f = []
            for i in range(3):
                d = axes[i][:, None] - tau[i] + np.arange(-nimg[i], nimg[i] + 1)[None, :]
                f.append(np.exp(-(d * L[i]) ** 2 / (2 * sigma ** 2)).sum(1))
            out += np.einsum("i,j,l->ijl", f[0], f[1], f[2])
    else:
        fr = _grid_points_frac(grid).reshape(-1, 3)
        acc = np.zeros(fr.shape[0])
        shifts = np.array([[i, j, l] for i in range(-nimg[0], nimg[0] + 1)
                           for j in range(-nimg[1], nimg[1] + 1)
                           for l in range(-nimg[2], nimg[2] + 1)], float)
        for tau in afrac:
            d = fr - tau
            d -= np.round(d)
            for s in shifts:
                x = (d + s) @ cell
                acc += np.exp(-(x * x).sum(1) / (2 * sigma ** 2))
        out = acc.reshape(grid)
    return depth * out


def beta_gaussian(cell, atoms, k_cryst, miller, sigma=SIGMA):
    """<k+G|beta_i> for s, px, py, pz on every atom; complex128 [4*nat, npw]."""
    b = _recip(cell)
    omega = abs(np.linalg.det(cell))
    q = miller.astype(float) @ b + np.asarray(k_cryst, float) @ b     # [npw, 3]
    q2 = (q * q).sum(1)
    g = (2 * math.pi * sigma ** 2) ** 1.5 * np.exp(-0.5 * sigma ** 2 * q2) / math.sqrt(omega)
    ns = math.pi ** -0.75 * sigma ** -1.5
    npn = math.sqrt(2.0 / (math.pi ** 1.5 * sigma ** 5))
    nat = atoms.shape[0]
    out = np.empty((4 * nat, q.shape[0]), np.complex128)
    for a in range(nat):
        ph = np.exp(-1j * (q @ atoms[a])) * g
        out[4 * a] = ns * ph
        for al in range(3):
            out[4 * a + 1 + al] = (-1j * sigma ** 2 * npn) * q[:, al] * ph
    return out


def dmat_sp(nat):
    """Block-diagonal KB coefficients, one diag(1.5, 0.8, 0.8, 0.8) Ha block per atom."""
    return np.diag(np.tile(np.array(D_DIAG), nat)).astype(np.float64)


def random_bands(nbnd, npw, seed):
    """Complex Gaussian coefficients, unit 2-norm per band (seeded PCG64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.standard_normal((nbnd, npw)) + 1j * rng.standard_normal((nbnd, npw))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    return x


# ----------------------------------------------------------------------------- configs
@dataclasses.dataclass
class Workload:
    name: str
    cell: np.ndarray
    atoms: np.ndarray
    ecut_ry: float
    grid: tuple
    k_cryst: np.ndarray
    nbnd: int
    index: int                      # used to derive seeds: 1000*index + purpose

    def __post_init__(self):
        self.recip = _recip(self.cell)
        self.k_cart = self.k_cryst @ self.recip
        self.miller = [miller_sphere(self.cell, self.ecut_ry, k, self.grid) for k in self.k_cryst]
        self.npw = np.array([m.shape[0] for m in self.miller], np.int32)
        self.nproj = 4 * self.atoms.shape[0]

    @property
    def nk(self):
        return len(self.miller)

    def vloc_r(self):
        return vloc_gaussian(self.cell, self.atoms, self.grid)

    def beta(self, ik):
        return beta_gaussian(self.cell, self.atoms, self.k_cryst[ik], self.miller[ik])

    def dmat(self):
        return dmat_sp(self.atoms.shape[0])

    def psi(self, ik, purpose=1, nbnd=None):
        nb = self.nbnd if nbnd is None else nbnd
        return random_bands(nb, int(self.npw[ik]), 1000 * self.index + 10 * ik + purpose)


def config_names():
    return ["c1", "c2", "c3", "c4", "c5"]


def make_workload(name: str, nk_limit: int | None = None) -> Workload:
    """The five workload shapes: c1 fcc 2-atom 12 Ry 20^3 Gamma 8 bands; c2 8-atom cubic
    25 Ry 40^3 4 k 32 bands; c3 64-atom 30 Ry 72^3 16 k 160 bands; c4 the c3 cell with
    Gamma + 16 k; c5 216-atom 30 Ry 108^3 Gamma 500 bands; t2 the 8-atom cell at 30 Ry with
    12 k and 20 bands (training data for the learned preconditioner)."""
    name = name.lower()
    if name == "c1":
        cell, atoms = cell_fcc2()
        w = dict(ecut_ry=12.0, grid=(20, 20, 20), k_cryst=np.zeros((1, 3)), nbnd=8, index=1)
    elif name == "c2":
        cell, atoms = cell_sc_diamond(1)
        w = dict(ecut_ry=25.0, grid=(40, 40, 40), k_cryst=kmesh_c2(), nbnd=32, index=2)
    elif name == "c3":
        cell, atoms = cell_sc_diamond(2)
        w = dict(ecut_ry=30.0, grid=(72, 72, 72), k_cryst=kmesh_c3(), nbnd=160, index=3)
    elif name == "c4":
        cell, atoms = cell_sc_diamond(2)
        w = dict(ecut_ry=30.0, grid=(72, 72, 72),
                 k_cryst=np.concatenate([np.zeros((1, 3)), kmesh_c3()]), nbnd=160, index=4)
    elif name == "t2":
        # training cell for the learned preconditioner: the 8-atom cell at the 64-atom
        # cell's cutoff, k-points {0, 1/2}^3 (the 64-atom Gamma point unfolded) plus the
        # c2 mesh, 20 bands per k (the 64-atom cell's 160 bands per 8 unfolded k-points)
        cell, atoms = cell_sc_diamond(1)
        kf = np.array([[a, b, c] for a in (0, .5) for b in (0, .5) for c in (0, .5)], float)
        w = dict(ecut_ry=30.0, grid=(40, 40, 40), k_cryst=np.concatenate([kf, kmesh_c2()]),
                 nbnd=20, index=6)
    elif name == "c5":
        cell, atoms = cell_sc_diamond(3)
        w = dict(ecut_ry=30.0, grid=(108, 108, 108), k_cryst=np.zeros((1, 3)), nbnd=500, index=5)
    else:
        raise ValueError(f"unknown workload {name}")
    if nk_limit is not None:
        w["k_cryst"] = w["k_cryst"][:nk_limit]
    return Workload(name=name, cell=cell, atoms=atoms, **w)
