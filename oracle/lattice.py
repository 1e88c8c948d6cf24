"""Lattices and units (Sec. 4.2, the Lattice/RealLattice/ReciLattice description).

Cell matrices hold the primitive vectors a_i as rows, in bohr.  The reciprocal
vectors b_i satisfy a_i . b_j = 2 pi delta_ij, i.e. B = 2 pi (A^-1)^T.
"""
import numpy as np

BOHR_IN_ANGSTROM = 0.529177210903      # CODATA 2018 Bohr radius
ANGSTROM = 1.0 / BOHR_IN_ANGSTROM      # one angstrom in bohr
TWO_PI = 2.0 * np.pi


def from_alat(alat, axes_alat):
    """Cell (rows a_i, bohr) from a lattice parameter and axes in units of alat."""
    return float(alat) * np.asarray(axes_alat, dtype=np.float64)


def reciprocal(cell):
    """Rows b_i with a_i . b_j = 2 pi delta_ij."""
    return TWO_PI * np.linalg.inv(np.asarray(cell, np.float64)).T


def volume(cell):
    return abs(float(np.linalg.det(np.asarray(cell, np.float64))))


def tpiba(alat):
    return TWO_PI / float(alat)


def cryst2cart(cell, v_cryst):
    """Crystal (fractional) components -> cartesian; v_cryst [..., 3]."""
    return np.asarray(v_cryst, np.float64) @ np.asarray(cell, np.float64)


def cart2cryst(cell, v_cart):
    return np.asarray(v_cart, np.float64) @ np.linalg.inv(np.asarray(cell, np.float64))
