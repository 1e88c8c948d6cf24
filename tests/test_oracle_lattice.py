"""Oracle lattice code against the values the paper prints (Sec. 4.2)."""
import numpy as np

from oracle import lattice


def test_bcc_5p1_angstrom(golden):
    g = golden("lattice_bcc_5p1A.txt")
    axes = 0.5 * np.array([[1, 1, 1], [-1, 1, 1], [-1, -1, 1]], float)
    alat = 5.1 * lattice.ANGSTROM
    assert abs(alat - g["alat"][0]) <= 1e-12 * alat
    cell = lattice.from_alat(alat, axes)
    tp = lattice.tpiba(alat)
    assert abs(tp - g["tpiba"][0]) <= 1e-12 * tp
    b = lattice.reciprocal(cell)
    np.testing.assert_allclose(b / tp, np.reshape(g["axes_tpiba"], (3, 3)), atol=1e-14)
    v = np.array([[1, 0, 0], [0, 1, 0], [1, 1, 0], [0, 1, 1]], float)
    cart = lattice.cryst2cart(cell, v)
    np.testing.assert_allclose(cart, np.reshape(g["vec_cart"], (4, 3)), atol=5e-9)
    np.testing.assert_allclose(cart / alat, np.reshape(g["vec_alat"], (4, 3)), atol=1e-14)
    np.testing.assert_allclose(np.linalg.norm(cart, axis=1) / alat, g["len_over_alat"], atol=5e-9)
    # round trip and duality a_i . b_j = 2 pi delta_ij
    np.testing.assert_allclose(lattice.cart2cryst(cell, cart), v, atol=1e-13)
    np.testing.assert_allclose(cell @ b.T, 2 * np.pi * np.eye(3), atol=1e-13)


def test_fe_bcc_printout(golden):
    g = golden("crystal_fe_bcc.txt")
    cell = lattice.from_alat(g["alat"][0], np.reshape(g["axes_alat"], (3, 3)))
    assert abs(lattice.volume(cell) - g["volume"][0]) <= 5e-6
    tp = lattice.tpiba(g["alat"][0])
    assert abs(tp - g["tpiba"][0]) <= 5e-6
    np.testing.assert_allclose(lattice.reciprocal(cell) / tp, np.reshape(g["axes_tpiba"], (3, 3)),
                               atol=1e-14)
