"""Oracle G-space against the paper's GSpace example (Sec. 4.3) and the workloads."""
import numpy as np
import pytest

from oracle import gspace, lattice
import workload


def _fe_cell(golden):
    g = golden("crystal_fe_bcc.txt")
    return lattice.from_alat(g["alat"][0], np.reshape(g["axes_alat"], (3, 3)))


def test_gspace_example(golden):
    cell = _fe_cell(golden)
    g = golden("gspace_fe_160ry.txt")
    grid = gspace.grid_rule(cell, 160.0)
    assert list(grid) == [int(x) for x in g["grid_shape"]]
    assert int(np.prod(grid)) == int(g["size_r"][0])
    m = gspace.sphere(cell, 160.0, grid)
    assert m.shape[0] == int(g["size_g"][0])
    for ax, name in enumerate(("g1", "g2", "g3")):
        np.testing.assert_array_equal(m[:5, ax], g[name + "_head"])
        np.testing.assert_array_equal(m[-5:, ax], g[name + "_tail"])
    n2 = gspace.norm2(cell, m)
    np.testing.assert_allclose(np.round(n2[:5], 1), g["gnorm2_head"], atol=1e-9)
    np.testing.assert_allclose(np.round(n2[-5:], 1), g["gnorm2_tail"], atol=1e-9)


def test_sphere_boundary_reading(golden):
    """'<=' and '<' give the same count for the printed example (no G on the boundary)."""
    cell = _fe_cell(golden)
    grid = gspace.grid_rule(cell, 160.0)
    a = gspace.sphere(cell, 160.0, grid, slack=1e-12)
    b = gspace.sphere(cell, 160.0 * (1 - 1e-9), grid)
    assert a.shape == b.shape


def test_r2g_identity():
    """r2g equals fftn followed by taking the sphere, and g2r inverts it on the sphere."""
    rng = np.random.default_rng(3)
    cell, _ = workload.cell_fcc2()
    grid = (12, 10, 9)
    m = gspace.sphere(cell, 4.0, grid)
    c = rng.standard_normal(m.shape[0]) + 1j * rng.standard_normal(m.shape[0])
    np.testing.assert_allclose(gspace.r2g(gspace.g2r(c, m, grid), m, grid), c, atol=1e-13)
    f = rng.standard_normal(grid) + 1j * rng.standard_normal(grid)
    full = np.fft.fftn(f).reshape(-1)
    np.testing.assert_allclose(gspace.r2g(f, m, grid), full[gspace.idxgrid(m, grid)], atol=1e-12)


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_workload_sphere_matches_oracle(name):
    """The input generator's Miller lists are exactly the oracle's sphere, in the same order."""
    w = workload.make_workload(name)
    for ik in range(w.nk):
        ref = gspace.sphere(w.cell, w.ecut_ry, w.grid, w.k_cryst[ik])
        np.testing.assert_array_equal(w.miller[ik], ref)


def test_grid_rule_configs():
    """Workload grids are at least the rule's minimum; the 72^3 and 108^3 grids equal it."""
    for name, exact in (("c1", False), ("c2", False), ("c3", True), ("c5", True)):
        w = workload.make_workload(name, nk_limit=1)
        rule = gspace.grid_rule(w.cell, 4 * w.ecut_ry)
        assert all(a >= b for a, b in zip(w.grid, rule))
        if exact:
            assert tuple(w.grid) == tuple(rule)
