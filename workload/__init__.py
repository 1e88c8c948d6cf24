"""Seeded synthetic inputs shared by the GPU path's tests/bench and the oracle.

This package builds *inputs only*: cells, atom positions, k-points, the
plane-wave basis (Miller lists), a Gaussian model local potential V(r) on the
FFT grid, Gaussian s+p Kleinman-Bylander projectors beta(k+G) with their
coefficient matrix D, and seeded random band coefficients.  It holds none of
the Hamiltonian arithmetic (no H|psi>, no FFT, no eigen-solver); both the
oracle and the HIP library consume the arrays it returns.

Units are Hartree atomic units (bohr, Ha).  A cutoff "X Ry" selects plane
waves with |k+G|^2 <= X bohr^-2 (kinetic energy |k+G|^2/2 <= X/2 Ha), the
Kohn-Sham basis truncation of Sec. 2.2 (eq. KSHamMat and the cutoff below it).
"""
from .synth import (  # noqa: F401
    Workload, make_workload, config_names, cell_fcc2, cell_sc_diamond,
    kmesh_c2, kmesh_c3, miller_sphere, vloc_gaussian, beta_gaussian,
    dmat_sp, random_bands, A_SI,
)
