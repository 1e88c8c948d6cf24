"""FP64 CPU oracle for the plane-wave Kohn-Sham H|psi> and block-Davidson path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) may import, call or link anything here; only the tests, the
smoke check and the CPU-baseline leg of the benchmark do.  The oracle shares no
code with the GPU path: it is plain NumPy/SciPy in float64, written from the
paper's definitions, and each function cites the passage it follows.

Modules
  lattice      real/reciprocal lattice, volumes, coordinate transforms (Sec. 4.2)
  gspace       G-sphere, FFT grid rule, G ordering, r2g/g2r (Sec. 4.3)
  dft_direct   brute-force O(N^2) discrete Fourier transform (pins numpy.fft)
  hamiltonian  kinetic, local (dense and FFT), Kleinman-Bylander non-local,
               dense H_GG' and apply_h_ref (Secs. 2.2, 2.3, 4.3)
  davidson     block Davidson with Teter preconditioner (Sec. 5 'dft' module)
  mlp          2-layer residual->correction MLP: forward, backward, Adam, loss
  density      electron density, Hartree potential and energy, Hartree-only SCF (Sec. 2.1)
  tddft        Taylor exponential, ETRS propagation of the Hartree-only model (Secs. 2.4, 5)
  gw           plane-wave matrix elements M_nn'(k, q, G) of the GW polarizability (Sec. 5)

Parity pins live in tests/ (``-m "not gpu"``); functions without a pin say
"parity unpinned" in their docstring.
"""
