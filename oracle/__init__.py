"""Plain FP64 CPU oracle for real-space DFT+U Chebyshev-filtered subspace
iteration (arXiv:2507.23612, Sec. II).

TEST INFRASTRUCTURE ONLY.  This package is the independent reference that the
HIP library is checked against.  Only the test suite, the smoke entry point
and the CPU-baseline leg of the benchmark may import it; the product path
never does.  It shares no code with the HIP path: it computes its own
finite-difference weights, potentials, atomic functions, operator, filter,
Rayleigh-Ritz, occupations and mixing, in float64 (complex128 for k != 0),
with numpy/scipy primitives and no blocking or fusion.

Modules
  fd          finite-difference weights and the periodic/Bloch Laplacian
  atoms       real spherical harmonics, radial functions, truncation radii,
              Bloch-mapped atom-centred functions and the local potential
  hamiltonian the discrete operator H[D] (matrix-free and assembled)
  chfsi       Lanczos bound, scaled Chebyshev filter, Rayleigh-Ritz
  scf         occupations, occupation matrices, E_U, density, free energy,
              Pulay mixing and the SCF loop
  mlp         two-hidden-layer SiLU MLP (forward/backward) and descriptors

Parity status of each function is stated in its module header.
"""
