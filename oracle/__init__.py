"""Plain FP64 CPU oracle for gauge-canonical-form PEPS variational Monte Carlo of pure Z_N
lattice gauge theory on an open L x L square lattice (arXiv:2503.20566).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its Python
binding) may import, call or link anything in this package; only the tests, the smoke
check and the CPU-baseline leg of the benchmark use it.  It shares no code with the GPU
path: the two meet only through the seeded input generator, which draws random numbers
and holds none of the method's arithmetic.

Modules, each following the passage of the paper it cites:
  lattice   - link labels, Gauss law, plaquette moves           (Hamiltonian section, SM S-2)
  layout    - block-sparse parameter layout and projection       (eq. A, eq. gcf, SM S-2)
  contract  - exact contraction and canonical boundary MPS       (VMC section, SM S-2 eq. project)
  energy    - Hamiltonian tables and the local energy            (eqs. H_b, electric; SM S-1 eq. Es)
  ed        - exact diagonalisation in the link basis            (used only to pin `energy`)
  logderiv  - log-derivatives O_k by reverse-mode autodiff       (SM S-1, definition of O_m)
  sr        - stochastic-reconfiguration force and overlap       (SM S-1 eq. gradient, SM S-3 S_mn)

Every function works in float64 unless it says otherwise.
"""
