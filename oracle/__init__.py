"""FP64 CPU oracle for the LRI-G0W0 imaginary-frequency screening and
self-energy path of Ren et al., "All-electron periodic G0W0 implementation
with numerical atomic orbital basis functions: algorithm and benchmarks"
(arXiv:2011.01400).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
NumPy implementation written from the paper's equations.  It exists to check
the HIP library; only the test suite, the smoke check and the CPU-baseline leg
of the benchmark may import it.  It shares no code with the HIP path and the
product never calls it.

Modules
  grids          k/q grids, index maps, modified Gauss-Legendre frequencies
  lri            Bloch transform of the two-centre coefficients (Eqs.
                 expan_coeff_FT1/2), AO triple coefficients (Eq.
                 AO_triple_split2), AO->MO transform (Eq. AO_MO_transform)
  response       chi0 on the auxiliary basis (Eq. chi0_matrix), both the
                 time-reversal form and the literal Adler-Wiser sum
  screening      symmetrised dielectric matrix, its inverse and W^c (Eqs.
                 symm_dielec_func, screened_W_matr), Gamma-point treatment in
                 the Coulomb eigenbasis (Eq. dielectric_func_gamma)
  selfenergy     correlation self-energy (Eq. GW_selfe_element with W -> W^c)
  continuation   Thiele Pade continued fraction and the quasiparticle equation
  contour        Sigma^c at real energies by contour deformation (imaginary-axis
                 integral plus residues, W^c below the smallest transition)
  pipeline       the whole path for one synthetic cell

Pins live in tests/test_oracle_*.py.  Functions without an independent pin
say so in their docstring ("parity unpinned").
"""
