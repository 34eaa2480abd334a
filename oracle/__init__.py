"""CPU oracle for one IMEX step of spherical quasi-geostrophic convection.

TEST INFRASTRUCTURE ONLY.  Plain, slow, FP64 NumPy/SciPy code written from
the paper (Gastine, "pizza: an open-source pseudo-spectral code for
spherical quasi-geostrophic convection", arXiv:1902.07092).  Only the test
suite, the entry point's smoke check and the benchmark's CPU-baseline leg
may import it.  It shares no code with the HIP library and imports nothing
from it.

Modules
  grid        radii, Gauss-Lobatto nodes, conducting background (Sect. 2)
  transforms  Fourier pair (eq. fft/ifft) and Chebyshev pair (eq. cheb/icheb)
  operators   Chebyshev-integration operators A,B,C,D,E,F and tau rows
              (Sect. 3.2, eqs. psi_int, uphi_int, temp_int, bc_d3psi_coll)
  bordered    bordered (almost-banded) direct solve (Appendix A)
  step        explicit terms, CNAB2 and BPR353 IMEX steps (Sect. 4)
  diagnostics kinetic/zonal/thermal energy, enstrophy, Re, Ro, CFL (Sect. 6)
  collocation Chebyshev-collocation variant (Sect. 3.1), cross-check only
  eigen       linear eigen-solver for the onset problem (eq. lin), test tool

Every function states the passage of the paper it follows.  Readings taken
where the paper is silent or inconsistent are listed in the module that
takes them.
"""
