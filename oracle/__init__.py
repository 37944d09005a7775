"""Plain FP64 CPU oracle for the coupled BSSN + Valencia GRMHD spectral RK stage.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library or its Python binding
imports, calls or links anything under ``oracle/``.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` use it.

The oracle is written to be read against the paper (arXiv 2508.18221), not to be
fast: every function takes the paper's route (Chebyshev coefficients through
``numpy.polynomial.chebyshev.chebder``, FFT derivatives with the paper's k set,
modal filtering, classic RK4) or, where the method only approaches a result
that has a plain definition (con2prim), computes that definition directly by a
bracketed root search.  Where the paper is garbled the standard published form
it names (Valencia GRMHD, BSSN as in Alcubierre's textbook) is used; every such
reading is stated in the docstring of the function that takes it.

Modules
  spectral     grid nodes, maps, derivative and filter operators (Methods,
               "Grid Discretization", "Spectral Derivative Operators",
               "Dealiasing and Spectral Filtering")
  kerr_schild  Kerr metric in Kerr-Schild form and its 3+1 split
               (Results, "The Kerr-Schild Metric and 3+1 Decomposition")
  grmhd        EOS, conserved variables, con2prim, fluxes, 3+1 sources
               (Results, "GRMHD Conservative Form"; Methods, "Primitive Variable
               Recovery", "Conserved Fluxes and Geometric Source Terms")
  bssn         BSSN + 1+log + Gamma-driver right-hand side (Methods,
               "BSSN Evolution Equations", "Gauge Conditions")
  initial_data Kerr-Schild BSSN data, Michel accretion, monopole field,
               seeded perturbation
  evolve       full RHS, boundary freeze, RK4 step, filter, CFL time step
               (Methods, "Time Integration", "The Stability and Complexity")
  diagnostics  Hamiltonian constraint, rest mass, discrete entropy E^n
"""

from . import spectral, kerr_schild, grmhd, bssn, initial_data, evolve, diagnostics  # noqa: F401
