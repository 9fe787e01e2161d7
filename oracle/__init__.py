"""FP64 CPU oracle for the finite-element P3M method (Beams, Olson & Freund,
"A Finite Element Based P3M Method for N-body Problems").

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package; only the tests, the smoke check and the benchmark's CPU
baseline leg use it.  It shares no code with the HIP library: every step is
written here again from the paper, in plain NumPy/SciPy, in float64, with
exact linear algebra (dense eigen-decompositions) in place of iterative
solves.

Modules
  geometry  wrap and bin charges into elements (Section 2, element offsets)
  fe1d      1-D order-p Lagrange elements, Gauss quadrature, K1/M1 matrices
  screens   one-element polynomial screens, dual functions (eq. moment1d)
  potential exact free-space potential of a screen density (eq. screenintegral)
  tables    screen-potential tables as Dirichlet FE solutions (Remark, Section 4)
  mesh      load vector (eq. defineassign) and exact periodic FE solve
  fep3m     the whole method, stage by stage (Algorithm 1)
  ewald     classic Ewald summation and direct image sums (ground truth)
"""
