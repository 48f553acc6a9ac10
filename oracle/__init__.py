"""FP64 CPU oracle for the npFEM red-blood-cell time step.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference that the GPU path is checked against.  Only the test suite, the smoke
check and the benchmark's CPU-baseline leg may import it; the product library never
does, and it shares no code, tables or helpers with the HIP path.

It follows Kotsalos, Latt & Chopard, "Bridging the computational gap between
mesoscopic and continuum modeling of red blood cells for fully resolved blood flow"
(arXiv:1903.06479):

  model.py   rest data of a mesh (section 2.1.2 and Appendix B), lumped masses
             (section 2.1), the PD matrix L (eq. fullyDeveloped_g), M~ = M + hC
             (eq. preOptimizationNewton, section 2.1.4) and H~ = M~/h^2 + L (section 2.1.1)
  energy.py  local-area PD energy (section 2.1.2, SL(2) projection), bending PD energy
             (eq. BendingDiscretizedPotential), global-volume PD energy (section 2.1.2),
             modified Skalak energy and its forces (section 2.1.3)
  step.py    objective and gradient (eqs. GeneralizedObjectiveFunction and
             GeneralizedObjectiveFunctionDerivative), first guess, L-BFGS with H~ as
             initial Hessian and halving line search (Algorithm 1), velocity update and
             the post-convergence dissipation (section 2.1.4)
  collision.py  contact search between cells and the collision term (section 4.7)
  newton.py  brute-force Newton with a finite-difference Jacobian (test pin)
  mpnn.py    FP64 forward/backward of the learned warm-start network

Every floating-point quantity is float64.  Units are whatever the caller uses
consistently (the tests use um, us, pN, fg).
"""
