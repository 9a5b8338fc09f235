"""Plain FP64 CPU oracle for the Newton-Krylov-BDDC/FETI-DP deluxe Bidomain solver.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and
the CPU-baseline leg of the benchmark may import this package; the device
path never calls it and shares no code with it.

Every function follows one passage of Huynh, Pavarino, Scacchi,
"Parallel Newton-Krylov-BDDC and FETI-DP deluxe solvers for implicit time
discretizations of the cardiac Bidomain equations" (arXiv:2101.02959), cited
by section and equation.  Arithmetic is NumPy/SciPy in float64; there is no
blocking, fusion or reordering beyond what the definitions state.

Modules
  fem      Q1 mesh, conductivity tensors, stiffness and lumped mass (Sec. 2, 3a);
           the truncated ellipsoid with isoparametric Q1 elements (Sec. 6)
  ionic    Rogers-McCulloch model and the Step-1 gating update (Sec. 2, 3b)
  bidomain residual, Jacobian and direct sparse Newton in (v, u_e) (Sec. 3b-c)
  dd       subdomains, N_x classes, local Schur complements (Sec. 4.1)
  bddc     deluxe scaling, vertex+edge-average coarse space, BDDC (Sec. 4.2, 4.4)
  fetidp   jump operators and the FETI-DP operator/preconditioner (Sec. 4.3)
  krylov   PCG with a Lanczos condition estimate (Sec. 4.1, 6)
  newton   Newton with backtracking on the DD-preconditioned PCG (Sec. 3c, 6)
  cnn      FP64 reference of the learned Newton initial-guess network
"""
