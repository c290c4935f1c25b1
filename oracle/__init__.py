"""Oracle for the least-action propagator: plain, slow, CPU-only, FP64.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this package.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.

What it computes (Walters, "An efficient parallel method for relaxing to the
minimum action wavefunction"):

* the time-basis matrices U, Q and the initial/final values of the Legendre
  time functions (Sec. "Implementation with Legendre Polynomials");
* the least-action linear system of one time step: the stationarity rows of
  Eq. (stationaryphase) plus one Lagrange-multiplier row per spatial function
  for the initial condition (Sec. "Review of the Least Action Principle");
* its direct solution, the action residual of Eq. (actionresidual) and the
  residual norm of Eq. (residnorm);
* the reference semantics of the subvolume relaxation of Sec. "Iterative
  relaxation to the least action solution" (correction form,
  Eq. (leastaction_correction)) and of the coarse-grid correction of
  Sec. "Multigrid Relaxation", Eqs. (residual_rough) and (correction_fine);
* the adjoint of the step system and the gradients of a loss with respect to
  the potential and to pulse coefficients.

Spatial discretisation (a reading; the paper tests on Legendre elements): one
spatial function per finite-difference grid point, overlap O = identity,
H0 = -(1/2m) times the (2d+1)-point Laplacian with zero values one spacing
outside the grid (or periodic wrap), V_ijnm = delta_ij * int T_n T_m V(x_j,t).

Every function is written from the definitions, with library primitives
(sparse LU, dense solve, Gauss-Legendre nodes, eigh) as steps.  It shares no
code with the HIP library.

Parity status of each part is stated in the module that holds it.
"""
