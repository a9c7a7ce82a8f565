"""CPU FP64 oracle for the LAPW+LO real-time TDDFT hot path — TEST INFRASTRUCTURE.

This package is the plain, slow reference against which the GPU library is
checked.  It is not part of the product: only the test-suite, the smoke check
and the CPU-baseline leg of the benchmark may import it.  It shares no code with
the GPU path; both read the same seeded inputs from ``synth``.

Modules (each function cites the passage of Pela & Draxl, "Speeding up
all-electron real-time TDDFT demonstrated by the exciting package", that it
follows):

* ``operators`` — the LAPW+LO operators H0, S, P_z, T, V: dense assembly from
  their matrix elements, and the matrix-free applies (FFT route and MM route).
* ``subspace`` — projection onto the auxiliary basis, Rayleigh-Ritz ground
  state stand-in, the per-step potential rebuild.
* ``propagate`` — the subspace propagator (exponential midpoint rule),
  observables (current, dipole change, energy), the critical time step.
* ``adjoint`` — the discrete adjoint of the propagation for pulse gradients.

Readings taken where the paper is silent (also listed in the design notes):

* R1 propagator: exponential midpoint rule, theta_{n+1} = exp(-i dt
  S_sub^{-1} H_sub(t_n + dt/2)) theta_n, evaluated through the Cholesky factor
  of S_sub and a Hermitian eigendecomposition.
* R2 non-orthonormal subspace: S_sub theta' = -i H_sub theta.
* R3 the "^T" on the LO-LAPW block of the muffin-tin potential is read as a
  Hermitian conjugate.
* R4 interstitial matrix elements use the discrete transform
  f~(q) = (1/N) sum_j f_j exp(-2 pi i q.j/N) (grid of N points), so that the
  FFT and the matrix-matrix routes agree exactly.
* R5 the step function is 0 strictly inside a sphere image, 1 elsewhere.
* R6 interstitial kinetic element 1/2 (G+k).(G'+k) Theta~(g-g'); the
  muffin-tin kinetic energy is part of the synthetic block h_alpha.
* R7 momentum: interstitial 1/2 [(G+k)_z + (G'+k)_z] Theta~(g-g'), muffin-tin
  block p_z,alpha (synthetic).
* R8 current J = -(f/Omega) sum_j Re theta_j^H (P_sub + (A/c) S_sub) theta_j,
  f = 2, J_ind = J - J(0), dipole change by the trapezoid rule.
* R9 theta(0) = first N_states unit vectors; the auxiliary basis is the lowest
  eigenvectors of (H0, S) (dense, small systems) or Rayleigh-Ritz vectors of a
  start block (large systems).
* R10 time grid t_n = n dt, pulse sampled at t_n and t_n + dt/2.
* R11 per-step rebuild: only the potential part of H_sub is rebuilt each step.

Parity: every function here is pinned by the tests in ``tests/test_oracle_*``
(brute force, closed forms, an independent matrix exponential, finite
differences, the paper's printed timing/speedup table).  Physics against the
paper's figures is *parity unpinned*: the paper prints no numeric outputs for
any system that can be rebuilt without its data.
"""
