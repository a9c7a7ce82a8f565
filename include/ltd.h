/*
 * ltd.h — LAPW+LO real-time TDDFT hot path on one AMD Instinct MI355X (gfx950).
 *
 * The library applies the velocity-gauge Hamiltonian and the overlap of an
 * LAPW+LO basis to blocks of coefficient vectors without assembling either
 * matrix, projects them onto an auxiliary subspace, and propagates the subspace
 * coefficients (Pela & Draxl, "Speeding up all-electron real-time TDDFT
 * demonstrated by the exciting package": Sec. 2.1 Eqs. (9)-(10), Sec. 2.2
 * Eqs. (11)-(14), Sec. 2.3 Eqs. (15)-(19), App. A Eqs. (A.1)-(A.7)).
 *
 * Conventions for every entry point:
 *  - Pointers are DEVICE pointers unless marked (host).
 *  - Complex numbers are complex128: interleaved (re, im) float64 pairs, 16-byte
 *    aligned (the storage of a torch.complex128 tensor).
 *  - Matrices are column-major with an explicit leading dimension (in
 *    elements).  A contiguous C-order array of shape (cols, rows) is the
 *    column-major rows x cols matrix with leading dimension rows.
 *  - Real-space grids hold N = N1*N2*N3 float64 values, x fastest:
 *    index j1 + N1*(j2 + N2*j3).
 *  - A basis vector of k-point k has N_basis(k) = n_g[k] + N_LO rows: the
 *    plane-wave (LAPW) block first, then the local orbitals of atom 0, atom 1, ...
 *  - `stream` is a hipStream_t passed as void* (NULL: the null stream).
 *    Every call only enqueues work on `stream` (except where it says it
 *    synchronises) and returns before the work ends.
 *  - Status: 0 ok; negative: the arguments were rejected on the host and
 *    nothing was enqueued; positive: a HIP call failed, or the device latched
 *    a failure (read it with ltd_sync_status).  No exception crosses the ABI
 *    and nothing is printed.
 *  - Ownership: the caller owns every buffer, including the workspace.  The
 *    library keeps the device pointers of the system description and of the
 *    bound auxiliary basis, which must stay valid while the system is used.
 *  - Threading: one system is used by one host thread and one stream at a time.
 */
#ifndef LTD_H
#define LTD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ltd_system ltd_system;
typedef int ltd_status;

enum {
  LTD_OK = 0,
  LTD_EINVAL = -1,      /* null pointer, bad enum, non-finite scalar */
  LTD_ESHAPE = -2,      /* sizes or leading dimensions inconsistent */
  LTD_EALIGN = -3,      /* complex pointer not 16-byte aligned */
  LTD_ESTATE = -4,      /* call out of order (no workspace / no subspace bound) */
  LTD_EWORKSPACE = -5,  /* bound workspace smaller than ltd_create asked for */
  LTD_EUNSUPPORTED = -6,/* grid length or mode this build does not handle */
  LTD_ESTEP = -7,       /* time step above the critical time step of the explicit propagator */
  LTD_EHIP = 1,         /* a HIP runtime call failed */
  LTD_ECAPTURE = 5,     /* graph capture: a stream forked from the capture stream was not joined back */
  LTD_ENOTSPD = 2,      /* device: S_sub Cholesky met a pivot <= 0 */
  LTD_ENONFINITE = 3,   /* device: non-finite current, energy or step Hamiltonian */
  LTD_ESPECTRUM = 4     /* device: subspace spectrum left the propagator's interval */
};

typedef enum { LTD_FP64 = 0, LTD_FP32_RESID = 1, LTD_BF16X3_RESID = 2 } ltd_precision;
typedef enum { LTD_STEP_REBUILD = 0, LTD_STEP_AFFINE = 1 } ltd_step_mode;

/* The system: one cell, one real-space grid, n_k k-points, n_atoms atoms.
 * Muffin-tin channels of atom a: n_mt[a] (= n_rad (lmax+1)^2); local orbitals
 * n_lo[a]; N_A = sum n_mt, N_LO = sum n_lo.  Sec. 2.1 Eqs. (6)-(9). */
typedef struct {
  int n_k;                 /* number of k-points, >= 1 */
  const int *n_g;          /* (host) [n_k] plane waves per k-point */
  const int32_t *g_int;    /* (host) [sum n_g][3] integer G triples, k-points concatenated;
                              grid index of G is g mod (N1,N2,N3) and must be injective */
  const double *gk_cart;   /* (host) [sum n_g][3] Cartesian G+k (bohr^-1) */
  int grid[3];             /* N1, N2, N3 (each a product of 2, 3, 5; at most 192) */
  const double *theta_r;   /* [N] step function: 1 interstitial, 0 in spheres (App. A, Eq. (A.2)) */
  const double *v_r;       /* [N] reference Kohn-Sham potential (Ha) */
  int n_atoms;
  const int *n_mt;         /* (host) [n_atoms] */
  const int *n_lo;         /* (host) [n_atoms] */
  const void *amat;        /* per k: N_A x n_g[k] matching coefficients (ld N_A), k-points
                              concatenated; rows = atom 0 channels, atom 1, ... */
  const void *h;           /* per atom: s_a x s_a Hermitian block, s_a = n_mt[a]+n_lo[a], ld s_a,
                              atoms concatenated: muffin-tin Hamiltonian (kinetic + potential) */
  const void *o;           /* same layout: muffin-tin overlap block (positive definite) */
  const void *pz;          /* same layout: muffin-tin momentum block, z component */
  double omega;            /* cell volume (bohr^3) */
  double c_light;          /* speed of light (a.u.) */
  double occ;              /* occupation of every propagated state */
  const double *k_weight;  /* (host) [n_k] k-point weights */
  int n_aux;               /* auxiliary-subspace dimension N_aux (all k) */
  int n_states;            /* propagated states N_states <= n_aux (all k) */
  int max_cols;            /* most columns ever passed to ltd_apply_HS */
  int interstitial_route;  /* LTD_ROUTE_FFT (0): the interstitial plane-wave blocks applied by FFT
                              convolution with the step function (Sec. 2.3, second route);
                              LTD_ROUTE_MM (1): as dense N_G x N_G matrices of Fourier coefficients
                              at G - G' applied by GEMM (Sec. 2.3, first route; App. A, Eq. (A.7)):
                              five N_G^2 complex128 matrices per k-point in the workspace, FP64 only;
                              LTD_ROUTE_FFT_PLANES (2): the FFT route with the apply's transforms as
                              whole-plane x-y passes and z lines on every grid (LTD_ROUTE_FFT takes
                              box arrays and the rebuild's x/z and y kernels where the grid has
                              them); the same sums up to rounding order */
} ltd_system_desc;

enum { LTD_ROUTE_FFT = 0, LTD_ROUTE_MM = 1, LTD_ROUTE_FFT_PLANES = 2 };

/* Validates the description, copies its host arrays and plans every kernel;
 * returns in *workspace_bytes the device workspace the caller must bind.
 * precision: LTD_FP64, or a mixed mode for the per-step potential rebuild
 * (LTD_FP32_RESID: FP32 rebuild of the potential difference on top of the FP64
 * reference).  No device memory is allocated. */
ltd_status ltd_create(const ltd_system_desc *desc, int precision, size_t *workspace_bytes,
                      ltd_system **out);

/* Binds a caller-allocated device workspace of at least the size ltd_create
 * asked for, uploads the plan tables and clears the device status word.
 * Synchronises `stream`. */
ltd_status ltd_bind_workspace(ltd_system *sys, void *workspace, size_t bytes, void *stream);

/* Frees the host-side state; the workspace stays the caller's. */
ltd_status ltd_destroy(ltd_system *sys);

const char *ltd_status_string(ltd_status status);

/* Synchronises `stream`, returns the latched device status (LTD_OK if none)
 * and clears it. */
ltd_status ltd_sync_status(ltd_system *sys, void *stream);

/* HC = H(t) C and SC = S C for the n columns of C at k-point k, with the
 * velocity-gauge H(t) = H0 + (A_z/c) P_z + (A_z^2/2c^2) S (Sec. 2, Eq. (2)
 * expanded as Eq. (15)); H0 = T + V.  The muffin-tin part goes through the
 * matching coefficients and per-atom blocks (Eq. (19); App. A, Eqs.
 * (A.4)-(A.6)), the interstitial part by FFT convolution with the step
 * function (Sec. 2.3, second route; App. A, Eq. (A.7)).  a_vec (host) holds
 * A(t) = (A_x, A_y, A_z); only A_z can enter (the system carries the z
 * momentum block only): a nonzero A_x or A_y returns LTD_EUNSUPPORTED.
 * C, HC, SC: N_basis(k) x n, leading dimensions >= N_basis(k); outputs must
 * not overlap C or each other.  n <= max_cols. */
ltd_status ltd_apply_HS(ltd_system *sys, int k, const double a_vec[3], const void *C, int ldc,
                        int n, void *HC, int ldhc, void *SC, int ldsc, void *stream);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same HC = H(t) C,
 * SC = S C as ltd_apply_HS (same arguments, same kernels), with every scratch
 * buffer of the apply (FFT slabs, muffin-tin vectors and products, effective
 * blocks, GEMM partial sums) taken from a fixed array of
 * LTD_STATIC_SCRATCH_BYTES in the library, one per device, held until the
 * process ends, instead of the bound workspace.  Nothing is allocated or freed.
 * Columns are processed in passes that fit the array; when not even one column
 * fits (an FFT slab of 9 x nbz x N1 x N2 complex values per column plus the
 * blocks) the call returns LTD_EUNSUPPORTED and enqueues nothing.  The system
 * must be bound (its read-only tables stay in the workspace).  Every call on a
 * device shares that device's array: calls that overlap on one device (several
 * streams or host threads) race and must be serialised by the caller.  n has no
 * max_cols limit. */
#define LTD_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
ltd_status ltd_apply_HS_static(ltd_system *sys, int k, const double a_vec[3], const void *C, int ldc,
                               int n, void *HC, int ldhc, void *SC, int ldsc, void *stream);

/* Conventional propagation in the full LAPW+LO basis, the reference the
 * auxiliary subspace is measured against (Sec. 2.1, Eq. (10); Sec. 3.1): the n
 * columns of C (N_basis(k) x n, ld ldc, in/out) are advanced n_steps explicit
 * steps of S dC/dt = -i H(t) C, each the exponential of -i dt S^{-1} H(t_n +
 * dt/2) truncated after `order` Taylor terms about c0 times the exact phase
 * exp(-i dt c0).  Every term applies H by ltd_apply_HS and solves with S by
 * conjugate gradients (one system per column; S is Hermitian positive
 * definite), stopping when every column's relative residual is below cg_tol
 * (checked every 8 iterations) or after cg_max_iter iterations.  The explicit
 * step diverges beyond dt_cr = 0.2 / (eps_max - eps_min) of the full (H0, S)
 * (Sec. 3.1, Eq. (20)); the caller chooses dt (ltd_full_spectrum estimates
 * eps_max).  Host-driven launches (not graph-captured); synchronises `stream`. */
typedef struct {
  double dt;
  int order;               /* Taylor terms, 1..8 */
  double c0;               /* expansion centre (Ha), e.g. (eps_max + eps_min) / 2 */
  const double *a_mid;     /* (host) [n_steps] A_z(t_n + dt/2) */
  int cg_max_iter;         /* >= 1 */
  double cg_tol;           /* > 0 */
  double *cg_resid;        /* (host, optional) out: largest final relative residual of any solve */
  int *cg_iters;           /* (host, optional) out: most iterations any solve used */
} ltd_full_args;
ltd_status ltd_propagate_full(ltd_system *sys, int k, void *C, int ldc, int n, const ltd_full_args *args,
                              int n_steps, void *stream);

/* Largest eigenvalue of the full (H0, S) of k-point k by power iteration on
 * S^{-1} H0 from the start vector x0 (N_basis(k) complex128, device; the
 * caller's seeded draw): `iters` iterations, each one H apply and one CG solve
 * (cg_max_iter, cg_tol as above); *eps_max (host) is the last Rayleigh quotient
 * x^H H0 x / x^H S x.  Synchronises `stream`. */
ltd_status ltd_full_spectrum(ltd_system *sys, int k, const void *x0, int iters, int cg_max_iter, double cg_tol,
                             double *eps_max, void *stream);

/* Binds the auxiliary basis Phi (N_basis(k) x n_aux, ld ldphi; caller-owned,
 * must stay valid and unchanged while the system propagates k) and prepares
 * the subspace (Sec. 2.2, Eq. (14); Sec. 2.3, Eqs. (15)-(16)): applies T, V,
 * P_z and S to Phi, projects them (T_sub, V_sub, P_sub, S_sub, each made
 * Hermitian), factors S_sub = L L^H, caches R = [A Phi_G; Phi_LO] and the
 * plane-wave part of Phi on the real-space grid for the per-step rebuild, and
 * computes the subspace spectrum.  Outputs, each optional (NULL skips):
 * h0_sub, s_sub: n_aux x n_aux (ld n_aux); if C (N_basis x n_states, ld ldc)
 * is given, theta = S_sub^{-1} Phi^H S C (n_aux x n_states, ld n_aux).
 * n_aux must equal the description's.  Synchronises `stream` (the host reads
 * back the spectrum bounds).  A non-positive-definite S_sub returns
 * LTD_ENOTSPD. */
ltd_status ltd_project_subspace(ltd_system *sys, int k, const void *phi, int ldphi, int n_aux,
                                void *h0_sub, void *s_sub, const void *C, int ldc, int n_states,
                                void *theta, void *stream);

/* Rotates the block X (N_basis(k) x n_aux, ld ldx, overwritten) into the
 * Rayleigh-Ritz vectors of (H0, S) over span(X): X <- X W with W^H (X^H S X) W
 * = I and W^H (X^H H0 X) W = diag(eps), eps ascending, written to eps (device,
 * n_aux doubles) if non-NULL.  A stand-in for the ground-state orbitals that
 * form the auxiliary basis (Sec. 2.2, Eq. (11)).  Synchronises `stream`. */
ltd_status ltd_ritz_basis(ltd_system *sys, int k, void *x, int ldx, double *eps, void *stream);

/* Tuner of the per-step rebuild's launch shapes (batched k-points, with the
 * tiles chosen by a tuner rather than fixed): times, on the bound subspaces, every
 * launch shape of the x/z transform kernel (three shapes of the two-factor
 * kernel, whose results do not depend on the shape, and for the FP32 residual
 * on a 64-point rebuild grid a fourth, register-resident kernel: the same
 * transforms in another summation order) and four block targets (256, 512,
 * 1024, 2048) of the K split of the projection GEMM (another summation order),
 * and keeps the fastest of each for the following steps.  choice (host, 3
 * ints): the shape index and the block target chosen, and the number of shapes
 * timed; times_us (host, optional, 8 doubles): the timings, shapes first.
 * Every k-point must be bound.  Synchronises `stream`; invalidates a captured
 * step graph. */
ltd_status ltd_autotune(ltd_system *sys, int *choice, double *times_us, void *stream);

/* Sets the two tuned choices directly (host, 2 ints: x/z launch-shape index in
 * [0, number of shapes of this system), projection block target in [64, 8192]), e.g. to reuse
 * a tuning result saved from an earlier run.  LTD_EINVAL for values outside
 * those ranges.  Invalidates a captured step graph. */
ltd_status ltd_set_tuning(ltd_system *sys, const int *choice);

/* S-orthonormality of the propagated states (mixed precision: S-reorthonormalisation
 * with the drift reported): for every k, G = theta^H S_sub theta (n_states x
 * n_states); *drift (host) = max over k and entries of |G - I|.  With
 * reorthonormalize != 0 the states are replaced by Loewdin's symmetric
 * orthonormalisation theta G^{-1/2} (G = V diag(w) V^H by the device Jacobi
 * solver; the S-orthonormal set closest to theta, spanning the same space).
 * theta (device): n_k x n_states x n_aux as in ltd_step_args, in/out.  Every
 * k-point must be bound.  Synchronises `stream`. */
ltd_status ltd_state_drift(ltd_system *sys, void *theta, int reorthonormalize, double *drift, void *stream);

/* Host read-out of the FFT lengths of the per-step rebuild (lengths[3], host):
 * the smallest supported lengths >= 4 b_i + 1 (b_i the largest |g_i| of the
 * G+k sets) and <= the grid's, so that every difference of two G-box
 * frequencies stays distinct and the convolution with Theta V(t) (Sec. 2.3,
 * Eq. (17)) is exact on them; the grid's own lengths when none is smaller. */
ltd_status ltd_rebuild_grid(const ltd_system *sys, int *lengths);

/* Host read-out of the bound subspace of k: extreme eigenvalues of (H0_sub,
 * S_sub) and the critical time step f/(eps_max - eps_min) with f = 0.2
 * (Sec. 3.1, Eq. (20)).  Any output may be NULL. */
ltd_status ltd_subspace_info(ltd_system *sys, int k, double *eps_min, double *eps_max,
                             double *dt_cr);

typedef struct {
  int mode;               /* LTD_STEP_REBUILD (the potential part is rebuilt from the
                             potential handed in for the step) or LTD_STEP_AFFINE */
  double dt;              /* time step (a.u.), may be negative */
  const double *a_t;      /* [n_steps+1] A_z(t_n), t_n = n dt */
  const double *a_mid;    /* [n_steps]   A_z(t_n + dt/2) */
  int *step;              /* device int n: the step taken is n -> n+1; advanced on the device */
  const double *v_r_t;    /* REBUILD: [N] potential for this step (NULL: the reference) */
  const void *h_t;        /* REBUILD: per-atom Hamiltonian blocks for this step (NULL: reference) */
  void *theta;            /* per k: n_aux x n_states (ld n_aux), k-points concatenated; in/out */
  void *c_out;            /* optional: per k the map-back C = Phi theta, N_basis(k) x n_states
                             (ld N_basis(k)), k-points concatenated; NULL skips */
  double *j_out;          /* [n_steps+1] k-weighted current along z at t_n */
  double *e_out;          /* [n_steps+1] energy at t_n */
  double *dmu_out;        /* [n_steps+1] dipole change along z at t_n */
  long long v_stride;     /* REBUILD: doubles between the potentials of consecutive steps in
                             v_r_t: step n reads v_r_t + n v_stride (0: one potential) */
  long long h_stride;     /* REBUILD: complex elements between the blocks of consecutive steps
                             in h_t: step n reads h_t + n h_stride (0: one set of blocks) */
  int taylor_order;       /* 0: exponential midpoint rule (Chebyshev series to double precision);
                             1..8: explicit step, the Taylor series of exp(-i dt (H~ - c0)) truncated
                             after that many terms (c0 the centre of the bound spectrum), allowed
                             only for |dt| <= 0.2 / (eps_max - eps_min) of every k-point (Sec. 3.1,
                             Eq. (20)); a larger step returns LTD_ESTEP */
  double *nexc_out;       /* optional [n_steps+1]: excited electrons at t_n,
                             f sum_k w_k sum_j (|theta_j|_S^2 - sum_{i < N_states} |<phi_i|S|psi_j>|^2),
                             the states' weight outside the first N_states auxiliary functions
                             (Secs. 3.2-3.3); NULL skips */
  void *theta_hist;       /* optional: before step n the states theta_n are copied to slot
                             n mod hist_len of this buffer (hist_len slots of n_k x n_states x
                             n_aux complex128, the layout of theta): the recomputed segment of a
                             checkpointed backward pass, recorded inside the replayed graph;
                             NULL skips */
  int hist_len;           /* slots of theta_hist (>= 1 when it is set) */
} ltd_step_args;

/* One time step n -> n+1 for every k-point (Sec. 2.2, Eqs. (12)-(13); Sec. 2.3
 * text after Eq. (16): only the potential part is rebuilt): V_sub(t) =
 * sum_a R_a^H h_a(t) R_a + Phi_G^H F[Theta V(t) F^{-1}(Phi_G)] (Eqs. (17)-(19),
 * REBUILD) or the bound reference (AFFINE); H_sub = T_sub + V_sub + (A/c) P_sub
 * + (A^2/2c^2) S_sub at A = a_mid[n] (Eq. (15)); theta <- exp(-i dt
 * S_sub^{-1} H_sub) theta (exponential midpoint rule, FP64 Chebyshev series);
 * optional map-back C = Phi theta (Eq. (12)); then at t_{n+1}: the current
 * J = -(f/Omega) sum_k w_k sum_j Re theta_j^H (P_sub + (A/c) S_sub) theta_j,
 * the energy, and the dipole change delta mu = Omega int J_ind dt (Eq. (4),
 * trapezoid rule).  On the first step (n = 0) entry 0 of the series is
 * written too.  Every k-point needs a bound subspace. */
ltd_status ltd_propagate_step(ltd_system *sys, const ltd_step_args *args, void *stream);

/* n_steps calls of ltd_propagate_step, recorded once into hipGraphs of 32, 8
 * and 1 steps and replayed, the largest that fit first (the device step
 * counter selects the pulse samples and, with nonzero strides, the potential
 * of the step).  REBUILD re-reads v_r_t / h_t every step and is pipelined: the
 * rebuild of V_sub for step n + 1 runs beside the exponential of step n on
 * library-owned streams that join `stream` before the call's work ends, with
 * their own step indices clamped to the call's last step.  The results are
 * bit-identical to n_steps calls of ltd_propagate_step.  The graphs are kept
 * and replayed again while the arguments stay the same. */
ltd_status ltd_propagate(ltd_system *sys, const ltd_step_args *args, int n_steps, void *stream);

/* Captures and instantiates the graphs that a call of ltd_propagate with the
 * same arguments and n_steps replays, without running any step: a caller that
 * times ltd_propagate calls this first so that the capture is outside its timed
 * region (ltd_propagate itself captures on first use).  Enqueues nothing on
 * `stream`. */
ltd_status ltd_propagate_prepare(ltd_system *sys, const ltd_step_args *args, int n_steps, void *stream);

typedef struct {
  const ltd_step_args *fwd; /* the step description (mode, dt, pulse, potential);
                               fwd->theta holds theta_n; fwd->step is not used */
  int n;                    /* (host) the step n -> n+1 to differentiate, 0 <= n < N;
                               with terminal = 1, the last time point n = N */
  int terminal;             /* 1: initialise at t_N: mu_N = dt w_N g_N, no propagator term */
  int n_steps;              /* N, the length of the propagation (trapezoid weights) */
  const void *mu_next;      /* per k: mu_{n+1}, n_aux x n_states (ld n_aux), concatenated */
  void *mu_out;             /* per k: mu_n = U_n^H mu_{n+1} + dt w_n g_n (may equal mu_next) */
  double *dl_da_mid;        /* [N]   entry n: dL/dA(t_n + dt/2) */
  double *dl_da_t;          /* [N+1] entry n: explicit dL/dA(t_n) */
} ltd_adjoint_args;

/* The loss of the pulse-gradient workload, L = dt sum_n w_n (J_n - J_0) =
 * delta mu(T) / Omega (Eq. (4), trapezoid weights): *loss = dmu[n_steps] / Omega
 * on the device, dmu the dipole series a propagation of n_steps wrote. */
ltd_status ltd_pulse_loss(ltd_system *sys, const double *dmu, int n_steps, double *loss, void *stream);

/* One step of the discrete adjoint of ltd_propagate_step for the loss
 * L = dt sum_n w_n (J_n - J_0) (trapezoid weights; L = delta mu(T)/Omega by
 * Eq. (4)): mu_n = U_n^H mu_{n+1} + dt w_n g_n with g_n = -(2f/Omega) w_k
 * (P_sub + (A_n/c) S_sub) theta_n, dL/dA(t_n+dt/2) = Re <mu_{n+1}, (dU_n/dA)
 * theta_n> (derivative of the same Chebyshev series), and the explicit
 * dL/dA(t_n) = dt w_n dJ_n/dA_n (minus T dJ_0/dA_0 at n = 0).  The caller
 * recomputes theta_n (checkpointing).  Does not advance the step counter. */
ltd_status ltd_propagate_step_adjoint(ltd_system *sys, const ltd_adjoint_args *args,
                                      void *stream);

/* Diagnostics (profiling).  Stage durations come from HIP events recorded on
 * `stream` between the stages of an eager (not graph-replayed) run; the host
 * synchronises after every step.  stage_ms: (host) LTD_PROFILE_STAGES doubles.
 *
 * ltd_profile_steps: n_steps calls of ltd_propagate_step (advancing the step
 * counter); stage_ms[i] is the mean per step of stage i: 0 Theta V(t) on the
 * grid, 1 x/z transforms and Theta V product per y plane (the mean of four
 * back-to-back launches of that kernel, which rewrite the same output, so the
 * figure is its launch duration without the latency after the event), 2 y transforms and
 * sphere read-out, 3 muffin-tin block products, 4 projection of V~ (Phi~^H Y), 5 subspace
 * exponential and observables, 6 map-back.
 *
 * ltd_profile_apply: one ltd_apply_HS at A = 0 (HC, SC: N_basis(k) x n, ld ldo);
 * stage_ms[i] is the total of: 0 inverse plane transforms, 1 z lines and
 * products, 2 forward plane transforms, 3 A C (muffin-tin gather GEMM), 4 block
 * products, 5 A^H Y (scatter GEMM) and local-orbital rows. */
#define LTD_PROFILE_STAGES 8
ltd_status ltd_profile_steps(ltd_system *sys, const ltd_step_args *args, int n_steps, double *stage_ms,
                             void *stream);
ltd_status ltd_profile_apply(ltd_system *sys, int k, const void *C, int ldc, int n, void *HC, void *SC,
                             int ldo, double *stage_ms, void *stream);

/* Piecewise-linear pulse on n_knots uniform knots over [0, t_end] (both ends
 * included): a_t[n] = A(n dt), n = 0..n_steps, a_mid[n] = A((n+1/2) dt).
 * knots: [n_knots]. */
ltd_status ltd_knot_samples(const double *knots, int n_knots, double t_end, double dt,
                            int n_steps, double *a_t, double *a_mid, void *stream);

/* Chain rule of ltd_knot_samples: dl_dq[k] = sum_n dl_da_t[n] phi_k(t_n) +
 * sum_n dl_da_mid[n] phi_k(t_n + dt/2), phi_k the hat functions. */
ltd_status ltd_knot_gradient(const double *dl_da_t, const double *dl_da_mid, int n_steps,
                             double dt, int n_knots, double t_end, double *dl_dq, void *stream);

/* Vector potential samples of the paper's excitations along z:
 * a_t[n] = A(n dt), n = 0..n_steps, a_mid[n] = A((n + 1/2) dt), n < n_steps.
 * kind / params (host, 4 doubles):
 *   LTD_PULSE_SIN2: (A0, w, t0, T_p): A0 cos(w t) sin^2[pi (t - t0)/T_p] for
 *     t0 <= t <= t0 + T_p, 0 outside (the laser of Sec. 3.2);
 *   LTD_PULSE_KICK: (E0, c, -, -): an impulsive field E0 delta(t - 0+), i.e.
 *     A = -c E0 for t > 0 and 0 at t = 0 (the kick of Sec. 3.1);
 *   LTD_PULSE_GAUSS_SIN: (A0, w, t0, width): A0 sin(w t) exp(-((t - t0)/width)^2).
 * Non-finite parameters, T_p, width or c <= 0 return LTD_EINVAL. */
enum { LTD_PULSE_GAUSS_SIN = 0, LTD_PULSE_SIN2 = 1, LTD_PULSE_KICK = 2 };
ltd_status ltd_pulse_samples(int kind, const double *params, double dt, int n_steps, double *a_t, double *a_mid,
                             void *stream);

/* Dynamical polarizability alpha_zz(w) = (i Omega / w) J(w) / E(w) (Sec. 2,
 * Eq. (5)) from the current series j[0..n_steps] (J at t_n = n dt, as written by
 * the propagation; J_ind = J - J(0)) and the potential samples a_t[0..n_steps]:
 *   J(w) = dt sum_n w_n J_ind(t_n) exp((i w - gamma) t_n), trapezoid weights,
 *   E(w) = -(1/c) sum_n (A(t_{n+1}) - A(t_n)) exp((i w - gamma) t_{n+1/2}),
 * the field E = -(1/c) dA/dt of the sampled A; gamma >= 0 damps the tail.
 * w: [n_w] nonzero frequencies (a.u.); alpha: [n_w] complex128 out.  One
 * workgroup per frequency, fixed-order sums. */
ltd_status ltd_polarizability(const double *j, const double *a_t, int n_steps, double dt, double omega_cell,
                              double c_light, const double *w, int n_w, double gamma, void *alpha, void *stream);

/* Coefficients of the Chebyshev series exp(-i tau x) = sum_k c_k T_k(x) on
 * [-1, 1]: c_k = (2 - delta_k0) (-i)^k J_k(tau) (host; Bessel functions by
 * Miller's backward recurrence).  Writes kmax+1 complex values (interleaved
 * re, im) to coef (host) and returns the truncation degree in *degree. */
ltd_status ltd_chebyshev_coefficients(double tau, int kmax, double *coef, int *degree);

#ifdef __cplusplus
}
#endif
#endif /* LTD_H */
