// Device-side state of a bound auxiliary subspace and the launch contexts of
// the per-step kernels.
#pragma once

#include "common.h"

namespace ltd {

constexpr int CHEB_KMAX = 96;  // largest Chebyshev degree of the step exponential
constexpr int TAYLOR_MAX = 8;  // largest order of the explicit (truncated Taylor) step
constexpr int PART_STRIDE = 6; // per-state partial sums of the step and adjoint kernels
// The per-step projection V~ = Phi~^H Y computes only the PROJ_BLK x PROJ_BLK
// blocks on and above the block diagonal (V~ is Hermitian): block rows of
// PROJ_BLK rows starting at the diagonal.
constexpr int PROJ_BLK = 64;

// Per k-point subspace state (lives in the workspace; matrices n_aux x n_aux,
// column-major, in the S-orthonormal basis Phi~ = Phi L^{-H} unless noted).
struct SubDev {
  const double2 *tt;       // T~ (interstitial kinetic)
  const double2 *pt;       // P~ (momentum, z)
  const double2 *vt_ref;   // V~ of the reference potential
  const double2 *h0t;      // H~0 = T~ + V~_ref
  double2 *vt_step;        // V~ rebuilt for the current step (raw, made Hermitian on use)
  const double2 *L;        // Cholesky factor of S_sub (Phi basis), lower
  const double2 *Linv;     // L^{-1}
  const double2 *LH;       // L^H (explicit, for coalesced products)
  const double2 *LinvH;    // L^{-H}
  double2 *work;           // n_states x n_aux^2 scratch when H~ does not fit in LDS
  double2 *hm;             // (H~(t_n + dt/2) - c0)/r of the current step (n_aux^2)
  double *dev;             // per-block partial sums of ||H~(t) - H~0||_F^2
  double kw;               // k-point weight
  double c0, r;            // Chebyshev interval [c0 - r, c0 + r]
  double margin;           // largest ||H~(t) - H~0||_F the interval covers
  int K;                   // series degree for the current dt
  double2 phase;           // exp(-i dt c0)
  double2 coef[CHEB_KMAX + 1];
};

struct StepCtx {
  const SubDev *sub;       // device array [n_k]
  int n_aux, n_states, n_k;
  int h_in_lds;
  int p_in_lds;            // P~ also resident in LDS
  int rebuild;
  int resid;               // rebuilt matrix is the residual V~(t) - V~_ref (FP32 rebuild)
  const int *step;         // device step counter n
  int *step_rw;            // same pointer, advanced by the finaliser
  const double *a_t, *a_mid;
  double c_light, occ, omega, dt;
  double2 *theta;          // [n_k][n_states][n_aux]
  double *part;            // [n_k * n_states][PART_STRIDE] partial sums
  int taylor;              // 0: exponential (Chebyshev series); else order of the truncated Taylor step
  double *nexc_out;        // optional [n_steps+1] excited electrons at t_n
  int *status;
  int *done;               // blocks of the step kernel finished (zero between launches)
  double *j_out, *e_out, *dmu_out;
};

struct AdjCtx {
  int n;                   // step index (forward step n -> n+1), or N when terminal
  int terminal;
  int n_steps;
  const double2 *mu_next;
  double2 *mu_out;
  double *dl_da_mid, *dl_da_t;
};

// dst[i] = src[off + i], i < n, off = (*step) * stride (step on the device) or
// host_off when step is NULL.
// sub != NULL: dst[i] = src[off + i] - sub[i].
hipError_t launch_copy_step(double2 *dst, const double2 *src, long long n, const int *step, long long stride,
                            long long host_off, const double2 *sub, hipStream_t s);
hipError_t launch_copy_rows(double2 *dst, int ldd, const double2 *src, int lds, int rows, int cols, bool zero,
                            hipStream_t s);
// dst[i] = complex64(src[off + i] - sub[i]), i < n (off as launch_copy_step)
hipError_t launch_copy_step32(float2 *dst, const double2 *src, long long n, const int *step, long long stride,
                              long long host_off, const double2 *sub, hipStream_t s);
// complex64 copy of the rows of src (ld lds): rows r < ng as they are, then row
// ng + i from src row ng + perm[i], i < nperm; cols columns
hipError_t launch_rows_to_c64(float2 *dst, int ldd, const double2 *src, int lds, int ng, const int *perm, int nperm,
                              int cols, hipStream_t s);
hipError_t launch_herm_split(const double2 *x, int ldx, int n, int nb, double2 *out, hipStream_t s);
hipError_t launch_axpby(double2 *out, const double2 *a, const double2 *b, double sa, double sb, long long n,
                        hipStream_t s);
hipError_t launch_heff(double2 *out, const double2 *h, const double2 *p, const double2 *o, double al, double be,
                       long long n, hipStream_t s);
hipError_t launch_thv(double *out, const double *th, const double *v, long long n, hipStream_t s);
hipError_t launch_cholesky(const double2 *S, double2 *L, int n, int *status, int *fail, hipStream_t s);
hipError_t launch_trtri(const double2 *L, double2 *Li, int n, hipStream_t s);
// Hermitian eigendecomposition by cyclic Jacobi: A (n x n, destroyed) -> w
// ascending, V (optional) the eigenvectors.  n <= JACOBI_ONE_BLOCK (or no work
// buffer): one block, asynchronous; larger n: one launch per half round with the
// host reading the sweep test (synchronises s), work = jacobi_work_bytes(n).
constexpr int JACOBI_ONE_BLOCK = 128, JACOBI_MAXN = 1024;
size_t jacobi_work_bytes(int n);
hipError_t launch_jacobi(double2 *A, double2 *V, double *w, int n, hipStream_t s, void *work = nullptr);
// dst[i + c ldd] = src[idx[i] + c lds], i < rows, c < cols (row gather)
hipError_t launch_gather_rows(double2 *dst, int ldd, const double2 *src, int lds, const int *idx, int rows, int cols,
                              hipStream_t s);
// out[:, j] = V[:, j] / sqrt(w[j]) (n x n, ld n)
hipError_t launch_scale_cols(double2 *out, const double2 *V, const double *w, int n, hipStream_t s);
size_t step_lds_bytes(int n, bool h_in_lds, bool adjoint, bool p_in_lds = false);
hipError_t launch_conj_transpose(const double2 *a, double2 *out, int n, hipStream_t s);
void subspace_init_attrs();  // LDS limits of the step kernels (call outside graph capture)
hipError_t launch_step(const StepCtx &c, hipStream_t s);
// The two halves of launch_step: H~(mid) of the step (k_assemble), then the
// exponential, observables and step counter (k_step).
hipError_t launch_assemble(const StepCtx &c, hipStream_t s);
// beside: the launch runs beside other kernels (the pipelined rebuild), which
// prefers fewer, longer blocks for the large-subspace form
hipError_t launch_step_only(const StepCtx &c, hipStream_t s, bool beside = false);
// rs[0] = rs[2] = *step, rs[1] = rs[3] = *step + n_steps - 1 (two step-index counters
// of one propagate call, each with its last step)
hipError_t launch_lookahead_init(const int *step, int n_steps, int *rs, hipStream_t s);
// rs[0] = min(rs[0] + 1, rs[1]): the step whose V~ the pipelined rebuild computes
hipError_t launch_lookahead(int *rs, hipStream_t s);
int assemble_blocks(int n);
// hist + (*step mod hist_len) n_k n_states n_aux <- theta (the states before the step)
hipError_t launch_record_theta(const StepCtx &c, double2 *hist, int hist_len, hipStream_t s);
// Block conjugate gradients of the full-basis propagation, one column per
// system (columns of N rows, ld ld): out[j] = sum_i conj(a_ij) b_ij (fixed order,
// one workgroup per column)
hipError_t launch_col_dots(const double2 *a, const double2 *b, int rows, int cols, int ld, double2 *out,
                           hipStream_t s);
// alpha_j = rr_j / Re pq_j; x_j += alpha_j p_j; r_j -= alpha_j q_j
hipError_t launch_cg_step(double2 *x, double2 *r, const double2 *p, const double2 *q, const double2 *rr,
                          const double2 *pq, int rows, int cols, int ld, hipStream_t s);
// beta_j = rrn_j / rr_j; p_j = r_j + beta_j p_j; rr_j = rrn_j
hipError_t launch_cg_dir(double2 *p, const double2 *r, double2 *rr, const double2 *rrn, int rows, int cols, int ld,
                         hipStream_t s);
// y = f (x - c0 z) (f complex), and acc += y when acc is set
hipError_t launch_taylor_term(double2 *y, const double2 *x, const double2 *z, double2 f, double c0, double2 *acc,
                              int rows, int cols, int ld, hipStream_t s);
// y = f y
hipError_t launch_scale_block(double2 *y, double2 f, int rows, int cols, int ld, hipStream_t s);
// *loss = dmu[n] / omega
hipError_t launch_pulse_loss(const double *dmu, int n, double omega, double *loss, hipStream_t s);
hipError_t launch_adjoint(const StepCtx &c, const AdjCtx &a, hipStream_t s);
hipError_t launch_knot_samples(const double *q, int nk, double t_end, double dt, int ns, double *a_t,
                               double *a_mid, hipStream_t s);
hipError_t launch_knot_gradient(const double *g_t, const double *g_mid, int ns, double dt, int nk, double t_end,
                                double *g_q, hipStream_t s);

}  // namespace ltd
