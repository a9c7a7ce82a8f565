// Subspace kernels: small dense FP64 linear algebra (Cholesky, triangular
// inverse, Hermitian Jacobi eigensolver), the per-step propagation of the
// subspace coefficients with observables, the adjoint step, and helpers of
// the muffin-tin chain.
//
// The propagation works in the S-orthonormal basis Phi~ = Phi L^{-H}
// (S_sub = L L^H): there H~ = L^{-1} H_sub L^{-H} is Hermitian, the step
// propagator of the exponential midpoint rule is exp(-i dt H~(t_n + dt/2))
// (Pela & Draxl, Sec. 2.2, Eq. (13); Sec. 2.1, Eq. (10)), and theta~ = L^H
// theta.  The exponential is applied to each state as a Chebyshev series,
// exp(-i dt H~) = exp(-i dt c0) sum_k c_k T_k(X), X = (H~ - c0)/r, with the
// spectrum of H~ inside [c0 - r, c0 + r] and c_k = (2 - delta_k0) (-i)^k
// J_k(r dt).  One workgroup propagates one state of one k-point; H~ stays in
// LDS for the whole series.
#include "common.h"
#include "subspace.h"

#include <cmath>

namespace ltd {

namespace {

__device__ inline void latch(int *status, int code) {
  if (status) atomicCAS(status, 0, code);
}

// Block-wide y = op(A) v, A n x n column-major with leading dimension lda
// (LDS or global); v, y in LDS (y must not alias v); red: blockDim doubles2.
template <bool CONJT>
__device__ void matvec(const double2 *A, int lda, const double2 *v, double2 *y, int n, double2 *red) {
  const int t = threadIdx.x, nt = blockDim.x;
  if (n <= nt) {
    const int np = nt / n;
    const int i = t % n, part = t / n;
    double2 s = make_double2(0.0, 0.0);
    if (part < np) {
      const int k0 = (part * n) / np, k1 = ((part + 1) * n) / np;
#pragma unroll 8
      for (int k = k0; k < k1; ++k) {
        if (CONJT) s = cfma(cconj(A[(long long)k + (long long)i * lda]), v[k], s);
        else s = cfma(A[(long long)i + (long long)k * lda], v[k], s);
      }
    }
    red[t] = s;
    __syncthreads();
    if (t < n) {
      double2 acc = red[t];
      for (int p = 1; p < np; ++p) acc = cadd(acc, red[p * n + t]);
      y[t] = acc;
    }
    __syncthreads();
  } else {
    for (int i = t; i < n; i += nt) {
      double2 s = make_double2(0.0, 0.0);
      for (int k = 0; k < n; ++k) {
        if (CONJT) s = cfma(cconj(A[(long long)k + (long long)i * lda]), v[k], s);
        else s = cfma(A[(long long)i + (long long)k * lda], v[k], s);
      }
      y[i] = s;
    }
    __syncthreads();
  }
}

// Block-wide y = A v for A in global memory (n x n, column-major, ld lda), v and
// y in LDS: lane l of wave w accumulates rows l + 64 r (r < RPL) over the
// columns k = w, w + NW, ... (NW waves), four columns per iteration so that
// 4 RPL independent loads are in flight; the waves' partial sums meet in red
// (NW n values) and are added in wave order.  Row indices are clamped so that
// every load is in bounds and branch-free.
template <int RPL>
__device__ void matvec_wide(const double2 *__restrict__ A, int lda, const double2 *v, double2 *y, int n,
                            double2 *red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  double2 acc[RPL];
  int row[RPL];
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    acc[r] = make_double2(0.0, 0.0);
    const int i = lane + 64 * r;
    row[r] = i < n ? i : n - 1;
  }
  int k = w;
  for (; k + 3 * nw < n; k += 4 * nw) {
    double2 a[4][RPL];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int r = 0; r < RPL; ++r) a[u][r] = A[(long long)row[r] + (long long)(k + u * nw) * lda];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double2 vk = v[k + u * nw];
#pragma unroll
      for (int r = 0; r < RPL; ++r) acc[r] = cfma(a[u][r], vk, acc[r]);
    }
  }
  for (; k < n; k += nw) {
    const double2 vk = v[k];
#pragma unroll
    for (int r = 0; r < RPL; ++r) acc[r] = cfma(A[(long long)row[r] + (long long)k * lda], vk, acc[r]);
  }
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    const int i = lane + 64 * r;
    if (i < n) red[(long long)w * n + i] = acc[r];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double2 t = red[i];
    for (int q = 1; q < nw; ++q) t = cadd(t, red[(long long)q * n + i]);
    y[i] = t;
  }
  __syncthreads();
}

// matvec_wide for n <= 320 (rows per lane ceil(n / 64))
__device__ void matvec_g(const double2 *__restrict__ A, int lda, const double2 *v, double2 *y, int n, double2 *red) {
  switch ((n + 63) / 64) {
    case 1: matvec_wide<1>(A, lda, v, y, n, red); break;
    case 2: matvec_wide<2>(A, lda, v, y, n, red); break;
    case 3: matvec_wide<3>(A, lda, v, y, n, red); break;
    case 4: matvec_wide<4>(A, lda, v, y, n, red); break;
    default: matvec_wide<5>(A, lda, v, y, n, red); break;
  }
}

// Block-wide sum of one double per thread (fixed order); result valid in all threads.
__device__ double block_sum(double x, double *sred) {
  const int t = threadIdx.x;
  sred[t] = x;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) sred[t] += sred[t + s];
    __syncthreads();
  }
  const double r = sred[0];
  __syncthreads();
  return r;
}

// Sums of three doubles over the block: butterfly within each wavefront, then
// the per-wave sums in wave order (deterministic).  sred: >= 3 * (blockDim/64).
__device__ inline double wave_sum(double x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}
__device__ void block_sum3(double &a, double &b, double &c, double *sred) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  if (lane == 0) {
    sred[3 * wv] = a;
    sred[3 * wv + 1] = b;
    sred[3 * wv + 2] = c;
  }
  __syncthreads();
  a = b = c = 0.0;
  for (int q = 0; q < nw; ++q) {
    a += sred[3 * q];
    b += sred[3 * q + 1];
    c += sred[3 * q + 2];
  }
  __syncthreads();
}

__global__ void k_conj_transpose(const double2 *a, double2 *out, int n) {
  const long long tot = (long long)n * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), j = (int)(e / n);
    out[e] = cconj(a[j + (long long)i * n]);
  }
}

// Re sum_i conj(a_i) b_i over n entries in LDS (block-wide, fixed order).
__device__ double dot_re(const double2 *a, const double2 *b, int n, double *sred) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += a[i].x * b[i].x + a[i].y * b[i].y;
  return block_sum(s, sred);
}

// ---------------------------------------------------------------------------
// Elementwise helpers
// ---------------------------------------------------------------------------
__global__ void k_copy_rows(double2 *dst, int ldd, const double2 *src, int lds, int rows, int cols, int zero) {
  const long long tot = (long long)rows * cols;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(e % rows), j = (int)(e / rows);
    dst[r + (long long)j * ldd] = zero ? make_double2(0.0, 0.0) : src[r + (long long)j * lds];
  }
}

__global__ void k_herm_split(const double2 *x, int ldx, int n, int nb, double2 *out) {
  // out[b] (n x n, contiguous) = (X_b + X_b^H)/2 with X_b = x[:, b*n:(b+1)*n]
  const long long tot = (long long)nb * n * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const int b = (int)(e / ((long long)n * n));
    const int r = (int)(e % ((long long)n * n));
    const int i = r % n, j = r / n;
    const double2 a = x[i + (long long)(b * n + j) * ldx];
    const double2 c = x[j + (long long)(b * n + i) * ldx];
    out[e] = make_double2(0.5 * (a.x + c.x), 0.5 * (a.y - c.y));
  }
}

__global__ void k_axpby_n2(double2 *out, const double2 *a, const double2 *b, double sa, double sb, long long n) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
    out[e] = make_double2(sa * a[e].x + sb * b[e].x, sa * a[e].y + sb * b[e].y);
}

__global__ void k_heff(double2 *out, const double2 *h, const double2 *p, const double2 *o, double al, double be,
                       long long n) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
    out[e] = make_double2(h[e].x + al * p[e].x + be * o[e].x, h[e].y + al * p[e].y + be * o[e].y);
}

__global__ void k_copy_step(double2 *__restrict__ dst, const double2 *__restrict__ src, long long n,
                            const int *step, long long stride, long long host_off, const double2 *__restrict__ sub) {
  const long long off = step ? (long long)(*step) * stride : host_off;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    dst[i] = sub ? csub(src[off + i], sub[i]) : src[off + i];
}

// dst[i] = complex64(src[off + i] - sub[i]) (the FP32 residual's block difference)
__global__ void k_copy_step32(float2 *__restrict__ dst, const double2 *__restrict__ src, long long n, const int *step,
                              long long stride, long long host_off, const double2 *__restrict__ sub) {
  const long long off = step ? (long long)(*step) * stride : host_off;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double2 v = csub(src[off + i], sub[i]);
    dst[i] = make_float2((float)v.x, (float)v.y);
  }
}

// dst rows (complex64, ld ldd): rows r < ng copy src row r; row ng + i copies src row ng + perm[i]
__global__ void k_rows_to_c64(float2 *dst, int ldd, const double2 *src, int lds, int ng, const int *perm, int nperm,
                              int cols) {
  const int rows = ng + nperm;
  const long long tot = (long long)rows * cols;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(e % rows), c = (int)(e / rows);
    const int sr = r < ng ? r : ng + perm[r - ng];
    const double2 v = src[sr + (long long)c * lds];
    dst[r + (long long)c * ldd] = make_float2((float)v.x, (float)v.y);
  }
}

__global__ void k_thv(double *out, const double *th, const double *v, long long n) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
    out[e] = th[e] * v[e];
}

// ---------------------------------------------------------------------------
// Cholesky S = L L^H (lower), one workgroup, left-looking by columns.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_cholesky(const double2 *S, double2 *L, int n, int *status, int *fail) {
  __shared__ double2 col[320];
  __shared__ int bad;
  const int t = threadIdx.x;
  if (t == 0) bad = 0;
  for (long long e = t; e < (long long)n * n; e += blockDim.x) L[e] = make_double2(0.0, 0.0);
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    for (int i = j + t; i < n; i += blockDim.x) {
      double2 s = S[i + (long long)j * n];
      for (int k = 0; k < j; ++k) s = csub(s, cmul(L[i + (long long)k * n], cconj(L[j + (long long)k * n])));
      col[i] = s;
    }
    __syncthreads();
    const double d = col[j].x;
    if (!(d > 0.0) || !isfinite(d)) {
      if (t == 0) bad = 1;
      __syncthreads();
      break;
    }
    const double sd = sqrt(d);
    for (int i = j + t; i < n; i += blockDim.x)
      L[i + (long long)j * n] = (i == j) ? make_double2(sd, 0.0) : cscale(col[i], 1.0 / sd);
    __syncthreads();
  }
  if (t == 0) {
    if (bad) latch(status, 2);
    if (fail) *fail = bad;
  }
}

// Inverse of a lower-triangular matrix, one thread per column (forward substitution).
__global__ void k_trtri(const double2 *L, double2 *Li, int n) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  for (int i = 0; i < c; ++i) Li[i + (long long)c * n] = make_double2(0.0, 0.0);
  for (int i = c; i < n; ++i) {
    double2 s = (i == c) ? make_double2(1.0, 0.0) : make_double2(0.0, 0.0);
    for (int k = c; k < i; ++k) s = csub(s, cmul(L[i + (long long)k * n], Li[k + (long long)c * n]));
    const double2 d = L[i + (long long)i * n];
    const double den = d.x * d.x + d.y * d.y;
    Li[i + (long long)c * n] = make_double2((s.x * d.x + s.y * d.y) / den, (s.y * d.x - s.x * d.y) / den);
  }
}

// ---------------------------------------------------------------------------
// Hermitian eigensolver: cyclic two-sided Jacobi with round-robin parallel
// ordering (disjoint rotations applied together), one workgroup.  A (n x n,
// column-major, global) is overwritten; V (if non-null) receives the
// eigenvectors as columns; w the eigenvalues, ascending (V sorted along).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_jacobi(double2 *A, double2 *V, double *w, int n, int max_sweeps) {
  __shared__ double sc[160], ss[160];
  __shared__ double2 se[160];
  __shared__ int sp[160], sq[160];
  __shared__ double sred[1024];
  __shared__ int perm[320];
  const int t = threadIdx.x, nt = blockDim.x;
  const int m = (n + 1) & ~1;  // players (one dummy if n is odd)
  const int half = m / 2;
  if (V)
    for (long long e = t; e < (long long)n * n; e += nt) {
      const int i = (int)(e % n), j = (int)(e / n);
      V[e] = make_double2(i == j ? 1.0 : 0.0, 0.0);
    }
  __syncthreads();
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    // keep A exactly Hermitian (the two triangles are updated by different
    // rounded operations): the lower triangle from the upper, real diagonal
    for (long long e = t; e < (long long)n * n; e += nt) {
      const int i = (int)(e % n), j = (int)(e / n);
      if (i > j) A[e] = cconj(A[j + (long long)i * n]);
      else if (i == j) A[e].y = 0.0;
    }
    __syncthreads();
    double off = 0.0, tot = 0.0;
    for (long long e = t; e < (long long)n * n; e += nt) {
      const int i = (int)(e % n), j = (int)(e / n);
      const double a2 = A[e].x * A[e].x + A[e].y * A[e].y;
      tot += a2;
      if (i != j) off += a2;
    }
    off = block_sum(off, sred);
    tot = block_sum(tot, sred);
    // ||offdiag||_F <= 1e-14 ||A||_F bounds every eigenvalue's error by that
    // (Weyl); the rounding floor of the off-diagonal sum lies near 1e-30 ||A||_F^2
    if (off <= 1e-28 * tot || off == 0.0) break;
    for (int round = 0; round < m - 1; ++round) {
      for (int s = t; s < half; s += nt) {
        // circle method: position 0 fixed, others rotate
        auto player = [&](int pos) { return pos == 0 ? 0 : 1 + (pos - 1 + round) % (m - 1); };
        int p = player(s), q = player(m - 1 - s);
        if (p > q) {
          const int x = p;
          p = q;
          q = x;
        }
        sp[s] = p;
        sq[s] = q;
        double c = 1.0, sn = 0.0;
        double2 e = make_double2(1.0, 0.0);
        if (q < n) {
          const double2 apq = A[p + (long long)q * n];
          const double mag = sqrt(apq.x * apq.x + apq.y * apq.y);
          const double app = A[p + (long long)p * n].x, aqq = A[q + (long long)q * n].x;
          if (mag > 0.0) {
            e = make_double2(apq.x / mag, apq.y / mag);
            const double zeta = (aqq - app) / (2.0 * mag);
            const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            c = 1.0 / sqrt(1.0 + tt * tt);
            sn = tt * c;
          }
        }
        sc[s] = c;
        ss[s] = sn;
        se[s] = e;
      }
      __syncthreads();
      // columns: A[:,p], A[:,q] <- c A_p - s conj(e) A_q,  s A_p + c conj(e) A_q ; same for V
      for (long long e2 = t; e2 < (long long)half * n; e2 += nt) {
        const int s = (int)(e2 / n), i = (int)(e2 % n);
        const int p = sp[s], q = sq[s];
        if (q >= n || ss[s] == 0.0) continue;
        const double c = sc[s], sn = ss[s];
        const double2 ec = cconj(se[s]);
        double2 *ap = A + i + (long long)p * n, *aq = A + i + (long long)q * n;
        const double2 x = *ap, y = cmul(ec, *aq);
        *ap = make_double2(c * x.x - sn * y.x, c * x.y - sn * y.y);
        *aq = make_double2(sn * x.x + c * y.x, sn * x.y + c * y.y);
        if (V) {
          double2 *vp = V + i + (long long)p * n, *vq = V + i + (long long)q * n;
          const double2 vx = *vp, vy = cmul(ec, *vq);
          *vp = make_double2(c * vx.x - sn * vy.x, c * vx.y - sn * vy.y);
          *vq = make_double2(sn * vx.x + c * vy.x, sn * vx.y + c * vy.y);
        }
      }
      __syncthreads();
      // rows: A[p,:], A[q,:] <- c A_p - s e A_q,  s A_p + c e A_q
      for (long long e2 = t; e2 < (long long)half * n; e2 += nt) {
        const int s = (int)(e2 / n), j = (int)(e2 % n);
        const int p = sp[s], q = sq[s];
        if (q >= n || ss[s] == 0.0) continue;
        const double c = sc[s], sn = ss[s];
        const double2 ev = se[s];
        double2 *ap = A + p + (long long)j * n, *aq = A + q + (long long)j * n;
        const double2 x = *ap, y = cmul(ev, *aq);
        *ap = make_double2(c * x.x - sn * y.x, c * x.y - sn * y.y);
        *aq = make_double2(sn * x.x + c * y.x, sn * x.y + c * y.y);
      }
      __syncthreads();
    }
  }
  // sort ascending (selection by rank, ties by index)
  for (int i = t; i < n; i += nt) {
    const double di = A[i + (long long)i * n].x;
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double dj = A[j + (long long)j * n].x;
      rank += (dj < di) || (dj == di && j < i);
    }
    perm[rank] = i;
  }
  __syncthreads();
  for (int r = t; r < n; r += nt) w[r] = A[perm[r] + (long long)perm[r] * n].x;
  if (V) {
    // permute columns through A's strictly-lower part is not possible in place; use A as scratch
    __syncthreads();
    for (long long e = t; e < (long long)n * n; e += nt) A[e] = V[e];
    __syncthreads();
    for (long long e = t; e < (long long)n * n; e += nt) {
      const int i = (int)(e % n), r = (int)(e / n);
      V[e] = A[i + (long long)perm[r] * n];
    }
  }
}

// The same cyclic Jacobi for larger n, one launch per half round: every pair
// (p, q) of a round gets a block, which computes its rotation from the current
// A (the elements of its own two columns) and applies it to columns p, q of A
// and V (k_jac_cols); the row updates follow in a second launch (k_jac_rows).
// The rotations, their order and their arithmetic are those of k_jacobi; the
// sweep test (k_jac_check: symmetrise, then off(A) <= 1e-28 ||A||^2) is read
// by the host between sweeps.  JacRot: c, s and the phase e of each pair.
struct JacRot {
  double c, sn;
  double2 e;
  int p, q;
};

__device__ inline int jac_player(int pos, int round, int m) { return pos == 0 ? 0 : 1 + (pos - 1 + round) % (m - 1); }

__global__ __launch_bounds__(256) void k_jac_init(double2 *V, int n) {
  const long long tot = (long long)n * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), j = (int)(e / n);
    V[e] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
}

__global__ __launch_bounds__(1024) void k_jac_check(double2 *A, int n, int *done) {
  __shared__ double sred[1024];
  const int t = threadIdx.x, nt = blockDim.x;
  for (long long e = t; e < (long long)n * n; e += nt) {
    const int i = (int)(e % n), j = (int)(e / n);
    if (i > j) A[e] = cconj(A[j + (long long)i * n]);
    else if (i == j) A[e].y = 0.0;
  }
  __syncthreads();
  double off = 0.0, tot = 0.0;
  for (long long e = t; e < (long long)n * n; e += nt) {
    const int i = (int)(e % n), j = (int)(e / n);
    const double a2 = A[e].x * A[e].x + A[e].y * A[e].y;
    tot += a2;
    if (i != j) off += a2;
  }
  off = block_sum(off, sred);
  tot = block_sum(tot, sred);
  if (t == 0) *done = (off <= 1e-28 * tot || off == 0.0) ? 1 : 0;
}

// grid (m / 2): block s takes pair s of the round
__global__ __launch_bounds__(256) void k_jac_cols(double2 *A, double2 *V, int n, int round, JacRot *rot) {
  __shared__ JacRot r;
  const int m = (n + 1) & ~1, s = blockIdx.x;
  if (threadIdx.x == 0) {
    int p = jac_player(s, round, m), q = jac_player(m - 1 - s, round, m);
    if (p > q) {
      const int x = p;
      p = q;
      q = x;
    }
    double c = 1.0, sn = 0.0;
    double2 e = make_double2(1.0, 0.0);
    if (q < n) {
      const double2 apq = A[p + (long long)q * n];
      const double mag = sqrt(apq.x * apq.x + apq.y * apq.y);
      const double app = A[p + (long long)p * n].x, aqq = A[q + (long long)q * n].x;
      if (mag > 0.0) {
        e = make_double2(apq.x / mag, apq.y / mag);
        const double zeta = (aqq - app) / (2.0 * mag);
        const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        c = 1.0 / sqrt(1.0 + tt * tt);
        sn = tt * c;
      }
    }
    r = JacRot{c, sn, e, p, q};
    rot[s] = r;
  }
  __syncthreads();
  if (r.q >= n || r.sn == 0.0) return;
  const double2 ec = cconj(r.e);
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double2 *ap = A + i + (long long)r.p * n, *aq = A + i + (long long)r.q * n;
    const double2 x = *ap, y = cmul(ec, *aq);
    *ap = make_double2(r.c * x.x - r.sn * y.x, r.c * x.y - r.sn * y.y);
    *aq = make_double2(r.sn * x.x + r.c * y.x, r.sn * x.y + r.c * y.y);
    if (V) {
      double2 *vp = V + i + (long long)r.p * n, *vq = V + i + (long long)r.q * n;
      const double2 vx = *vp, vy = cmul(ec, *vq);
      *vp = make_double2(r.c * vx.x - r.sn * vy.x, r.c * vx.y - r.sn * vy.y);
      *vq = make_double2(r.sn * vx.x + r.c * vy.x, r.sn * vx.y + r.c * vy.y);
    }
  }
}

__global__ __launch_bounds__(256) void k_jac_rows(double2 *A, int n, const JacRot *rot) {
  const JacRot r = rot[blockIdx.x];
  if (r.q >= n || r.sn == 0.0) return;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    double2 *ap = A + r.p + (long long)j * n, *aq = A + r.q + (long long)j * n;
    const double2 x = *ap, y = cmul(r.e, *aq);
    *ap = make_double2(r.c * x.x - r.sn * y.x, r.c * x.y - r.sn * y.y);
    *aq = make_double2(r.sn * x.x + r.c * y.x, r.sn * x.y + r.c * y.y);
  }
}

// eigenvalues ascending (ties by index) into w, the columns of V in that order
__global__ __launch_bounds__(1024) void k_jac_sort(double2 *A, double2 *V, double *w, int n) {
  __shared__ int perm[JACOBI_MAXN];
  const int t = threadIdx.x, nt = blockDim.x;
  for (int i = t; i < n; i += nt) {
    const double di = A[i + (long long)i * n].x;
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double dj = A[j + (long long)j * n].x;
      rank += (dj < di) || (dj == di && j < i);
    }
    perm[rank] = i;
  }
  __syncthreads();
  for (int r = t; r < n; r += nt) w[r] = A[perm[r] + (long long)perm[r] * n].x;
  if (V) {
    __syncthreads();
    for (long long e = t; e < (long long)n * n; e += nt) A[e] = V[e];
    __syncthreads();
    for (long long e = t; e < (long long)n * n; e += nt) {
      const int i = (int)(e % n), r = (int)(e / n);
      V[e] = A[i + (long long)perm[r] * n];
    }
  }
}

// ---------------------------------------------------------------------------
// Per-step propagation of one state (blockIdx.x) of one k-point (blockIdx.y).
// ---------------------------------------------------------------------------
// (H~(mid) - c0)/r for every k-point, one thread per element, and per-block
// partial sums of ||H~(mid) - H~0||_F^2 for the spectral-interval check.
// grid (assemble_blocks(n), n_k).
// Element (a, b) of the Hermitian part of the step's V~, of which the projection
// wrote the PROJ_BLK-blocks on and above the block diagonal: the mean of the
// element and its mirror inside a diagonal block, else the written one.
__device__ inline double2 vt_herm(const double2 *v, int a, int b, int n) {
  const int ba = a / PROJ_BLK, bb = b / PROJ_BLK;
  if (ba < bb) return v[a + (long long)b * n];
  const double2 y = v[b + (long long)a * n];
  if (ba > bb) return make_double2(y.x, -y.y);
  const double2 x = v[a + (long long)b * n];
  return make_double2(0.5 * (x.x + y.x), 0.5 * (x.y - y.y));
}

__global__ __launch_bounds__(256) void k_assemble(const StepCtx c) {
  __shared__ double sred[16];
  const int k = blockIdx.y;
  const SubDev &S = c.sub[k];
  const int n = c.n_aux;
  const long long n2 = (long long)n * n;
  const int step = *c.step;
  const double am = c.a_mid[step];
  const double cl = c.c_light;
  const double al = am / cl, be = am * am / (2.0 * cl * cl);
  const double ir = 1.0 / S.r;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double dev2 = 0.0;
  if (e < n2) {
    const int a = (int)(e % n), b = (int)(e / n);
    double2 vv;
    if (c.rebuild) {  // Hermitian part of the rebuilt matrix (plus the reference for a residual)
      vv = vt_herm(S.vt_step, a, b, n);
      if (c.resid) vv = cadd(vv, S.vt_ref[e]);
    } else {
      vv = S.vt_ref[e];
    }
    double2 h = cadd(S.tt[e], vv);
    h = cadd(h, cscale(S.pt[e], al));
    if (a == b) h.x += be;
    const double2 d = csub(h, S.h0t[e]);
    dev2 = d.x * d.x + d.y * d.y;
    if (a == b) h.x -= S.c0;
    S.hm[e] = cscale(h, ir);
  }
  dev2 = wave_sum(dev2);
  if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = dev2;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += sred[q];
    S.dev[blockIdx.x] = t;
  }
}

// Copies n elements global -> LDS, eight loads in flight per thread.
__device__ __forceinline__ void stage_to_lds(double2 *dst, const double2 *src, long long n) {
  stage8<double2>((int)n, [&](int e) { return src[e]; }, [&](int e, double2 x) { dst[e] = x; });
}

// Sums the per-state partials in a fixed order, writes the series, advances
// the step (one thread, after every state of the step has written its partials).
__device__ void finalize_step(const StepCtx &c, int step) {
  const int np = c.n_k * c.n_states;
  double j1 = 0.0, e1 = 0.0, j0 = 0.0, e0 = 0.0;
  double x1 = 0.0, x0 = 0.0;
  for (int p = 0; p < np; ++p) {
    j1 += c.part[PART_STRIDE * p + 0];
    e1 += c.part[PART_STRIDE * p + 1];
    j0 += c.part[PART_STRIDE * p + 2];
    e0 += c.part[PART_STRIDE * p + 3];
    x1 += c.part[PART_STRIDE * p + 4];
    x0 += c.part[PART_STRIDE * p + 5];
  }
  if (step == 0) {
    c.j_out[0] = j0;
    c.e_out[0] = e0;
    c.dmu_out[0] = 0.0;
    if (c.nexc_out) c.nexc_out[0] = x0;
  }
  if (c.nexc_out) c.nexc_out[step + 1] = x1;
  const double jz = c.j_out[0];
  c.j_out[step + 1] = j1;
  c.e_out[step + 1] = e1;
  c.dmu_out[step + 1] = c.dmu_out[step] + c.omega * c.dt * 0.5 * ((c.j_out[step] - jz) + (j1 - jz));
  if (!isfinite(j1) || !isfinite(e1)) latch(c.status, 3);
  *c.step_rw = step + 1;
}

// Threads per state block of the forward step (512 measured no faster).
constexpr int STEP_NT = 256;
// the row-per-thread step: the largest n (six vectors per state in LDS, one
// thread per row, at most 1024 threads)
constexpr int STEP_MULTI_MAXN = 768;

// reduction slots (double2) of the forward step kernel: one per thread, or the
// NW n partial sums of the wide products when H~ is not LDS-resident
__host__ __device__ inline int step_red_slots(int n, bool h_in_lds, int nt) {
  return h_in_lds ? nt : (nt / 64 * n > nt ? nt / 64 * n : nt);
}

// HL / PL: H~(mid) / P~ staged in LDS (compile-time, so that their reads are
// LDS reads rather than generic ones).  The block that finishes last sums the
// partials of every state (finalize_step).
template <bool HL, bool PL>
__global__ __launch_bounds__(STEP_NT) void k_step(const StepCtx c) {
  extern __shared__ double2 sm[];
  const int j = blockIdx.x, k = blockIdx.y;
  const SubDev &S = c.sub[k];
  const int n = c.n_aux;
  const long long n2 = (long long)n * n;
  constexpr bool hl = HL, pl = PL;
  double2 *Hm = hl ? sm : S.hm;  // (H~(mid) - c0)/r
  double2 *Pl = pl ? sm + n2 : nullptr;
  double2 *vec = sm + (hl ? n2 : 0) + (pl ? n2 : 0);
  const double2 *P = pl ? Pl : S.pt;
  double2 *v = vec, *t0 = vec + n, *t1 = vec + 2 * n, *acc = vec + 3 * n, *tmp = vec + 4 * n, *w = vec + 5 * n;
  double2 *red = vec + 6 * n;
  double *sred = reinterpret_cast<double *>(red + step_red_slots(n, HL, blockDim.x));
  // products with matrices in global memory: the wide form when the subspace
  // Hamiltonian does not fit in LDS (large n); the LDS-resident ones as they are
  const auto mvg = [&](const double2 *A, const double2 *x, double2 *y) {
    if constexpr (!HL) matvec_g(A, n, x, y, n, red);
    else matvec<false>(A, n, x, y, n, red);
  };
  const int step = *c.step;
  const double am = c.a_mid[step], a1 = c.a_t[step + 1];
  const double cl = c.c_light;

  // 1. the assembled (H~(mid) - c0)/r (k_assemble) into LDS; spectral check
  if constexpr (HL) stage_to_lds(sm, S.hm, n2);
  if constexpr (PL) stage_to_lds(sm + n2, S.pt, n2);
  if (j == 0 && threadIdx.x < 64) {  // one wave: the partials load in parallel, fixed-order sum
    double dev2 = 0.0;
    const int nb = (int)((n2 + 255) / 256);
    for (int q = threadIdx.x; q < nb; q += 64) dev2 += S.dev[q];
    dev2 = wave_sum(dev2);
    // a non-finite H~(mid) (a non-finite potential handed in) is reported as such;
    // a finite one outside the series' interval as a spectrum error
    if (threadIdx.x == 0 && !isfinite(dev2)) latch(c.status, 3);
    else if (threadIdx.x == 0 && !(sqrt(dev2) <= S.margin)) latch(c.status, 4);
  }
  __syncthreads();

  // 2. theta~ = L^H theta
  double2 *th = c.theta + (long long)k * n * c.n_states + (long long)j * n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) tmp[i] = th[i];
  __syncthreads();
  mvg(S.LH, tmp, v);

  // observables of theta~ in v at A = a (H~(a) v built from M v):
  //   J = -(f/Omega) w_k Re(v^H P~ v + (a/c) v^H v),  E = f w_k Re v^H H~(a) v
  // ref = false: H~(a) v from the step's M = (H~(mid) - c0)/r;
  // ref = true:  H~(a) v from H~0 (the reference potential, the only one known at t_0)
  auto observe = [&](double a, double *jo, double *eo, bool ref) {
    if (ref) mvg(S.h0t, v, t0);  // t0 = H~0 v
    else if constexpr (HL) matvec<false>(Hm, n, v, t0, n, red);  // t0 = M v
    else mvg(Hm, v, t0);
    if constexpr (PL) matvec<false>(P, n, v, t1, n, red);  // t1 = P~ v
    else mvg(P, v, t1);
    double vv = 0.0, vp = 0.0, vm = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      vv += v[i].x * v[i].x + v[i].y * v[i].y;
      vp += v[i].x * t1[i].x + v[i].y * t1[i].y;
      vm += v[i].x * t0[i].x + v[i].y * t0[i].y;
    }
    block_sum3(vv, vp, vm, sred);
    // v^H H~(a) v = r vm + c0 vv + ((a - am)/c) vp + ((a^2 - am^2)/2c^2) vv   (step matrix)
    //             = vm + (a/c) vp + (a^2/2c^2) vv                              (reference)
    const double vh = ref ? vm + (a / cl) * vp + (a * a / (2.0 * cl * cl)) * vv
                          : S.r * vm + S.c0 * vv + ((a - am) / cl) * vp + ((a * a - am * am) / (2.0 * cl * cl)) * vv;
    if (threadIdx.x == 0) {
      *jo = -(c.occ / c.omega) * S.kw * (vp + (a / cl) * vv);
      *eo = c.occ * S.kw * vh;
    }
  };
  double *part = c.part + PART_STRIDE * ((long long)k * c.n_states + j);
  // excited electrons of this state: f w_k (theta~^H theta~ - sum_{i < N_s} |(S_sub theta)_i|^2),
  // S_sub theta = L theta~ (the overlaps with the first N_s auxiliary functions)
  auto excited = [&](double *xo) {
    double nn = 0.0, oc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) nn += v[i].x * v[i].x + v[i].y * v[i].y;
    for (int i = threadIdx.x; i < c.n_states; i += blockDim.x) {
      double2 sv = make_double2(0.0, 0.0);
      for (int q = 0; q <= i; ++q) sv = cfma(S.L[i + (long long)q * n], v[q], sv);
      oc += sv.x * sv.x + sv.y * sv.y;
    }
    double z = 0.0;
    block_sum3(nn, oc, z, sred);
    if (threadIdx.x == 0) *xo = c.occ * S.kw * (nn - oc);
  };
  if (step == 0) {
    observe(c.a_t[0], part + 2, part + 3, true);
    if (c.nexc_out) excited(part + 5);
  }

  if (c.taylor > 0) {
    // 3'. explicit step: the Taylor series of exp(-i dt (H~ - c0)) truncated after
    //     c.taylor terms (H~ - c0 = r M), term_q = (-i dt r / q) M term_{q-1}
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      t0[i] = v[i];
      acc[i] = v[i];
    }
    __syncthreads();
    for (int q = 1; q <= c.taylor; ++q) {
      if constexpr (HL) matvec<false>(Hm, n, t0, tmp, n, red);
      else mvg(Hm, t0, tmp);
      const double fq = c.dt * S.r / q;
      for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double2 tn = make_double2(fq * tmp[i].y, -fq * tmp[i].x);  // -i fq tmp
        t0[i] = tn;
        acc[i] = cadd(acc[i], tn);
      }
      __syncthreads();
    }
  } else {
  // 3. Chebyshev series
  const int K = S.K;
  for (int i = threadIdx.x; i < n; i += blockDim.x) t0[i] = v[i];
  if constexpr (HL) matvec<false>(Hm, n, v, t1, n, red);
  else mvg(Hm, v, t1);
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc[i] = cadd(cmul(S.coef[0], t0[i]), cmul(S.coef[1], t1[i]));
  __syncthreads();
  double2 *pa = t0, *pb = t1;  // T_{k-2}, T_{k-1}
  for (int q = 2; q <= K; ++q) {
    if constexpr (HL) matvec<false>(Hm, n, pb, tmp, n, red);
    else mvg(Hm, pb, tmp);
    const double2 cq = S.coef[q];
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const double2 tn = make_double2(2.0 * tmp[i].x - pa[i].x, 2.0 * tmp[i].y - pa[i].y);
      pa[i] = tn;  // becomes T_q
      acc[i] = cfma(cq, tn, acc[i]);
    }
    __syncthreads();
    double2 *x = pa;
    pa = pb;
    pb = x;
  }
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) v[i] = cmul(S.phase, acc[i]);
  __syncthreads();

  // 4. theta = L^{-H} theta~
  mvg(S.LinvH, v, w);
  for (int i = threadIdx.x; i < n; i += blockDim.x) th[i] = w[i];

  // 5. observables at t_{n+1} (v still holds theta~)
  observe(a1, part + 0, part + 1, false);
  if (c.nexc_out) excited(part + 4);

  // 6. the last block to finish: fixed-order sum, series, step counter
  __syncthreads();
  int *last = reinterpret_cast<int *>(sred);
  if (threadIdx.x == 0) {
    __threadfence();
    *last = atomicAdd(c.done, 1) == (int)(gridDim.x * gridDim.y) - 1;
  }
  __syncthreads();
  if (!*last || threadIdx.x != 0) return;
  __threadfence();
  finalize_step(c, step);
  *c.done = 0;
}

// ---------------------------------------------------------------------------
// The same step for NS states per block (blockIdx.x covers states NS x, ...,
// NS x + NS - 1), for subspaces whose matrices stay in global memory: one block
// thread per matrix row (blockDim = 64 ceil(n / 64)), each product Y_s = A X_s
// reads A once for all NS states (row i of every product in thread i, columns
// in order, no cross-wave reduction).  Per state the arithmetic is that of
// k_step<false, false> except the summation order inside the products.  The
// stepwise REBUILD step and the step beside the rebuild of the next one use
// this form, so that the two give the same bits.
// ---------------------------------------------------------------------------
template <int NS, int UN>
__device__ void matvec_rows(const double2 *__restrict__ A, int lda, const double2 *X, double2 *Y, int n) {
  const int i = threadIdx.x;
  if (i < n) {
    double2 acc[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) acc[s] = make_double2(0.0, 0.0);
    const double2 *a = A + i;
    int k = 0;
    for (; k + UN <= n; k += UN) {
      double2 av[UN];
#pragma unroll
      for (int u = 0; u < UN; ++u) av[u] = a[(long long)(k + u) * lda];
#pragma unroll
      for (int u = 0; u < UN; ++u)
#pragma unroll
        for (int s = 0; s < NS; ++s) acc[s] = cfma(av[u], X[s * n + k + u], acc[s]);
    }
    for (; k < n; ++k) {
      const double2 av = a[(long long)k * lda];
#pragma unroll
      for (int s = 0; s < NS; ++s) acc[s] = cfma(av, X[s * n + k], acc[s]);
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) Y[s * n + i] = acc[s];
  }
  __syncthreads();
}

// The products of the AFFINE step, where the exponential is the whole step:
// P threads per row (blockDim = P x 64 ceil(n / 64), parts are whole waves),
// part p summing the columns of its contiguous range in order with UN loads in
// flight (the range's last, partial batch too: loads at clamped indices, the
// products predicated), the parts added in the order p = 0, 1, ... through red.
// Each thread's chain of dependent loads is P times shorter than in matvec_rows.
template <int NS, int UN, int P>
__device__ void matvec_split(const double2 *__restrict__ A, int lda, const double2 *X, double2 *Y, int n,
                             double2 *red) {
  const int nr = blockDim.x / P;
  const int i = threadIdx.x % nr, p = threadIdx.x / nr;
  const int chunk = ((n + P - 1) / P + UN - 1) / UN * UN;  // columns per part
  const int kb = p * chunk, ke = min(n, kb + chunk);
  double2 acc[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) acc[s] = make_double2(0.0, 0.0);
  if (i < n) {
    const double2 *a = A + i;
    int k = kb;
    for (; k + UN <= ke; k += UN) {
      double2 av[UN];
#pragma unroll
      for (int u = 0; u < UN; ++u) av[u] = a[(long long)(k + u) * lda];
#pragma unroll
      for (int u = 0; u < UN; ++u)
#pragma unroll
        for (int s = 0; s < NS; ++s) acc[s] = cfma(av[u], X[s * n + k + u], acc[s]);
    }
    if (k < ke) {
      double2 av[UN];
#pragma unroll
      for (int u = 0; u < UN; ++u) av[u] = a[(long long)min(k + u, ke - 1) * lda];
#pragma unroll
      for (int u = 0; u < UN; ++u)
        if (k + u < ke)
#pragma unroll
          for (int s = 0; s < NS; ++s) acc[s] = cfma(av[u], X[s * n + k + u], acc[s]);
    }
    if (p > 0)
#pragma unroll
      for (int s = 0; s < NS; ++s) red[((p - 1) * NS + s) * n + i] = acc[s];
  }
  __syncthreads();
  if (p == 0 && i < n)
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      double2 y = acc[s];
      for (int q = 1; q < P; ++q) y = cadd(y, red[((q - 1) * NS + s) * n + i]);
      Y[s * n + i] = y;
    }
  __syncthreads();
}

template <int NS, int UN, int P>
__global__ __launch_bounds__(1024) void k_step_multi(const StepCtx c) {
  extern __shared__ double2 sm[];
  const int k = blockIdx.y;
  const int j0 = blockIdx.x * NS;
  const int ns = (c.n_states - j0) < NS ? (c.n_states - j0) : NS;  // states of this block
  const SubDev &S = c.sub[k];
  const int n = c.n_aux;
  const int bd = blockDim.x;
  double2 *v = sm, *t0 = sm + NS * n, *t1 = sm + 2 * NS * n, *acc = sm + 3 * NS * n, *tmp = sm + 4 * NS * n;
  double2 *w = sm + 5 * NS * n;
  double2 *red = sm + 6 * NS * n;  // partial sums of parts 1 .. P-1
  double *sred = reinterpret_cast<double *>(sm + (5 + P) * NS * n);
  const auto mv = [&](const double2 *A, const double2 *x, double2 *y) {
    if constexpr (P == 1) matvec_rows<NS, UN>(A, n, x, y, n);
    else matvec_split<NS, UN, P>(A, n, x, y, n, red);
  };
  const int step = *c.step;
  const double am = c.a_mid[step], a1 = c.a_t[step + 1];
  const double cl = c.c_light;
  const double2 *Hm = S.hm;

  if (blockIdx.x == 0 && threadIdx.x < 64) {  // spectral check (one wave, fixed-order sum)
    double dev2 = 0.0;
    const long long n2 = (long long)n * n;
    const int nb = (int)((n2 + 255) / 256);
    for (int q = threadIdx.x; q < nb; q += 64) dev2 += S.dev[q];
    dev2 = wave_sum(dev2);
    if (threadIdx.x == 0 && !isfinite(dev2)) latch(c.status, 3);
    else if (threadIdx.x == 0 && !(sqrt(dev2) <= S.margin)) latch(c.status, 4);
  }

  // theta~ = L^H theta (states past n_states: zero vectors, results discarded)
  double2 *th0 = c.theta + (long long)k * n * c.n_states + (long long)j0 * n;
  for (int e = threadIdx.x; e < NS * n; e += bd) tmp[e] = (e / n < ns) ? th0[e] : make_double2(0.0, 0.0);
  __syncthreads();
  mv(S.LH, tmp, v);

  auto observe = [&](double a, int slot_j, int slot_e, bool ref) {
    mv(ref ? S.h0t : Hm, v, t0);
    mv(S.pt, v, t1);
    for (int s = 0; s < ns; ++s) {
      double vv = 0.0, vp = 0.0, vm = 0.0;
      for (int i = threadIdx.x; i < n; i += bd) {
        const double2 x = v[s * n + i], p = t1[s * n + i], m = t0[s * n + i];
        vv += x.x * x.x + x.y * x.y;
        vp += x.x * p.x + x.y * p.y;
        vm += x.x * m.x + x.y * m.y;
      }
      block_sum3(vv, vp, vm, sred);
      const double vh = ref ? vm + (a / cl) * vp + (a * a / (2.0 * cl * cl)) * vv
                            : S.r * vm + S.c0 * vv + ((a - am) / cl) * vp + ((a * a - am * am) / (2.0 * cl * cl)) * vv;
      if (threadIdx.x == 0) {
        double *part = c.part + PART_STRIDE * ((long long)k * c.n_states + j0 + s);
        part[slot_j] = -(c.occ / c.omega) * S.kw * (vp + (a / cl) * vv);
        part[slot_e] = c.occ * S.kw * vh;
      }
    }
  };
  auto excited = [&](int slot) {
    for (int s = 0; s < ns; ++s) {
      double nn = 0.0, oc = 0.0;
      for (int i = threadIdx.x; i < n; i += bd) nn += v[s * n + i].x * v[s * n + i].x + v[s * n + i].y * v[s * n + i].y;
      for (int i = threadIdx.x; i < c.n_states; i += bd) {
        double2 sv = make_double2(0.0, 0.0);
        for (int q = 0; q <= i; ++q) sv = cfma(S.L[i + (long long)q * n], v[s * n + q], sv);
        oc += sv.x * sv.x + sv.y * sv.y;
      }
      double z = 0.0;
      block_sum3(nn, oc, z, sred);
      if (threadIdx.x == 0) c.part[PART_STRIDE * ((long long)k * c.n_states + j0 + s) + slot] = c.occ * S.kw * (nn - oc);
    }
  };
  if (step == 0) {
    observe(c.a_t[0], 2, 3, true);
    if (c.nexc_out) excited(5);
  }

  if (c.taylor > 0) {
    for (int e = threadIdx.x; e < NS * n; e += bd) {
      t0[e] = v[e];
      acc[e] = v[e];
    }
    __syncthreads();
    for (int q = 1; q <= c.taylor; ++q) {
      mv(Hm, t0, tmp);
      const double fq = c.dt * S.r / q;
      for (int e = threadIdx.x; e < NS * n; e += bd) {
        const double2 tn = make_double2(fq * tmp[e].y, -fq * tmp[e].x);
        t0[e] = tn;
        acc[e] = cadd(acc[e], tn);
      }
      __syncthreads();
    }
  } else {
    const int K = S.K;
    for (int e = threadIdx.x; e < NS * n; e += bd) t0[e] = v[e];
    mv(Hm, v, t1);
    for (int e = threadIdx.x; e < NS * n; e += bd) acc[e] = cadd(cmul(S.coef[0], t0[e]), cmul(S.coef[1], t1[e]));
    __syncthreads();
    double2 *pa = t0, *pb = t1;
    for (int q = 2; q <= K; ++q) {
      mv(Hm, pb, tmp);
      const double2 cq = S.coef[q];
      for (int e = threadIdx.x; e < NS * n; e += bd) {
        const double2 tn = make_double2(2.0 * tmp[e].x - pa[e].x, 2.0 * tmp[e].y - pa[e].y);
        pa[e] = tn;
        acc[e] = cfma(cq, tn, acc[e]);
      }
      __syncthreads();
      double2 *x = pa;
      pa = pb;
      pb = x;
    }
  }
  for (int e = threadIdx.x; e < NS * n; e += bd) v[e] = cmul(S.phase, acc[e]);
  __syncthreads();
  mv(S.LinvH, v, w);
  for (int e = threadIdx.x; e < ns * n; e += bd) th0[e] = w[e];
  observe(a1, 0, 1, false);
  if (c.nexc_out) excited(4);

  __syncthreads();
  int *last = reinterpret_cast<int *>(sred);
  if (threadIdx.x == 0) {
    __threadfence();
    *last = atomicAdd(c.done, 1) == (int)(gridDim.x * gridDim.y) - 1;
  }
  __syncthreads();
  if (!*last || threadIdx.x != 0) return;
  __threadfence();
  finalize_step(c, step);
  *c.done = 0;
}

// ---------------------------------------------------------------------------
// Adjoint step for one state (blockIdx.x) of one k-point (blockIdx.y).
// In the S-orthonormal basis (theta~ = L^H theta, mu~ = L^{-1} mu, so that
// Re <mu, d theta> = Re <mu~, d theta~>):
//   mu~_n = U~^H mu~_{n+1} + dt w_n g~_n,  g~_n = -(2f/Omega) w_k (P~ + A_n/c) theta~_n
//   dL/dA_mid = Re <mu~_{n+1}, (dU~/dA) theta~_n>,
// where dU~/dA is the derivative of the same Chebyshev series:
//   T'_0 = 0, T'_1 = E, T'_q = 2 E T_{q-1} + 2 X T'_{q-1} - T'_{q-2},
//   E = dX/dA = (P~/c + (A/c^2) I)/r,
// and U~^H = conj(phase) sum conj(c_q) T_q(X) (X Hermitian).
// Per-state partials: part[4p+0] midpoint term, part[4p+1] dt w_n dJ_n/dA_n,
// part[4p+2] dJ_n/dA_n.
// ---------------------------------------------------------------------------
template <bool HL>
__global__ __launch_bounds__(256) void k_adjoint(const StepCtx c, const AdjCtx ac) {
  extern __shared__ double2 sm[];
  const int j = blockIdx.x, k = blockIdx.y;
  const SubDev &S = c.sub[k];
  const int n = c.n_aux;
  constexpr bool hl = HL;
  double2 *Hm = hl ? sm : S.work + (long long)j * n * n;
  double2 *vec = hl ? sm + (long long)n * n : sm;
  double2 *v = vec, *mu = vec + n, *ta = vec + 2 * n, *tb = vec + 3 * n, *da = vec + 4 * n;
  double2 *db = vec + 5 * n, *tmp = vec + 6 * n, *tmp2 = vec + 7 * n, *xdt = vec + 8 * n;
  double2 *acc = vec + 9 * n, *dacc = vec + 10 * n;
  double2 *red = vec + 11 * n;
  double *sred = reinterpret_cast<double *>(red + blockDim.x);
  const int step = ac.n;
  const double cl = c.c_light;
  const double an = c.a_t[step];
  const double wn = (step == 0 || step == ac.n_steps) ? 0.5 : 1.0;
  const double ir = 1.0 / S.r;
  const double gs = -(2.0 * c.occ / c.omega) * S.kw;
  double *part = c.part + PART_STRIDE * ((long long)k * c.n_states + j);
  double2 *mo = ac.mu_out + (long long)k * n * c.n_states + (long long)j * n;

  const double2 *th = c.theta + (long long)k * n * c.n_states + (long long)j * n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) tmp[i] = th[i];
  __syncthreads();
  matvec<false>(S.LH, n, tmp, v, n, red);  // theta~_n
  const double vv = dot_re(v, v, n, sred);
  const double djda = -(c.occ / (c.omega * cl)) * S.kw * vv;
  matvec<false>(S.pt, n, v, tmp2, n, red);  // P~ theta~_n (for the source term)

  if (ac.terminal) {
    for (int i = threadIdx.x; i < n; i += blockDim.x)
      tmp[i] = cscale(cadd(tmp2[i], cscale(v[i], an / cl)), gs * c.dt * wn);
    __syncthreads();
    matvec<false>(S.L, n, tmp, acc, n, red);  // mu_N = L mu~_N
    for (int i = threadIdx.x; i < n; i += blockDim.x) mo[i] = acc[i];
    if (threadIdx.x == 0) {
      part[0] = 0.0;
      part[1] = c.dt * wn * djda;
      part[2] = djda;
    }
    return;
  }
  // keep the source term: xdt <- dt w_n g~_n (zero at n = 0: the initial state is fixed)
  const double sw = (step >= 1) ? gs * c.dt * wn : 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) xdt[i] = cscale(cadd(tmp2[i], cscale(v[i], an / cl)), sw);

  const double am = c.a_mid[step];
  const double al = am / cl, be = am * am / (2.0 * cl * cl);
  for (long long e = threadIdx.x; e < (long long)n * n; e += blockDim.x) {
    const int a = (int)(e % n), b = (int)(e / n);
    double2 vv2;
    if (c.rebuild) {
      vv2 = vt_herm(S.vt_step, a, b, n);
      if (c.resid) vv2 = cadd(vv2, S.vt_ref[e]);
    } else {
      vv2 = S.vt_ref[e];
    }
    double2 h = cadd(S.tt[e], vv2);
    h = cadd(h, cscale(S.pt[e], al));
    if (a == b) h.x += be - S.c0;
    Hm[e] = cscale(h, ir);
  }
  // mu~_{n+1} = L^{-1} mu_{n+1}
  const double2 *mn = ac.mu_next + (long long)k * n * c.n_states + (long long)j * n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) tmp[i] = mn[i];
  __syncthreads();
  matvec<false>(S.Linv, n, tmp, mu, n, red);

  // derivative of the series applied to theta~_n
  auto apply_e = [&](const double2 *y, double2 *out) {  // out = E y
    matvec<false>(S.pt, n, y, tmp2, n, red);
    for (int i = threadIdx.x; i < n; i += blockDim.x)
      out[i] = cscale(cadd(cscale(tmp2[i], 1.0 / cl), cscale(y[i], am / (cl * cl))), ir);
    __syncthreads();
  };
  const int K = S.K;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    ta[i] = v[i];
    da[i] = make_double2(0.0, 0.0);
  }
  __syncthreads();
  matvec<false>(Hm, n, v, tb, n, red);  // T_1 v
  apply_e(v, db);                        // T'_1 v
  for (int i = threadIdx.x; i < n; i += blockDim.x) dacc[i] = cmul(S.coef[1], db[i]);
  __syncthreads();
  for (int q = 2; q <= K; ++q) {
    double2 *et = acc;                    // scratch: E T_{q-1} v
    apply_e(tb, et);
    matvec<false>(Hm, n, db, tmp, n, red);  // X T'_{q-1} v
    double2 *xt = tmp2;
    matvec<false>(Hm, n, tb, xt, n, red);  // X T_{q-1} v
    const double2 cq = S.coef[q];
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const double2 tn = make_double2(2.0 * xt[i].x - ta[i].x, 2.0 * xt[i].y - ta[i].y);
      const double2 dn = make_double2(2.0 * et[i].x + 2.0 * tmp[i].x - da[i].x,
                                      2.0 * et[i].y + 2.0 * tmp[i].y - da[i].y);
      ta[i] = tn;
      da[i] = dn;
      dacc[i] = cfma(cq, dn, dacc[i]);
    }
    __syncthreads();
    double2 *x = ta;
    ta = tb;
    tb = x;
    x = da;
    da = db;
    db = x;
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) dacc[i] = cmul(S.phase, dacc[i]);
  __syncthreads();
  const double dmid = dot_re(mu, dacc, n, sred);

  // U~^H mu~_{n+1}
  for (int i = threadIdx.x; i < n; i += blockDim.x) ta[i] = mu[i];
  __syncthreads();
  matvec<false>(Hm, n, mu, tb, n, red);
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    acc[i] = cadd(cmul(cconj(S.coef[0]), ta[i]), cmul(cconj(S.coef[1]), tb[i]));
  __syncthreads();
  for (int q = 2; q <= K; ++q) {
    matvec<false>(Hm, n, tb, tmp, n, red);
    const double2 cq = cconj(S.coef[q]);
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const double2 tn = make_double2(2.0 * tmp[i].x - ta[i].x, 2.0 * tmp[i].y - ta[i].y);
      ta[i] = tn;
      acc[i] = cfma(cq, tn, acc[i]);
    }
    __syncthreads();
    double2 *x = ta;
    ta = tb;
    tb = x;
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) tmp[i] = cadd(cmul(cconj(S.phase), acc[i]), xdt[i]);
  __syncthreads();
  matvec<false>(S.L, n, tmp, ta, n, red);  // mu_n = L mu~_n
  for (int i = threadIdx.x; i < n; i += blockDim.x) mo[i] = ta[i];
  if (threadIdx.x == 0) {
    part[0] = dmid;
    part[1] = c.dt * wn * djda;
    part[2] = djda;
  }
}

// Sums the adjoint partials in a fixed order.
__global__ void k_adjoint_finalize(const StepCtx c, const AdjCtx ac) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int np = c.n_k * c.n_states;
  double dm = 0.0, dt_ = 0.0, dj = 0.0;
  for (int p = 0; p < np; ++p) {
    dm += c.part[PART_STRIDE * p + 0];
    dt_ += c.part[PART_STRIDE * p + 1];
    dj += c.part[PART_STRIDE * p + 2];
  }
  if (!ac.terminal) ac.dl_da_mid[ac.n] = dm;
  // the J_0 subtracted in J_ind: L contains -T J_0, T = N dt
  if (ac.n == 0) dt_ -= ac.n_steps * c.dt * dj;
  ac.dl_da_t[ac.n] = dt_;
}

// ---------------------------------------------------------------------------
// Piecewise-linear pulse on uniform knots and its chain rule.
// ---------------------------------------------------------------------------
__device__ inline void hat_pair(double t, int nk, double h, int *i0, double *w1) {
  int i = (int)floor(t / h);
  if (i < 0) i = 0;
  if (i > nk - 2) i = nk - 2;
  *i0 = i;
  *w1 = (t - i * h) / h;
}

__global__ void k_knot_samples(const double *q, int nk, double t_end, double dt, int ns, double *a_t,
                               double *a_mid) {
  const double h = t_end / (nk - 1);
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < 2 * ns + 1; e += gridDim.x * blockDim.x) {
    const bool mid = e > ns;
    const int n = mid ? e - ns - 1 : e;
    const double t = (n + (mid ? 0.5 : 0.0)) * dt;
    int i0;
    double w1;
    hat_pair(t, nk, h, &i0, &w1);
    const double v = (1.0 - w1) * q[i0] + w1 * q[i0 + 1];
    if (mid) a_mid[n] = v;
    else a_t[n] = v;
  }
}

// One thread per knot sums its support in time order (deterministic).
__global__ void k_knot_gradient(const double *g_t, const double *g_mid, int ns, double dt, int nk, double t_end,
                                double *g_q) {
  const int kq = blockIdx.x * blockDim.x + threadIdx.x;
  if (kq >= nk) return;
  const double h = t_end / (nk - 1);
  double s = 0.0;
  for (int e = 0; e < 2 * ns + 1; ++e) {
    const bool mid = e > ns;
    const int n = mid ? e - ns - 1 : e;
    const double t = (n + (mid ? 0.5 : 0.0)) * dt;
    int i0;
    double w1;
    hat_pair(t, nk, h, &i0, &w1);
    const double g = mid ? g_mid[n] : g_t[n];
    if (i0 == kq) s += (1.0 - w1) * g;
    if (i0 + 1 == kq) s += w1 * g;
  }
  g_q[kq] = s;
}

}  // namespace

hipError_t launch_copy_rows(double2 *dst, int ldd, const double2 *src, int lds, int rows, int cols, bool zero,
                            hipStream_t s) {
  const long long tot = (long long)rows * cols;
  if (tot <= 0) return hipSuccess;
  const int nb = (int)((tot + 255) / 256 < 4096 ? (tot + 255) / 256 : 4096);
  hipLaunchKernelGGL(k_copy_rows, dim3(nb), dim3(256), 0, s, dst, ldd, src, lds, rows, cols, zero ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_herm_split(const double2 *x, int ldx, int n, int nb, double2 *out, hipStream_t s) {
  const long long tot = (long long)nb * n * n;
  if (tot <= 0) return hipSuccess;
  const int g = (int)((tot + 255) / 256 < 4096 ? (tot + 255) / 256 : 4096);
  hipLaunchKernelGGL(k_herm_split, dim3(g), dim3(256), 0, s, x, ldx, n, nb, out);
  return hipGetLastError();
}

hipError_t launch_axpby(double2 *out, const double2 *a, const double2 *b, double sa, double sb, long long n,
                        hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int g = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  hipLaunchKernelGGL(k_axpby_n2, dim3(g), dim3(256), 0, s, out, a, b, sa, sb, n);
  return hipGetLastError();
}

hipError_t launch_heff(double2 *out, const double2 *h, const double2 *p, const double2 *o, double al, double be,
                       long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int g = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  hipLaunchKernelGGL(k_heff, dim3(g), dim3(256), 0, s, out, h, p, o, al, be, n);
  return hipGetLastError();
}

hipError_t launch_copy_step(double2 *dst, const double2 *src, long long n, const int *step, long long stride,
                            long long host_off, const double2 *sub, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int blocks = (int)std::min<long long>((n + 255) / 256, 2048);
  hipLaunchKernelGGL(k_copy_step, dim3(blocks), dim3(256), 0, s, dst, src, n, step, stride, host_off, sub);
  return hipGetLastError();
}

hipError_t launch_copy_step32(float2 *dst, const double2 *src, long long n, const int *step, long long stride,
                              long long host_off, const double2 *sub, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int blocks = (int)std::min<long long>((n + 255) / 256, 2048);
  hipLaunchKernelGGL(k_copy_step32, dim3(blocks), dim3(256), 0, s, dst, src, n, step, stride, host_off, sub);
  return hipGetLastError();
}

hipError_t launch_rows_to_c64(float2 *dst, int ldd, const double2 *src, int lds, int ng, const int *perm, int nperm,
                              int cols, hipStream_t s) {
  const long long tot = (long long)(ng + nperm) * cols;
  if (tot <= 0) return hipSuccess;
  const int nb = (int)((tot + 255) / 256 < 4096 ? (tot + 255) / 256 : 4096);
  hipLaunchKernelGGL(k_rows_to_c64, dim3(nb), dim3(256), 0, s, dst, ldd, src, lds, ng, perm, nperm, cols);
  return hipGetLastError();
}

hipError_t launch_thv(double *out, const double *th, const double *v, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int g = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  hipLaunchKernelGGL(k_thv, dim3(g), dim3(256), 0, s, out, th, v, n);
  return hipGetLastError();
}

hipError_t launch_cholesky(const double2 *S, double2 *L, int n, int *status, int *fail, hipStream_t s) {
  hipLaunchKernelGGL(k_cholesky, dim3(1), dim3(1024), 0, s, S, L, n, status, fail);
  return hipGetLastError();
}

hipError_t launch_trtri(const double2 *L, double2 *Li, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_trtri, dim3((n + 63) / 64), dim3(64), 0, s, L, Li, n);
  return hipGetLastError();
}

size_t jacobi_work_bytes(int n) { return (size_t)((n + 1) / 2) * sizeof(JacRot) + 256; }

hipError_t launch_jacobi(double2 *A, double2 *V, double *w, int n, hipStream_t s, void *work) {
  if (n <= JACOBI_ONE_BLOCK || !work) {
    hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(1024), 0, s, A, V, w, n, 40);
    return hipGetLastError();
  }
  if (n > JACOBI_MAXN) return hipErrorInvalidValue;
  const int m = (n + 1) & ~1;
  int *done = static_cast<int *>(work);
  JacRot *rot = reinterpret_cast<JacRot *>(static_cast<char *>(work) + 256);
  if (V) hipLaunchKernelGGL(k_jac_init, dim3(std::min(1024, (n * n + 255) / 256)), dim3(256), 0, s, V, n);
  for (int sweep = 0; sweep < 40; ++sweep) {
    hipLaunchKernelGGL(k_jac_check, dim3(1), dim3(1024), 0, s, A, n, done);
    int hd = 0;
    hipError_t e = hipMemcpyAsync(&hd, done, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    if (hd) break;
    for (int round = 0; round < m - 1; ++round) {
      hipLaunchKernelGGL(k_jac_cols, dim3(m / 2), dim3(256), 0, s, A, V, n, round, rot);
      hipLaunchKernelGGL(k_jac_rows, dim3(m / 2), dim3(256), 0, s, A, n, rot);
    }
  }
  hipLaunchKernelGGL(k_jac_sort, dim3(1), dim3(1024), 0, s, A, V, w, n);
  return hipGetLastError();
}

size_t step_multi_lds_bytes(int n, int ns, int parts) {
  return ((size_t)(5 + parts) * ns * n) * sizeof(double2) + 3 * 16 * sizeof(double) + 64;
}

size_t step_lds_bytes(int n, bool h_in_lds, bool adjoint, bool p_in_lds) {
  const size_t vecs = adjoint ? 11 : 6;
  const size_t mats = (h_in_lds ? (size_t)n * n : 0) + ((!adjoint && p_in_lds) ? (size_t)n * n : 0);
  // reduction slots: one per thread, or the wave partials of the wide products
  const size_t nt = adjoint ? 256 : step_red_slots(n, h_in_lds, STEP_NT);
  return (mats + vecs * n + nt) * sizeof(double2) + 256 * sizeof(double);
}

hipError_t launch_conj_transpose(const double2 *a, double2 *out, int n, hipStream_t s) {
  const long long tot = (long long)n * n;
  const int g = (int)((tot + 255) / 256 < 4096 ? (tot + 255) / 256 : 4096);
  hipLaunchKernelGGL(k_conj_transpose, dim3(g), dim3(256), 0, s, a, out, n);
  return hipGetLastError();
}

static bool g_step_attr = false;

int assemble_blocks(int n) { return (int)(((long long)n * n + 255) / 256); }

void subspace_init_attrs() {
  if (g_step_attr) return;
  for (const void *k : {(const void *)k_step<true, true>, (const void *)k_step<true, false>,
                        (const void *)k_step<false, false>, (const void *)k_step_multi<1, 16, 1>,
                        (const void *)k_step_multi<1, 12, 3>,
                        (const void *)k_step_multi<2, 8, 1>,
                        (const void *)k_adjoint<true>,
                        (const void *)k_adjoint<false>})
    (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  g_step_attr = true;
}

hipError_t launch_assemble(const StepCtx &c, hipStream_t s) {
  hipLaunchKernelGGL(k_assemble, dim3(assemble_blocks(c.n_aux), c.n_k), dim3(256), 0, s, c);
  return hipGetLastError();
}

__global__ void k_record_theta(const double2 *__restrict__ th, double2 *__restrict__ hist, const int *step,
                               int hist_len, long long len) {
  const long long off = (long long)((*step) % hist_len) * len;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < len; i += (long long)gridDim.x * blockDim.x)
    hist[off + i] = th[i];
}

hipError_t launch_record_theta(const StepCtx &c, double2 *hist, int hist_len, hipStream_t s) {
  const long long len = (long long)c.n_k * c.n_states * c.n_aux;
  const int blocks = (int)std::min<long long>((len + 255) / 256, 1024);
  hipLaunchKernelGGL(k_record_theta, dim3(blocks), dim3(256), 0, s, c.theta, hist, c.step, hist_len, len);
  return hipGetLastError();
}

__global__ void k_pulse_loss(const double *dmu, int n, double omega, double *loss) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *loss = dmu[n] / omega;
}

hipError_t launch_pulse_loss(const double *dmu, int n, double omega, double *loss, hipStream_t s) {
  hipLaunchKernelGGL(k_pulse_loss, dim3(1), dim3(64), 0, s, dmu, n, omega, loss);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_col_dots(const double2 *a, const double2 *b, int rows, int ld,
                                                 double2 *out) {
  __shared__ double2 red[256];
  const int c = blockIdx.x;
  const double2 *ac = a + (long long)c * ld, *bc = b + (long long)c * ld;
  double2 s = make_double2(0.0, 0.0);
  for (int i = threadIdx.x; i < rows; i += 256) s = cadd(s, cmulc(ac[i], bc[i]));
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] = cadd(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = red[0];
}

hipError_t launch_col_dots(const double2 *a, const double2 *b, int rows, int cols, int ld, double2 *out,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_col_dots, dim3(cols), dim3(256), 0, s, a, b, rows, ld, out);
  return hipGetLastError();
}

__global__ void k_cg_step(double2 *x, double2 *r, const double2 *p, const double2 *q, const double2 *rr,
                          const double2 *pq, int rows, int cols, int ld) {
  const long long tot = (long long)rows * cols;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % rows), c = (int)(e / rows);
    const double den = pq[c].x;
    const double al = den != 0.0 ? rr[c].x / den : 0.0;
    const long long o = (long long)i + (long long)c * ld;
    x[o] = cadd(x[o], cscale(p[o], al));
    r[o] = csub(r[o], cscale(q[o], al));
  }
}

hipError_t launch_cg_step(double2 *x, double2 *r, const double2 *p, const double2 *q, const double2 *rr,
                          const double2 *pq, int rows, int cols, int ld, hipStream_t s) {
  const long long tot = (long long)rows * cols;
  const int nb = (int)std::min<long long>((tot + 255) / 256, 4096);
  hipLaunchKernelGGL(k_cg_step, dim3(nb), dim3(256), 0, s, x, r, p, q, rr, pq, rows, cols, ld);
  return hipGetLastError();
}

__global__ void k_cg_dir(double2 *p, const double2 *r, double2 *rr, const double2 *rrn, int rows, int cols, int ld) {
  const long long tot = (long long)rows * cols;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % rows), c = (int)(e / rows);
    const double be = rr[c].x != 0.0 ? rrn[c].x / rr[c].x : 0.0;
    const long long o = (long long)i + (long long)c * ld;
    p[o] = cadd(r[o], cscale(p[o], be));
  }
}

__global__ void k_copy_scalars(double2 *dst, const double2 *src, int n) {
  if (threadIdx.x < n) dst[threadIdx.x] = src[threadIdx.x];
}

hipError_t launch_cg_dir(double2 *p, const double2 *r, double2 *rr, const double2 *rrn, int rows, int cols, int ld,
                         hipStream_t s) {
  const long long tot = (long long)rows * cols;
  const int nb = (int)std::min<long long>((tot + 255) / 256, 4096);
  hipLaunchKernelGGL(k_cg_dir, dim3(nb), dim3(256), 0, s, p, r, rr, rrn, rows, cols, ld);
  hipLaunchKernelGGL(k_copy_scalars, dim3(1), dim3(1024), 0, s, rr, rrn, cols);
  return hipGetLastError();
}

__global__ void k_taylor_term(double2 *y, const double2 *x, const double2 *z, double2 f, double c0, double2 *acc,
                              int rows, int cols, int ld) {
  const long long tot = (long long)rows * cols;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % rows), c = (int)(e / rows);
    const long long o = (long long)i + (long long)c * ld;
    const double2 v = cmul(f, csub(x[o], cscale(z[o], c0)));
    y[o] = v;
    if (acc) acc[o] = cadd(acc[o], v);
  }
}

hipError_t launch_taylor_term(double2 *y, const double2 *x, const double2 *z, double2 f, double c0, double2 *acc,
                              int rows, int cols, int ld, hipStream_t s) {
  const long long tot = (long long)rows * cols;
  const int nb = (int)std::min<long long>((tot + 255) / 256, 4096);
  hipLaunchKernelGGL(k_taylor_term, dim3(nb), dim3(256), 0, s, y, x, z, f, c0, acc, rows, cols, ld);
  return hipGetLastError();
}

__global__ void k_scale_block(double2 *y, double2 f, int rows, int cols, int ld) {
  const long long tot = (long long)rows * cols;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % rows), c = (int)(e / rows);
    const long long o = (long long)i + (long long)c * ld;
    y[o] = cmul(f, y[o]);
  }
}

hipError_t launch_scale_block(double2 *y, double2 f, int rows, int cols, int ld, hipStream_t s) {
  const long long tot = (long long)rows * cols;
  const int nb = (int)std::min<long long>((tot + 255) / 256, 4096);
  hipLaunchKernelGGL(k_scale_block, dim3(nb), dim3(256), 0, s, y, f, rows, cols, ld);
  return hipGetLastError();
}

hipError_t launch_step(const StepCtx &c, hipStream_t s) {
  const hipError_t e0 = launch_assemble(c, s);
  if (e0 != hipSuccess) return e0;
  return launch_step_only(c, s);
}

hipError_t launch_step_only(const StepCtx &c, hipStream_t s, bool beside) {
  subspace_init_attrs();
  // matrices in global memory: one thread per row.  Alone (stepwise, AFFINE)
  // one state per block with 16 column loads in flight per thread (the
  // shortest step); beside the rebuild of the next step two states per block
  // (half the blocks, so that the x/z transforms keep more CUs; measured on the
  // heterostructure: exponential 267 / 318 us, pipelined step 1.281 / 1.265 ms,
  // against 513 us and 1.349 ms for the column-split product)
  if (!c.h_in_lds && c.n_aux <= STEP_MULTI_MAXN) {
    const int nt = 64 * ((c.n_aux + 63) / 64);
#define LTD_SM(NS, UN, P)                                                                              \
  hipLaunchKernelGGL((k_step_multi<NS, UN, P>), dim3((c.n_states + NS - 1) / NS, c.n_k), dim3(P * nt), \
                     step_multi_lds_bytes(c.n_aux, NS, P), s, c)
    if (beside) LTD_SM(2, 8, 1);
    else if (c.rebuild || 3 * nt > 1024) LTD_SM(1, 16, 1);
    else LTD_SM(1, 12, 3);  // AFFINE: three parts of each row (n <= 320 at creation: 960 threads at most)
#undef LTD_SM
    return hipGetLastError();
  }
  const size_t lds = step_lds_bytes(c.n_aux, c.h_in_lds, false, c.p_in_lds);
  if (c.h_in_lds && c.p_in_lds)
    hipLaunchKernelGGL((k_step<true, true>), dim3(c.n_states, c.n_k), dim3(STEP_NT), lds, s, c);
  else if (c.h_in_lds)
    hipLaunchKernelGGL((k_step<true, false>), dim3(c.n_states, c.n_k), dim3(STEP_NT), lds, s, c);
  else
    hipLaunchKernelGGL((k_step<false, false>), dim3(c.n_states, c.n_k), dim3(STEP_NT), lds, s, c);
  return hipGetLastError();
}

__global__ void k_lookahead_init(const int *step, int n_steps, int *rs) {
  rs[0] = rs[2] = *step;
  rs[1] = rs[3] = *step + n_steps - 1;
}

__global__ void k_lookahead(int *rs) { rs[0] = min(rs[0] + 1, rs[1]); }

hipError_t launch_lookahead_init(const int *step, int n_steps, int *rs, hipStream_t s) {
  hipLaunchKernelGGL(k_lookahead_init, dim3(1), dim3(1), 0, s, step, n_steps, rs);
  return hipGetLastError();
}

hipError_t launch_lookahead(int *rs, hipStream_t s) {
  hipLaunchKernelGGL(k_lookahead, dim3(1), dim3(1), 0, s, rs);
  return hipGetLastError();
}

__global__ void k_gather_rows(double2 *dst, int ldd, const double2 *src, int lds, const int *idx, int rows,
                              int cols) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)rows * cols) return;
  const int i = (int)(e % rows), c = (int)(e / rows);
  dst[i + (long long)c * ldd] = src[idx[i] + (long long)c * lds];
}

hipError_t launch_gather_rows(double2 *dst, int ldd, const double2 *src, int lds, const int *idx, int rows, int cols,
                              hipStream_t s) {
  const long long tot = (long long)rows * cols;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, dst, ldd, src, lds, idx,
                     rows, cols);
  return hipGetLastError();
}

__global__ void k_scale_cols(double2 *out, const double2 *V, const double *w, int n) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < (long long)n * n) out[e] = cscale(V[e], 1.0 / sqrt(w[e / n]));
}

hipError_t launch_scale_cols(double2 *out, const double2 *V, const double *w, int n, hipStream_t s) {
  const long long tot = (long long)n * n;
  hipLaunchKernelGGL(k_scale_cols, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, out, V, w, n);
  return hipGetLastError();
}

hipError_t launch_adjoint(const StepCtx &c, const AdjCtx &a, hipStream_t s) {
  subspace_init_attrs();
  const size_t lds = step_lds_bytes(c.n_aux, c.h_in_lds, true);
  if (c.h_in_lds)
    hipLaunchKernelGGL((k_adjoint<true>), dim3(c.n_states, c.n_k), dim3(256), lds, s, c, a);
  else
    hipLaunchKernelGGL((k_adjoint<false>), dim3(c.n_states, c.n_k), dim3(256), lds, s, c, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_adjoint_finalize, dim3(1), dim3(64), 0, s, c, a);
  return hipGetLastError();
}

hipError_t launch_knot_samples(const double *q, int nk, double t_end, double dt, int ns, double *a_t,
                               double *a_mid, hipStream_t s) {
  const int tot = 2 * ns + 1;
  hipLaunchKernelGGL(k_knot_samples, dim3((tot + 255) / 256), dim3(256), 0, s, q, nk, t_end, dt, ns, a_t, a_mid);
  return hipGetLastError();
}

hipError_t launch_knot_gradient(const double *g_t, const double *g_mid, int ns, double dt, int nk, double t_end,
                                double *g_q, hipStream_t s) {
  hipLaunchKernelGGL(k_knot_gradient, dim3((nk + 63) / 64), dim3(64), 0, s, g_t, g_mid, ns, dt, nk, t_end, g_q);
  return hipGetLastError();
}

}  // namespace ltd
