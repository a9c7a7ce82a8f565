// Interstitial part of the LAPW+LO operators by matrix-matrix multiplication
// (Pela & Draxl, Sec. 2.3, first route; App. A, Eqs. (A.4), (A.7)): the
// plane-wave blocks are dense N_G x N_G matrices whose elements are Fourier
// coefficients of the step function and of Theta V at differences of G vectors,
//   S_GG' = Theta~(g - g'),          T_GG' = 1/2 (G+k).(G'+k) Theta~(g - g'),
//   V_GG' = (Theta V)~(g - g'),      P_GG' = 1/2 [(G+k)_z + (G'+k)_z] Theta~(g - g'),
// with f~(q) = (1/N) sum_j f_j exp(-2 pi i q.j / N), and are applied by the
// complex GEMM.  Storage and work grow as N_G^2 (the route's cost the paper
// compares with the flat cost of the FFT route, Sec. 3.2).
//
// The coefficients are needed only in the box of differences |q_d| <= 2 b_d
// (b_d the largest |g_d|), computed by three separable DFT passes over the
// real grid field (x, then y, then z), each keeping only the box frequencies.
#include "common.h"

namespace ltd {
namespace {

// exp(-2 pi i q j / n) from the twiddle table of length n (q may be negative)
__device__ inline double2 twq(const double2 *tw, int q, int j, int n) {
  long long m = ((long long)q * j) % n;
  if (m < 0) m += n;
  return tw[m];
}

// pass x: A[z][y][qx] = sum_x f(z, y, x) exp(-2 pi i qx x / n1), f = th v, or th
// alone when v is NULL (v read at v + (*step) stride when step is set)
__global__ void k_box_x(const double *__restrict__ th, const double *__restrict__ v, const int *step,
                        long long stride, int n1, int n2, int n3, int qx, const double2 *__restrict__ tw1,
                        double2 *__restrict__ out) {
  if (step) v += (long long)(*step) * stride;
  const int nqx = 2 * qx + 1;
  const long long tot = (long long)n3 * n2 * nqx;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const int iq = (int)(e % nqx);
    const long long zy = e / nqx;
    const int q = iq - qx;
    const double *row = v ? v + zy * n1 : nullptr;
    const double *trow = th + zy * n1;
    double2 acc = make_double2(0.0, 0.0);
    for (int x = 0; x < n1; ++x) {
      const double f = row ? trow[x] * row[x] : trow[x];
      const double2 w = twq(tw1, q, x, n1);
      acc.x = fma(f, w.x, acc.x);
      acc.y = fma(f, w.y, acc.y);
    }
    out[e] = acc;
  }
}

// pass y: B[z][qy][qx] = sum_y A[z][y][qx] exp(-2 pi i qy y / n2)
__global__ void k_box_y(const double2 *__restrict__ in, int n2, int n3, int nqx, int qy,
                        const double2 *__restrict__ tw2, double2 *__restrict__ out) {
  const int nqy = 2 * qy + 1;
  const long long tot = (long long)n3 * nqy * nqx;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const int ix = (int)(e % nqx);
    const int iy = (int)((e / nqx) % nqy);
    const int z = (int)(e / ((long long)nqx * nqy));
    const int q = iy - qy;
    double2 acc = make_double2(0.0, 0.0);
    for (int y = 0; y < n2; ++y) acc = cfma(in[((long long)z * n2 + y) * nqx + ix], twq(tw2, q, y, n2), acc);
    out[e] = acc;
  }
}

// pass z: F[qz][qy][qx] = (1/N) sum_z B[z][qy][qx] exp(-2 pi i qz z / n3)
__global__ void k_box_z(const double2 *__restrict__ in, int n3, int nqxy, int qz, double inv_n,
                        const double2 *__restrict__ tw3, double2 *__restrict__ out) {
  const int nqz = 2 * qz + 1;
  const long long tot = (long long)nqz * nqxy;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const int ixy = (int)(e % nqxy);
    const int q = (int)(e / nqxy) - qz;
    double2 acc = make_double2(0.0, 0.0);
    for (int z = 0; z < n3; ++z) acc = cfma(in[(long long)z * nqxy + ixy], twq(tw3, q, z, n3), acc);
    out[e] = cscale(acc, inv_n);
  }
}

// Dense N_G x N_G block (column-major, ld) of one operator at the G vectors
// g[idx[i]] (rows) and g[idx[j]] (columns); idx = NULL: natural order.
// which: 0 S (Theta~), 1 T, 2 V ((Theta V)~ from fv), 3 P_z.
__global__ void k_dense(int which, const int *__restrict__ gint, const double *__restrict__ gk,
                        const int *__restrict__ idx, int ng, const double2 *__restrict__ ft,
                        const double2 *__restrict__ fv, int qx, int qy, int qz, double2 *__restrict__ out, long long ld) {
  const long long tot = (long long)ng * ng;
  const int nqx = 2 * qx + 1, nqy = 2 * qy + 1;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % ng), j = (int)(e / ng);
    const int a = idx ? idx[i] : i, b = idx ? idx[j] : j;
    const int dx = gint[3 * a] - gint[3 * b], dy = gint[3 * a + 1] - gint[3 * b + 1],
              dz = gint[3 * a + 2] - gint[3 * b + 2];
    const long long q = ((long long)(dz + qz) * nqy + (dy + qy)) * nqx + (dx + qx);
    double2 val;
    if (which == 2) {
      val = fv[q];
    } else {
      const double2 t = ft[q];
      double f = 1.0;
      if (which == 1)
        f = 0.5 * (gk[3 * a] * gk[3 * b] + gk[3 * a + 1] * gk[3 * b + 1] + gk[3 * a + 2] * gk[3 * b + 2]);
      else if (which == 3)
        f = 0.5 * (gk[3 * a + 2] + gk[3 * b + 2]);
      val = cscale(t, f);
    }
    out[(long long)i + (long long)j * ld] = val;
  }
}

int blocks_for(long long tot) { return (int)std::min<long long>((tot + 255) / 256, 16384); }

}  // namespace

size_t mm_box_values(const Grid &g) { return (size_t)(4 * g.bx + 1) * (4 * g.by + 1) * (4 * g.bz + 1); }

size_t mm_box_scratch(const Grid &g) {
  const size_t a = (size_t)g.n3 * g.n2 * (4 * g.bx + 1), b = (size_t)g.n3 * (4 * g.by + 1) * (4 * g.bx + 1);
  return a + b;
}

hipError_t mm_box_coefficients(const Grid &g, const double *th, const double *v, const int *step, long long stride,
                               double2 *scratch, double2 *out, hipStream_t s) {
  const int qx = 2 * g.bx, qy = 2 * g.by, qz = 2 * g.bz;
  const int nqx = 2 * qx + 1, nqy = 2 * qy + 1;
  double2 *a = scratch, *b = scratch + (size_t)g.n3 * g.n2 * nqx;
  long long tot = (long long)g.n3 * g.n2 * nqx;
  hipLaunchKernelGGL(k_box_x, dim3(blocks_for(tot)), dim3(256), 0, s, th, v, step, stride, g.n1, g.n2, g.n3, qx, g.tw1,
                     a);
  tot = (long long)g.n3 * nqy * nqx;
  hipLaunchKernelGGL(k_box_y, dim3(blocks_for(tot)), dim3(256), 0, s, a, g.n2, g.n3, nqx, qy, g.tw2, b);
  tot = (long long)(2 * qz + 1) * nqy * nqx;
  const double inv_n = 1.0 / ((double)g.n1 * g.n2 * g.n3);
  hipLaunchKernelGGL(k_box_z, dim3(blocks_for(tot)), dim3(256), 0, s, b, g.n3, nqx * nqy, qz, inv_n, g.tw3, out);
  return hipGetLastError();
}

hipError_t mm_dense(int which, const Grid &g, const int *gint, const double *gk, const int *idx, int ng,
                    const double2 *ft, const double2 *fv, double2 *out, long long ld, hipStream_t s) {
  const long long tot = (long long)ng * ng;
  hipLaunchKernelGGL(k_dense, dim3(blocks_for(tot)), dim3(256), 0, s, which, gint, gk, idx, ng, ft, fv, 2 * g.bx,
                     2 * g.by, 2 * g.bz, out, ld);
  return hipGetLastError();
}

}  // namespace ltd
