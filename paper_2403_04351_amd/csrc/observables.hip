// Pulses and spectra of the propagation: the sampled vector potential of the
// paper's excitations (impulsive kick, Sec. 3.1; sin^2-envelope laser, Sec. 3.2;
// the Gaussian-envelope pulse of the benchmark workloads) and the dynamical
// polarizability alpha_zz(w) = (i Omega / w) J(w) / E(w) (Sec. 2, Eq. (5)).
#include "ltd.h"

#include <cmath>

#include "common.h"

namespace ltd {
namespace {

__device__ double pulse_at(int kind, const double *p, double t) {
  if (kind == LTD_PULSE_SIN2) {  // A0 cos(w t) sin^2[pi (t - t0)/T_p] on [t0, t0 + T_p]
    if (t < p[2] || t > p[2] + p[3]) return 0.0;
    const double s = sin(M_PI * (t - p[2]) / p[3]);
    return p[0] * cos(p[1] * t) * s * s;
  }
  if (kind == LTD_PULSE_KICK) return t > 0.0 ? -p[1] * p[0] : 0.0;  // E0 delta(t - 0+): A = -c E0
  const double x = (t - p[2]) / p[3];  // A0 sin(w t) exp(-((t - t0)/width)^2)
  return p[0] * sin(p[1] * t) * exp(-x * x);
}

__global__ void k_pulse(int kind, double p0, double p1, double p2, double p3, double dt, int n_steps, double *a_t,
                        double *a_mid) {
  const double p[4] = {p0, p1, p2, p3};
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i <= n_steps; i += gridDim.x * blockDim.x) {
    a_t[i] = pulse_at(kind, p, i * dt);
    if (i < n_steps) a_mid[i] = pulse_at(kind, p, (i + 0.5) * dt);
  }
}

// One block per frequency: J(w) = dt sum_n w_n (J_n - J_0) e^{(i w - gamma) t_n}
// (trapezoid weights) and E(w) = -(1/c) sum_n (A_{n+1} - A_n) e^{(i w - gamma) t_{n+1/2}};
// alpha = (i Omega / w) J / E.  Fixed-order block reduction.
constexpr int POL_NT = 256;
__global__ __launch_bounds__(POL_NT) void k_polarizability(const double *j, const double *a, int n, double dt,
                                                           double omega_cell, double c_light, const double *w,
                                                           double gamma, double2 *alpha) {
  __shared__ double red[4][POL_NT];
  const double om = w[blockIdx.x];
  const double j0 = j[0];
  double jr = 0.0, ji = 0.0, er = 0.0, ei = 0.0;
  for (int i = threadIdx.x; i <= n; i += POL_NT) {
    const double t = i * dt;
    const double wt = (i == 0 || i == n) ? 0.5 : 1.0;
    double s, c;
    sincos(om * t, &s, &c);
    const double g = exp(-gamma * t) * wt * (j[i] - j0);
    jr += g * c;
    ji += g * s;
    if (i < n) {
      const double tm = (i + 0.5) * dt;
      sincos(om * tm, &s, &c);
      const double f = -(a[i + 1] - a[i]) / c_light * exp(-gamma * tm);
      er += f * c;
      ei += f * s;
    }
  }
  red[0][threadIdx.x] = jr;
  red[1][threadIdx.x] = ji;
  red[2][threadIdx.x] = er;
  red[3][threadIdx.x] = ei;
  __syncthreads();
  for (int h = POL_NT / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h)
      for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double2 jw = make_double2(dt * red[0][0], dt * red[1][0]);
    const double2 ew = make_double2(red[2][0], red[3][0]);
    const double den = ew.x * ew.x + ew.y * ew.y;
    const double2 q = make_double2((jw.x * ew.x + jw.y * ew.y) / den, (jw.y * ew.x - jw.x * ew.y) / den);
    const double s = omega_cell / om;  // i s q
    alpha[blockIdx.x] = make_double2(-s * q.y, s * q.x);
  }
}

}  // namespace
}  // namespace ltd

using namespace ltd;

extern "C" {

ltd_status ltd_pulse_samples(int kind, const double *params, double dt, int n_steps, double *a_t, double *a_mid,
                             void *stream) {
  if (!params || !a_t || !a_mid) return LTD_EINVAL;
  if (kind != LTD_PULSE_GAUSS_SIN && kind != LTD_PULSE_SIN2 && kind != LTD_PULSE_KICK) return LTD_EINVAL;
  if (n_steps < 1 || !(dt > 0.0) || !std::isfinite(dt)) return LTD_ESHAPE;
  for (int i = 0; i < 4; ++i)
    if (!std::isfinite(params[i])) return LTD_EINVAL;
  if (kind == LTD_PULSE_SIN2 && !(params[3] > 0.0)) return LTD_EINVAL;
  if (kind == LTD_PULSE_GAUSS_SIN && !(params[3] > 0.0)) return LTD_EINVAL;
  if (kind == LTD_PULSE_KICK && !(params[1] > 0.0)) return LTD_EINVAL;
  const int blocks = std::min(1024, (n_steps + 256) / 256);
  hipLaunchKernelGGL(k_pulse, dim3(blocks), dim3(256), 0, reinterpret_cast<hipStream_t>(stream), kind, params[0],
                     params[1], params[2], params[3], dt, n_steps, a_t, a_mid);
  return hipGetLastError() == hipSuccess ? LTD_OK : LTD_EHIP;
}

ltd_status ltd_polarizability(const double *j, const double *a_t, int n_steps, double dt, double omega_cell,
                              double c_light, const double *w, int n_w, double gamma, void *alpha, void *stream) {
  if (!j || !a_t || !w || !alpha) return LTD_EINVAL;
  if (n_steps < 1 || n_w < 1 || n_w > 65535) return LTD_ESHAPE;
  if (!(dt > 0.0) || !(omega_cell > 0.0) || !(c_light > 0.0) || !(gamma >= 0.0) || !std::isfinite(gamma))
    return LTD_EINVAL;
  if (((uintptr_t)alpha & 15u) != 0) return LTD_EALIGN;
  hipLaunchKernelGGL(k_polarizability, dim3(n_w), dim3(POL_NT), 0, reinterpret_cast<hipStream_t>(stream), j, a_t,
                     n_steps, dt, omega_cell, c_light, w, gamma, reinterpret_cast<double2 *>(alpha));
  return hipGetLastError() == hipSuccess ? LTD_OK : LTD_EHIP;
}

}  // extern "C"
