// Plan construction and per-form dispatch (internal).
#pragma once

#include <complex>

#include "rw_common.h"

namespace rw {

int validate_plan(const rwpsf_optics* o, const rwpsf_grid* g, const rwpsf_numerics* nm);
int validate_stacks(const rwpsf_optics* o, const rwpsf_grid* g, const rwpsf_numerics* nm, int n,
                    const rwpsf_stack* s);
int plan_init(rwpsf_plan* p, const rwpsf_optics& o, const rwpsf_grid& g, const rwpsf_numerics& nm);
int fourier_compute(rwpsf_plan* p, int n, const rwpsf_stack* s, float2* E, float* I, hipStream_t st);
int fourier_build_pupils(rwpsf_plan* p, const rwpsf_stack* s, int nb, hipStream_t st);
int fourier_build_folded(rwpsf_plan* p, const rwpsf_stack* s, int nb, float2* Pf, hipStream_t st);
int fourier_adjoint(rwpsf_plan* p, int n, const rwpsf_stack* s, const float2* E, const float* dLdI,
                    int n_zernike, float* dc, float* dW0, hipStream_t st);
int czt_plan_init(rwpsf_plan* p);
int czt_compute(rwpsf_plan* p, int n, const rwpsf_stack* s, float2* E, float* I, hipStream_t st);
int bessel_compute(rwpsf_plan* p, int n, const rwpsf_stack* s, float2* E, float* I, hipStream_t st);
int bessel_compute_noalloc(rwpsf_plan* p, int n, const rwpsf_stack* s, float2* E, float* I, hipStream_t st);
int bessel_adjoint(rwpsf_plan* p, int n, const rwpsf_stack* s, const float2* E, const float* dLdI, float* dc,
                   float* dts, float* dz, hipStream_t st);

// Products q_s, q_p of the Fresnel transmission coefficients (Sec. 3.3) of the
// interfaces sample (n_s) -> coverslip (n_g) -> immersion (n_i) for the ray of immersion
// angle theta: n_m sin t_m = n_i sin t, n_m cos t_m = sqrt(n_m^2 - (n_i sin t)^2) on the
// principal branch, q_s^m = 2 n_m cos t_m / (n_m cos t_m + n_{m+1} cos t_{m+1}),
// q_p^m = 2 n_m cos t_m / (n_{m+1} cos t_m + n_m cos t_{m+1}).  1 when off.
inline void fresnel_q(const rwpsf_optics& o, double sin_t, std::complex<double>* qs,
                      std::complex<double>* qp) {
  *qs = 1.0;
  *qp = 1.0;
  if (!o.fresnel) return;
  const double inv2 = (o.n_i * sin_t) * (o.n_i * sin_t);
  const double media[3] = {o.n_s, o.n_g, o.n_i};
  for (int m = 0; m < 2; ++m) {
    const double n1 = media[m], n2 = media[m + 1];
    const std::complex<double> nc1 = std::sqrt(std::complex<double>(n1 * n1 - inv2, 0.0));
    const std::complex<double> nc2 = std::sqrt(std::complex<double>(n2 * n2 - inv2, 0.0));
    *qs *= 2.0 * nc1 / (nc1 + nc2);
    *qp *= 2.0 * nc1 / (n2 * (nc1 / n1) + n1 * (nc2 / n2));
  }
}

// Vectorial far field e_inf of Sec. 3.3 eq. "field Gaussian sphere" for e_inc =
// (ex, ey, 0) at direction (theta, phi) given by cos/sin values, with the Fresnel
// products qs, qp.
inline void far_field(std::complex<double> ex, std::complex<double> ey, double cos_t, double sin_t,
                      double cp, double sp, std::complex<double> qs, std::complex<double> qp,
                      std::complex<double> out[3]) {
  const double c2 = cp * cp - sp * sp, s2 = 2.0 * sp * cp;
  const std::complex<double> vx[3] = {qs * (1.0 - c2) + qp * ((1.0 + c2) * cos_t), (qp * cos_t - qs) * s2,
                                      -2.0 * cp * sin_t * qp};
  const std::complex<double> vy[3] = {(qp * cos_t - qs) * s2, qs * (1.0 + c2) + qp * ((1.0 - c2) * cos_t),
                                      -2.0 * sp * sin_t * qp};
  for (int c = 0; c < 3; ++c) out[c] = 0.5 * (vx[c] * ex + vy[c] * ey);
}

// amplitude factors a(s) of Sec. 3.4.3-3.4.4, and the optional extra s_z factor
inline double amplitude(const rwpsf_optics& o, double cos_t, double sin_t) {
  double a = 1.0;
  if (o.apodization) a *= std::sqrt(cos_t);
  if (o.s_env > 0.0) a *= std::exp(-(sin_t * sin_t) / (o.s_env * o.s_env));
  if (o.extra_sz) a *= cos_t;
  return a;
}

// Base pupil of one cell of the Cartesian grid, ds^2 a(s) e_inf,c(s) / s_z for the
// vectorial model (nc = 3) or ds^2 a(s) / s_z for the scalar model (nc = 1).
inline void base_pupil_cell(const rwpsf_optics& o, int nc, double ds, double sx, double sy,
                            std::complex<double> out[3]) {
  const double s2 = sx * sx + sy * sy;
  const double sin_t = std::sqrt(s2), cos_t = std::sqrt(1.0 - s2);
  const double w = ds * ds * amplitude(o, cos_t, sin_t) / cos_t;
  if (nc == 1) {
    out[0] = w;
    out[1] = out[2] = 0.0;
    return;
  }
  const double cp = sin_t > 0 ? sx / sin_t : 1.0, sp = sin_t > 0 ? sy / sin_t : 0.0;
  std::complex<double> qs, qp;
  fresnel_q(o, sin_t, &qs, &qp);
  far_field(std::complex<double>(o.ex_re, o.ex_im), std::complex<double>(o.ey_re, o.ey_im), cos_t, sin_t,
            cp, sp, qs, qp, out);
  for (int c = 0; c < 3; ++c) out[c] *= w;
}

template <class T>
int dev_alloc(rwpsf_plan* p, T** ptr, size_t count) {
  void* d = nullptr;
  const size_t bytes = count * sizeof(T);
  hipError_t e = hipMalloc(&d, bytes ? bytes : 16);
  if (e != hipSuccess) {
    set_hip_error(e);
    return RWPSF_ERR_OOM;
  }
  p->allocations.push_back(d);
  p->device_bytes += bytes;
  *ptr = (T*)d;
  return RWPSF_OK;
}

inline int hip_check(hipError_t e) {
  if (e == hipSuccess) return RWPSF_OK;
  set_hip_error(e);
  return RWPSF_ERR_HIP;
}

}  // namespace rw
