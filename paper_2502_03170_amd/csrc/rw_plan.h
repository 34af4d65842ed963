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
int fourier_adjoint(rwpsf_plan* p, int n, const rwpsf_stack* s, const float2* E, const float* dLdI,
                    int n_zernike, float* dc, float* dW0, hipStream_t st);
int czt_plan_init(rwpsf_plan* p);
int czt_compute(rwpsf_plan* p, int n, const rwpsf_stack* s, float2* E, float* I, hipStream_t st);
int bessel_compute(rwpsf_plan* p, int n, const rwpsf_stack* s, float2* E, float* I, hipStream_t st);

// Vectorial far field e_inf of Sec. 3.3 eq. "field Gaussian sphere" with q_s = q_p = 1,
// for e_inc = (ex, ey, 0) at direction (theta, phi) given by cos/sin values.
inline void far_field(std::complex<double> ex, std::complex<double> ey, double cos_t, double sin_t,
                      double cp, double sp, std::complex<double> out[3]) {
  const double c2 = cp * cp - sp * sp, s2 = 2.0 * sp * cp;
  const double vx[3] = {(1.0 - c2) + (1.0 + c2) * cos_t, (cos_t - 1.0) * s2, -2.0 * cp * sin_t};
  const double vy[3] = {(cos_t - 1.0) * s2, (1.0 + c2) + (1.0 - c2) * cos_t, -2.0 * sp * sin_t};
  for (int c = 0; c < 3; ++c) out[c] = 0.5 * (vx[c] * ex + vy[c] * ey);
}

// amplitude factors a(s) of Sec. 3.4.3-3.4.4
inline double amplitude(const rwpsf_optics& o, double cos_t, double sin_t) {
  double a = 1.0;
  if (o.apodization) a *= std::sqrt(cos_t);
  if (o.s_env > 0.0) a *= std::exp(-(sin_t * sin_t) / (o.s_env * o.s_env));
  return a;
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
