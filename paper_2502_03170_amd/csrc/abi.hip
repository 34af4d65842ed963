// C ABI entry points: status strings, validation, host reference routines,
// plan lifetime and the compute dispatch (see include/rwpsf.h).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "rw_common.h"
#include "rw_plan.h"

namespace rw {

static thread_local int g_last_hip = 0;
void set_hip_error(hipError_t e) { g_last_hip = (int)e; }

// n-point Gauss-Legendre rule on [a, b].  Newton's method on f(theta) = P_n(cos theta)
// from theta_i = pi (i + 3/4) / (n + 1/2); P_n, P_{n-1} by the three-term recurrence
// (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}.  With x = cos theta,
// d/dtheta P_n = n (x P_n - P_{n-1}) / sin theta, and the weight
// 2 (1 - x^2) / (n P_{n-1})^2 takes 1 - x^2 = sin^2 theta without cancellation.
int gauss_legendre(int n, double a, double b, double* x, double* w) {
  if (n < 1 || !x || !w || !std::isfinite(a) || !std::isfinite(b)) return RWPSF_ERR_INVALID_ARG;
  const double half = 0.5 * (b - a), mid = 0.5 * (b + a);
  if (n == 1) {
    x[0] = mid;
    w[0] = 2.0 * half;
    return RWPSF_OK;
  }
  auto legendre = [n](double t, double* pn, double* pm) {
    double p0 = 1.0, p1 = t;
    for (int k = 1; k < n; ++k) {
      const double p2 = ((2.0 * k + 1.0) * t * p1 - k * p0) / (k + 1.0);
      p0 = p1;
      p1 = p2;
    }
    *pn = p1;
    *pm = p0;
  };
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double th = kPi * (i + 0.75) / (n + 0.5);
    for (int it = 0; it < 100; ++it) {
      const double t = std::cos(th), st = std::sin(th);
      double pn, pm;
      legendre(t, &pn, &pm);
      const double dpdth = n * (t * pn - pm) / st;   // d/dtheta P_n(cos theta)
      const double d = pn / dpdth;
      th -= d;
      if (std::fabs(d) < 1e-17 * (1.0 + th)) break;
    }
    const double t = std::cos(th), st = std::sin(th);
    double pn, pm;
    legendre(t, &pn, &pm);
    const double wt = 2.0 * st * st / ((n * pm) * (n * pm));
    x[n - 1 - i] = mid + half * t;
    w[n - 1 - i] = half * wt;
    x[i] = mid - half * t;
    w[i] = half * wt;
  }
  return RWPSF_OK;
}

static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int validate_plan(const rwpsf_optics* o, const rwpsf_grid* g, const rwpsf_numerics* nm) {
  if (!o || !g || !nm) return RWPSF_ERR_INVALID_ARG;
  if (!finite_pos(o->na) || !finite_pos(o->n_i) || !(o->na < o->n_i)) return RWPSF_ERR_INVALID_ARG;
  if (!finite_pos(o->wavelength_nm) || !finite_pos(o->focal_length)) return RWPSF_ERR_INVALID_ARG;
  const double pol[4] = {o->ex_re, o->ex_im, o->ey_re, o->ey_im};
  double pn = 0;
  for (double p : pol) {
    if (!std::isfinite(p)) return RWPSF_ERR_INVALID_ARG;
    pn += p * p;
  }
  if (pn == 0.0) return RWPSF_ERR_INVALID_ARG;
  if (!std::isfinite(o->s_env) || o->s_env < 0.0) return RWPSF_ERR_INVALID_ARG;
  if (o->apodization != 0 && o->apodization != 1) return RWPSF_ERR_INVALID_ARG;
  if (o->gibson_lanni != 0 && o->gibson_lanni != 1) return RWPSF_ERR_INVALID_ARG;
  if (o->gibson_lanni) {
    if (!finite_pos(o->n_s) || !finite_pos(o->n_g) || !finite_pos(o->n_g_design) ||
        !finite_pos(o->n_i_design))
      return RWPSF_ERR_INVALID_ARG;
    const double t[3] = {o->t_g_nm, o->t_g_design_nm, o->t_i_design_nm};
    for (double v : t)
      if (!std::isfinite(v) || v < 0.0) return RWPSF_ERR_INVALID_ARG;
  }
  if (o->fresnel != 0 && o->fresnel != 1) return RWPSF_ERR_INVALID_ARG;
  if (o->extra_sz != 0 && o->extra_sz != 1) return RWPSF_ERR_INVALID_ARG;
  if (o->fresnel && (!finite_pos(o->n_s) || !finite_pos(o->n_g))) return RWPSF_ERR_INVALID_ARG;
  if (nm->model != RWPSF_MODEL_VECTORIAL && nm->model != RWPSF_MODEL_SCALAR) return RWPSF_ERR_INVALID_ARG;
  if (nm->theta_rule < RWPSF_THETA_GAUSS || nm->theta_rule > RWPSF_THETA_RIEMANN) return RWPSF_ERR_INVALID_ARG;
  if (nm->model == RWPSF_MODEL_SCALAR && o->fresnel) return RWPSF_ERR_UNSUPPORTED;
  if (g->nx < 1 || g->ny < 1 || g->nx > 8192 || g->ny > 8192) return RWPSF_ERR_INVALID_ARG;
  if (!finite_pos(g->dx_nm) || !finite_pos(g->dy_nm)) return RWPSF_ERR_INVALID_ARG;
  if (g->nz < 1 || g->nz > 65536 || !g->z_nm) return RWPSF_ERR_INVALID_ARG;
  for (int i = 0; i < g->nz; ++i)
    if (!std::isfinite(g->z_nm[i])) return RWPSF_ERR_INVALID_ARG;
  if (nm->form == RWPSF_FORM_FOURIER) {
    if (nm->n_pupil < 2 || nm->n_pupil > 1024) return RWPSF_ERR_INVALID_ARG;
  } else if (nm->form == RWPSF_FORM_CHIRPZ) {
    if (nm->n_pupil < 2 || nm->n_pupil > 1024) return RWPSF_ERR_INVALID_ARG;
    if (nm->n_pupil + std::max(g->nx, g->ny) - 1 > 2048) return RWPSF_ERR_UNSUPPORTED;
  } else if (nm->form == RWPSF_FORM_BESSEL) {
    if (nm->n_theta < 2 || nm->n_theta > 4096) return RWPSF_ERR_INVALID_ARG;
    if (nm->theta_rule == RWPSF_THETA_SIMPSON && (nm->n_theta < 3 || nm->n_theta % 2 == 0))
      return RWPSF_ERR_INVALID_ARG;
    if (nm->n_rho < 8 || nm->n_rho > 65536) return RWPSF_ERR_INVALID_ARG;
  } else {
    return RWPSF_ERR_INVALID_ARG;
  }
  return RWPSF_OK;
}

int validate_stacks(const rwpsf_optics* o, const rwpsf_grid* g, const rwpsf_numerics* nm, int n,
                    const rwpsf_stack* s) {
  if (n < 1 || n > RWPSF_MAX_STACKS_PER_CALL || !s) return RWPSF_ERR_INVALID_ARG;
  for (int i = 0; i < n; ++i) {
    const rwpsf_stack& st = s[i];
    if (!std::isfinite(st.t_s_nm) || !std::isfinite(st.x0_nm) || !std::isfinite(st.y0_nm) ||
        !std::isfinite(st.z_offset_nm))
      return RWPSF_ERR_INVALID_ARG;
    if (st.t_s_nm < 0.0) return RWPSF_ERR_INVALID_ARG;
    if (st.n_zernike < 0 || st.n_zernike > RWPSF_MAX_ZERNIKE) return RWPSF_ERR_INVALID_ARG;
    if (st.n_zernike > 0 && !st.zernike_waves) return RWPSF_ERR_INVALID_ARG;
    for (int q = 0; q < st.n_zernike; ++q)
      if (!std::isfinite(st.zernike_waves[q])) return RWPSF_ERR_INVALID_ARG;
    if (nm->form == RWPSF_FORM_BESSEL) {
      if (st.phase_map) return RWPSF_ERR_NOT_AXISYMMETRIC;
      for (int q = 0; q < st.n_zernike; ++q) {
        int zn, zm;
        noll_nm(q + 1, &zn, &zm);
        if (zm != 0 && st.zernike_waves[q] != 0.0) return RWPSF_ERR_NOT_AXISYMMETRIC;
      }
      // the radial table covers lateral emitter shifts up to one pixel
      if (std::fabs(st.x0_nm) > g->dx_nm || std::fabs(st.y0_nm) > g->dy_nm)
        return RWPSF_ERR_INVALID_ARG;
    }
  }
  (void)o;
  return RWPSF_OK;
}

}  // namespace rw

static hipEvent_t pool_get(std::vector<hipEvent_t>& pool) {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

int rwpsf_plan::time_begin(int kernel, hipStream_t st) {
  if (!timing) return -1;
  TimingRec r{kernel, pool_get(event_pool), pool_get(event_pool)};
  if (!r.a || !r.b || hipEventRecord(r.a, st) != hipSuccess) {   // this launch is then not timed
    if (r.a) event_pool.push_back(r.a);
    if (r.b) event_pool.push_back(r.b);
    return -1;
  }
  timing_recs.push_back(r);
  return (int)timing_recs.size() - 1;
}

void rwpsf_plan::time_end(int rec, hipStream_t st) {
  // a failed record leaves the end event unrecorded; timing_flush then skips this launch
  if (rec >= 0) (void)hipEventRecord(timing_recs[rec].b, st);
}

void rwpsf_plan::timing_flush() {
  for (TimingRec& r : timing_recs) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      timing_ms[r.kernel] += ms;
      timing_launches[r.kernel] += 1;
    }
    event_pool.push_back(r.a);
    event_pool.push_back(r.b);
  }
  timing_recs.clear();
}

rwpsf_plan::~rwpsf_plan() {   // teardown: failures cannot be reported and are ignored
  for (TimingRec& r : timing_recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (hipEvent_t e : event_pool) (void)hipEventDestroy(e);
  for (void* p : allocations) (void)hipFree(p);
}

extern "C" {

int rwpsf_abi_version(void) { return RWPSF_ABI_VERSION; }

const char* rwpsf_status_string(int s) {
  switch (s) {
    case RWPSF_OK: return "ok";
    case RWPSF_ERR_INVALID_ARG: return "invalid argument";
    case RWPSF_ERR_NOT_AXISYMMETRIC: return "the Bessel form needs an axisymmetric pupil";
    case RWPSF_ERR_UNSUPPORTED: return "unsupported option";
    case RWPSF_ERR_OOM: return "out of memory";
    case RWPSF_ERR_HIP: return "HIP runtime error";
    case RWPSF_ERR_NO_DEVICE: return "no usable gfx950 device";
    case RWPSF_ERR_SCRATCH_LIMIT:
      return "one stack needs more than the fixed scratch of the allocation-free entry point";
    default: return "unknown status";
  }
}

int rwpsf_last_hip_error(void) { return rw::g_last_hip; }

int rwpsf_validate(const rwpsf_optics* o, const rwpsf_grid* g, const rwpsf_numerics* nm) {
  return rw::validate_plan(o, g, nm);
}

int rwpsf_validate_stacks(const rwpsf_optics* o, const rwpsf_grid* g, const rwpsf_numerics* nm,
                          int n, const rwpsf_stack* s) {
  int st = rw::validate_plan(o, g, nm);
  if (st != RWPSF_OK) return st;
  return rw::validate_stacks(o, g, nm, n, s);
}

int rwpsf_gauss_legendre(int n, double a, double b, double* x, double* w) {
  return rw::gauss_legendre(n, a, b, x, w);
}

int rwpsf_bessel_j(int order, int count, const double* x, double* out) {
  if (order < 0 || order > 8 || count < 0 || (count > 0 && (!x || !out))) return RWPSF_ERR_INVALID_ARG;
  for (int i = 0; i < count; ++i) {
    if (!std::isfinite(x[i]) || x[i] < 0.0) return RWPSF_ERR_INVALID_ARG;
    out[i] = rw::bessel_j(order, x[i]);
  }
  return RWPSF_OK;
}

int rwpsf_zernike(int j, int count, const double* r, const double* phi, double* out) {
  if (j < 1 || count < 0 || (count > 0 && (!r || !phi || !out))) return RWPSF_ERR_INVALID_ARG;
  for (int i = 0; i < count; ++i) out[i] = rw::zernike_noll(j, r[i], std::cos(phi[i]), std::sin(phi[i]));
  return RWPSF_OK;
}

int rwpsf_plan_create(const rwpsf_optics* o, const rwpsf_grid* g, const rwpsf_numerics* nm,
                      rwpsf_plan** out) {
  if (!out) return RWPSF_ERR_INVALID_ARG;
  *out = nullptr;
  int st = rw::validate_plan(o, g, nm);
  if (st != RWPSF_OK) return st;
  rwpsf_plan* p = new (std::nothrow) rwpsf_plan();
  if (!p) return RWPSF_ERR_OOM;
  st = rw::plan_init(p, *o, *g, *nm);
  if (st != RWPSF_OK) {
    delete p;
    return st;
  }
  *out = p;
  return RWPSF_OK;
}

void rwpsf_plan_destroy(rwpsf_plan* p) {   // teardown: HIP failures are ignored
  if (!p) return;
  int cur = 0;
  const bool had = hipGetDevice(&cur) == hipSuccess;
  (void)hipSetDevice(p->device);
  (void)hipDeviceSynchronize();
  delete p;
  if (had) (void)hipSetDevice(cur);
}

size_t rwpsf_plan_device_bytes(const rwpsf_plan* p) { return p ? p->device_bytes : 0; }

int rwpsf_plan_set_timing(rwpsf_plan* p, int enable) {
  if (!p) return RWPSF_ERR_INVALID_ARG;
  p->timing_flush();
  for (int i = 0; i < RWPSF_KERNEL_COUNT; ++i) {
    p->timing_ms[i] = 0.0;
    p->timing_launches[i] = 0;
  }
  p->timing = enable != 0;
  return RWPSF_OK;
}

int rwpsf_plan_timing(rwpsf_plan* p, int kernel, double* total_ms, int64_t* launches) {
  if (!p || kernel < 0 || kernel >= RWPSF_KERNEL_COUNT || !total_ms || !launches)
    return RWPSF_ERR_INVALID_ARG;
  p->timing_flush();
  *total_ms = p->timing_ms[kernel];
  *launches = p->timing_launches[kernel];
  return RWPSF_OK;
}

int rwpsf_compute(rwpsf_plan* p, int n, const rwpsf_stack* s, void* E, float* I, void* stream) {
  if (!p) return RWPSF_ERR_INVALID_ARG;
  if (!E && !I) return RWPSF_ERR_INVALID_ARG;
  int st = rw::validate_stacks(&p->opt, &p->grid, &p->num, n, s);
  if (st != RWPSF_OK) return st;
  if (p->num.form == RWPSF_FORM_FOURIER)
    return rw::fourier_compute(p, n, s, (float2*)E, I, (hipStream_t)stream);
  if (p->num.form == RWPSF_FORM_CHIRPZ) return rw::czt_compute(p, n, s, (float2*)E, I, (hipStream_t)stream);
  return rw::bessel_compute(p, n, s, (float2*)E, I, (hipStream_t)stream);
}

int rwpsf_compute_noalloc(rwpsf_plan* p, int n, const rwpsf_stack* s, void* E, float* I, void* stream) {
  if (!p) return RWPSF_ERR_INVALID_ARG;
  if (!E && !I) return RWPSF_ERR_INVALID_ARG;
  if (p->num.form != RWPSF_FORM_BESSEL) return RWPSF_ERR_UNSUPPORTED;
  int st = rw::validate_stacks(&p->opt, &p->grid, &p->num, n, s);
  if (st != RWPSF_OK) return st;
  return rw::bessel_compute_noalloc(p, n, s, (float2*)E, I, (hipStream_t)stream);
}

int rwpsf_adjoint(rwpsf_plan* p, int n, const rwpsf_stack* s, const void* E, const float* dLdI,
                  int n_zernike, float* dc, float* dW0, void* stream) {
  if (!p || !E || !dLdI) return RWPSF_ERR_INVALID_ARG;
  if (n_zernike < 0 || n_zernike > RWPSF_MAX_ZERNIKE || (n_zernike > 0 && !dc)) return RWPSF_ERR_INVALID_ARG;
  if (p->num.form != RWPSF_FORM_FOURIER || p->num.model != RWPSF_MODEL_VECTORIAL) return RWPSF_ERR_UNSUPPORTED;
  int st = rw::validate_stacks(&p->opt, &p->grid, &p->num, n, s);
  if (st != RWPSF_OK) return st;
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != p->device) return RWPSF_ERR_INVALID_ARG;
  return rw::fourier_adjoint(p, n, s, (const float2*)E, dLdI, n_zernike, dc, dW0, (hipStream_t)stream);
}

int rwpsf_adjoint_bessel(rwpsf_plan* p, int n, const rwpsf_stack* s, const void* E, const float* dLdI,
                         float* dc, float* dts, float* dz, void* stream) {
  if (!p || !E || !dLdI) return RWPSF_ERR_INVALID_ARG;
  if (p->num.form != RWPSF_FORM_BESSEL) return RWPSF_ERR_UNSUPPORTED;
  int st = rw::validate_stacks(&p->opt, &p->grid, &p->num, n, s);
  if (st != RWPSF_OK) return st;
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != p->device) return RWPSF_ERR_INVALID_ARG;
  return rw::bessel_adjoint(p, n, s, (const float2*)E, dLdI, dc, dts, dz, (hipStream_t)stream);
}

}  // extern "C"
