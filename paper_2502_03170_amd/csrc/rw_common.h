// Internal declarations of the rwpsf library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <vector>

#include "rwpsf.h"

#define RW_HD __host__ __device__ inline

namespace rw {

constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 6.28318530717958647692;

// ---------------------------------------------------------------------------
// Bessel functions of the first kind, J_n(x) = (1/pi) int_0^pi cos(n t - x sin t) dt.
// The integrand is 2 pi periodic and even about pi, so the M-point trapezoid rule
// on [0, 2 pi) is exact up to the aliased orders J_{n +- M} (Jacobi-Anger).  J_nu(x)
// decays past the turning point nu = x on the scale x^(1/3) (Airy transition), so
// M = n + x + 12 x^(1/3) + 32 keeps the aliased terms below 1e-20.
// ---------------------------------------------------------------------------
RW_HD double bessel_j(int n, double x) {
  if (x == 0.0) return n == 0 ? 1.0 : 0.0;
  const double ax = fabs(x);
  int m = n + (int)ceil(ax + 12.0 * cbrt(ax)) + 32;
  m += m & 1;
  const double h = kTwoPi / m;
  double s = 0.0;
  for (int i = 0; i < m; ++i) {
    const double t = h * i;
    s += cos(n * t - x * sin(t));
  }
  return s / m;
}

// ---------------------------------------------------------------------------
// Noll-indexed Zernike polynomials, orthonormal on the unit disk (Sec. 3.4.2).
// ---------------------------------------------------------------------------
RW_HD void noll_nm(int j, int* n_out, int* m_out) {
  int n = 0;
  while ((n + 1) * (n + 2) / 2 < j) ++n;
  const int p = j - n * (n + 1) / 2 - 1;
  const int am = (n % 2 == 0) ? 2 * ((p + 1) / 2) : 2 * (p / 2) + 1;
  *n_out = n;
  *m_out = (am == 0) ? 0 : ((j % 2 == 0) ? am : -am);
}

RW_HD double factorial_d(int k) {
  double f = 1.0;
  for (int i = 2; i <= k; ++i) f *= i;
  return f;
}

// Coefficient of r^(n-2s) in R_n^|m|, times the orthonormalisation factor.
RW_HD double zernike_radial_coef(int n, int am, int s) {
  const double sign = (s & 1) ? -1.0 : 1.0;
  return sign * factorial_d(n - s) /
         (factorial_d(s) * factorial_d((n + am) / 2 - s) * factorial_d((n - am) / 2 - s));
}

RW_HD double zernike_noll(int j, double r, double cp, double sp) {
  int n, m;
  noll_nm(j, &n, &m);
  const int am = m < 0 ? -m : m;
  double rad = 0.0;
  for (int s = 0; s <= (n - am) / 2; ++s) rad += zernike_radial_coef(n, am, s) * pow(r, n - 2 * s);
  if (m == 0) return sqrt((double)(n + 1)) * rad;
  // cos(am p), sin(am p) by the angle-addition recurrence
  double c = 1.0, s = 0.0;
  for (int i = 0; i < am; ++i) {
    const double c2 = c * cp - s * sp;
    s = s * cp + c * sp;
    c = c2;
  }
  return sqrt(2.0 * (n + 1)) * rad * (m > 0 ? c : s);
}

// ---------------------------------------------------------------------------
// Gibson-Lanni OPD (Sec. 3.4.1, eq. "stratified layers general formula"), with
// t_i from the focusing condition eq. "gibson lanni t_i" as printed.  Returns
// W = (re, im): a principal-branch square root makes im >= 0 past a critical angle.
// ---------------------------------------------------------------------------
struct GLParams {
  double k0;  // 2 pi / lambda
  double n_i, n_s, n_g, n_g_d, n_i_d;
  double t_g, t_g_d, t_i_d;
};

RW_HD double gl_ti(const GLParams& g, double t_s) {
  return t_s + g.n_i * (-t_s / g.n_s - g.t_g / g.n_g + g.t_g_d / g.n_g_d + g.t_i_d / g.n_i_d);
}

// sqrt(n^2 - q) for real arguments, principal branch: (re, im)
RW_HD void csqrt_real(double v, double* re, double* im) {
  if (v >= 0.0) {
    *re = sqrt(v);
    *im = 0.0;
  } else {
    *re = 0.0;
    *im = sqrt(-v);
  }
}

RW_HD void gl_opd(const GLParams& g, double t_s, double sin_t, double* w_re, double* w_im) {
  const double q = g.n_i * g.n_i * sin_t * sin_t;
  const double t_i = gl_ti(g, t_s);
  const double n[5] = {g.n_s, g.n_i, g.n_i_d, g.n_g, g.n_g_d};
  const double t[5] = {t_s, t_i, -g.t_i_d, g.t_g, -g.t_g_d};
  double re = 0.0, im = 0.0;
  for (int i = 0; i < 5; ++i) {
    double a, b;
    csqrt_real(n[i] * n[i] - q, &a, &b);
    re += t[i] * a;
    im += t[i] * b;
  }
  *w_re = g.k0 * re;
  *w_im = g.k0 * im;
}

// Reduce an FP64 phase to [-pi, pi] before it is rounded to FP32.
RW_HD double reduce_2pi(double p) { return p - kTwoPi * rint(p * (1.0 / kTwoPi)); }

// sin and cos of 2 pi t: t is reduced to [-1/2, 1/2] in FP64 and rounded once to FP32,
// then the hardware sine and cosine, which take their argument in revolutions (on
// [-1/2, 1/2] their largest error measured 1.3e-7, that of sincosf 1.5e-7).
__device__ __forceinline__ void sincos_rev(double t, float* s, float* c) {
  const float r = (float)(t - rint(t));
  *s = __builtin_amdgcn_sinf(r);
  *c = __builtin_amdgcn_cosf(r);
}

// ---------------------------------------------------------------------------
// Host helpers
// ---------------------------------------------------------------------------
int gauss_legendre(int n, double a, double b, double* x, double* w);
void set_hip_error(hipError_t e);

struct PlanDevice;  // per-form device state

}  // namespace rw

// ---------------------------------------------------------------------------
// Plan
// ---------------------------------------------------------------------------
struct rwpsf_plan {
  int device = 0;
  rwpsf_optics opt{};
  rwpsf_grid grid{};
  rwpsf_numerics num{};
  std::vector<double> z;
  double k = 0, s_max = 0, theta_max = 0;
  int nc = 3;                   // output channels: 3 (vectorial model) or 1 (scalar model)
  rw::GLParams gl{};
  size_t device_bytes = 0;
  std::vector<void*> allocations;

  // Fourier form (device operands zero-padded to whole GEMM tiles)
  int np = 0, nxp = 0, nyp = 0; // padded pupil size and output widths
  double* d_z = nullptr;        // [nz]
  double* d_ksz = nullptr;      // [np][np] k * s_z (0 outside the disk)
  float2* d_Q = nullptr;        // [3][np][np] ds^2 a e_inf,c / s_z (0 outside)
  int nhp = 0;                  // folded pupil cells per axis, padded (2 nhp = np)
  double* d_kszf = nullptr;     // [nhp][nhp] k * s_z on the folded cells
  float* d_B1 = nullptr;        // [nyp][2 nhp] cos / sin (k s_y[lf] y_n)
  float* d_A2T = nullptr;       // [nxp][2 nhp] pref cos / sin (k s_x[jf] x_m), pref = f k / 2 pi
  float* d_ztab = nullptr;      // [RWPSF_MAX_ZERNIKE][N][N] Noll basis on the pupil cells
  float2* d_P = nullptr;        // workspace [chunk][3][np][np]
  float2* d_Pf = nullptr;       // workspace [chunk][3][2 nhp][2 nhp] folded pupils
  float2* d_T = nullptr;        // workspace [planes][3][2 nhp][nyp]
  size_t T_planes = 0;          // capacity of d_T in stack-planes
  // adjoint (built on first use)
  float* d_CxT = nullptr;       // [2 nhp][nxp] folded x table (prefactor included), pixels contiguous
  float* d_CyT = nullptr;       // [2 nhp][nyp] folded y table, pixels contiguous
  float2* d_H = nullptr;        // [32 stacks][nz][3][nxp][2 nhp] folded H
  float2* d_adjPf = nullptr;    // [32 stacks][3][2 nhp][2 nhp] folded pupils of an adjoint group
  float* d_partial = nullptr;   // [stacks * 3][np][np] per-(stack, component) dL/dPhi
  int partial_groups = 0;
  double* d_dphi = nullptr;     // [N][N]
  float2* d_adjD = nullptr;     // [nz][np][np] exp(i k s_z z) of the plan's planes
  double* d_runs = nullptr;     // [partial runs][N][N] first level of the dL/dPhi reduction
  int P_stacks = 0;             // capacity of d_P in stacks

  // chirp-z evaluation of the Fourier form
  int czt_Ly = 0, czt_Lx = 0, czt_cb = 0;   // FFT lengths, output columns per workgroup
  float2* d_czt = nullptr;       // tables: pre/post/chat along y, then along x
  float2 *czt_pre_y = nullptr, *czt_post_y = nullptr, *czt_chat_y = nullptr;
  float2 *czt_pre_x = nullptr, *czt_post_x = nullptr, *czt_chat_x = nullptr;
  float2* d_czt_T = nullptr;     // workspace [planes][3][N][ny]
  size_t czt_planes = 0;

  // Bessel form
  int n_theta_total = 0;        // nodes after the critical-angle split
  double* d_theta = nullptr;    // [T] nodes
  double* d_wtheta = nullptr;   // [T] weights
  double* d_node = nullptr;     // [T][4] Bessel form: sin, cos, stack-independent amplitude, k cos of each node
  int bessel_mode = 0;          // 0 vectorial, 1 vectorial with Fresnel factors, 2 scalar
  float* d_btab = nullptr;      // [T][G][R] w_t h_g(t) J_{n_g}(k rho_r sin t)
  double* d_fq = nullptr;       // [T][4] Fresnel products q_s, q_p per node (Fresnel mode)
  float2* d_phi = nullptr;      // workspace [T][stacks][nz][V] pupil x defocus (x q_v)
  float2* d_In = nullptr;       // workspace [stacks][nz][V][re/im][G][R]
  int bessel_stacks = 0;        // capacity of the Bessel workspaces
  std::vector<double> fused_cum;   // Bessel, few stacks: accumulated cost per radial base sample
  float* scratch = nullptr;     // device address of the allocation-free entry point's fixed array
  double drho = 0;              // radial sample pitch
  // Bessel-form adjoint (built on first use)
  float* d_btabT = nullptr;     // [G][R][T] transposed table
  float* d_GInT = nullptr;      // workspace [G][R][2 stacks nz V] gradients of the radial samples
  float* d_GPhi = nullptr;      // workspace [2 stacks nz V][T] gradient of Phi
  double2* d_adjX = nullptr;    // workspace [stacks][T] sum_z conj(G_Phi) Phi
  double* d_adjnode = nullptr;  // [T][7] k cos t, dW/dt_s (re, im), 2 pi Z_{1,4,11,22}
  double* d_dcp = nullptr;      // [max stacks][4] per-stack shares of dL/dc

  // per-kernel timing (opt-in)
  struct TimingRec {
    int kernel;
    hipEvent_t a, b;
  };
  bool timing = false;
  std::vector<TimingRec> timing_recs;
  std::vector<hipEvent_t> event_pool;
  double timing_ms[RWPSF_KERNEL_COUNT] = {};
  int64_t timing_launches[RWPSF_KERNEL_COUNT] = {};
  int time_begin(int kernel, hipStream_t st);   // returns a record index or -1
  void time_end(int rec, hipStream_t st);
  void timing_flush();

  ~rwpsf_plan();
};
