// Plan construction (FP64 tables on the host, uploaded once) and the Fourier-form
// dispatch.  Tables of the Fourier form (Sec. 3.3 eq. "cartesian vectorial",
// Sec. 3.4 correction factors) on the cell-centred pupil grid
//   s_x[j] = (2j + 1 - N) s_max / N,  s_y[l] likewise,  cell area ds^2 = (2 s_max / N)^2,
// disk mask (2j+1-N)^2 + (2l+1-N)^2 <= N^2 decided in integers:
//   Q_c[j,l]  = ds^2 a(s) e_inf,c(s) / s_z          (complex64, 0 outside the disk;
//               one channel ds^2 a(s) / s_z for the scalar model, Sec. 3.2)
//   ksz[j,l]  = k s_z                                (FP64, for the defocus phase)
// and of the folded transforms (jf, lf < nh = ceil(N/2), the mirror-symmetric half):
//   kszf[jf,lf]   = k s_z                            (FP64)
//   B1[n][2lf]    = cos(k s_y[lf] y_n),  B1[n][2lf+1] = sin(k s_y[lf] y_n)
//   A2[m][2jf]    = pref cos(k s_x[jf] x_m),  A2[m][2jf+1] = pref sin(...),  pref = f k / 2 pi
// (both with the contraction index contiguous)
// with x_m = (m - nx/2) dx, y_n = (n - ny/2) dy.
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "rw_common.h"
#include "rw_fourier.h"
#include "rw_plan.h"

namespace rw {

int bessel_plan_init(rwpsf_plan* p);

static int fourier_plan_init(rwpsf_plan* p) {
  const int N = p->num.n_pupil, nx = p->grid.nx, ny = p->grid.ny;
  const int np = round_up(N, kPadPupil), nxp = pad_axis(nx), nyp = pad_axis(ny);
  p->np = np;
  p->nxp = nxp;
  p->nyp = nyp;
  const double s_max = p->s_max, k = p->k;
  const size_t npp = (size_t)np * np;
  std::vector<float2> Q(3 * npp, make_float2(0.f, 0.f));
  std::vector<double> ksz(npp, 0.0);
  const double ds = 2.0 * s_max / N;
  for (int j = 0; j < N; ++j)
    for (int l = 0; l < N; ++l) {
      const long u = 2L * j + 1 - N, v = 2L * l + 1 - N;
      if (u * u + v * v > (long)N * N) continue;
      const size_t cell = (size_t)j * np + l;
      const double sx = u * s_max / N, sy = v * s_max / N;
      std::complex<double> e[3];
      base_pupil_cell(p->opt, p->nc, ds, sx, sy, e);
      for (int c = 0; c < p->nc; ++c) Q[c * npp + cell] = make_float2((float)e[c].real(), (float)e[c].imag());
      ksz[cell] = k * std::sqrt(1.0 - (sx * sx + sy * sy));
    }
  const int nh = (N + 1) / 2, nhp = round_up(nh, kFoldPad), w = 2 * nhp;
  p->nhp = nhp;
  std::vector<double> kszf((size_t)nhp * nhp, 0.0);
  for (int jf = 0; jf < nh; ++jf)
    for (int lf = 0; lf < nh; ++lf) kszf[(size_t)jf * nhp + lf] = ksz[(size_t)jf * np + lf];
  std::vector<float> B1((size_t)w * nyp, 0.f), A2T((size_t)w * nxp, 0.f);
  const double pref = p->opt.focal_length * k / kTwoPi;  // C = -i pref
  for (int lf = 0; lf < nh; ++lf) {
    const double sy = (2.0 * lf + 1.0 - N) * s_max / N;
    for (int n = 0; n < ny; ++n) {
      const double ph = k * sy * (double)(n - ny / 2) * p->grid.dy_nm;
      B1[(size_t)n * w + 2 * lf] = (float)std::cos(ph);
      B1[(size_t)n * w + 2 * lf + 1] = (float)std::sin(ph);
    }
  }
  for (int jf = 0; jf < nh; ++jf) {
    const double sx = (2.0 * jf + 1.0 - N) * s_max / N;
    for (int m = 0; m < nx; ++m) {
      const double ph = k * sx * (double)(m - nx / 2) * p->grid.dx_nm;
      A2T[(size_t)m * w + 2 * jf] = (float)(pref * std::cos(ph));
      A2T[(size_t)m * w + 2 * jf + 1] = (float)(pref * std::sin(ph));
    }
  }
  int st;
  if ((st = dev_alloc(p, &p->d_Q, 3 * npp))) return st;
  if ((st = dev_alloc(p, &p->d_ksz, npp))) return st;
  if ((st = dev_alloc(p, &p->d_kszf, kszf.size()))) return st;
  if ((st = dev_alloc(p, &p->d_B1, B1.size()))) return st;
  if ((st = dev_alloc(p, &p->d_A2T, A2T.size()))) return st;
  if ((st = dev_alloc(p, &p->d_ztab, (size_t)RWPSF_MAX_ZERNIKE * N * N))) return st;
  if ((st = dev_alloc(p, &p->d_z, (size_t)p->grid.nz))) return st;
  p->P_stacks = kPupilStacks;
  if ((st = dev_alloc(p, &p->d_P, (size_t)p->P_stacks * 3 * npp))) return st;
  const bool gemm = p->num.form == RWPSF_FORM_FOURIER;   // the chirp-z form needs no GEMM workspaces
  if (gemm && (st = dev_alloc(p, &p->d_Pf, (size_t)kGemmStacks * 3 * w * w))) return st;
  // plane workspace: whole group of stacks x planes, capped at 1 GiB
  const size_t plane_bytes = 3 * (size_t)w * nyp * sizeof(float2);
  const size_t want = (size_t)kGemmStacks * p->grid.nz;
  p->T_planes = std::max<size_t>(1, std::min(want, ((size_t)1 << 30) / plane_bytes));
  if (gemm && (st = dev_alloc(p, &p->d_T, p->T_planes * 3 * (size_t)w * nyp))) return st;

  if ((st = hip_check(hipMemcpy(p->d_Q, Q.data(), Q.size() * sizeof(float2), hipMemcpyHostToDevice)))) return st;
  if ((st = hip_check(hipMemcpy(p->d_ksz, ksz.data(), ksz.size() * sizeof(double), hipMemcpyHostToDevice)))) return st;
  if ((st = hip_check(hipMemcpy(p->d_kszf, kszf.data(), kszf.size() * sizeof(double), hipMemcpyHostToDevice)))) return st;
  if ((st = hip_check(hipMemcpy(p->d_B1, B1.data(), B1.size() * sizeof(float), hipMemcpyHostToDevice)))) return st;
  if ((st = hip_check(hipMemcpy(p->d_A2T, A2T.data(), A2T.size() * sizeof(float), hipMemcpyHostToDevice)))) return st;
  if ((st = hip_check(hipMemcpy(p->d_z, p->z.data(), p->z.size() * sizeof(double), hipMemcpyHostToDevice)))) return st;
  if ((st = hip_check(launch_zernike_table(p->d_ztab, N, RWPSF_MAX_ZERNIKE, 0)))) return st;
  if ((st = hip_check(fourier_kernel_attributes()))) return st;
  return hip_check(hipDeviceSynchronize());
}

int plan_init(rwpsf_plan* p, const rwpsf_optics& o, const rwpsf_grid& g, const rwpsf_numerics& nm) {
  int dev_count = 0;
  if (hipGetDeviceCount(&dev_count) != hipSuccess || dev_count < 1) return RWPSF_ERR_NO_DEVICE;
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) return hip_check(e);
  p->opt = o;
  p->grid = g;
  p->num = nm;
  p->z.assign(g.z_nm, g.z_nm + g.nz);
  p->grid.z_nm = nullptr;
  p->nc = nm.model == RWPSF_MODEL_SCALAR ? 1 : 3;
  p->k = kTwoPi * o.n_i / o.wavelength_nm;
  p->s_max = o.na / o.n_i;
  p->theta_max = std::asin(p->s_max);
  p->gl.k0 = kTwoPi / o.wavelength_nm;
  p->gl.n_i = o.n_i;
  p->gl.n_s = o.n_s;
  p->gl.n_g = o.n_g;
  p->gl.n_g_d = o.n_g_design;
  p->gl.n_i_d = o.n_i_design;
  p->gl.t_g = o.t_g_nm;
  p->gl.t_g_d = o.t_g_design_nm;
  p->gl.t_i_d = o.t_i_design_nm;
  if (nm.form == RWPSF_FORM_FOURIER) return fourier_plan_init(p);
  if (nm.form == RWPSF_FORM_CHIRPZ) {
    const int st = fourier_plan_init(p);
    return st ? st : czt_plan_init(p);
  }
  return bessel_plan_init(p);
}

// Pupil arguments of nb <= NS stacks.
template <int NS>
static void fill_pupil_args(const rwpsf_plan* p, const rwpsf_stack* s, int nb, PupilArgsT<NS>& pa) {
  pa.n = p->num.n_pupil;
  pa.np = p->np;
  pa.nstk = nb;
  pa.gibson_lanni = p->opt.gibson_lanni;
  pa.nc = p->nc;
  pa.s_max = p->s_max;
  pa.k = p->k;
  pa.gl = p->gl;
  int maxz = 0;
  for (int i = 0; i < nb; ++i) {
    const rwpsf_stack& x = s[i];
    PupilStack& d = pa.s[i];
    d.t_s = x.t_s_nm;
    d.x0 = x.x0_nm;
    d.y0 = x.y0_nm;
    for (int q = 0; q < RWPSF_MAX_ZERNIKE; ++q) d.coef[q] = q < x.n_zernike ? x.zernike_waves[q] : 0.0;
    d.w0 = x.phase_map;
    maxz = std::max(maxz, x.n_zernike);
  }
  pa.max_zernike = maxz;
}

// Base pupils P_{b,c} of up to 8 stacks into the plan's pupil workspace.
int fourier_build_pupils(rwpsf_plan* p, const rwpsf_stack* s, int nb, hipStream_t st) {
  PupilArgs pa{};
  fill_pupil_args(p, s, nb, pa);
  const int tr = p->time_begin(RWPSF_KERNEL_PUPIL_BUILD, st);
  const int rc = hip_check(launch_pupil_build(pa, p->d_Q, p->d_ztab, p->d_P, st));
  p->time_end(tr, st);
  return rc;
}

// Mirror-folded pupils of up to 8 stacks into Pf ([nb][nc][2 nhp][2 nhp]).
int fourier_build_folded(rwpsf_plan* p, const rwpsf_stack* s, int nb, float2* Pf, hipStream_t st) {
  PupilArgs pa{};
  fill_pupil_args(p, s, nb, pa);
  const int tr = p->time_begin(RWPSF_KERNEL_PUPIL_BUILD, st);
  const int rc = hip_check(launch_pupil_build_folded(pa, p->d_Q, p->d_ztab, Pf, p->nhp, st));
  p->time_end(tr, st);
  return rc;
}

// --------------------------------------------------------------------------
// Fourier dispatch: chunks of up to 64 stacks (folded pupils in launches of 8), then
// slabs of stack-planes through the two GEMM kernels.
// --------------------------------------------------------------------------
static int fourier_gemms(rwpsf_plan* p, int s_local, int ns, const double* zoff, int s_global, int z0, int nzs,
                         float2* E, float* I, hipStream_t st) {
  const int w = 2 * p->nhp;
  Gemm1Args g1{};
  g1.Pf = p->d_Pf + (size_t)s_local * p->nc * w * w;
  g1.kszf = p->d_kszf;
  g1.z = p->d_z;
  g1.B1 = p->d_B1;
  g1.T = p->d_T;
  for (int i = 0; i < ns; ++i) g1.zoff[i] = zoff[i];
  g1.n = p->num.n_pupil;
  g1.nhp = p->nhp;
  g1.nyp = p->nyp;
  g1.nstk = ns;
  g1.z0 = z0;
  g1.nzs = nzs;
  g1.nc = p->nc;
  int tr = p->time_begin(RWPSF_KERNEL_GEMM_PUPIL, st);
  int rc = hip_check(launch_gemm_pupil(g1, st));
  if (rc) return rc;
  p->time_end(tr, st);
  Gemm2Args g2{};
  g2.A2 = p->d_A2T;
  g2.T = p->d_T;
  g2.E = E;
  g2.I = I;
  g2.nhp = p->nhp;
  g2.nxp = p->nxp;
  g2.nyp = p->nyp;
  g2.nx = p->grid.nx;
  g2.ny = p->grid.ny;
  g2.nz = p->grid.nz;
  g2.nstk = ns;
  g2.s_base = s_global;
  g2.z0 = z0;
  g2.nzs = nzs;
  g2.nc = p->nc;
  tr = p->time_begin(RWPSF_KERNEL_GEMM_IMAGE, st);
  if ((rc = hip_check(launch_gemm_image(g2, st)))) return rc;
  p->time_end(tr, st);
  return RWPSF_OK;
}

int fourier_compute(rwpsf_plan* p, int n, const rwpsf_stack* s, float2* E, float* I, hipStream_t st) {
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != p->device) return RWPSF_ERR_INVALID_ARG;
  const int nz = p->grid.nz;
  for (int b0 = 0; b0 < n; b0 += kGemmStacks) {
    const int nb = std::min(kGemmStacks, n - b0);
    int rc;
    // folded pupils of the group in launches of up to kPupilStacks, side by side
    for (int c0 = 0; c0 < nb; c0 += kPupilStacks)
      if ((rc = fourier_build_folded(p, s + b0 + c0, std::min(kPupilStacks, nb - c0),
                                     p->d_Pf + (size_t)c0 * p->nc * 4 * p->nhp * p->nhp, st)))
        return rc;
    double zoff[kGemmStacks];
    for (int i = 0; i < nb; ++i) zoff[i] = s[b0 + i].z_offset_nm;
    // slabs over (stack, plane): a slab is a run of planes of one or more stacks
    const size_t cap = p->T_planes;
    if ((size_t)nz <= cap) {
      const int stk_per = (int)std::min<size_t>(nb, cap / nz);
      for (int s0 = 0; s0 < nb; s0 += stk_per) {
        const int ns = std::min(stk_per, nb - s0);
        if ((rc = fourier_gemms(p, s0, ns, zoff + s0, b0 + s0, 0, nz, E, I, st))) return rc;
      }
    } else {
      for (int i = 0; i < nb; ++i)
        for (int z0 = 0; z0 < nz; z0 += (int)cap) {
          const int nzs = (int)std::min<size_t>(cap, nz - z0);
          if ((rc = fourier_gemms(p, i, 1, zoff + i, b0 + i, z0, nzs, E, I, st))) return rc;
        }
    }
  }
  return RWPSF_OK;
}

}  // namespace rw
