// Fourier (Cartesian) form of the vectorial Richards-Wolf integral on gfx950.
//
// Sec. 3.3 eq. "cartesian vectorial" with the correction factors of Sec. 3.4:
// each z-plane of each field component is the 2-D transform of the pupil
//   P~_c[j,l] = P_c[j,l] exp(i k s_z[j,l] z),  P_c = ds^2 a exp(iW) e_inf,c / s_z
// to the pixel grid.  It is evaluated as the separable matrix DFT
//   E_c = Ax P~_c Ay^T,  Ax[m,j] = C exp(i k s_x[j] x_m),  Ay[n,l] = exp(i k s_y[l] y_n)
// (C = -i f k / 2 pi), i.e. two complex GEMMs per component-plane on the FP32
// matrix cores:
//   K1 pupil_build   P_c for up to 8 stacks (FP64 phase: Gibson-Lanni, Zernike,
//                    free phase map, lateral emitter shift), complex64 [s][c][j][l]
//   K2 gemm_pupil    T = P~ Ay^T; the defocus factor is formed while the pupil
//                    tile is staged (FP64 phase, reduced mod 2 pi, FP32 sincos)
//   K3 gemm_image    E_c = Ax T_c for c = x, y, z in one workgroup, writing E and
//                    I = sum_c |E_c|^2 from registers.
#include "cgemm.h"
#include "rw_common.h"
#include "rw_fourier.h"

namespace rw {

// --------------------------------------------------------------------------
// Plan-time table: orthonormal Noll Zernike basis on the cell-centred pupil grid.
// --------------------------------------------------------------------------
__global__ void zernike_table_kernel(float* __restrict__ out, int n, int nj, double s_max_unused) {
  const int cell = blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= n * n) return;
  const int j = cell / n, l = cell % n;
  const double u = (2.0 * j + 1.0 - n) / n, v = (2.0 * l + 1.0 - n) / n;  // unit-disk coords
  const double r = sqrt(u * u + v * v);
  const double cp = r > 0 ? u / r : 1.0, sp = r > 0 ? v / r : 0.0;
  for (int q = 1; q <= nj; ++q)
    out[(size_t)(q - 1) * n * n + cell] = (float)zernike_noll(q, r, cp, sp);
}

// --------------------------------------------------------------------------
// K1: base pupil of each stack.
// --------------------------------------------------------------------------
__global__ void __launch_bounds__(256) pupil_build_kernel(PupilArgs a, const float2* __restrict__ Q,
                                                          const float* __restrict__ ztab,
                                                          float2* __restrict__ P) {
  const int n = a.n, np = a.np;
  const size_t npp = (size_t)np * np;
  const int pcell = blockIdx.x * blockDim.x + threadIdx.x;   // padded cell
  if (pcell >= np * np) return;
  const int j = pcell / np, l = pcell % np;
  float2 q0 = make_float2(0.f, 0.f), q1 = q0, q2 = q0;
  if (j < n && l < n) {
    q0 = Q[pcell];
    q1 = Q[npp + pcell];
    q2 = Q[2 * npp + pcell];
  }
  const bool inside = (q0.x != 0.f || q0.y != 0.f || q1.x != 0.f || q1.y != 0.f || q2.x != 0.f ||
                       q2.y != 0.f);
  if (!inside) {
    for (int s = 0; s < a.nstk; ++s)
      for (int c = 0; c < 3; ++c) P[((size_t)s * 3 + c) * npp + pcell] = make_float2(0.f, 0.f);
    return;
  }
  const int cell = j * n + l;   // unpadded index: Zernike table and user phase map
  const double sx = (2.0 * j + 1.0 - n) * a.s_max / n;
  const double sy = (2.0 * l + 1.0 - n) * a.s_max / n;
  const double sin_t = sqrt(sx * sx + sy * sy);

  double w_re[kPupilStacks], w_im[kPupilStacks];
  for (int s = 0; s < kPupilStacks; ++s) {
    w_re[s] = 0.0;
    w_im[s] = 0.0;
  }
  for (int s = 0; s < a.nstk; ++s) {
    const PupilStack& st = a.s[s];
    if (a.gibson_lanni) {
      double gr, gi;
      gl_opd(a.gl, st.t_s, sin_t, &gr, &gi);
      w_re[s] += gr;
      w_im[s] += gi;
    }
    w_re[s] -= a.k * (sx * st.x0 + sy * st.y0);
    if (st.w0) w_re[s] += (double)st.w0[cell];
  }
  for (int q = 0; q < a.max_zernike; ++q) {
    const double zq = (double)ztab[(size_t)q * n * n + cell];
    for (int s = 0; s < a.nstk; ++s) w_re[s] += kTwoPi * a.s[s].coef[q] * zq;
  }
  for (int s = 0; s < a.nstk; ++s) {
    const float ph = (float)reduce_2pi(w_re[s]);
    const float amp = (float)exp(-w_im[s]);
    float sn, cs;
    sincosf(ph, &sn, &cs);
    const float er = amp * cs, ei = amp * sn;
    float2* out = P + (size_t)s * 3 * npp + pcell;
    out[0] = make_float2(q0.x * er - q0.y * ei, q0.x * ei + q0.y * er);
    out[npp] = make_float2(q1.x * er - q1.y * ei, q1.x * ei + q1.y * er);
    out[2 * npp] = make_float2(q2.x * er - q2.y * ei, q2.x * ei + q2.y * er);
  }
}

// --------------------------------------------------------------------------
// A operand of K2: pupil rows j, contraction index l, with the defocus factor
// exp(i k s_z z) applied on the way into LDS.  The phase k s_z z is formed and
// reduced in FP64; only the reduced angle goes through FP32 sincos.
// --------------------------------------------------------------------------
template <class Cfg>
struct DefocusLoader {
  static constexpr int PAIRS = Cfg::BK / 2;
  static constexpr int PER_THREAD = Cfg::BM * PAIRS / Cfg::NT;
  static_assert(Cfg::BM * PAIRS % Cfg::NT == 0, "loader shape");
  const float2* P;    // [np][np] of this stack and component, rows from row0
  const double* ksz;  // [np][np], rows from row0
  double z;
  int ld;
  float4 v[PER_THREAD];
  double2 kz[PER_THREAD];

  __device__ void load(int k0, int tid) {
#pragma unroll
    for (int i = 0; i < PER_THREAD; ++i) {
      const int idx = tid + i * Cfg::NT;
      const int row = idx / PAIRS, kk = 2 * (idx % PAIRS);
      const size_t off = (size_t)row * ld + k0 + kk;
      v[i] = *reinterpret_cast<const float4*>(P + off);
      kz[i] = *reinterpret_cast<const double2*>(ksz + off);
    }
  }
  __device__ void store(float* re, float* im, int ldl, int tid) const {
#pragma unroll
    for (int i = 0; i < PER_THREAD; ++i) {
      const int idx = tid + i * Cfg::NT;
      const int row = idx / PAIRS, kk = 2 * (idx % PAIRS);
      float s0, c0, s1, c1;
      sincosf((float)reduce_2pi(kz[i].x * z), &s0, &c0);
      sincosf((float)reduce_2pi(kz[i].y * z), &s1, &c1);
      re[kk * ldl + row] = v[i].x * c0 - v[i].y * s0;
      im[kk * ldl + row] = v[i].x * s0 + v[i].y * c0;
      re[(kk + 1) * ldl + row] = v[i].z * c1 - v[i].w * s1;
      im[(kk + 1) * ldl + row] = v[i].z * s1 + v[i].w * c1;
    }
  }
};

#ifndef RW_PUPIL_BK
#define RW_PUPIL_BK 16
#endif
#ifndef RW_IMAGE_BK
#define RW_IMAGE_BK 8
#endif
#ifndef RW_PUPIL_OCC
#define RW_PUPIL_OCC 2
#endif
#ifndef RW_IMAGE_OCC
#define RW_IMAGE_OCC 2
#endif
static_assert(kPadPupil % 64 == 0 && kPadY % 128 == 0 && kPadX % 64 == 0, "tile padding");
using CfgPupil = CgCfg<64, 128, RW_PUPIL_BK, 64, 32>;
using CfgImage = CgCfg<64, 128, RW_IMAGE_BK, 64, 32>;

// K2: T[s][z][c] = P~[s][c](z) * Ay^T   ([n x n] * [n x ny])
__global__ void __launch_bounds__(CfgPupil::NT, RW_PUPIL_OCC) gemm_pupil_kernel(Gemm1Args a) {
  using Cfg = CfgPupil;
  extern __shared__ float lds[];
  const int tiles_m = a.np / Cfg::BM;
  const int tiles_n = a.nyp / Cfg::BN;
  const int nblocks = a.nstk * a.nzs * 3 * tiles_m * tiles_n;
  int id = xcd_remap(blockIdx.x, nblocks);
  const int tn = id % tiles_n; id /= tiles_n;
  const int tm = id % tiles_m; id /= tiles_m;
  const int zi = id % a.nzs; id /= a.nzs;
  const int c = id % 3; id /= 3;
  const int s = id;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wrow = (wave / Cfg::WAVES_N) * Cfg::WM, wcol = (wave % Cfg::WAVES_N) * Cfg::WN;
  const size_t npp = (size_t)a.np * a.np;
  const int row0 = tm * Cfg::BM, col0 = tn * Cfg::BN;

  DefocusLoader<Cfg> la;
  la.P = a.P + ((size_t)s * 3 + c) * npp + (size_t)row0 * a.np;
  la.ksz = a.ksz + (size_t)row0 * a.np;
  la.z = a.z[a.z0 + zi] + a.zoff[s];
  la.ld = a.np;
  KMajorLoader<Cfg, Cfg::BN> lb;
  lb.src = a.AyT + col0;
  lb.ld = a.nyp;

  // The pupil is zero outside the disk (2j+1-n)^2 + (2l+1-n)^2 <= n^2: this row block only
  // needs the columns l that its row nearest the centre reaches.
  int k_begin = 0, k_end = a.np;
  {
    const int n = a.n;
    const int r_lo = row0, r_hi = min(row0 + Cfg::BM, n) - 1;
    if (r_lo >= n) {
      k_end = Cfg::BK;   // padding rows only: one (zero) stage
    } else {
      const int u_lo = 2 * r_lo + 1 - n, u_hi = 2 * r_hi + 1 - n;
      const int umin = (u_lo <= 0 && u_hi >= 0) ? 0 : min(abs(u_lo), abs(u_hi));
      const int vmax = (int)floorf(sqrtf((float)n * n - (float)umin * umin)) + 1;   // generous
      const int l_lo = max(0, (n - 1 - vmax) / 2), l_hi = min(n - 1, (n - 1 + vmax) / 2 + 1);
      k_begin = (l_lo / Cfg::BK) * Cfg::BK;
      k_end = min(a.np, (l_hi / Cfg::BK + 1) * Cfg::BK);
    }
  }
  CgAcc<Cfg> acc;
  acc.zero();
  cg_mainloop<Cfg>(acc, la, lb, k_begin, k_end, lds, tid, wrow, wcol, lane);

  float2* T = a.T + (((size_t)s * a.nzs + zi) * 3 + c) * (size_t)a.np * a.nyp;
#pragma unroll
  for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
    for (int jj = 0; jj < Cfg::TN; ++jj) {
      const int col = col0 + cg_col(wcol, jj, lane);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = row0 + cg_row(wrow, i, r, lane);
        T[(size_t)row * a.nyp + col] = make_float2(acc.re[i][jj][r], acc.im[i][jj][r]);
      }
    }
}

// K3: E[s][z][c] = Ax T[s][z][c] for c = 0..2 and I = sum_c |E_c|^2
__global__ void __launch_bounds__(CfgImage::NT, RW_IMAGE_OCC) gemm_image_kernel(Gemm2Args a) {
  using Cfg = CfgImage;
  extern __shared__ float lds[];
  const int tiles_m = a.nxp / Cfg::BM;
  const int tiles_n = a.nyp / Cfg::BN;
  const int nblocks = a.nstk * a.nzs * tiles_m * tiles_n;
  int id = xcd_remap(blockIdx.x, nblocks);
  const int tn = id % tiles_n; id /= tiles_n;
  const int tm = id % tiles_m; id /= tiles_m;
  const int zi = id % a.nzs; id /= a.nzs;
  const int s = id;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wrow = (wave / Cfg::WAVES_N) * Cfg::WM, wcol = (wave % Cfg::WAVES_N) * Cfg::WN;
  const size_t plane = (size_t)a.nx * a.ny;
  const size_t gstk = (size_t)(a.s_base + s), gz = (size_t)(a.z0 + zi);
  const int row0 = tm * Cfg::BM, col0 = tn * Cfg::BN;

  float isum[Cfg::TM][Cfg::TN][16];
#pragma unroll
  for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
    for (int jj = 0; jj < Cfg::TN; ++jj)
#pragma unroll
      for (int r = 0; r < 16; ++r) isum[i][jj][r] = 0.f;

#pragma unroll 1
  for (int c = 0; c < 3; ++c) {
    KMajorLoader<Cfg, Cfg::BM> la;
    la.src = a.AxT + row0;
    la.ld = a.nxp;
    KMajorLoader<Cfg, Cfg::BN> lb;
    lb.src = a.T + (((size_t)s * a.nzs + zi) * 3 + c) * (size_t)a.np * a.nyp + col0;
    lb.ld = a.nyp;
    CgAcc<Cfg> acc;
    acc.zero();
    cg_mainloop<Cfg>(acc, la, lb, a.np, lds, tid, wrow, wcol, lane);

    float2* E = a.E ? a.E + ((gstk * a.nz + gz) * 3 + c) * plane : nullptr;
#pragma unroll
    for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
      for (int jj = 0; jj < Cfg::TN; ++jj) {
        const int col = col0 + cg_col(wcol, jj, lane);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = row0 + cg_row(wrow, i, r, lane);
          const float er = acc.re[i][jj][r], ei = acc.im[i][jj][r];
          isum[i][jj][r] += er * er + ei * ei;
          if (E && row < a.nx && col < a.ny) E[(size_t)row * a.ny + col] = make_float2(er, ei);
        }
      }
  }
  if (a.I) {
    float* I = a.I + (gstk * a.nz + gz) * plane;
#pragma unroll
    for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
      for (int jj = 0; jj < Cfg::TN; ++jj) {
        const int col = col0 + cg_col(wcol, jj, lane);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = row0 + cg_row(wrow, i, r, lane);
          if (row < a.nx && col < a.ny) I[(size_t)row * a.ny + col] = isum[i][jj][r];
        }
      }
  }
}

// --------------------------------------------------------------------------
// Host-side launchers
// --------------------------------------------------------------------------
hipError_t launch_zernike_table(float* out, int n, int nj, hipStream_t st) {
  const int cells = n * n;
  hipLaunchKernelGGL(zernike_table_kernel, dim3((cells + 255) / 256), dim3(256), 0, st, out, n, nj,
                     0.0);
  return hipGetLastError();
}

hipError_t launch_pupil_build(const PupilArgs& a, const float2* Q, const float* ztab, float2* P,
                              hipStream_t st) {
  const int cells = a.np * a.np;
  hipLaunchKernelGGL(pupil_build_kernel, dim3((cells + 255) / 256), dim3(256), 0, st, a, Q, ztab, P);
  return hipGetLastError();
}

hipError_t launch_gemm_pupil(const Gemm1Args& a, hipStream_t st) {
  using Cfg = CfgPupil;
  const int tiles = (a.np / Cfg::BM) * (a.nyp / Cfg::BN);
  const int nblocks = a.nstk * a.nzs * 3 * tiles;
  hipLaunchKernelGGL(gemm_pupil_kernel, dim3(nblocks), dim3(Cfg::NT), Cfg::LDS_BYTES, st, a);
  return hipGetLastError();
}

hipError_t launch_gemm_image(const Gemm2Args& a, hipStream_t st) {
  using Cfg = CfgImage;
  const int tiles = (a.nxp / Cfg::BM) * (a.nyp / Cfg::BN);
  const int nblocks = a.nstk * a.nzs * tiles;
  hipLaunchKernelGGL(gemm_image_kernel, dim3(nblocks), dim3(Cfg::NT), Cfg::LDS_BYTES, st, a);
  return hipGetLastError();
}

hipError_t fourier_kernel_attributes() {
  hipError_t e = hipFuncSetAttribute((const void*)gemm_pupil_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, CfgPupil::LDS_BYTES);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)gemm_image_kernel,
                             hipFuncAttributeMaxDynamicSharedMemorySize, CfgImage::LDS_BYTES);
}

}  // namespace rw
