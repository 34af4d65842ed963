// Fourier (Cartesian) form of the vectorial Richards-Wolf integral on gfx950.
//
// Sec. 3.3 eq. "cartesian vectorial" with the correction factors of Sec. 3.4:
// each z-plane of each field component is the 2-D transform of the pupil
//   P~_c[j,l] = P_c[j,l] exp(i k s_z z),  P_c = ds^2 a exp(iW) e_inf,c / s_z
// to the pixel grid, E_c = C sum_{j,l} P~_c[j,l] e^{i k (s_x[j] x + s_y[l] y)},
// C = -i f k / 2 pi.  The sample grid is symmetric (s[n-1-j] = -s[j]), so each 1-D
// transform folds into even and odd parts with real coefficients cos / sin, and the
// separable transform becomes two real GEMMs on the FP32 matrix cores with half the
// flops of the complex matrix DFT:
//   K1  pupil_build_folded   mirror-folded pupils Pf (four parities per folded cell)
//                     of up to 8 stacks, each cell's P_c formed on the way (FP64
//                     phase: Gibson-Lanni, Zernike, free phase map, lateral emitter
//                     shift); the chirp-z and adjoint paths take the unfolded P_c of
//                     pupil_build
//   K2  gemm_pupil    T = Pf~ B1 (fold along y); the defocus factor is formed while the
//                     pupil tile is staged (FP64 phase, reduced mod 2 pi, FP32 sincos)
//   K3  gemm_image    E'_c = A2 T_c (fold along x) for c = x, y, z in one workgroup,
//                     writing E = -i E' and I = sum_c |E_c|^2 from registers.
#include "cgemm.h"
#include "rgemm.h"
#include "rw_common.h"
#include "rw_fourier.h"

namespace rw {

// --------------------------------------------------------------------------
// Plan-time table: orthonormal Noll Zernike basis on the cell-centred pupil grid.
// --------------------------------------------------------------------------
__global__ void zernike_table_kernel(float* __restrict__ out, int n, int nj) {
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
// exp(i W) (times the evanescent decay of a Gibson-Lanni layer) at cell (j, l) of stack
// st.  The Zernike loads are unrolled to the maximum term count, so that a thread has
// them all in flight at once instead of waiting for each in turn.
template <class Args>
__device__ __forceinline__ float2 pupil_phase_factor(const Args& a, const PupilStack& st,
                                                     const float* __restrict__ ztab, int j, int l) {
  const int n = a.n;
  const int cell = j * n + l;   // unpadded index: Zernike table and user phase map
  const double sx = (2.0 * j + 1.0 - n) * a.s_max / n;
  const double sy = (2.0 * l + 1.0 - n) * a.s_max / n;
  const double sin_t = sqrt(sx * sx + sy * sy);
  float zv[RWPSF_MAX_ZERNIKE];
#pragma unroll
  for (int k = 0; k < RWPSF_MAX_ZERNIKE; ++k) zv[k] = k < a.max_zernike ? ztab[(size_t)k * n * n + cell] : 0.f;
  double w_re = 0.0, w_im = 0.0;
  if (a.gibson_lanni) gl_opd(a.gl, st.t_s, sin_t, &w_re, &w_im);
  w_re -= a.k * (sx * st.x0 + sy * st.y0);
  if (st.w0) w_re += (double)st.w0[cell];
#pragma unroll
  for (int k = 0; k < RWPSF_MAX_ZERNIKE; ++k) w_re += kTwoPi * st.coef[k] * (double)zv[k];
  // the evanescent decay in FP32 (relative error ~1e-7, far below the tolerance), the
  // phase reduced in FP64 in revolutions before the hardware sine and cosine
  const float amp = w_im > 0.0 ? expf((float)-w_im) : 1.f;
  float sn, cs;
  sincos_rev(w_re * (1.0 / kTwoPi), &sn, &cs);
  return make_float2(amp * cs, amp * sn);
}

// One thread per (padded cell, stack): grid.y is the stack.
__global__ void __launch_bounds__(256) pupil_build_kernel(PupilArgs a, const float2* __restrict__ Q,
                                                          const float* __restrict__ ztab,
                                                          float2* __restrict__ P) {
  const int n = a.n, np = a.np;
  const size_t npp = (size_t)np * np;
  const int pcell = blockIdx.x * blockDim.x + threadIdx.x;   // padded cell
  const int s = blockIdx.y;
  if (pcell >= np * np) return;
  const int j = pcell / np, l = pcell % np;
  const int nc = a.nc;
  float2* out = P + (size_t)s * nc * npp + pcell;
  float2 q[3] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
  bool inside = false;
  if (j < n && l < n)
    for (int c = 0; c < nc; ++c) {
      q[c] = Q[c * npp + pcell];
      inside = inside || q[c].x != 0.f || q[c].y != 0.f;
    }
  if (!inside) {
    for (int c = 0; c < nc; ++c) out[c * npp] = make_float2(0.f, 0.f);
    return;
  }
  const float2 e = pupil_phase_factor(a, a.s[s], ztab, j, l);
  for (int c = 0; c < nc; ++c) out[c * npp] = make_float2(q[c].x * e.x - q[c].y * e.y, q[c].x * e.y + q[c].y * e.x);
}

// --------------------------------------------------------------------------
// K1 of the Fourier form: mirror-folded pupils.
//
// The cell-centred grid is symmetric, s[n-1-j] = -s[j], so with jf < nh = ceil(n/2)
// and its mirror j' = n-1-jf each 1-D transform splits into even and odd parts:
//   sum_j p_j e^{i k s_j x} = sum_jf cos(k s_jf x) (p_jf + p_j') + sin(k s_jf x) i (p_jf - p_j')
// Folding both pupil axes gives, per folded cell (jf, lf) and parities (pj, pl),
//   Pf_{pj,pl} = i^(pj+pl) sum_{a,b in {0,1}} (-1)^(a pj + b pl) P[mir_a(jf), mir_b(lf)]
// (a mirror equal to the cell itself -- the middle row of an odd n -- is counted once
// and has no odd part).  Both transforms then have real coefficients (cos, sin), so
// each is one real GEMM with half the flops of the complex one.  The defocus factor
// depends on s_x^2 + s_y^2 only and is the same for all four mirrors.
// Layout: Pf[s][c][q = 2 jf + pj][kk = 2 lf + pl], complex, (2 nhp) x (2 nhp).
// The four mirror cells' pupils are formed in registers, so P never reaches memory.
// --------------------------------------------------------------------------
// The values of v in the four lanes of this lane's quad (DPP quad_perm(k, k, k, k)).
__device__ __forceinline__ float4 quad_values(float v) {
  const int b = __float_as_int(v);
  return make_float4(__int_as_float(__builtin_amdgcn_update_dpp(0, b, 0x00, 0xF, 0xF, false)),
                     __int_as_float(__builtin_amdgcn_update_dpp(0, b, 0x55, 0xF, 0xF, false)),
                     __int_as_float(__builtin_amdgcn_update_dpp(0, b, 0xAA, 0xF, 0xF, false)),
                     __int_as_float(__builtin_amdgcn_update_dpp(0, b, 0xFF, 0xF, 0xF, false)));
}

// Four lanes per (folded cell, stack), grid.y the stack: lane m of a quad forms the pupil
// of mirror m = 2 a + b, i.e. of cell (mir_a(jf), mir_b(lf)), broadcasts it to the quad
// (DPP quad permutes) and writes parity (pj, pl) = (m / 2, m % 2) of every channel.
__global__ void __launch_bounds__(256) pupil_build_folded_kernel(PupilArgs a, const float2* __restrict__ Q,
                                                                 const float* __restrict__ ztab,
                                                                 float2* __restrict__ Pf, int nhp) {
  const int n = a.n, np = a.np, nh = (a.n + 1) / 2;
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int cell = gid >> 2, m = gid & 3;
  const int s = blockIdx.y;
  if (cell >= nhp * nhp) return;   // whole quads
  const int jf = cell / nhp, lf = cell % nhp;
  const int pj = m >> 1, pl = m & 1;
  const size_t npp = (size_t)np * np, fpp = (size_t)4 * nhp * nhp;
  const int w = 2 * nhp, nc = a.nc;
  float2* out = Pf + (size_t)s * nc * fpp + (size_t)(2 * jf + pj) * w + 2 * lf + pl;
  const float2 zero = make_float2(0.f, 0.f);
  if (jf >= nh || lf >= nh) {   // whole quads
#pragma unroll
    for (int c = 0; c < 3; ++c)
      if (c < nc) out[c * fpp] = make_float2(0.f, 0.f);
    return;
  }
  const int j1 = n - 1 - jf, l1 = n - 1 - lf;
  const bool dj = j1 != jf, dl = l1 != lf;
  // this lane's mirror; a mirror equal to the cell itself is absent (zero)
  const int j = pj ? j1 : jf, l = pl ? l1 : lf;
  const bool present = (pj ? dj : true) && (pl ? dl : true);
  float2 q[3];
  bool inside = false;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    q[c] = present && c < nc ? Q[c * npp + (size_t)j * np + l] : zero;
    inside = inside || q[c].x != 0.f || q[c].y != 0.f;
  }
  if (inside) {
    const float2 e = pupil_phase_factor(a, a.s[s], ztab, j, l);
#pragma unroll
    for (int c = 0; c < 3; ++c) q[c] = make_float2(q[c].x * e.x - q[c].y * e.y, q[c].x * e.y + q[c].y * e.x);
  }
  // the mirror's sign in this lane's parity: (-1)^(a pj + b pl) for mirror (a, b)
  const float s01 = pl ? -1.f : 1.f, s10 = pj ? -1.f : 1.f;
  const bool odd_ok = (!pj || dj) && (!pl || dl);   // odd parts of a self-mirrored row vanish
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (c >= nc) break;
    const float4 vr = quad_values(q[c].x), vi = quad_values(q[c].y);
    // mirrors (0,0) + s01 (0,1) + s10 [(1,0) + s01 (1,1)]
    float re = (vr.x + s01 * vr.y) + s10 * (vr.z + s01 * vr.w);
    float im = (vi.x + s01 * vi.y) + s10 * (vi.z + s01 * vi.w);
    if (!odd_ok) re = im = 0.f;
    // times i^(pj + pl)
    float2 v;
    if (pj + pl == 0) v = make_float2(re, im);
    else if (pj + pl == 1) v = make_float2(-im, re);
    else v = make_float2(-re, -im);
    out[c * fpp] = v;
  }
}

// --------------------------------------------------------------------------
// A operand of K2: rows 2q + ri (q = 2 jf + pj, ri = re/im) and contraction index
// kk = 2 lf + pl of the folded pupil, with the defocus factor exp(i k s_z z) applied
// on the way into LDS.  One thread takes one folded cell (jf, lf): its four values
// share one defocus factor, whose phase is formed and reduced in FP64 (in revolutions)
// before the FP32 hardware sine and cosine.
// --------------------------------------------------------------------------
template <class Cfg>
struct FoldDefocusLoader {
  static constexpr int JF = Cfg::BM / 4, LF = Cfg::BK / 2;
  static constexpr int PER_THREAD = JF * LF / Cfg::NT;
  static_assert(JF * LF % Cfg::NT == 0, "loader shape");
  const float2* Pf;    // [2 nhp][2 nhp] of this stack and component, from folded row jf0
  const double* kszf;  // [nhp][nhp], from row jf0
  double zrev;         // z / 2 pi, so that k s_z zrev is the phase in revolutions
  int w, nhp;          // w = 2 nhp
  struct Regs {
    float4 v0[PER_THREAD], v1[PER_THREAD];
    double kz[PER_THREAD];
  };

  __device__ Regs load(int k0, int tid) const {
    Regs r;
#pragma unroll
    for (int i = 0; i < PER_THREAD; ++i) {
      const int idx = tid + i * Cfg::NT;
      const int jl = idx / LF, ll = idx % LF;
      const size_t off = (size_t)(2 * jl) * w + k0 + 2 * ll;
      r.v0[i] = *reinterpret_cast<const float4*>(Pf + off);       // pj = 0, pl = 0, 1
      r.v1[i] = *reinterpret_cast<const float4*>(Pf + off + w);   // pj = 1
      r.kz[i] = kszf[(size_t)jl * nhp + k0 / 2 + ll];
    }
    return r;
  }
  // LDS tile [row][k]: rows 4 jl + 2 pj + ri, columns 2 ll + pl
  __device__ void store(float* dst, int tid, const Regs& r) const {
    const float4* v0 = r.v0;
    const float4* v1 = r.v1;
    const double* kz = r.kz;
#pragma unroll
    for (int i = 0; i < PER_THREAD; ++i) {
      const int idx = tid + i * Cfg::NT;
      const int jl = idx / LF, ll = idx % LF;
      float sn, cs;
      sincos_rev(kz[i] * zrev, &sn, &cs);
      float* d = dst + (4 * jl) * Cfg::LDK + 2 * ll;
      *reinterpret_cast<float2*>(d) = make_float2(v0[i].x * cs - v0[i].y * sn, v0[i].z * cs - v0[i].w * sn);
      *reinterpret_cast<float2*>(d + Cfg::LDK) =
          make_float2(v0[i].x * sn + v0[i].y * cs, v0[i].z * sn + v0[i].w * cs);
      *reinterpret_cast<float2*>(d + 2 * Cfg::LDK) =
          make_float2(v1[i].x * cs - v1[i].y * sn, v1[i].z * cs - v1[i].w * sn);
      *reinterpret_cast<float2*>(d + 3 * Cfg::LDK) =
          make_float2(v1[i].x * sn + v1[i].y * cs, v1[i].z * sn + v1[i].w * cs);
    }
  }
};

#ifndef RW_F1_BM
#define RW_F1_BM 128
#endif
#ifndef RW_F1_BN
#define RW_F1_BN 128
#endif
#ifndef RW_F1_BK
#define RW_F1_BK 16
#endif
#ifndef RW_F1_WM
#define RW_F1_WM 64
#endif
#ifndef RW_F1_WN
#define RW_F1_WN 64
#endif
#ifndef RW_F1_OCC
#define RW_F1_OCC 4
#endif
#ifndef RW_F2_BM
#define RW_F2_BM 128
#endif
#ifndef RW_F2_BN
#define RW_F2_BN 256
#endif
#ifndef RW_F2_BK
#define RW_F2_BK 16
#endif
#ifndef RW_F2_WM
#define RW_F2_WM 64
#endif
#ifndef RW_F2_WN
#define RW_F2_WN 64
#endif
#ifndef RW_F2_OCC
#define RW_F2_OCC 2
#endif
using CfgPupil = RgCfg<RW_F1_BM, RW_F1_BN, RW_F1_BK, RW_F1_WM, RW_F1_WN>;
// image GEMM: 128 x 256 tiles (a whole padded row of re/im columns at 128-pixel width) on
// eight 64 x 64 waves; launches whose padded width 2 nyp is not a multiple of 256, or
// that would underfill the GPU, take CfgImageS
using CfgImage = RgCfg<RW_F2_BM, RW_F2_BN, RW_F2_BK, RW_F2_WM, RW_F2_WN>;
// pupils whose folded row count 4 nhp is a multiple of 256 take 256-row tiles (8 waves;
// the y-table tile is then shared by twice the rows)
using CfgPupilL = RgCfg<256, 128, 16, 64, 64>;
// outputs of at most 64 pixels per axis are padded to 64 and use half-height tiles
// (256 rows when the folded row count allows, as above)
using CfgPupilS = RgCfg<128, 64, 16, 64, 32>;
using CfgPupilSL = RgCfg<256, 64, 16, 64, 64>;
using CfgImageS = RgCfg<64, 64, 32, 32, 32>;
static_assert((4 * kFoldPad) % CfgPupil::BM == 0 && (2 * kFoldPad) % CfgPupil::BK == 0, "pupil GEMM padding");
static_assert((4 * kFoldPad) % CfgPupilS::BM == 0 && kPadSmall % CfgPupilS::BN == 0 && kPadSmall % CfgImageS::BM == 0 &&
                  (2 * kPadSmall) % CfgImageS::BN == 0 && (2 * kFoldPad) % CfgImageS::BK == 0,
              "small-output padding");
static_assert(kPadY % CfgPupil::BN == 0 && kPadX % CfgImage::BM == 0 && (2 * kPadY) % CfgImage::BN == 0 &&
                  (2 * kFoldPad) % CfgImage::BK == 0,
              "image GEMM padding");

// K2: T[s][z][c] = (Pf~ B1) with rows 2q + ri, i.e. the complex [2 nhp] x [nyp] matrix
// T[q][n] = sum_kk Pf~[q][kk] B1[kk][n], B1[2lf][n] = cos(k s_lf y_n), B1[2lf+1][n] = sin(...)
template <class Cfg, int OCC>
__global__ void __launch_bounds__(Cfg::NT, OCC) gemm_pupil_kernel(Gemm1Args a) {
  extern __shared__ float lds[];
  const int w = 2 * a.nhp;
  const int tiles_m = 2 * w / Cfg::BM;
  const int tiles_n = a.nyp / Cfg::BN;
  const int nblocks = a.nstk * a.nzs * a.nc * tiles_m * tiles_n;
  int id = xcd_remap(blockIdx.x, nblocks);
  const int tn = id % tiles_n; id /= tiles_n;
  const int tm = id % tiles_m; id /= tiles_m;
  const int zi = id % a.nzs; id /= a.nzs;
  const int c = id % a.nc; id /= a.nc;
  const int s = id;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wrow = (wave / Cfg::WAVES_N) * Cfg::WM, wcol = (wave % Cfg::WAVES_N) * Cfg::WN;
  const size_t fpp = (size_t)w * w;
  const int row0 = tm * Cfg::BM, col0 = tn * Cfg::BN;
  const int jf0 = row0 / 4;

  FoldDefocusLoader<Cfg> la;
  la.Pf = a.Pf + ((size_t)s * a.nc + c) * fpp + (size_t)(2 * jf0) * w;
  la.kszf = a.kszf + (size_t)jf0 * a.nhp;
  la.zrev = (a.z[a.z0 + zi] + a.zoff[s]) * (1.0 / kTwoPi);
  la.w = w;
  la.nhp = a.nhp;
  RRowLoader<Cfg, Cfg::BN> lb;
  lb.src = a.B1 + (size_t)col0 * w;
  lb.ld = w;

  // The pupil is zero outside the disk (2j+1-n)^2 + (2l+1-n)^2 <= n^2: this row block
  // needs the folded columns lf that its row nearest the centre (largest jf) reaches.
  int k_begin = 0, k_end = w;
  {
    const int n = a.n, nh = (a.n + 1) / 2;
    const int jf_hi = min(jf0 + Cfg::BM / 4, nh) - 1;
    if (jf_hi < jf0) {
      k_end = Cfg::BK;   // padding rows only: one (zero) stage
    } else {
      const int umin = abs(2 * jf_hi + 1 - n);
      const int vmax = (int)floorf(sqrtf((float)n * n - (float)umin * umin)) + 1;   // generous
      const int lf_lo = max(0, (n - 1 - vmax) / 2);
      k_begin = (2 * lf_lo / Cfg::BK) * Cfg::BK;
    }
  }
  RgAcc<Cfg> acc;
  acc.zero();
  // unordered: the compiler's interleaving of the defocus arithmetic measured faster here
  rg_mainloop<Cfg, kOrderFree>(acc, la, lb, k_begin, k_end, lds, tid, wrow, wcol, lane);

  // rows 2q + ri: registers r and r + 1 (r even) are the re/im parts of one T[q][n]
  float2* T = a.T + (((size_t)s * a.nzs + zi) * a.nc + c) * (size_t)w * a.nyp;
#pragma unroll
  for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
    for (int jj = 0; jj < Cfg::TN; ++jj) {
      const int col = col0 + rg_col(wcol, jj, lane);
#pragma unroll
      for (int r = 0; r < 16; r += 2) {
        const int q = (row0 + rg_row(wrow, i, r, lane)) >> 1;
        T[(size_t)q * a.nyp + col] = make_float2(acc.c[i][jj][r], acc.c[i][jj][r + 1]);
      }
    }
}

// K3: E'[m][(n, ri)] = sum_kk A2[m][kk] T[kk][(n, ri)] with A2[m][2jf] = pref cos(k s_jf x_m),
// A2[m][2jf+1] = pref sin(...) for all channels in one workgroup; E = -i E' and
// I = sum_c |E_c|^2 are written from registers.
// One channel of an output tile of K3: the GEMM (its first stage already in ra, rb),
// then the next channel's first stage is loaded, then this channel's fields are stored
// and its intensity accumulated.  The loads go first so that the wait before they are
// staged in LDS does not also wait for the stores.
template <class Cfg, bool FULL, bool HAS_E, class LA, class LB>
__device__ __forceinline__ void image_channel(const Gemm2Args& a, float* lds, int c, const LA& la, LB& lb,
                                              typename LA::Regs& ra, typename LB::Regs& rb, const float* tsrc,
                                              size_t tch, float* E, int row0, int col0, float (*isum)[Cfg::TN][8]) {
  const int w = 2 * a.nhp;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wrow = (wave / Cfg::WAVES_N) * Cfg::WM, wcol = (wave % Cfg::WAVES_N) * Cfg::WN;
  const int ri = lane & 1;   // columns alternate re/im with the lane index
  RgAcc<Cfg> acc;
  acc.zero();
  rg_mainloop_pre<Cfg, kOrderFull>(acc, la, lb, ra, rb, 0, w, lds, tid, wrow, wcol, lane);
  // first stage of the next channel (the last channel reloads its own, unused)
  lb.src = tsrc + (size_t)min(c + 1, a.nc - 1) * tch;
  ra = la.load(0, tid);
  rb = lb.load(0, tid);
  __builtin_amdgcn_sched_barrier(0);

  // Lane 2t holds Re E' and lane 2t+1 Im E' of one pixel: E = -i E' = (Im E', -Re E'),
  // so the odd lane writes E.x = v and the even lane E.y = -v.  A DPP swap within lane
  // pairs gives each lane its partner's value for the intensity.
  // The store offsets are the same for every channel; keeping them opaque here stops
  // them from being hoisted out of the channel loop (32 live offsets would spill).
  int mbase = row0 + rg_row(wrow, 0, 0, lane);
  asm volatile("" : "+v"(mbase));
#pragma unroll
  for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
    for (int jj = 0; jj < Cfg::TN; ++jj) {
      const int n = (col0 + rg_col(wcol, jj, lane)) >> 1;
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        float q[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int rr = r + 8 * h;
          const int m = mbase + 32 * i + (rr >> 2) * 8 + (rr & 3);
          const float v = acc.c[i][jj][rr];
          const float u = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
          q[h] = v * v + u * u;
          if (HAS_E && (FULL || (m < a.nx && n < a.ny))) E[2 * ((size_t)m * a.ny + n) + 1 - ri] = ri ? v : -v;
        }
        isum[i][jj][r] += ri ? q[1] : q[0];
      }
    }
}

// One output tile of K3 for every channel.  FULL: the tile lies inside the nx x ny
// image, so its stores need no per-lane bounds and run as straight-line code.  The
// first channel is peeled so that every entry into the channel loop follows a batch of
// stores issued after the loads it waits for.
template <class Cfg, bool FULL, bool HAS_E>
__device__ __forceinline__ void image_tile(const Gemm2Args& a, float* lds, int s, int zi, int row0, int col0) {
  const int w = 2 * a.nhp;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wrow = (wave / Cfg::WAVES_N) * Cfg::WM, wcol = (wave % Cfg::WAVES_N) * Cfg::WN;
  const size_t plane = (size_t)a.nx * a.ny;
  const size_t gstk = (size_t)(a.s_base + s), gz = (size_t)(a.z0 + zi);
  const int ri = lane & 1;

  // intensity of the lane pair's 16 pixels per block: the even lane keeps those of
  // registers 0-7, the odd lane those of registers 8-15
  float isum[Cfg::TM][Cfg::TN][8];
#pragma unroll
  for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
    for (int jj = 0; jj < Cfg::TN; ++jj)
#pragma unroll
      for (int r = 0; r < 8; ++r) isum[i][jj][r] = 0.f;

  RRowLoader<Cfg, Cfg::BM> la;
  la.src = a.A2 + (size_t)row0 * w;
  la.ld = w;
  RColLoader<Cfg, Cfg::BN> lb;
  const float* tsrc = reinterpret_cast<const float*>(a.T + ((size_t)s * a.nzs + zi) * a.nc * (size_t)w * a.nyp) + col0;
  const size_t tch = 2 * (size_t)w * a.nyp;   // floats per channel of T
  lb.src = tsrc;
  lb.ld = 2 * a.nyp;
  auto ra = la.load(0, tid);
  auto rb = lb.load(0, tid);
  float* E0 = HAS_E ? reinterpret_cast<float*>(a.E + (gstk * a.nz + gz) * a.nc * plane) : nullptr;
  image_channel<Cfg, FULL, HAS_E>(a, lds, 0, la, lb, ra, rb, tsrc, tch, E0, row0, col0, isum);
#pragma unroll 1
  for (int c = 1; c < a.nc; ++c)
    image_channel<Cfg, FULL, HAS_E>(a, lds, c, la, lb, ra, rb, tsrc, tch, HAS_E ? E0 + 2 * c * plane : nullptr,
                                    row0, col0, isum);
  if (a.I) {
    float* I = a.I + (gstk * a.nz + gz) * plane;
#pragma unroll
    for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
      for (int jj = 0; jj < Cfg::TN; ++jj) {
        const int n = (col0 + rg_col(wcol, jj, lane)) >> 1;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          const int m = row0 + rg_row(wrow, i, r + 8 * ri, lane);
          if (FULL || (m < a.nx && n < a.ny)) I[(size_t)m * a.ny + n] = isum[i][jj][r];
        }
      }
  }
}

template <class Cfg, int OCC>
__global__ void __launch_bounds__(Cfg::NT, OCC) gemm_image_kernel(Gemm2Args a) {
  extern __shared__ float lds[];
  const int tiles_m = a.nxp / Cfg::BM;
  const int tiles_n = 2 * a.nyp / Cfg::BN;
  const int nblocks = a.nstk * a.nzs * tiles_m * tiles_n;
  int id = xcd_remap(blockIdx.x, nblocks);
  const int tn = id % tiles_n; id /= tiles_n;
  const int tm = id % tiles_m; id /= tiles_m;
  const int zi = id % a.nzs; id /= a.nzs;
  const int s = id;
  const int row0 = tm * Cfg::BM, col0 = tn * Cfg::BN;
  const bool full = row0 + Cfg::BM <= a.nx && col0 + Cfg::BN <= 2 * a.ny;
  if (a.E) {
    if (full)
      image_tile<Cfg, true, true>(a, lds, s, zi, row0, col0);
    else
      image_tile<Cfg, false, true>(a, lds, s, zi, row0, col0);
  } else {
    if (full)
      image_tile<Cfg, true, false>(a, lds, s, zi, row0, col0);
    else
      image_tile<Cfg, false, false>(a, lds, s, zi, row0, col0);
  }
}

// --------------------------------------------------------------------------
// Host-side launchers
// --------------------------------------------------------------------------
hipError_t launch_zernike_table(float* out, int n, int nj, hipStream_t st) {
  const int cells = n * n;
  hipLaunchKernelGGL(zernike_table_kernel, dim3((cells + 255) / 256), dim3(256), 0, st, out, n, nj);
  return hipGetLastError();
}

hipError_t launch_pupil_build(const PupilArgs& a, const float2* Q, const float* ztab, float2* P,
                              hipStream_t st) {
  const int cells = a.np * a.np;
  hipLaunchKernelGGL(pupil_build_kernel, dim3((cells + 255) / 256, a.nstk), dim3(256), 0, st, a, Q, ztab, P);
  return hipGetLastError();
}

hipError_t launch_pupil_build_folded(const PupilArgs& a, const float2* Q, const float* ztab, float2* Pf, int nhp,
                                     hipStream_t st) {
  const int lanes = 4 * nhp * nhp;
  hipLaunchKernelGGL(pupil_build_folded_kernel, dim3((lanes + 255) / 256, a.nstk), dim3(256), 0, st, a, Q, ztab, Pf,
                     nhp);
  return hipGetLastError();
}

template <class Cfg, int OCC>
static hipError_t gemm_pupil_launch(const Gemm1Args& a, hipStream_t st) {
  const int tiles = (4 * a.nhp / Cfg::BM) * (a.nyp / Cfg::BN);
  const int nblocks = a.nstk * a.nzs * a.nc * tiles;
  hipLaunchKernelGGL((gemm_pupil_kernel<Cfg, OCC>), dim3(nblocks), dim3(Cfg::NT), Cfg::LDS_BYTES, st, a);
  return hipGetLastError();
}

template <class Cfg, int OCC>
static hipError_t gemm_image_launch(const Gemm2Args& a, hipStream_t st) {
  const int tiles = (a.nxp / Cfg::BM) * (2 * a.nyp / Cfg::BN);
  const int nblocks = a.nstk * a.nzs * tiles;
  hipLaunchKernelGGL((gemm_image_kernel<Cfg, OCC>), dim3(nblocks), dim3(Cfg::NT), Cfg::LDS_BYTES, st, a);
  return hipGetLastError();
}

// Compute units of the current device (queried once per device).
static int device_cus() {
  static int cus[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cus[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cus[dev] = n;
  }
  return cus[dev];
}

// The tile height follows the padding the plan chose (multiples of 128, or of 64 for
// outputs of at most 64 pixels along that axis).  A launch whose large tiles would give
// fewer than two workgroups per CU (a few planes, e.g. one image) takes the small tiles
// instead: its time is then set by how many CUs work on it, not by the tile efficiency.
hipError_t launch_gemm_pupil(const Gemm1Args& a, hipStream_t st) {
  const long long work = (long long)a.nstk * a.nzs * a.nc;
  const bool few = work * ((4 * a.nhp + 127) / 128) * ((a.nyp + 127) / 128) < 2LL * device_cus();
  if (!few && a.nyp % CfgPupilL::BN == 0 && (4 * a.nhp) % CfgPupilL::BM == 0)
    return gemm_pupil_launch<CfgPupilL, 2>(a, st);
  if (!few && a.nyp % CfgPupil::BN == 0) return gemm_pupil_launch<CfgPupil, RW_F1_OCC>(a, st);
  if (!few && (4 * a.nhp) % CfgPupilSL::BM == 0) return gemm_pupil_launch<CfgPupilSL, 2>(a, st);
  return gemm_pupil_launch<CfgPupilS, 4>(a, st);
}

hipError_t launch_gemm_image(const Gemm2Args& a, hipStream_t st) {
  const long long work = (long long)a.nstk * a.nzs;
  const bool few = work * ((a.nxp + 127) / 128) * ((2 * a.nyp + 127) / 128) < 2LL * device_cus();
  if (!few && a.nxp % CfgImage::BM == 0 && (2 * a.nyp) % CfgImage::BN == 0)
    return gemm_image_launch<CfgImage, RW_F2_OCC>(a, st);
  return gemm_image_launch<CfgImageS, 4>(a, st);
}

hipError_t fourier_kernel_attributes() {
  const void* k[6] = {(const void*)gemm_pupil_kernel<CfgPupil, RW_F1_OCC>, (const void*)gemm_pupil_kernel<CfgPupilS, 4>,
                      (const void*)gemm_image_kernel<CfgImage, RW_F2_OCC>, (const void*)gemm_image_kernel<CfgImageS, 4>,
                      (const void*)gemm_pupil_kernel<CfgPupilL, 2>, (const void*)gemm_pupil_kernel<CfgPupilSL, 2>};
  const int bytes[6] = {CfgPupil::LDS_BYTES, CfgPupilS::LDS_BYTES, CfgImage::LDS_BYTES, CfgImageS::LDS_BYTES,
                        CfgPupilL::LDS_BYTES, CfgPupilSL::LDS_BYTES};
  for (int i = 0; i < 6; ++i) {
    const hipError_t e = hipFuncSetAttribute(k[i], hipFuncAttributeMaxDynamicSharedMemorySize, bytes[i]);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace rw
