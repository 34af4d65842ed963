// Hand-written adjoint of the Fourier form.
//
// Forward (per stack b, plane z, component c): E = Ax' P~ Ay^T with
// P~ = P_{b,c} exp(i k s_z z), P_{b,c} = Q_c exp(i Phi_b) (read from the forward's
// mirror-folded pupils: each lane recovers its own mirror cell from the four parities).
// For a real loss L(I), I = sum_c |E_c|^2, with g = dL/dI:
//   dL/dPhi[j,l] = sum_{b,z,c} Im( G[j,l] conj(P~[j,l]) ),  G = Ax'^H (2 g E) conj(Ay)
//   dL/dW0 = dL/dPhi,  dL/dc_q = 2 pi sum_cells dL/dPhi Z_q.
// The pupil grid is mirror-symmetric (s[N-1-j] = -s[j]), so with theta = k s_jf x_m and
// phi = k s_lf y_n (jf, lf < N/2 the folded indices, j' = N-1-jf, l' = N-1-lf):
//   H[m][lf], H[m][l'] = Hc -+ i Hs,   Hc, Hs = sum_n (2 g E)[m][n] {cos, sin} phi
//   G = i pref (CC -+ i CS -+ i SC ...)  with  CC = sum_m cos theta Hc, CS = sum_m cos theta Hs,
//   SC = sum_m sin theta Hc, SS = sum_m sin theta Hs (pref = f k / 2 pi), i.e.
//   G[jf,lf] = i pref (CC - iCS - iSC - SS)    G[jf,l'] = i pref (CC + iCS - iSC + SS)
//   G[j',lf] = i pref (CC - iCS + iSC + SS)    G[j',l'] = i pref (CC + iCS + iSC - SS)
// Kernels (real-coefficient GEMMs on the FP32 matrix cores, FP32 accumulate):
//   adj_h_kernel   H'[b,z,c][m][2lf + p] = {Hc, Hs}: rows 2m + re/im of 2 g E (the scaling
//                  applied while E is staged) times the folded y table
//   adj_g_kernel   for each (stack, component, plane group) and folded pupil tile, over
//                  the planes in order: Q = {cos, sin}(theta) H', then the four mirror
//                  values of G from each lane quad, acc += Im(G conj(P~)) -- one partial
//                  per (stack, component, plane group), no atomics
//   adj_reduce_*   dL/dPhi = sum of the partials in a fixed order (FP64), dL/dW0
//   adj_zernike_kernel dL/dc_q by a fixed-shape tree reduction (FP64)
// The result does not depend on scheduling: every sum runs in a fixed order.
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "cgemm.h"
#include "rgemm.h"
#include "rw_common.h"
#include "rw_fourier.h"
#include "rw_plan.h"

namespace rw {

constexpr int kAdjStacks = 32;   // stacks per adj_h / adj_g launch (fewer kernel prologues and tails)
using CfgAdjH = RgCfg<128, 64, 16, 64, 32>;   // rows 2m + re/im, columns 2lf + p, k = n
using CfgAdjG = RgCfg<64, 128, 16, 32, 64>;   // rows 2jf + p, columns 2(2lf + p) + re/im, k = m

// A operand of adj_h: rows 2m + ri of 2 g E ([nx][ny] complex, k = n contiguous); rows
// past nx read row nx - 1 with a zero factor (no branches in the load path).
template <class Cfg>
struct ScaledFieldLoader {
  static constexpr int ROWS = Cfg::BM / 2, PAIRS = Cfg::BK / 2;
  static constexpr int PER_THREAD = ROWS * PAIRS / Cfg::NT;
  static_assert(ROWS * PAIRS % Cfg::NT == 0, "loader shape");
  const float2* E;
  const float* g;
  int ld, nrows, row0;
  struct Regs {
    float4 v[PER_THREAD];
    float2 f[PER_THREAD];
  };

  __device__ Regs load(int k0, int tid) const {
    Regs r;
    float4* v = r.v;
    float2* f = r.f;
#pragma unroll
    for (int i = 0; i < PER_THREAD; ++i) {
      const int idx = tid + i * Cfg::NT;
      const int row = idx / PAIRS, kk = 2 * (idx % PAIRS);
      const int gr = min(row0 + row, nrows - 1);
      const size_t off = (size_t)gr * ld + k0 + kk;
      v[i] = *reinterpret_cast<const float4*>(E + off);
      const float2 gg = *reinterpret_cast<const float2*>(g + off);
      const float keep = (row0 + row < nrows) ? 2.f : 0.f;
      f[i] = make_float2(keep * gg.x, keep * gg.y);
    }
    return r;
  }
  __device__ void store(float* dst, int tid, const Regs& r) const {
    const float4* v = r.v;
    const float2* f = r.f;
#pragma unroll
    for (int i = 0; i < PER_THREAD; ++i) {
      const int idx = tid + i * Cfg::NT;
      const int row = idx / PAIRS, kk = 2 * (idx % PAIRS);
      float* d = dst + (2 * row) * Cfg::LDK + kk;
      *reinterpret_cast<float2*>(d) = make_float2(f[i].x * v[i].x, f[i].y * v[i].z);
      *reinterpret_cast<float2*>(d + Cfg::LDK) = make_float2(f[i].x * v[i].y, f[i].y * v[i].w);
    }
  }
};

struct AdjHArgs {
  const float2* E;     // [stacks][nz][3][nx][ny] (the caller's fields)
  const float* g;      // [stacks][nz][nx][ny]
  const float* CyT;    // [w][nyp] rows 2lf + p: {cos, sin}(k s_lf y_n)
  float2* H;           // [chunk][nz][3][nxp][w]
  int s0, nstk, nz, nx, ny, nyp, nxp, w;
};

__global__ void __launch_bounds__(CfgAdjH::NT, 2) adj_h_kernel(AdjHArgs a) {
  using Cfg = CfgAdjH;
  extern __shared__ float lds[];
  const int tiles_m = 2 * a.nxp / Cfg::BM, tiles_n = a.w / Cfg::BN;
  const int nblocks = a.nstk * a.nz * 3 * tiles_m * tiles_n;
  int id = xcd_remap(blockIdx.x, nblocks);
  const int tn = id % tiles_n; id /= tiles_n;
  const int tm = id % tiles_m; id /= tiles_m;
  const int item = id;   // (s, z, c) within the chunk
  const int c = item % 3, z = (item / 3) % a.nz, s = item / (3 * a.nz);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wrow = (wave / Cfg::WAVES_N) * Cfg::WM, wcol = (wave % Cfg::WAVES_N) * Cfg::WN;
  const size_t plane = (size_t)a.nx * a.ny;
  const size_t gs = (size_t)(a.s0 + s);
  const int row0 = tm * Cfg::BM, col0 = tn * Cfg::BN;
  ScaledFieldLoader<Cfg> la;
  la.E = a.E + ((gs * a.nz + z) * 3 + c) * plane;
  la.g = a.g + (gs * a.nz + z) * plane;
  la.ld = a.ny;
  la.nrows = a.nx;
  la.row0 = row0 / 2;
  RRowLoader<Cfg, Cfg::BN> lb;
  lb.src = a.CyT + (size_t)col0 * a.nyp;
  lb.ld = a.nyp;
  RgAcc<Cfg> acc;
  acc.zero();
  rg_mainloop<Cfg, kOrderFull>(acc, la, lb, 0, a.ny, lds, tid, wrow, wcol, lane);
  // rows 2m + ri: registers r and r + 1 (r even) are the re/im parts of one H'[m][col]
  float2* H = a.H + (size_t)item * a.nxp * a.w;
#pragma unroll
  for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
    for (int jj = 0; jj < Cfg::TN; ++jj) {
      const int col = col0 + rg_col(wcol, jj, lane);
#pragma unroll
      for (int r = 0; r < 16; r += 2) {
        const int m = (row0 + rg_row(wrow, i, r, lane)) >> 1;
        H[(size_t)m * a.w + col] = make_float2(acc.c[i][jj][r], acc.c[i][jj][r + 1]);
      }
    }
}

struct AdjGArgs {
  const float* CxT;    // [w][nxp] rows 2jf + p: pref {cos, sin}(k s_jf x_m)
  const float2* H;     // [chunk][nz][3][nxp][w]
  const float2* Pf;    // [chunk][3][w][w] mirror-folded pupils (the forward's fold)
  const double* ksz;   // [np][np]
  const float2* D;     // [nz][np][np] exp(i k s_z z) of the plan's planes
  float* partial;      // [stacks * 3 * zgroups][np][np]
  double zoff[kAdjStacks];
  int s0, nstk, nz, nxp, w, n;
  int zgroups, zper;   // planes are split into zgroups runs of zper (the last may be shorter)
};

// quad_perm DPP: lane 4t + q reads lane 4t + sel[q]
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// at most 168 VGPRs, so that three 4-wave workgroups share a CU
__global__ void __launch_bounds__(CfgAdjG::NT, 3) adj_g_kernel(AdjGArgs a) {
  using Cfg = CfgAdjG;
  extern __shared__ float lds[];
  const int tiles_m = a.w / Cfg::BM, tiles_n = 2 * a.w / Cfg::BN;
  const int nblocks = a.nstk * 3 * a.zgroups * tiles_m * tiles_n;
  int id = xcd_remap(blockIdx.x, nblocks);
  const int tn = id % tiles_n; id /= tiles_n;
  const int tm = id % tiles_m; id /= tiles_m;
  const int g = id % a.zgroups; id /= a.zgroups;
  const int c = id % 3, s = id / 3;
  const int z_begin = g * a.zper, z_end = min(a.nz, z_begin + a.zper);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wrow = (wave / Cfg::WAVES_N) * Cfg::WM, wcol = (wave % Cfg::WAVES_N) * Cfg::WN;
  const int row0 = tm * Cfg::BM, col0 = tn * Cfg::BN;
  const int n = a.n, nh = (n + 1) / 2;
  const size_t npp = (size_t)a.w * a.w;
  const float2* Pf = a.Pf + ((size_t)s * 3 + c) * npp;
  // lane quad q = lane & 3 of columns 2(2lf + p) + ri: q = 2p + ri.  After the exchange the
  // lane owns mirror cell q: (jf, lf), (jf, l'), (j', lf), (j', l').
  const int q = lane & 3;
  // The defocus of plane z for stack s is exp(i k s_z z) exp(i k s_z zoff_s): the second
  // factor is applied to the lane's pupil cells once, the first comes from the plan's table.
  float2 p0[Cfg::TM][Cfg::TN][8];
#pragma unroll
  for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
    for (int jj = 0; jj < Cfg::TN; ++jj) {
      const int lf = (col0 + rg_col(wcol, jj, lane)) >> 2;
#pragma unroll
      for (int r = 0; r < 16; r += 2) {
        const int jf = (row0 + rg_row(wrow, i, r, lane)) >> 1;
        const int jc = (q & 2) ? n - 1 - jf : jf, lc = (q & 1) ? n - 1 - lf : lf;
        const bool own = jf < nh && lf < nh && !((q & 2) && jc == jf) && !((q & 1) && lc == lf);
        float2 v = make_float2(0.f, 0.f);
        if (own) {
          // the pupil at mirror (a, b) = (q / 2, q % 2) from the four parities of the
          // folded cell: P_ab = sum_{pj, pl} (-1)^(a pj + b pl) (-i)^(pj + pl) Pf_{pj, pl},
          // over 2 per folded axis with two mirrors (a self-mirrored row has no odd part)
          const float2* f = Pf + (size_t)(2 * jf) * a.w + 2 * lf;
          const float2 f00 = f[0], f01 = f[1], f10 = f[a.w], f11 = f[a.w + 1];
          const float sb = (q & 1) ? -1.f : 1.f, sa = (q & 2) ? -1.f : 1.f;
          const float scale = (jf != n - 1 - jf ? 0.5f : 1.f) * (lf != n - 1 - lf ? 0.5f : 1.f);
          // (-i) (x + i y) = y - i x
          const float2 pp = make_float2(scale * (f00.x + sb * f01.y + sa * f10.y - sa * sb * f11.x),
                                        scale * (f00.y - sb * f01.x - sa * f10.x - sa * sb * f11.y));
          const size_t cell = (size_t)jc * a.w + lc;
          float sn, cs;
          sincosf((float)reduce_2pi(a.ksz[cell] * a.zoff[s]), &sn, &cs);
          v = make_float2(pp.x * cs - pp.y * sn, pp.x * sn + pp.y * cs);
        }
        p0[i][jj][r >> 1] = v;
      }
    }
  float dphi[Cfg::TM][Cfg::TN][8];
#pragma unroll
  for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
    for (int jj = 0; jj < Cfg::TN; ++jj)
#pragma unroll
      for (int r = 0; r < 8; ++r) dphi[i][jj][r] = 0.f;
  RRowLoader<Cfg, Cfg::BM> la;
  la.src = a.CxT + (size_t)row0 * a.nxp;
  la.ld = a.nxp;
  RColLoader<Cfg, Cfg::BN> lb;
  const float* hsrc = reinterpret_cast<const float*>(a.H) + col0;
  const size_t hplane = 2 * (size_t)a.nxp * a.w;   // floats per (stack, plane, channel) of H
  lb.src = hsrc + ((size_t)(s * a.nz + z_begin) * 3 + c) * hplane;
  lb.ld = 2 * a.w;
  auto ra = la.load(0, tid);
  auto rb = lb.load(0, tid);
#pragma unroll 1
  for (int zi = z_begin; zi < z_end; ++zi) {
    RgAcc<Cfg> acc;
    acc.zero();
    rg_mainloop_pre<Cfg, kOrderFree>(acc, la, lb, ra, rb, 0, a.nxp, lds, tid, wrow, wcol, lane);
    // the next plane's first stage (the last plane reloads its own, unused) is loaded
    // before this plane's epilogue, which hides its latency
    lb.src = hsrc + ((size_t)(s * a.nz + min(zi + 1, z_end - 1)) * 3 + c) * hplane;
    ra = la.load(0, tid);
    rb = lb.load(0, tid);
    // Per column block: the table cells of its 8 accumulator pairs (the lane's mirror
    // cell, or cell 0 where the lane owns none: its p0 is zero there, so the product
    // adds nothing) are all loaded before any is used.
    const float2* Dz = a.D + (size_t)zi * npp;
#pragma unroll
    for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
      for (int jj = 0; jj < Cfg::TN; ++jj) {
        const int lf = (col0 + rg_col(wcol, jj, lane)) >> 2;
        float2 dz[8];
#pragma unroll
        for (int r = 0; r < 16; r += 2) {
          const int jf = (row0 + rg_row(wrow, i, r, lane)) >> 1;
          const int jc = (q & 2) ? n - 1 - jf : jf, lc = (q & 1) ? n - 1 - lf : lf;
          const bool own = jf < nh && lf < nh && !((q & 2) && jc == jf) && !((q & 1) && lc == lf);
          dz[r >> 1] = Dz[own ? jc * a.w + lc : 0];
        }
#pragma unroll
        for (int r = 0; r < 16; r += 2) {
          // this lane holds row (jf, p = 0) in register r and (jf, 1) in r + 1, column q
          const float x0 = acc.c[i][jj][r], x1 = acc.c[i][jj][r + 1];
          // quad values: [q'] of register r -> C* , of register r + 1 -> S*
          const float c0 = dpp<0x00>(x0), c1 = dpp<0x55>(x0), c2 = dpp<0xAA>(x0), c3 = dpp<0xFF>(x0);
          const float s0 = dpp<0x00>(x1), s1 = dpp<0x55>(x1), s2 = dpp<0xAA>(x1), s3 = dpp<0xFF>(x1);
          // CC = c0 + i c1, CS = c2 + i c3, SC = s0 + i s1, SS = s2 + i s3
          const float sl = (q & 1) ? 1.f : -1.f;   // sign of i CS: - for lf, + for l'
          const float sj = (q & 2) ? 1.f : -1.f;   // sign of i SC: - for jf, + for j'
          const float ss = (q == 0 || q == 3) ? -1.f : 1.f;
          // T = CC + sl i CS + sj i SC + ss SS;  G = i pref T (pref is in the x table)
          const float tr = c0 - sl * c3 - sj * s1 + ss * s2;
          const float ti = c1 + sl * c2 + sj * s0 + ss * s3;
          const float gr = -ti, gi = tr;
          const float2 d = dz[r >> 1];
          const float2 pv = p0[i][jj][r >> 1];
          const float pr = pv.x * d.x - pv.y * d.y, pi = pv.x * d.y + pv.y * d.x;
          // Im(G conj(P~)) = Gi Pr - Gr Pi
          dphi[i][jj][r >> 1] += gi * pr - gr * pi;
        }
      }
  }
  float* out = a.partial + (((size_t)(a.s0 + s) * 3 + c) * a.zgroups + g) * npp;
#pragma unroll
  for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
    for (int jj = 0; jj < Cfg::TN; ++jj) {
      const int lf = (col0 + rg_col(wcol, jj, lane)) >> 2;
#pragma unroll
      for (int r = 0; r < 16; r += 2) {
        const int jf = (row0 + rg_row(wrow, i, r, lane)) >> 1;
        const int jc = (q & 2) ? n - 1 - jf : jf, lc = (q & 1) ? n - 1 - lf : lf;
        const bool own = jf < nh && lf < nh && !((q & 2) && jc == jf) && !((q & 1) && lc == lf);
        if (own) out[(size_t)jc * a.w + lc] = dphi[i][jj][r >> 1];
      }
    }
}

// dL/dPhi on the N x N cells: the partials are summed in group order (FP64) in two
// levels -- runs of kReduceRun groups (grid.y runs), then the runs in order.
constexpr int kReduceRun = 32;

__global__ void adj_reduce_runs_kernel(const float* __restrict__ partial, int groups, int n, int np,
                                       double* __restrict__ runs) {
  const int cell = blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= n * n) return;
  const int j = cell / n, l = cell % n;
  const size_t pc = (size_t)j * np + l, npp = (size_t)np * np;
  const int g0 = blockIdx.y * kReduceRun, g1 = min(groups, g0 + kReduceRun);
  double s = 0.0;
#pragma unroll 8
  for (int g = g0; g < g1; ++g) s += (double)partial[g * npp + pc];
  runs[(size_t)blockIdx.y * n * n + cell] = s;
}

__global__ void adj_reduce_kernel(const double* __restrict__ runs, int nruns, int n, double* __restrict__ dphi,
                                  float* __restrict__ dW0) {
  const int cell = blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= n * n) return;
  double s = 0.0;
  for (int r = 0; r < nruns; ++r) s += runs[(size_t)r * n * n + cell];
  dphi[cell] = s;
  if (dW0) dW0[cell] = (float)s;
}

// dL/dc_q = 2 pi sum_cells dL/dPhi Z_q: one workgroup of 1024 threads per q, fixed-shape tree.
constexpr int kZernThreads = 1024;
__global__ void __launch_bounds__(kZernThreads) adj_zernike_kernel(const double* __restrict__ dphi,
                                                                   const float* __restrict__ ztab, int nn,
                                                                   float* __restrict__ dc) {
  __shared__ double red[kZernThreads];
  const int q = blockIdx.x;
  double s = 0.0;
  for (int cell = threadIdx.x; cell < nn; cell += kZernThreads)
    s += dphi[cell] * (double)ztab[(size_t)q * nn + cell];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kZernThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) dc[q] = (float)(kTwoPi * red[0]);
}

hipError_t adjoint_kernel_attributes() {
  hipError_t e = hipFuncSetAttribute((const void*)adj_h_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     CfgAdjH::LDS_BYTES);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)adj_g_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                             CfgAdjG::LDS_BYTES);
}

// Lazily built adjoint tables and workspace of a Fourier plan.
// Plane groups of adj_g: enough workgroups to fill the chip (>= 4 per CU of 256).
static int adjoint_zgroups(const rwpsf_plan* p) {
  const int tiles = (p->np / CfgAdjG::BM) * (2 * p->np / CfgAdjG::BN);
  const int per_group = kAdjStacks * 3 * tiles;
  return std::max(1, std::min(p->grid.nz, (1024 + per_group - 1) / per_group));
}

// Lazily built adjoint tables and workspace of a Fourier plan: the folded DFT tables with
// the pixel index contiguous, CxT[2jf + p][m] = pref {cos, sin}(k s_jf x_m) and
// CyT[2lf + p][n] = {cos, sin}(k s_lf y_n) (zero past nx, ny and for jf, lf >= N/2).
// exp(i k s_z z) of every plan plane on the padded pupil cells (FP64 phase reduced
// mod 2 pi before the FP32 sincos); 0 outside the disk where k s_z is 0 -> factor 1.
__global__ void adj_defocus_kernel(const double* __restrict__ ksz, const double* __restrict__ z, int nz,
                                   int npp, float2* __restrict__ D) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)nz * npp) return;
  const int zi = (int)(idx / npp), cell = (int)(idx % npp);
  float sn, cs;
  sincosf((float)reduce_2pi(ksz[cell] * z[zi]), &sn, &cs);
  D[idx] = make_float2(cs, sn);
}

static int adjoint_prepare(rwpsf_plan* p, int n_stacks) {
  const int nx = p->grid.nx, ny = p->grid.ny, N = p->num.n_pupil, np = p->np;
  const int nxp = p->nxp, nyp = p->nyp, w = 2 * p->nhp, nh = (N + 1) / 2;
  int st;
  if (!p->d_CxT) {
    const double s_max = p->s_max, k = p->k;
    const double pref = p->opt.focal_length * k / kTwoPi;
    std::vector<float> CxT((size_t)w * nxp, 0.f), CyT((size_t)w * nyp, 0.f);
    for (int f = 0; f < nh; ++f) {
      const double sv = (2.0 * f + 1.0 - N) * s_max / N;
      for (int m = 0; m < nx; ++m) {
        const double ph = k * sv * (double)(m - nx / 2) * p->grid.dx_nm;
        CxT[(size_t)(2 * f) * nxp + m] = (float)(pref * std::cos(ph));
        CxT[(size_t)(2 * f + 1) * nxp + m] = (float)(pref * std::sin(ph));
      }
      for (int n = 0; n < ny; ++n) {
        const double ph = k * sv * (double)(n - ny / 2) * p->grid.dy_nm;
        CyT[(size_t)(2 * f) * nyp + n] = (float)std::cos(ph);
        CyT[(size_t)(2 * f + 1) * nyp + n] = (float)std::sin(ph);
      }
    }
    if ((st = dev_alloc(p, &p->d_CxT, CxT.size()))) return st;
    if ((st = dev_alloc(p, &p->d_CyT, CyT.size()))) return st;
    if ((st = dev_alloc(p, &p->d_dphi, (size_t)N * N))) return st;
    if ((st = dev_alloc(p, &p->d_H, (size_t)kAdjStacks * p->grid.nz * 3 * nxp * w))) return st;
    // folded pupils of a whole adjoint group
    if ((st = dev_alloc(p, &p->d_adjPf, (size_t)kAdjStacks * 3 * w * w))) return st;
    const size_t nzpp = (size_t)p->grid.nz * np * np;
    if ((st = dev_alloc(p, &p->d_adjD, nzpp))) return st;
    hipLaunchKernelGGL(adj_defocus_kernel, dim3((unsigned)((nzpp + 255) / 256)), dim3(256), 0, 0, p->d_ksz, p->d_z,
                       p->grid.nz, np * np, p->d_adjD);
    if ((st = hip_check(hipGetLastError()))) return st;
    // the table is written on the null stream; the caller's stream may not order after it
    if ((st = hip_check(hipDeviceSynchronize()))) return st;
    if ((st = hip_check(hipMemcpy(p->d_CxT, CxT.data(), CxT.size() * sizeof(float), hipMemcpyHostToDevice)))) return st;
    if ((st = hip_check(hipMemcpy(p->d_CyT, CyT.data(), CyT.size() * sizeof(float), hipMemcpyHostToDevice)))) return st;
    if ((st = hip_check(adjoint_kernel_attributes()))) return st;
  }
  const int groups = 3 * n_stacks * adjoint_zgroups(p);
  if (p->partial_groups < groups) {
    float* d = nullptr;
    if ((st = dev_alloc(p, &d, (size_t)groups * np * np))) return st;
    p->d_partial = d;
    p->partial_groups = groups;
    double* r = nullptr;
    if ((st = dev_alloc(p, &r, (size_t)((groups + kReduceRun - 1) / kReduceRun) * N * N))) return st;
    p->d_runs = r;
  }
  return RWPSF_OK;
}

int fourier_adjoint(rwpsf_plan* p, int n, const rwpsf_stack* s, const float2* E, const float* dLdI,
                    int n_zernike, float* dc, float* dW0, hipStream_t st) {
  const int nx = p->grid.nx, ny = p->grid.ny, nz = p->grid.nz, N = p->num.n_pupil, np = p->np;
  if (nx % 16 || ny % 16) return RWPSF_ERR_UNSUPPORTED;   // whole MFMA k-stages along x and y
  int rc = adjoint_prepare(p, n);
  if (rc) return rc;
  const int nxp = p->nxp, w = 2 * p->nhp;
  const int zg = adjoint_zgroups(p);
  for (int b0 = 0; b0 < n; b0 += kAdjStacks) {
    const int nb = std::min(kAdjStacks, n - b0);
    for (int c0 = 0; c0 < nb; c0 += kPupilStacks)
      if ((rc = fourier_build_folded(p, s + b0 + c0, std::min(kPupilStacks, nb - c0),
                                     p->d_adjPf + (size_t)c0 * 3 * w * w, st)))
        return rc;
    AdjHArgs ha{E, dLdI, p->d_CyT, p->d_H, b0, nb, nz, nx, ny, p->nyp, nxp, w};
    const int hblocks = nb * nz * 3 * (2 * nxp / CfgAdjH::BM) * (w / CfgAdjH::BN);
    int tr = p->time_begin(RWPSF_KERNEL_ADJ_H, st);
    hipLaunchKernelGGL(adj_h_kernel, dim3(hblocks), dim3(CfgAdjH::NT), CfgAdjH::LDS_BYTES, st, ha);
    if ((rc = hip_check(hipGetLastError()))) return rc;
    p->time_end(tr, st);
    AdjGArgs ga{};
    ga.CxT = p->d_CxT;
    ga.H = p->d_H;
    ga.Pf = p->d_adjPf;
    ga.ksz = p->d_ksz;
    ga.D = p->d_adjD;
    ga.partial = p->d_partial;
    for (int i = 0; i < nb; ++i) ga.zoff[i] = s[b0 + i].z_offset_nm;
    ga.s0 = b0;
    ga.nstk = nb;
    ga.nz = nz;
    ga.nxp = nxp;
    ga.w = w;
    ga.n = N;
    ga.zgroups = zg;
    ga.zper = (nz + zg - 1) / zg;
    const int gblocks = nb * 3 * zg * (w / CfgAdjG::BM) * (2 * w / CfgAdjG::BN);
    tr = p->time_begin(RWPSF_KERNEL_ADJ_G, st);
    hipLaunchKernelGGL(adj_g_kernel, dim3(gblocks), dim3(CfgAdjG::NT), CfgAdjG::LDS_BYTES, st, ga);
    if ((rc = hip_check(hipGetLastError()))) return rc;
    p->time_end(tr, st);
  }
  int tr = p->time_begin(RWPSF_KERNEL_ADJ_REDUCE, st);
  const int groups = 3 * n * zg, nruns = (groups + kReduceRun - 1) / kReduceRun;
  hipLaunchKernelGGL(adj_reduce_runs_kernel, dim3((N * N + 255) / 256, nruns), dim3(256), 0, st, p->d_partial,
                     groups, N, np, p->d_runs);
  if ((rc = hip_check(hipGetLastError()))) return rc;
  hipLaunchKernelGGL(adj_reduce_kernel, dim3((N * N + 255) / 256), dim3(256), 0, st, p->d_runs, nruns, N,
                     p->d_dphi, dW0);
  if ((rc = hip_check(hipGetLastError()))) return rc;
  if (n_zernike > 0) {
    hipLaunchKernelGGL(adj_zernike_kernel, dim3(n_zernike), dim3(kZernThreads), 0, st, p->d_dphi, p->d_ztab, N * N,
                       dc);
    if ((rc = hip_check(hipGetLastError()))) return rc;
  }
  p->time_end(tr, st);
  return RWPSF_OK;
}

}  // namespace rw
