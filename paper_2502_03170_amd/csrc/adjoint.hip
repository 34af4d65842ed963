// Hand-written adjoint of the Fourier form.
//
// Forward (per stack b, plane z, component c): E = Ax' P~ Ay^T with
// P~ = P_{b,c} exp(i k s_z z), P_{b,c} = Q_c exp(i Phi_b) (the pupil-build kernel).
// For a real loss L(I), I = sum_c |E_c|^2, with g = dL/dI:
//   dL/dPhi[j,l] = sum_{b,z,c} Im( G[j,l] conj(P~[j,l]) ),  G = Ax'^H (2 g E) conj(Ay)
//   dL/dW0 = dL/dPhi,  dL/dc_q = 2 pi sum_cells dL/dPhi Z_q.
// Kernels (complex FP32 GEMMs on the matrix cores, FP32 accumulate):
//   adj_h_kernel   H[b,z,c] = (2 g E) AyH,  AyH[n][l] = conj(Ay[n][l])   (the scaling
//                  2 g is applied while E is staged; H is [nx][np])
//   adj_g_kernel   for each (stack, component) and pupil tile, over the planes z in
//                  order: G = AxH^T H (AxH[m][j] = conj(Ax'[m][j])), then
//                  acc += Im(G conj(P~)) -- one partial per (stack, component), no atomics
//   adj_reduce_kernel  dL/dPhi = sum of the partials in a fixed order (FP64), dL/dW0
//   adj_zernike_kernel dL/dc_q by a fixed-shape tree reduction (FP64)
// The result does not depend on scheduling: every sum runs in a fixed order.
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "cgemm.h"
#include "rw_common.h"
#include "rw_fourier.h"
#include "rw_plan.h"

namespace rw {

using CfgAdj = CgCfg<64, 64, 16, 32, 32>;

// A operand of adj_h: rows m, contraction n, from E [nx][ny] scaled by 2 dL/dI.
// Rows past nx read row nx-1 with a zero factor (no branches in the load path).
template <class Cfg>
struct ScaledRowLoader {
  static constexpr int PAIRS = Cfg::BK / 2;
  static constexpr int PER_THREAD = Cfg::BM * PAIRS / Cfg::NT;
  static_assert(Cfg::BM * PAIRS % Cfg::NT == 0, "loader shape");
  const float2* E;
  const float* g;
  int ld, nrows, row0;
  float4 v[PER_THREAD];
  float2 f[PER_THREAD];

  __device__ void load(int k0, int tid) {
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
  }
  __device__ void store(float* re, float* im, int ldl, int tid) const {
#pragma unroll
    for (int i = 0; i < PER_THREAD; ++i) {
      const int idx = tid + i * Cfg::NT;
      const int row = idx / PAIRS, kk = 2 * (idx % PAIRS);
      re[kk * ldl + row] = f[i].x * v[i].x;
      im[kk * ldl + row] = f[i].x * v[i].y;
      re[(kk + 1) * ldl + row] = f[i].y * v[i].z;
      im[(kk + 1) * ldl + row] = f[i].y * v[i].w;
    }
  }
};

struct AdjHArgs {
  const float2* E;     // [stacks][nz][3][nx][ny] (the caller's fields)
  const float* g;      // [stacks][nz][nx][ny]
  const float2* AyH;   // [ny][np]
  float2* H;           // [chunk][nz][3][nxp][np]
  int s0, nstk, nz, nx, ny, nxp, np;
};

__global__ void __launch_bounds__(CfgAdj::NT, 2) adj_h_kernel(AdjHArgs a) {
  using Cfg = CfgAdj;
  extern __shared__ float lds[];
  const int tiles_m = a.nxp / Cfg::BM, tiles_n = a.np / Cfg::BN;
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
  ScaledRowLoader<Cfg> la;
  la.E = a.E + ((gs * a.nz + z) * 3 + c) * plane;
  la.g = a.g + (gs * a.nz + z) * plane;
  la.ld = a.ny;
  la.nrows = a.nx;
  la.row0 = tm * Cfg::BM;
  KMajorLoader<Cfg, Cfg::BN> lb;
  lb.src = a.AyH + tn * Cfg::BN;
  lb.ld = a.np;
  CgAcc<Cfg> acc;
  acc.zero();
  cg_mainloop<Cfg>(acc, la, lb, a.ny, lds, tid, wrow, wcol, lane);
  float2* H = a.H + (size_t)item * a.nxp * a.np;
#pragma unroll
  for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
    for (int jj = 0; jj < Cfg::TN; ++jj) {
      const int col = tn * Cfg::BN + cg_col(wcol, jj, lane);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = tm * Cfg::BM + cg_row(wrow, i, r, lane);
        H[(size_t)row * a.np + col] = make_float2(acc.re[i][jj][r], acc.im[i][jj][r]);
      }
    }
}

struct AdjGArgs {
  const float2* AxH;   // [nxp][np]
  const float2* H;     // [chunk][nz][3][nxp][np]
  const float2* P;     // [chunk][3][np][np]
  const double* ksz;   // [np][np]
  const double* z;     // [nz]
  float* partial;      // [stacks * 3 * zgroups][np][np]
  double zoff[kPupilStacks];
  int s0, nstk, nz, nx, nxp, np;
  int zgroups, zper;   // planes are split into zgroups runs of zper (the last may be shorter)
};

__global__ void __launch_bounds__(CfgAdj::NT, 2) adj_g_kernel(AdjGArgs a) {
  using Cfg = CfgAdj;
  extern __shared__ float lds[];
  const int tiles = a.np / Cfg::BM;
  const int nblocks = a.nstk * 3 * a.zgroups * tiles * tiles;
  int id = xcd_remap(blockIdx.x, nblocks);
  const int tn = id % tiles; id /= tiles;
  const int tm = id % tiles; id /= tiles;
  const int g = id % a.zgroups; id /= a.zgroups;
  const int c = id % 3, s = id / 3;
  const int z_begin = g * a.zper, z_end = min(a.nz, z_begin + a.zper);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wrow = (wave / Cfg::WAVES_N) * Cfg::WM, wcol = (wave % Cfg::WAVES_N) * Cfg::WN;
  const int row0 = tm * Cfg::BM, col0 = tn * Cfg::BN;
  const size_t npp = (size_t)a.np * a.np;
  const float2* P = a.P + ((size_t)s * 3 + c) * npp;
  float dphi[Cfg::TM][Cfg::TN][16];
#pragma unroll
  for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
    for (int jj = 0; jj < Cfg::TN; ++jj)
#pragma unroll
      for (int r = 0; r < 16; ++r) dphi[i][jj][r] = 0.f;
  const int K = (a.nx + Cfg::BK - 1) / Cfg::BK * Cfg::BK;   // H rows past nx are zero
#pragma unroll 1
  for (int z = z_begin; z < z_end; ++z) {
    KMajorLoader<Cfg, Cfg::BM> la;
    la.src = a.AxH + row0;
    la.ld = a.np;
    KMajorLoader<Cfg, Cfg::BN> lb;
    lb.src = a.H + ((size_t)(s * a.nz + z) * 3 + c) * a.nxp * a.np + col0;
    lb.ld = a.np;
    CgAcc<Cfg> acc;
    acc.zero();
    cg_mainloop<Cfg>(acc, la, lb, K, lds, tid, wrow, wcol, lane);
    const double zz = a.z[z] + a.zoff[s];
#pragma unroll
    for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
      for (int jj = 0; jj < Cfg::TN; ++jj) {
        const int col = col0 + cg_col(wcol, jj, lane);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = row0 + cg_row(wrow, i, r, lane);
          const size_t cell = (size_t)row * a.np + col;
          const float2 p = P[cell];
          float sn, cs;
          sincosf((float)reduce_2pi(a.ksz[cell] * zz), &sn, &cs);
          const float pr = p.x * cs - p.y * sn, pi = p.x * sn + p.y * cs;
          // Im(G conj(P~)) = Gi Pr - Gr Pi
          dphi[i][jj][r] += acc.im[i][jj][r] * pr - acc.re[i][jj][r] * pi;
        }
      }
  }
  float* out = a.partial + (((size_t)(a.s0 + s) * 3 + c) * a.zgroups + g) * npp;
#pragma unroll
  for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
    for (int jj = 0; jj < Cfg::TN; ++jj) {
      const int col = col0 + cg_col(wcol, jj, lane);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = row0 + cg_row(wrow, i, r, lane);
        out[(size_t)row * a.np + col] = dphi[i][jj][r];
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

// dL/dc_q = 2 pi sum_cells dL/dPhi Z_q: one workgroup per q, fixed-shape tree.
__global__ void __launch_bounds__(256) adj_zernike_kernel(const double* __restrict__ dphi,
                                                          const float* __restrict__ ztab, int nn,
                                                          float* __restrict__ dc) {
  __shared__ double red[256];
  const int q = blockIdx.x;
  double s = 0.0;
  for (int cell = threadIdx.x; cell < nn; cell += 256) s += dphi[cell] * (double)ztab[(size_t)q * nn + cell];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) dc[q] = (float)(kTwoPi * red[0]);
}

hipError_t adjoint_kernel_attributes() {
  hipError_t e = hipFuncSetAttribute((const void*)adj_h_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     CfgAdj::LDS_BYTES);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)adj_g_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                             CfgAdj::LDS_BYTES);
}

// Lazily built adjoint tables and workspace of a Fourier plan.
// Plane groups of adj_g: enough workgroups to fill the chip (>= 4 per CU of 256).
static int adjoint_zgroups(const rwpsf_plan* p) {
  const int tiles = p->np / CfgAdj::BM;
  const int per_group = kPupilStacks * 3 * tiles * tiles;
  return std::max(1, std::min(p->grid.nz, (1024 + per_group - 1) / per_group));
}

static int adjoint_prepare(rwpsf_plan* p, int n_stacks) {
  const int nx = p->grid.nx, ny = p->grid.ny, N = p->num.n_pupil, np = p->np;
  const int nxp = round_up(nx, 64);
  int st;
  if (!p->d_AxH) {
    const double s_max = p->s_max, k = p->k;
    const double pref = p->opt.focal_length * k / kTwoPi;
    std::vector<float2> AxH((size_t)nxp * np, make_float2(0.f, 0.f)), AyH((size_t)ny * np, make_float2(0.f, 0.f));
    for (int m = 0; m < nx; ++m)
      for (int j = 0; j < N; ++j) {
        const double sx = (2.0 * j + 1.0 - N) * s_max / N;
        const double ph = k * sx * (double)(m - nx / 2) * p->grid.dx_nm;
        // conj(-i pref e^{i ph}) = i pref e^{-i ph} = pref (sin ph + i cos ph)
        AxH[(size_t)m * np + j] = make_float2((float)(pref * std::sin(ph)), (float)(pref * std::cos(ph)));
      }
    for (int n = 0; n < ny; ++n)
      for (int l = 0; l < N; ++l) {
        const double sy = (2.0 * l + 1.0 - N) * s_max / N;
        const double ph = k * sy * (double)(n - ny / 2) * p->grid.dy_nm;
        AyH[(size_t)n * np + l] = make_float2((float)std::cos(ph), (float)(-std::sin(ph)));
      }
    if ((st = dev_alloc(p, &p->d_AxH, AxH.size()))) return st;
    if ((st = dev_alloc(p, &p->d_AyH, AyH.size()))) return st;
    if ((st = dev_alloc(p, &p->d_dphi, (size_t)N * N))) return st;
    if ((st = dev_alloc(p, &p->d_H, (size_t)kPupilStacks * p->grid.nz * 3 * nxp * np))) return st;
    if ((st = hip_check(hipMemcpy(p->d_AxH, AxH.data(), AxH.size() * sizeof(float2), hipMemcpyHostToDevice)))) return st;
    if ((st = hip_check(hipMemcpy(p->d_AyH, AyH.data(), AyH.size() * sizeof(float2), hipMemcpyHostToDevice)))) return st;
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
  const int nxp = round_up(nx, 64);
  const int zg = adjoint_zgroups(p);
  for (int b0 = 0; b0 < n; b0 += kPupilStacks) {
    const int nb = std::min(kPupilStacks, n - b0);
    if ((rc = fourier_build_pupils(p, s + b0, nb, st))) return rc;
    AdjHArgs ha{E, dLdI, p->d_AyH, p->d_H, b0, nb, nz, nx, ny, nxp, np};
    const int hblocks = nb * nz * 3 * (nxp / CfgAdj::BM) * (np / CfgAdj::BN);
    int tr = p->time_begin(RWPSF_KERNEL_ADJ_H, st);
    hipLaunchKernelGGL(adj_h_kernel, dim3(hblocks), dim3(CfgAdj::NT), CfgAdj::LDS_BYTES, st, ha);
    if ((rc = hip_check(hipGetLastError()))) return rc;
    p->time_end(tr, st);
    AdjGArgs ga{};
    ga.AxH = p->d_AxH;
    ga.H = p->d_H;
    ga.P = p->d_P;
    ga.ksz = p->d_ksz;
    ga.z = p->d_z;
    ga.partial = p->d_partial;
    for (int i = 0; i < nb; ++i) ga.zoff[i] = s[b0 + i].z_offset_nm;
    ga.s0 = b0;
    ga.nstk = nb;
    ga.nz = nz;
    ga.nx = nx;
    ga.nxp = nxp;
    ga.np = np;
    ga.zgroups = zg;
    ga.zper = (nz + zg - 1) / zg;
    const int t = np / CfgAdj::BM;
    tr = p->time_begin(RWPSF_KERNEL_ADJ_G, st);
    hipLaunchKernelGGL(adj_g_kernel, dim3(nb * 3 * zg * t * t), dim3(CfgAdj::NT), CfgAdj::LDS_BYTES, st, ga);
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
    hipLaunchKernelGGL(adj_zernike_kernel, dim3(n_zernike), dim3(256), 0, st, p->d_dphi, p->d_ztab, N * N, dc);
    if ((rc = hip_check(hipGetLastError()))) return rc;
  }
  p->time_end(tr, st);
  return RWPSF_OK;
}

}  // namespace rw
