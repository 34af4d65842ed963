// Batched emitters: the Fourier form (Sec. 3.3 eq. "cartesian vectorial" with the
// Sec. 3.4 correction factors) for thousands of emitters with individual sub-pixel
// position, axial position, Zernike vector (Sec. 3.4.2), crop size and plane count,
// in one persistent launch.
//
// Per emitter b the pupil phase is
//   Phi_b[j,l] = 2 pi sum_q c_bq Z_q(s) - k (s_x x0_b + s_y y0_b)
// formed for all emitters at once by one real GEMM on the matrix cores,
//   Phi[b][cell] = sum_k coef[k][b] basis[k][cell],  basis = (2 pi Z_1..Z_21, s_x, s_y).
// Each plane d of each field component c is then, with P~ = Q_c exp(i (Phi_b + k s_z z)),
//   U = Ax_S P~          (S x N, P~ generated in registers as the MFMA B operand)
//   E = U Ay_S^T         (S x S, U staged in LDS as the A operand)
// and I = sum_c |E_c|^2.  Ax_S / Ay_S are the rows of one 96-row DFT table that
// cover the crop (pixel i of an S-crop is table row i - S/2 + 32).  A workgroup
// takes whole emitters from an atomic counter over a cost-sorted (longest first)
// list until the list is exhausted; every workgroup exits when the counter passes n.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <numeric>
#include <vector>

#include "rw_common.h"
#include "rw_plan.h"

namespace rw {

hipError_t launch_rgemm(const float* A, int lda, const float* B, int ldb, float* C, int ldc, int M,
                        int N, int K, hipStream_t st);

typedef float f16v_t __attribute__((ext_vector_type(16)));

constexpr int kTabRows = 96;    // DFT table rows: x_r = (r - 32) * pixel
constexpr int kBasisRows = 32;  // 21 Zernike + s_x + s_y, zero-padded

struct BatchParam {
  double zoff;      // -z_e
  long long off;    // voxel offset of the emitter's output
  int S, D, SP, pad;
};

struct BatchArgs {
  const BatchParam* params;  // [n] cost-sorted
  const float2* Q;           // [3][N][N]
  const double* ksz;         // [N][N]
  const float* phi;          // [n][N*N], slot order
  const float2* AxT;         // [N][96]
  const float2* AyT;         // [N][96]
  float* I;
  float2* E;
  int* counter;
  int n, N;
  double pitch;
};

__global__ void batch_reset_kernel(int* counter) { *counter = 0; }

// MFMA 32x32x2 f32: A lane l -> A[l%32][l/32], B lane l -> B[l/32][l%32],
// C register r of lane l -> C[8(r/4) + 4(l/32) + r%4][l%32].
template <int SP>
__device__ __forceinline__ void batch_emitter(const BatchArgs& a, const BatchParam& bp, int slot,
                                              float* lds, int tid) {
  constexpr int TI = SP / 32;
  constexpr int LDU = SP + 1;
  const int lane = tid & 63, w = tid >> 6, h = lane >> 5, l32 = lane & 31;
  const int N = a.N, NN = N * N, S = bp.S;
  const int r0 = 32 - S / 2;
  const float* phi = a.phi + (size_t)slot * NN;
  float* Ure = lds;
  float* Uim = lds + N * LDU;
  for (int d = 0; d < bp.D; ++d) {
    const double z = (d - 0.5 * (bp.D - 1)) * a.pitch + bp.zoff;
    float isum64[16];   // SP = 64: this wave's 32x32 block of E, MFMA C layout
    float isum32[4];    // SP = 32: elements tid + 256 q of the 32x32 image
#pragma unroll
    for (int r = 0; r < 16; ++r) isum64[r] = 0.f;
#pragma unroll
    for (int q = 0; q < 4; ++q) isum32[q] = 0.f;
    for (int c = 0; c < 3; ++c) {
      const float2* Qc = a.Q + (size_t)c * NN;
      // ---- U[m][l] = sum_j Ax[r0 + m][j] P~[j][l], this wave's 32-column blocks of l
      for (int lb = w; lb < N / 32; lb += 4) {
        f16v_t ur[TI], ui[TI];
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            ur[i][r] = 0.f;
            ui[i][r] = 0.f;
          }
        const int l = 32 * lb + l32;
#pragma unroll 4
        for (int kp = 0; kp < N / 2; ++kp) {
          const int j = 2 * kp + h;
          const int cell = j * N + l;
          const float2 q = Qc[cell];
          float sn, cs;
          sincosf(phi[cell] + (float)reduce_2pi(a.ksz[cell] * z), &sn, &cs);
          const float br = q.x * cs - q.y * sn, bi = q.x * sn + q.y * cs;
#pragma unroll
          for (int i = 0; i < TI; ++i) {
            const float2 av = a.AxT[j * kTabRows + r0 + 32 * i + l32];
            ur[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(av.x, br, ur[i], 0, 0, 0);
            ui[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(av.x, bi, ui[i], 0, 0, 0);
          }
#pragma unroll
          for (int i = 0; i < TI; ++i) {
            const float2 av = a.AxT[j * kTabRows + r0 + 32 * i + l32];
            ur[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(-av.y, bi, ur[i], 0, 0, 0);
            ui[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(av.y, br, ui[i], 0, 0, 0);
          }
        }
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int m = 32 * i + 8 * (r >> 2) + 4 * h + (r & 3);
            Ure[l * LDU + m] = ur[i][r];
            Uim[l * LDU + m] = ui[i][r];
          }
      }
      __syncthreads();
      // ---- E[m][n] = sum_l U[m][l] Ay[r0 + n][l]
      f16v_t er, ei;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        er[r] = 0.f;
        ei[r] = 0.f;
      }
      const int mi = (SP == 64) ? (w >> 1) : 0, ni = (SP == 64) ? (w & 1) : 0;
      const int kp0 = (SP == 64) ? 0 : w * 16;               // SP = 32: K split over the waves
      const int kp1 = (SP == 64) ? N / 2 : min(N / 2, w * 16 + 16);
#pragma unroll 4
      for (int kp = kp0; kp < kp1; ++kp) {
        const int l = 2 * kp + h;
        const float ar = Ure[l * LDU + 32 * mi + l32], ai = Uim[l * LDU + 32 * mi + l32];
        const float2 b = a.AyT[l * kTabRows + r0 + 32 * ni + l32];
        er = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, b.x, er, 0, 0, 0);
        ei = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, b.y, ei, 0, 0, 0);
        er = __builtin_amdgcn_mfma_f32_32x32x2f32(-ai, b.y, er, 0, 0, 0);
        ei = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, b.x, ei, 0, 0, 0);
      }
      __syncthreads();   // U is consumed
      if (SP == 64) {
        float2* Ec = a.E ? a.E + 3 * bp.off + ((size_t)(d * 3 + c) * S) * S : nullptr;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int m = 32 * mi + 8 * (r >> 2) + 4 * h + (r & 3), n = 32 * ni + l32;
          isum64[r] += er[r] * er[r] + ei[r] * ei[r];
          if (Ec && m < S && n < S) Ec[m * S + n] = make_float2(er[r], ei[r]);
        }
      } else {
        // reduce the four K-partials through LDS (the U area is free now)
        float* pre = lds + w * 2 * 32 * 33;
        float* pim = pre + 32 * 33;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int m = 8 * (r >> 2) + 4 * h + (r & 3);
          pre[m * 33 + l32] = er[r];
          pim[m * 33 + l32] = ei[r];
        }
        __syncthreads();
        float2* Ec = a.E ? a.E + 3 * bp.off + ((size_t)(d * 3 + c) * S) * S : nullptr;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = tid + 256 * q, m = e >> 5, n = e & 31;
          float sr = 0.f, si = 0.f;
#pragma unroll
          for (int ww = 0; ww < 4; ++ww) {
            sr += lds[ww * 2 * 32 * 33 + m * 33 + n];
            si += lds[ww * 2 * 32 * 33 + 32 * 33 + m * 33 + n];
          }
          isum32[q] += sr * sr + si * si;
          if (Ec && m < S && n < S) Ec[m * S + n] = make_float2(sr, si);
        }
        __syncthreads();
      }
    }
    if (a.I) {
      float* Ip = a.I + bp.off + (size_t)d * S * S;
      if (SP == 64) {
        const int mi = w >> 1, ni = w & 1;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int m = 32 * mi + 8 * (r >> 2) + 4 * h + (r & 3), n = 32 * ni + l32;
          if (m < S && n < S) Ip[m * S + n] = isum64[r];
        }
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = tid + 256 * q, m = e >> 5, n = e & 31;
          if (m < S && n < S) Ip[m * S + n] = isum32[q];
        }
      }
    }
  }
}

constexpr int kBatchLdsBytes = 2 * 128 * 65 * 4;   // U for N <= 128, SP = 64

__global__ void __launch_bounds__(256, 2) batch_planes_kernel(BatchArgs a) {
  extern __shared__ float lds[];
  __shared__ int item;
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) item = atomicAdd(a.counter, 1);
    __syncthreads();
    const int slot = item;
    __syncthreads();
    if (slot >= a.n) break;
    const BatchParam bp = a.params[slot];
    if (bp.SP == 32)
      batch_emitter<32>(a, bp, slot, lds, tid);
    else
      batch_emitter<64>(a, bp, slot, lds, tid);
  }
}

}  // namespace rw

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
struct rwpsf_batch {
  int device = 0;
  rwpsf_optics opt{};
  int N = 0, max_emitters = 0, num_cus = 0;
  double px = 0, pitch = 0, k = 0, s_max = 0;
  std::vector<void*> allocations;
  float2* d_Q = nullptr;
  double* d_ksz = nullptr;
  float2* d_AxT = nullptr;
  float2* d_AyT = nullptr;
  float* d_basis = nullptr;
  float* d_phi = nullptr;
  char* d_upload = nullptr;     // params [max] then coefT [32][max_pad]
  int* d_counter = nullptr;
  char* h_staging = nullptr;    // pinned mirror of d_upload
  size_t upload_bytes = 0;
  int max_pad = 0;
  hipEvent_t upload_done = nullptr;
  bool upload_pending = false;
  rwpsf_batch_config cfg{2, 32};
  bool use_graph = false;
  hipGraphExec_t gexec = nullptr;
  struct Key {
    int n = -1;
    void* I = nullptr;
    void* E = nullptr;
    int wg = 0, small = 0;
    hipStream_t st = nullptr;
  } gkey;
  ~rwpsf_batch() {
    if (gexec) hipGraphExecDestroy(gexec);
    if (upload_done) hipEventDestroy(upload_done);
    if (h_staging) hipHostFree(h_staging);
    for (void* p : allocations) hipFree(p);
  }
};

namespace rw {

static int batch_validate(const rwpsf_batch* b, int n, const rwpsf_emitter* e) {
  if (!b || n < 1 || n > b->max_emitters || !e) return RWPSF_ERR_INVALID_ARG;
  for (int i = 0; i < n; ++i) {
    const rwpsf_emitter& x = e[i];
    if (!std::isfinite(x.x0_nm) || !std::isfinite(x.y0_nm) || !std::isfinite(x.z_nm))
      return RWPSF_ERR_INVALID_ARG;
    if (std::fabs(x.x0_nm) > 4 * b->px || std::fabs(x.y0_nm) > 4 * b->px) return RWPSF_ERR_INVALID_ARG;
    if (x.crop < 1 || x.crop > RWPSF_BATCH_MAX_CROP || x.planes < 1 || x.planes > 4096)
      return RWPSF_ERR_INVALID_ARG;
    for (int q = 0; q < RWPSF_BATCH_MAX_ZERNIKE; ++q)
      if (!std::isfinite(x.zernike_waves[q])) return RWPSF_ERR_INVALID_ARG;
  }
  return RWPSF_OK;
}

template <class T>
static int balloc(rwpsf_batch* b, T** p, size_t count) {
  void* d = nullptr;
  hipError_t e = hipMalloc(&d, std::max<size_t>(16, count * sizeof(T)));
  if (e != hipSuccess) {
    set_hip_error(e);
    return RWPSF_ERR_OOM;
  }
  b->allocations.push_back(d);
  *p = (T*)d;
  return RWPSF_OK;
}

// Fill the pinned staging area (cost-sorted params and the coefficient matrix).
static void batch_stage(rwpsf_batch* b, int n, const rwpsf_emitter* e) {
  std::vector<long long> off(n + 1, 0);
  for (int i = 0; i < n; ++i) off[i + 1] = off[i] + (long long)e[i].planes * e[i].crop * e[i].crop;
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  auto sp_of = [&](int i) { return e[i].crop <= b->cfg.small_tile_max_crop ? 32 : 64; };
  auto cost = [&](int i) { return (double)e[i].planes * sp_of(i) * (b->N + sp_of(i)); };
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost(x) > cost(y); });
  BatchParam* prm = (BatchParam*)b->h_staging;
  float* coefT = (float*)(b->h_staging + sizeof(BatchParam) * b->max_emitters);
  for (int slot = 0; slot < n; ++slot) {
    const int i = order[slot];
    prm[slot].zoff = -e[i].z_nm;
    prm[slot].off = off[i];
    prm[slot].S = e[i].crop;
    prm[slot].D = e[i].planes;
    prm[slot].SP = sp_of(i);
    prm[slot].pad = 0;
    for (int q = 0; q < kBasisRows; ++q) {
      double v = 0.0;
      if (q < RWPSF_BATCH_MAX_ZERNIKE) v = e[i].zernike_waves[q];
      else if (q == RWPSF_BATCH_MAX_ZERNIKE) v = -b->k * e[i].x0_nm;
      else if (q == RWPSF_BATCH_MAX_ZERNIKE + 1) v = -b->k * e[i].y0_nm;
      coefT[(size_t)q * b->max_pad + slot] = (float)v;
    }
  }
}

static int batch_enqueue(rwpsf_batch* b, int n, float* I, float2* E, hipStream_t st) {
  int rc;
  if ((rc = hip_check(hipMemcpyAsync(b->d_upload, b->h_staging, b->upload_bytes, hipMemcpyHostToDevice, st))))
    return rc;
  hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(1), 0, st, b->d_counter);
  if ((rc = hip_check(hipGetLastError()))) return rc;
  const float* coefT = (const float*)(b->d_upload + sizeof(BatchParam) * b->max_emitters);
  const int NN = b->N * b->N;
  if ((rc = hip_check(launch_rgemm(coefT, b->max_pad, b->d_basis, NN, b->d_phi, NN, n, NN, kBasisRows, st))))
    return rc;
  BatchArgs a{};
  a.params = (const BatchParam*)b->d_upload;
  a.Q = b->d_Q;
  a.ksz = b->d_ksz;
  a.phi = b->d_phi;
  a.AxT = b->d_AxT;
  a.AyT = b->d_AyT;
  a.I = I;
  a.E = E;
  a.counter = b->d_counter;
  a.n = n;
  a.N = b->N;
  a.pitch = b->pitch;
  const int grid = std::max(1, std::min(n, b->num_cus * b->cfg.wg_per_cu));
  hipLaunchKernelGGL(batch_planes_kernel, dim3(grid), dim3(256), kBatchLdsBytes, st, a);
  return hip_check(hipGetLastError());
}

}  // namespace rw

extern "C" {

int rwpsf_batch_offsets(int n, const rwpsf_emitter* e, int64_t* off) {
  if (n < 0 || (n > 0 && !e) || !off) return RWPSF_ERR_INVALID_ARG;
  off[0] = 0;
  for (int i = 0; i < n; ++i) {
    if (e[i].crop < 1 || e[i].planes < 1) return RWPSF_ERR_INVALID_ARG;
    off[i + 1] = off[i] + (int64_t)e[i].planes * e[i].crop * e[i].crop;
  }
  return RWPSF_OK;
}

int rwpsf_batch_create(const rwpsf_optics* o, int n_pupil, double pixel_nm, double pitch_nm,
                       int max_emitters, rwpsf_batch** out) {
  using namespace rw;
  if (!out) return RWPSF_ERR_INVALID_ARG;
  *out = nullptr;
  double zero = 0.0;
  rwpsf_grid g{1, 1, 1.0, 1.0, 1, &zero};
  rwpsf_numerics nm{RWPSF_FORM_FOURIER, n_pupil, 2, 8};
  int st = validate_plan(o, &g, &nm);
  if (st != RWPSF_OK) return st;
  if (o->gibson_lanni) return RWPSF_ERR_UNSUPPORTED;
  if (n_pupil < 32 || n_pupil > 128 || n_pupil % 32 != 0) return RWPSF_ERR_INVALID_ARG;
  if (!(pixel_nm > 0) || !std::isfinite(pixel_nm) || !(pitch_nm >= 0) || !std::isfinite(pitch_nm))
    return RWPSF_ERR_INVALID_ARG;
  if (max_emitters < 1 || max_emitters > (1 << 20)) return RWPSF_ERR_INVALID_ARG;
  int dev_count = 0;
  if (hipGetDeviceCount(&dev_count) != hipSuccess || dev_count < 1) return RWPSF_ERR_NO_DEVICE;
  rwpsf_batch* b = new (std::nothrow) rwpsf_batch();
  if (!b) return RWPSF_ERR_OOM;
  hipGetDevice(&b->device);
  hipDeviceGetAttribute(&b->num_cus, hipDeviceAttributeMultiprocessorCount, b->device);
  b->opt = *o;
  b->N = n_pupil;
  b->px = pixel_nm;
  b->pitch = pitch_nm;
  b->max_emitters = max_emitters;
  b->k = kTwoPi * o->n_i / o->wavelength_nm;
  b->s_max = o->na / o->n_i;
  const int N = n_pupil;
  const size_t NN = (size_t)N * N;
  const std::complex<double> ex(o->ex_re, o->ex_im), ey(o->ey_re, o->ey_im);
  std::vector<float2> Q(3 * NN, make_float2(0.f, 0.f));
  std::vector<double> ksz(NN, 0.0);
  std::vector<float> basis((size_t)kBasisRows * NN, 0.f);
  const double ds = 2.0 * b->s_max / N;
  for (int j = 0; j < N; ++j)
    for (int l = 0; l < N; ++l) {
      const long u = 2L * j + 1 - N, v = 2L * l + 1 - N;
      const size_t cell = (size_t)j * N + l;
      const double sx = u * b->s_max / N, sy = v * b->s_max / N;
      basis[(size_t)RWPSF_BATCH_MAX_ZERNIKE * NN + cell] = (float)sx;
      basis[(size_t)(RWPSF_BATCH_MAX_ZERNIKE + 1) * NN + cell] = (float)sy;
      const double ru = (double)u / N, rv = (double)v / N, r = std::sqrt(ru * ru + rv * rv);
      for (int q = 0; q < RWPSF_BATCH_MAX_ZERNIKE; ++q)
        basis[(size_t)q * NN + cell] =
            (float)(kTwoPi * zernike_noll(q + 1, r, r > 0 ? ru / r : 1.0, r > 0 ? rv / r : 0.0));
      if (u * u + v * v > (long)N * N) continue;
      const double s2 = sx * sx + sy * sy;
      const double sin_t = std::sqrt(s2), cos_t = std::sqrt(1.0 - s2);
      const double cp = sin_t > 0 ? sx / sin_t : 1.0, sp = sin_t > 0 ? sy / sin_t : 0.0;
      std::complex<double> e[3];
      far_field(ex, ey, cos_t, sin_t, cp, sp, e);
      const double w = ds * ds * amplitude(*o, cos_t, sin_t) / cos_t;
      for (int c = 0; c < 3; ++c) Q[c * NN + cell] = make_float2((float)(w * e[c].real()), (float)(w * e[c].imag()));
      ksz[cell] = b->k * cos_t;
    }
  std::vector<float2> AxT((size_t)N * kTabRows), AyT((size_t)N * kTabRows);
  const double pref = o->focal_length * b->k / kTwoPi;
  for (int j = 0; j < N; ++j) {
    const double s = (2.0 * j + 1.0 - N) * b->s_max / N;
    for (int r = 0; r < kTabRows; ++r) {
      const double x = (r - 32) * pixel_nm;
      const double ph = b->k * s * x;
      AxT[(size_t)j * kTabRows + r] = make_float2((float)(pref * std::sin(ph)), (float)(-pref * std::cos(ph)));
      AyT[(size_t)j * kTabRows + r] = make_float2((float)std::cos(ph), (float)std::sin(ph));
    }
  }
  b->max_pad = (max_emitters + 63) / 64 * 64;
  b->upload_bytes = sizeof(BatchParam) * max_emitters + sizeof(float) * kBasisRows * b->max_pad;
  int rc;
  if ((rc = balloc(b, &b->d_Q, 3 * NN)) || (rc = balloc(b, &b->d_ksz, NN)) ||
      (rc = balloc(b, &b->d_AxT, (size_t)N * kTabRows)) || (rc = balloc(b, &b->d_AyT, (size_t)N * kTabRows)) ||
      (rc = balloc(b, &b->d_basis, (size_t)kBasisRows * NN)) ||
      (rc = balloc(b, &b->d_phi, (size_t)max_emitters * NN)) || (rc = balloc(b, &b->d_upload, b->upload_bytes)) ||
      (rc = balloc(b, &b->d_counter, 1))) {
    delete b;
    return rc;
  }
  if (hipHostMalloc((void**)&b->h_staging, b->upload_bytes, hipHostMallocDefault) != hipSuccess) {
    b->h_staging = nullptr;
    delete b;
    return RWPSF_ERR_OOM;
  }
  std::memset(b->h_staging, 0, b->upload_bytes);
  if ((rc = hip_check(hipEventCreateWithFlags(&b->upload_done, hipEventDisableTiming))) ||
      (rc = hip_check(hipMemcpy(b->d_Q, Q.data(), Q.size() * sizeof(float2), hipMemcpyHostToDevice))) ||
      (rc = hip_check(hipMemcpy(b->d_ksz, ksz.data(), ksz.size() * sizeof(double), hipMemcpyHostToDevice))) ||
      (rc = hip_check(hipMemcpy(b->d_AxT, AxT.data(), AxT.size() * sizeof(float2), hipMemcpyHostToDevice))) ||
      (rc = hip_check(hipMemcpy(b->d_AyT, AyT.data(), AyT.size() * sizeof(float2), hipMemcpyHostToDevice))) ||
      (rc = hip_check(hipMemcpy(b->d_basis, basis.data(), basis.size() * sizeof(float), hipMemcpyHostToDevice))) ||
      (rc = hip_check(hipMemcpy(b->d_upload, b->h_staging, b->upload_bytes, hipMemcpyHostToDevice))) ||
      (rc = hip_check(hipFuncSetAttribute((const void*)batch_planes_kernel,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, kBatchLdsBytes))) ||
      (rc = hip_check(hipDeviceSynchronize()))) {
    delete b;
    return rc;
  }
  *out = b;
  return RWPSF_OK;
}

void rwpsf_batch_destroy(rwpsf_batch* b) {
  if (!b) return;
  int cur = 0;
  hipGetDevice(&cur);
  hipSetDevice(b->device);
  hipDeviceSynchronize();
  delete b;
  hipSetDevice(cur);
}

int rwpsf_batch_set_graph(rwpsf_batch* b, int enable) {
  if (!b) return RWPSF_ERR_INVALID_ARG;
  b->use_graph = enable != 0;
  return RWPSF_OK;
}

int rwpsf_batch_set_config(rwpsf_batch* b, const rwpsf_batch_config* c) {
  if (!b || !c || c->wg_per_cu < 1 || c->wg_per_cu > 4 ||
      (c->small_tile_max_crop != 0 && c->small_tile_max_crop != 32))
    return RWPSF_ERR_INVALID_ARG;
  b->cfg = *c;
  return RWPSF_OK;
}

int rwpsf_batch_get_config(const rwpsf_batch* b, rwpsf_batch_config* c) {
  if (!b || !c) return RWPSF_ERR_INVALID_ARG;
  *c = b->cfg;
  return RWPSF_OK;
}

int rwpsf_batch_compute(rwpsf_batch* b, int n, const rwpsf_emitter* e, float* I, void* E, void* stream) {
  using namespace rw;
  int rc = batch_validate(b, n, e);
  if (rc) return rc;
  if (!I && !E) return RWPSF_ERR_INVALID_ARG;
  int cur = -1;
  hipGetDevice(&cur);
  if (cur != b->device) return RWPSF_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  if (b->use_graph && !st) return RWPSF_ERR_INVALID_ARG;   // the legacy default stream cannot be captured
  // the previous upload must have left the pinned staging area before it is rewritten
  if (b->upload_pending && (rc = hip_check(hipEventSynchronize(b->upload_done)))) return rc;
  batch_stage(b, n, e);
  if (!b->use_graph) {
    rc = batch_enqueue(b, n, I, (float2*)E, st);
  } else {
    const bool same = b->gexec && b->gkey.n == n && b->gkey.I == I && b->gkey.E == E &&
                      b->gkey.wg == b->cfg.wg_per_cu && b->gkey.small == b->cfg.small_tile_max_crop &&
                      b->gkey.st == st;
    if (!same) {
      if (b->gexec) {
        hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
      }
      hipGraph_t g = nullptr;
      if ((rc = hip_check(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal)))) return rc;
      const int erc = batch_enqueue(b, n, I, (float2*)E, st);
      hipError_t ce = hipStreamEndCapture(st, &g);
      if (erc) {
        if (g) hipGraphDestroy(g);
        return erc;
      }
      if ((rc = hip_check(ce))) return rc;
      ce = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
      hipGraphDestroy(g);
      if ((rc = hip_check(ce))) return rc;
      b->gkey = {n, I, E, b->cfg.wg_per_cu, b->cfg.small_tile_max_crop, st};
    }
    rc = hip_check(hipGraphLaunch(b->gexec, st));
  }
  if (rc) return rc;
  if ((rc = hip_check(hipEventRecord(b->upload_done, st)))) return rc;
  b->upload_pending = true;
  return RWPSF_OK;
}

}  // extern "C"

namespace rw {

// Autotune cache: a flat JSON object {"key": [wg_per_cu, small_tile_max_crop, ms], ...}
// in the file named by RWPSF_AUTOTUNE_CACHE.  Anything that does not parse is ignored
// (and replaced on the next write).
static std::string tune_key(const rwpsf_batch* b, int n, const rwpsf_emitter* e) {
  int small = 0, large = 0;
  long long planes = 0;
  for (int i = 0; i < n; ++i) {
    (e[i].crop <= 32 ? small : large) += 1;
    planes += e[i].planes;
  }
  int nb = 1;
  while (nb < n) nb <<= 1;
  char buf[160];
  snprintf(buf, sizeof buf, "N%d_n%d_small%d_large%d_meanD%lld_cus%d", b->N, nb, (int)(16.0 * small / n),
           (int)(16.0 * large / n), planes / n, b->num_cus);
  return buf;
}

static std::map<std::string, std::pair<rwpsf_batch_config, double>> cache_read(const char* path) {
  std::map<std::string, std::pair<rwpsf_batch_config, double>> m;
  FILE* f = fopen(path, "r");
  if (!f) return m;
  std::string text;
  char chunk[4096];
  size_t got;
  while ((got = fread(chunk, 1, sizeof chunk, f)) > 0) text.append(chunk, got);
  fclose(f);
  size_t pos = text.find('{');
  if (pos == std::string::npos) return {};
  while (true) {
    const size_t k0 = text.find('"', pos);
    if (k0 == std::string::npos) break;
    const size_t k1 = text.find('"', k0 + 1);
    if (k1 == std::string::npos) return {};
    const size_t b0 = text.find('[', k1);
    const size_t b1 = text.find(']', b0 == std::string::npos ? k1 : b0);
    if (b0 == std::string::npos || b1 == std::string::npos) return {};
    int wg = 0, sm = 0;
    double ms = 0;
    if (sscanf(text.c_str() + b0, "[%d ,%d ,%lf]", &wg, &sm, &ms) != 3 &&
        sscanf(text.c_str() + b0, "[%d, %d, %lf]", &wg, &sm, &ms) != 3)
      return {};
    if (wg < 1 || wg > 4 || (sm != 0 && sm != 32)) return {};
    m[text.substr(k0 + 1, k1 - k0 - 1)] = {rwpsf_batch_config{wg, sm}, ms};
    pos = b1 + 1;
  }
  return m;
}

static void cache_write(const char* path, const std::map<std::string, std::pair<rwpsf_batch_config, double>>& m) {
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return;
  fprintf(f, "{\n");
  size_t i = 0;
  for (const auto& kv : m)
    fprintf(f, "  \"%s\": [%d, %d, %.6f]%s\n", kv.first.c_str(), kv.second.first.wg_per_cu,
            kv.second.first.small_tile_max_crop, kv.second.second, ++i < m.size() ? "," : "");
  fprintf(f, "}\n");
  fclose(f);
  rename(tmp.c_str(), path);
}

}  // namespace rw

extern "C" {

int rwpsf_batch_autotune(rwpsf_batch* b, int n, const rwpsf_emitter* e, float* I, void* stream,
                         rwpsf_batch_config* best_out, double* best_ms) {
  using namespace rw;
  int rc = batch_validate(b, n, e);
  if (rc) return rc;
  if (!I) return RWPSF_ERR_INVALID_ARG;
  const char* cache_path = getenv("RWPSF_AUTOTUNE_CACHE");
  std::string key;
  std::map<std::string, std::pair<rwpsf_batch_config, double>> cache;
  if (cache_path && *cache_path) {
    key = tune_key(b, n, e);
    cache = cache_read(cache_path);
    auto it = cache.find(key);
    if (it != cache.end()) {
      b->cfg = it->second.first;
      if (best_out) *best_out = it->second.first;
      if (best_ms) *best_ms = it->second.second;
      return RWPSF_OK;
    }
  }
  hipStream_t st = (hipStream_t)stream;
  const rwpsf_batch_config saved = b->cfg;
  const bool saved_graph = b->use_graph;
  b->use_graph = false;
  hipEvent_t t0, t1;
  hipEventCreate(&t0);
  hipEventCreate(&t1);
  rwpsf_batch_config best = saved;
  float best_t = 1e30f;
  const int wgs[3] = {1, 2, 3};
  const int smalls[2] = {0, 32};
  for (int wi = 0; wi < 3; ++wi)
    for (int si = 0; si < 2; ++si) {
      b->cfg = {wgs[wi], smalls[si]};
      if ((rc = rwpsf_batch_compute(b, n, e, I, nullptr, st))) break;   // warm-up
      hipEventRecord(t0, st);
      for (int r = 0; r < 2 && !rc; ++r) rc = rwpsf_batch_compute(b, n, e, I, nullptr, st);
      hipEventRecord(t1, st);
      if (rc) break;
      hipEventSynchronize(t1);
      float ms = 0.f;
      hipEventElapsedTime(&ms, t0, t1);
      ms *= 0.5f;
      if (ms < best_t) {
        best_t = ms;
        best = b->cfg;
      }
    }
  hipEventDestroy(t0);
  hipEventDestroy(t1);
  b->use_graph = saved_graph;
  b->cfg = rc ? saved : best;
  if (rc) return rc;
  if (best_out) *best_out = best;
  if (best_ms) *best_ms = best_t;
  if (cache_path && *cache_path) {
    cache[key] = {best, best_t};
    cache_write(cache_path, cache);
  }
  return RWPSF_OK;
}

}  // extern "C"
