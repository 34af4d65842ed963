// Learned surrogate of the PSF engine: (21 Noll coefficients, z) -> 64 x 64 intensity.
//
//   x  = (c / 0.05, z / 1000 nm)                                   22 features
//   h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2), h3 = relu(h2 W3 + b3)   256, 1024, 2048
//   d1 = relu(T(h3 as 32x8x8; K1) + c1)    16 x 16 x 16
//   d2 = relu(T(d1; K2) + c2)              8 x 32 x 32
//   y  = T(d2; K3) + c3                    64 x 64
// T: stride-2 transposed convolution, 4 x 4 kernel, 1 pixel padding,
//   out[co, oy, ox] = sum_{ci,ky,kx} in[ci, iy, ix] K[ci, co, ky, kx], oy = 2 iy - 1 + ky.
//
// Dense layers run on the BF16 matrix cores (v_mfma_f32_32x32x16_bf16, FP32
// accumulate).  In the accurate mode every operand is split x = hi + lo with hi,
// lo in BF16 and the product is hi*hi + hi*lo + lo*hi (relative error ~1e-5); the
// fast mode uses hi*hi only.  Transposed convolutions are direct FP32 kernels: the
// forward computes all output channels of one pixel per thread with the weights read
// as wave-uniform scalars; the backward kernels stage a sample in LDS.  Weight gradients of the convolutions
// and all bias gradients are reduced over the batch in a fixed order through
// per-chunk partial sums; training updates FP32 master weights with Adam.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "rw_common.h"
#include "rw_plan.h"

namespace rw {

typedef float f16v_s __attribute__((ext_vector_type(16)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------- dense GEMM
// C[M][N] = op(A) op(B) (+ bias[n]) (relu), op(A)[m][k] = TA ? A[k lda + m] : A[m lda + k],
// op(B)[k][n] = TB ? B[n ldb + k] : B[k ldb + n].  Workgroup 64 x 64, 4 waves of 32 x 32,
// k-stage 32 staged in LDS as FP32 ([row][k], k contiguous), split to BF16 at the MFMA.
constexpr int SBM = 64, SBN = 64, SBK = 32, SLD = SBK + 4;

template <bool TA, bool TB, int NSPLIT>
__global__ void __launch_bounds__(256) sg_gemm_kernel(const float* __restrict__ A, int lda,
                                                      const float* __restrict__ B, int ldb,
                                                      float* __restrict__ C, int ldc, int M, int N, int K,
                                                      const float* __restrict__ bias, int relu) {
  __shared__ float As[SBM * SLD];
  __shared__ float Bs[SBN * SLD];
  const int tiles_n = (N + SBN - 1) / SBN;
  const int tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int row0 = tm * SBM, col0 = tn * SBN;
  f16v_s acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.f;
  for (int k0 = 0; k0 < K; k0 += SBK) {
    // stage: 64 x 32 of A and of B, 8 elements per thread each, branch-free bounds
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int e = tid + 256 * i;
      int r, kk;
      if (TA) { kk = e / SBM; r = e % SBM; } else { r = e / SBK; kk = e % SBK; }
      const int gm = row0 + r, gk = k0 + kk;
      const int cm = min(gm, M - 1), ck = min(gk, K - 1);
      const float v = TA ? A[(size_t)ck * lda + cm] : A[(size_t)cm * lda + ck];
      As[r * SLD + kk] = (gm < M && gk < K) ? v : 0.f;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int e = tid + 256 * i;
      int c, kk;
      if (TB) { c = e / SBK; kk = e % SBK; } else { kk = e / SBN; c = e % SBN; }
      const int gn = col0 + c, gk = k0 + kk;
      const int cn = min(gn, N - 1), ck = min(gk, K - 1);
      const float v = TB ? B[(size_t)cn * ldb + ck] : B[(size_t)ck * ldb + cn];
      Bs[c * SLD + kk] = (gn < N && gk < K) ? v : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < SBK; ks += 16) {
      const int kb = ks + 8 * (lane >> 5);
      const float* ap = As + (wm + (lane & 31)) * SLD + kb;
      const float* bp = Bs + (wn + (lane & 31)) * SLD + kb;
      bf8_t ahi, alo, bhi, blo;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const float a = ap[q], b = bp[q];
        ahi[q] = (__bf16)a;
        bhi[q] = (__bf16)b;
        alo[q] = (__bf16)(a - (float)ahi[q]);
        blo[q] = (__bf16)(b - (float)bhi[q]);
      }
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, bhi, acc, 0, 0, 0);
      if (NSPLIT > 1) {
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, blo, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo, bhi, acc, 0, 0, 0);
      }
    }
    __syncthreads();
  }
  const int n = col0 + wn + (lane & 31);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int m = row0 + wm + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    if (m < M && n < N) {
      float v = acc[r] + (bias ? bias[n] : 0.f);
      if (relu) v = fmaxf(v, 0.f);
      C[(size_t)m * ldc + n] = v;
    }
  }
}

template <bool TA, bool TB>
static hipError_t sg_gemm(const float* A, int lda, const float* B, int ldb, float* C, int ldc, int M, int N,
                          int K, const float* bias, int relu, int nsplit, hipStream_t st) {
  const dim3 grid(((M + SBM - 1) / SBM) * ((N + SBN - 1) / SBN));
  if (nsplit > 1)
    hipLaunchKernelGGL((sg_gemm_kernel<TA, TB, 3>), grid, dim3(256), 0, st, A, lda, B, ldb, C, ldc, M, N, K,
                       bias, relu);
  else
    hipLaunchKernelGGL((sg_gemm_kernel<TA, TB, 1>), grid, dim3(256), 0, st, A, lda, B, ldb, C, ldc, M, N, K,
                       bias, relu);
  return hipGetLastError();
}

// ---------------------------------------------------------------- dense GEMM, aligned fast path
// C[M][N] = relu(A B + bias) for K % 32 == 0 and N % 128 == 0 (the 256 -> 1024 and
// 1024 -> 2048 layers).  A is FP32 [M][K], split into BF16 hi / lo while it is staged;
// B is given pre-split as k-contiguous BF16 planes Bt_hi / Bt_lo [N][K].  Workgroup
// 128 x 128, 4 waves of 64 x 64 (2 x 2 MFMA blocks of 32 x 32 x 16), k-stage 32, two LDS
// stages; each lane reads its 8 consecutive k of an operand with one 16-byte LDS read.
constexpr int FBM = 128, FBN = 128, FBK = 32, FLD = FBK + 8;   // LDS row: 40 bf16 (80 B)
typedef __bf16 bf4_t __attribute__((ext_vector_type(4)));

// W [K][N] FP32 -> Bt_hi / Bt_lo [N][K] BF16 (hi = bf16(w), lo = bf16(w - hi))
__global__ void sg_wsplit_kernel(const float* __restrict__ W, int K, int N, __bf16* __restrict__ hi,
                                 __bf16* __restrict__ lo) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K * N) return;
  const int k = i / N, n = i % N;
  const float w = W[i];
  const __bf16 h = (__bf16)w;
  hi[(size_t)n * K + k] = h;
  lo[(size_t)n * K + k] = (__bf16)(w - (float)h);
}

template <int NSPLIT>
__global__ void __launch_bounds__(256, 2) sg_gemm_fast_kernel(const float* __restrict__ A,
                                                              const __bf16* __restrict__ Bhi,
                                                              const __bf16* __restrict__ Blo,
                                                              float* __restrict__ C, int M, int N, int K,
                                                              const float* __restrict__ bias, int relu) {
  constexpr int PL = FBM * FLD;             // one bf16 plane of a tile
  constexpr int STAGE = 4 * PL;             // A hi, A lo, B hi, B lo
  extern __shared__ __bf16 shb[];
  const int tiles_n = N / FBN;
  const int tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int row0 = tm * FBM, col0 = tn * FBN;
  f16v_s acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
  // A: 128 rows x 32 k = 1024 float4, 4 per thread; B: 128 cols x 32 k bf16 = 512 x 16 B per plane
  struct Staged {
    float4 ra[4];
    uint4 rbh[2], rbl[2];
  };
  // the staged tile is returned by value, so that it stays in registers
  auto load = [&](int k0) {
    Staged g;
    float4* ra = g.ra;
    uint4* rbh = g.rbh;
    uint4* rbl = g.rbl;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int idx = tid + 256 * i, r = idx >> 3, kq = 4 * (idx & 7);
      const int gr = min(row0 + r, M - 1);   // rows past M are computed but not stored
      ra[i] = *reinterpret_cast<const float4*>(A + (size_t)gr * K + k0 + kq);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int idx = tid + 256 * i, c = idx >> 2, k8 = 8 * (idx & 3);
      rbh[i] = *reinterpret_cast<const uint4*>(Bhi + (size_t)(col0 + c) * K + k0 + k8);
      if (NSPLIT > 1) rbl[i] = *reinterpret_cast<const uint4*>(Blo + (size_t)(col0 + c) * K + k0 + k8);
    }
    return g;
  };
  auto store = [&](__bf16* st, const Staged& g) {
    const float4* ra = g.ra;
    const uint4* rbh = g.rbh;
    const uint4* rbl = g.rbl;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int idx = tid + 256 * i, r = idx >> 3, kq = 4 * (idx & 7);
      const float v[4] = {ra[i].x, ra[i].y, ra[i].z, ra[i].w};
      bf4_t h, l;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        h[t] = (__bf16)v[t];
        l[t] = (__bf16)(v[t] - (float)h[t]);
      }
      *reinterpret_cast<bf4_t*>(st + r * FLD + kq) = h;
      if (NSPLIT > 1) *reinterpret_cast<bf4_t*>(st + PL + r * FLD + kq) = l;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int idx = tid + 256 * i, c = idx >> 2, k8 = 8 * (idx & 3);
      *reinterpret_cast<uint4*>(st + 2 * PL + c * FLD + k8) = rbh[i];
      if (NSPLIT > 1) *reinterpret_cast<uint4*>(st + 3 * PL + c * FLD + k8) = rbl[i];
    }
  };
  const int KT = K / FBK;
  auto mma = [&](const __bf16* cur) {
#pragma unroll
    for (int ks = 0; ks < FBK; ks += 16) {
      const int kb = ks + 8 * (lane >> 5);
      bf8_t ah[2], al[2], bh[2], bl[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int r = (wm + 32 * i + (lane & 31)) * FLD + kb;
        ah[i] = *reinterpret_cast<const bf8_t*>(cur + r);
        if (NSPLIT > 1) al[i] = *reinterpret_cast<const bf8_t*>(cur + PL + r);
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int c = (wn + 32 * j + (lane & 31)) * FLD + kb;
        bh[j] = *reinterpret_cast<const bf8_t*>(cur + 2 * PL + c);
        if (NSPLIT > 1) bl[j] = *reinterpret_cast<const bf8_t*>(cur + 3 * PL + c);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
          if (NSPLIT > 1) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
          }
        }
    }
  };
  store(shb, load(0));
  __syncthreads();
  // the last stage is peeled, so that no branch surrounds the loads and stores
  for (int kt = 0; kt < KT - 1; ++kt) {
    const Staged g = load((kt + 1) * FBK);
    mma(shb + (kt & 1) * STAGE);
    store(shb + ((kt + 1) & 1) * STAGE, g);
    __syncthreads();
  }
  mma(shb + ((KT - 1) & 1) * STAGE);
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int n = col0 + wn + 32 * j + (lane & 31);
    const float bn = bias ? bias[n] : 0.f;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = row0 + wm + 32 * i + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (m < M) {
          float v = acc[i][j][r] + bn;
          if (relu) v = fmaxf(v, 0.f);
          C[(size_t)m * N + n] = v;
        }
      }
  }
}

static hipError_t sg_gemm_fast(const float* A, const __bf16* Bh, const __bf16* Bl, float* C, int M, int N, int K,
                               const float* bias, int nsplit, hipStream_t st) {
  const dim3 grid(((M + FBM - 1) / FBM) * (N / FBN));
  const int lds = 2 * 4 * FBM * FLD * (int)sizeof(__bf16);
  if (nsplit > 1)
    hipLaunchKernelGGL(sg_gemm_fast_kernel<3>, grid, dim3(256), lds, st, A, Bh, Bl, C, M, N, K, bias, 1);
  else
    hipLaunchKernelGGL(sg_gemm_fast_kernel<1>, grid, dim3(256), lds, st, A, Bh, Bl, C, M, N, K, bias, 1);
  return hipGetLastError();
}

// ---------------------------------------------------------------- elementwise
__global__ void sg_features_kernel(const float* __restrict__ coef, const float* __restrict__ z, int B,
                                   float* __restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B * 22) return;
  const int b = i / 22, f = i % 22;
  x[i] = f < 21 ? coef[b * 21 + f] * (1.f / 0.05f) : z[b] * (1.f / 1000.f);
}

// g *= (h > 0): derivative of relu through its output
__global__ void sg_relu_mask_kernel(float* __restrict__ g, const float* __restrict__ h, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) g[i] = h[i] > 0.f ? g[i] : 0.f;
}

// dY = 2 (y - t) / n and per-block partial sums of (y - t)^2
__global__ void __launch_bounds__(256) sg_mse_kernel(const float* __restrict__ y, const float* __restrict__ t,
                                                      size_t n, float* __restrict__ dy,
                                                      double* __restrict__ partial) {
  __shared__ double red[256];
  double s = 0.0;
  const float scale = 2.f / (float)n;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const float r = y[i] - t[i];
    dy[i] = scale * r;
    s += (double)r * r;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void sg_sum_kernel(const double* __restrict__ partial, int n, double inv, float* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += partial[i];
    out[0] = (float)(s * inv);
  }
}

// column sums of g [rows][cols] in row order, per column (bias gradients of dense layers)
__global__ void sg_colsum_kernel(const float* __restrict__ g, int rows, int cols, float* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  double s = 0.0;
  for (int r = 0; r < rows; ++r) s += g[(size_t)r * cols + c];
  out[c] = (float)s;
}

// ---------------------------------------------------------------- transposed convolution
// Weights re-laid for the forward kernel: Kt[ky][kx][ci][co] = K[ci][co][ky][kx].
__global__ void sg_deconv_wt_kernel(const float* __restrict__ K, int Ci, int Co, float* __restrict__ Kt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Ci * Co * 16) return;
  const int ci = i / (Co * 16), co = (i / 16) % Co, ky = (i / 4) % 4, kx = i % 4;
  Kt[((ky * 4 + kx) * Ci + ci) * Co + co] = K[i];
}

// Forward transposed convolution, one output pixel (all Co channels) per thread (used
// for the 32 -> 16 channel layer, where a 2 x 2 block would need 4 Co accumulators and
// too many scalar weights per step).  Output (oy, ox) = (2 iy + py, 2 ix + px): the taps
// of parity p are (iy, ky = 1), (iy - 1, ky = 3) for p = 0 and (iy + 1, ky = 0),
// (iy, ky = 2) for p = 1.  A workgroup covers 256 pixels of one sample ordered by parity
// class (4 classes of H x H), so the class -- and every weight address -- is the same
// across a wave (H * H >= 64) and the weights are read as scalars.
template <int Ci, int Co, int H>
__global__ void __launch_bounds__(256) sg_deconv_fwd_pix_kernel(const float* __restrict__ in,
                                                                const float* __restrict__ Kt,
                                                                const float* __restrict__ bias, int relu,
                                                                float* __restrict__ out) {
  static_assert(H * H >= 64 && (4 * H * H) % 256 == 0, "parity class uniform per wave");
  constexpr int BPS = 4 * H * H / 256;   // workgroups per sample
  const int b = blockIdx.x / BPS;
  const int pix = (blockIdx.x % BPS) * 256 + threadIdx.x;
  const int cls = __builtin_amdgcn_readfirstlane(pix / (H * H));
  const int q = pix % (H * H), iy = q / H, ix = q % H;
  const int py = cls >> 1, px = cls & 1;
  const float* x = in + (size_t)b * Ci * H * H;
  float acc[Co];
#pragma unroll
  for (int co = 0; co < Co; ++co) acc[co] = bias[co];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const int yy = py ? iy + 1 - a : iy - a, ky = py ? 2 * a : 1 + 2 * a;
    if (yy < 0 || yy >= H) continue;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int xx = px ? ix + 1 - c : ix - c, kx = px ? 2 * c : 1 + 2 * c;
      if (xx < 0 || xx >= H) continue;
      const float* w = Kt + (ky * 4 + kx) * Ci * Co;
      const float* xp = x + yy * H + xx;
#pragma unroll 4
      for (int ci = 0; ci < Ci; ++ci) {
        const float v = xp[ci * H * H];
#pragma unroll
        for (int co = 0; co < Co; ++co) acc[co] = fmaf(v, w[ci * Co + co], acc[co]);
      }
    }
  }
  const int oy = 2 * iy + py, ox = 2 * ix + px, HO = 2 * H;
  float* o = out + (size_t)b * Co * HO * HO + oy * HO + ox;
#pragma unroll
  for (int co = 0; co < Co; ++co) o[co * HO * HO] = relu ? fmaxf(acc[co], 0.f) : acc[co];
}

// Forward transposed convolution: a thread takes one input position (iy, ix) of one
// sample and computes the 2 x 2 output block (2 iy + py, 2 ix + px), all Co channels.
// Output row 2 iy + py gets taps (iy, ky = 1), (iy - 1, ky = 3) when py = 0 and
// (iy + 1, ky = 0), (iy, ky = 2) when py = 1 (likewise along x), so the block reads the
// 3 x 3 input neighbourhood; every weight address is the same across the wave (read as
// scalars), and the block is written as 8-byte pairs.
template <int Ci, int Co, int H>
__global__ void __launch_bounds__(256) sg_deconv_fwd2_kernel(const float* __restrict__ in,
                                                             const float* __restrict__ Kt,
                                                             const float* __restrict__ bias, int relu,
                                                             int B, float* __restrict__ out) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= B * H * H) return;   // no barrier below
  const int b = t / (H * H), q = t % (H * H), iy = q / H, ix = q % H;
  const float* x = in + (size_t)b * Ci * H * H;
  float acc[2][2][Co];
#pragma unroll
  for (int py = 0; py < 2; ++py)
#pragma unroll
    for (int px = 0; px < 2; ++px)
#pragma unroll
      for (int co = 0; co < Co; ++co) acc[py][px][co] = bias[co];
  // rows / columns of the neighbourhood: index 0 = iy - 1, 1 = iy, 2 = iy + 1
  const bool ry[3] = {iy > 0, true, iy + 1 < H}, rx[3] = {ix > 0, true, ix + 1 < H};
#pragma unroll 2
  for (int ci = 0; ci < Ci; ++ci) {
    float v[3][3];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
      for (int dx = 0; dx < 3; ++dx)
        v[dy][dx] = (ry[dy] && rx[dx]) ? x[(ci * H + iy + dy - 1) * H + ix + dx - 1] : 0.f;
#pragma unroll
    for (int py = 0; py < 2; ++py)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int dy = py ? 2 - a : 1 - a, ky = py ? 2 * a : 1 + 2 * a;
#pragma unroll
        for (int px = 0; px < 2; ++px)
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            const int dx = px ? 2 - c : 1 - c, kx = px ? 2 * c : 1 + 2 * c;
            const float* w = Kt + ((ky * 4 + kx) * Ci + ci) * Co;
#pragma unroll
            for (int co = 0; co < Co; ++co) acc[py][px][co] = fmaf(v[dy][dx], w[co], acc[py][px][co]);
          }
      }
  }
  constexpr int HO = 2 * H;
  float* o = out + (size_t)b * Co * HO * HO + (2 * iy) * HO + 2 * ix;
#pragma unroll
  for (int co = 0; co < Co; ++co)
#pragma unroll
    for (int py = 0; py < 2; ++py) {
      float a0 = acc[py][0][co], a1 = acc[py][1][co];
      if (relu) {
        a0 = fmaxf(a0, 0.f);
        a1 = fmaxf(a1, 0.f);
      }
      *reinterpret_cast<float2*>(o + co * HO * HO + py * HO) = make_float2(a0, a1);
    }
}

// dIn[ci, iy, ix] = sum_{co, ky, kx} dOut[co, 2 iy - 1 + ky, 2 ix - 1 + kx] K[ci, co, ky, kx]
__global__ void __launch_bounds__(256) sg_deconv_bwd_data_kernel(const float* __restrict__ dout,
                                                                  const float* __restrict__ K, int Ci, int Co,
                                                                  int H, float* __restrict__ din) {
  extern __shared__ float sh[];
  const int HO = 2 * H;
  float* g = sh;                   // [Co][HO][HO]
  float* kk = sh + Co * HO * HO;   // [Ci][Co][16]
  const int b = blockIdx.x;
  const float* src = dout + (size_t)b * Co * HO * HO;
  for (int i = threadIdx.x; i < Co * HO * HO; i += 256) g[i] = src[i];
  for (int i = threadIdx.x; i < Ci * Co * 16; i += 256) kk[i] = K[i];
  __syncthreads();
  float* dst = din + (size_t)b * Ci * H * H;
  for (int o = threadIdx.x; o < Ci * H * H; o += 256) {
    const int ci = o / (H * H), iy = (o / H) % H, ix = o % H;
    float s = 0.f;
    for (int ky = 0; ky < 4; ++ky) {
      const int oy = 2 * iy - 1 + ky;
      if (oy < 0 || oy >= HO) continue;
      for (int kx = 0; kx < 4; ++kx) {
        const int ox = 2 * ix - 1 + kx;
        if (ox < 0 || ox >= HO) continue;
        for (int co = 0; co < Co; ++co) s += g[(co * HO + oy) * HO + ox] * kk[(ci * Co + co) * 16 + ky * 4 + kx];
      }
    }
    dst[o] = s;
  }
}

// Per chunk of samples: partial dK[ci, co, ky, kx] and dbias[co], summed over the chunk's
// samples in order.  Each sample's input and output gradient are staged in LDS; every
// thread owns a fixed set of parameters and keeps their sums in LDS.
__global__ void __launch_bounds__(256) sg_deconv_bwd_weight_kernel(const float* __restrict__ in,
                                                                    const float* __restrict__ dout, int B,
                                                                    int chunk, int Ci, int Co, int H,
                                                                    float* __restrict__ partial) {
  extern __shared__ float sh[];
  const int HO = 2 * H, np = Ci * Co * 16, nin = Ci * H * H, nout = Co * HO * HO;
  float* xs = sh;                  // [Ci][H][H]
  float* gs = sh + nin;            // [Co][HO][HO]
  float* accs = gs + nout;         // [np + Co]
  const int b0 = blockIdx.x * chunk, b1 = min(B, b0 + chunk);
  for (int p = threadIdx.x; p < np + Co; p += 256) accs[p] = 0.f;
  for (int b = b0; b < b1; ++b) {
    __syncthreads();
    const float* xsrc = in + (size_t)b * nin;
    const float* gsrc = dout + (size_t)b * nout;
    for (int i = threadIdx.x; i < nin; i += 256) xs[i] = xsrc[i];
    for (int i = threadIdx.x; i < nout; i += 256) gs[i] = gsrc[i];
    __syncthreads();
    for (int p = threadIdx.x; p < np + Co; p += 256) {
      float s = 0.f;
      if (p < np) {
        const int ci = p / (Co * 16), co = (p / 16) % Co, ky = (p / 4) % 4, kx = p % 4;
        const float* x = xs + ci * H * H;
        const float* g = gs + co * HO * HO;
        // output rows oy = 2 iy - 1 + ky inside [0, HO): iy from (1 - ky + 1) / 2 when ky = 0
        const int iy0 = ky == 0 ? 1 : 0, iy1 = ky == 3 ? H - 1 : H;
        const int ix0 = kx == 0 ? 1 : 0, ix1 = kx == 3 ? H - 1 : H;
        for (int iy = iy0; iy < iy1; ++iy) {
          const float* xr = x + iy * H;
          const float* gr = g + (2 * iy - 1 + ky) * HO - 1 + kx;
          for (int ix = ix0; ix < ix1; ++ix) s += xr[ix] * gr[2 * ix];
        }
      } else {
        const float* g = gs + (p - np) * HO * HO;
        for (int i = 0; i < HO * HO; ++i) s += g[i];
      }
      accs[p] += s;
    }
  }
  __syncthreads();
  float* dst = partial + (size_t)blockIdx.x * (np + Co);
  for (int p = threadIdx.x; p < np + Co; p += 256) dst[p] = accs[p];
}

// sum partials [chunks][n] in chunk order
__global__ void sg_reduce_partials_kernel(const float* __restrict__ partial, int chunks, int n,
                                          float* __restrict__ out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  double s = 0.0;
  for (int c = 0; c < chunks; ++c) s += partial[(size_t)c * n + p];
  out[p] = (float)s;
}

__global__ void sg_adam_kernel(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                               float* __restrict__ v, size_t n, float lr, float b1, float b2, float eps,
                               float c1, float c2) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

}  // namespace rw

// ---------------------------------------------------------------- host side
namespace {
struct Layout {
  size_t W1, b1, W2, b2, W3, b3, K1, c1, K2, c2, K3, c3, total;
};
Layout layout() {
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t n) { size_t r = o; o += n; return r; };
  L.W1 = take(22 * 256); L.b1 = take(256);
  L.W2 = take(256 * 1024); L.b2 = take(1024);
  L.W3 = take(1024 * 2048); L.b3 = take(2048);
  L.K1 = take(32 * 16 * 16); L.c1 = take(16);
  L.K2 = take(16 * 8 * 16); L.c2 = take(8);
  L.K3 = take(8 * 1 * 16); L.c3 = take(1);
  L.total = o;
  return L;
}
constexpr int kMaxChunks = 256;   // partial sums of the convolution weight gradients per step
}  // namespace

struct rwpsf_sg {
  int device = 0, max_batch = 0;
  Layout L{};
  std::vector<void*> allocations;
  float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;   // [L.total]
  float *x = nullptr, *h1 = nullptr, *h2 = nullptr, *h3 = nullptr, *d1 = nullptr, *d2 = nullptr, *y = nullptr;
  float *gx = nullptr, *g1 = nullptr, *g2 = nullptr, *g3 = nullptr, *gd1 = nullptr, *gd2 = nullptr, *gy = nullptr;
  float* partial = nullptr;   // conv weight partials
  float* kt = nullptr;        // transposed convolution weights of the forward kernels
  __bf16* wsplit = nullptr;   // BF16 hi / lo planes of W2 and W3, [N][K]
  double* loss_partial = nullptr;
  int64_t step = 0;
  ~rwpsf_sg() {   // teardown: failures cannot be reported and are ignored
    for (void* p : allocations) (void)hipFree(p);
  }
};

namespace rw {

template <class T>
static int sg_alloc(rwpsf_sg* s, T** p, size_t count) {
  void* d = nullptr;
  hipError_t e = hipMalloc(&d, std::max<size_t>(16, count * sizeof(T)));
  if (e != hipSuccess) {
    set_hip_error(e);
    return RWPSF_ERR_OOM;
  }
  s->allocations.push_back(d);
  *p = (T*)d;
  return RWPSF_OK;
}

static int sg_forward_impl(rwpsf_sg* s, int B, const float* coef, const float* z, float* out, int nsplit,
                           hipStream_t st) {
  const Layout& L = s->L;
  int rc;
  hipLaunchKernelGGL(sg_features_kernel, dim3((B * 22 + 255) / 256), dim3(256), 0, st, coef, z, B, s->x);
  if ((rc = hip_check(hipGetLastError()))) return rc;
  if ((rc = hip_check(sg_gemm<false, false>(s->x, 22, s->w + L.W1, 256, s->h1, 256, B, 256, 22, s->w + L.b1, 1, nsplit, st)))) return rc;
  // the two wide layers on the aligned fast path, with the weights split to BF16 planes
  __bf16* w2h = s->wsplit;
  __bf16* w2l = w2h + 256 * 1024;
  __bf16* w3h = w2l + 256 * 1024;
  __bf16* w3l = w3h + 1024 * 2048;
  hipLaunchKernelGGL(sg_wsplit_kernel, dim3(256 * 1024 / 256), dim3(256), 0, st, s->w + L.W2, 256, 1024, w2h, w2l);
  hipLaunchKernelGGL(sg_wsplit_kernel, dim3(1024 * 2048 / 256), dim3(256), 0, st, s->w + L.W3, 1024, 2048, w3h, w3l);
  if ((rc = hip_check(hipGetLastError()))) return rc;
  if ((rc = hip_check(sg_gemm_fast(s->h1, w2h, w2l, s->h2, B, 1024, 256, s->w + L.b2, nsplit, st)))) return rc;
  if ((rc = hip_check(sg_gemm_fast(s->h2, w3h, w3l, s->h3, B, 2048, 1024, s->w + L.b3, nsplit, st)))) return rc;
  float* kt1 = s->kt;
  float* kt2 = kt1 + 32 * 16 * 16;
  float* kt3 = kt2 + 16 * 8 * 16;
  hipLaunchKernelGGL(sg_deconv_wt_kernel, dim3(32), dim3(256), 0, st, s->w + L.K1, 32, 16, kt1);
  hipLaunchKernelGGL(sg_deconv_wt_kernel, dim3(8), dim3(256), 0, st, s->w + L.K2, 16, 8, kt2);
  hipLaunchKernelGGL(sg_deconv_wt_kernel, dim3(1), dim3(256), 0, st, s->w + L.K3, 8, 1, kt3);
  if ((rc = hip_check(hipGetLastError()))) return rc;
  // one thread per input position (B * H * H threads)
  hipLaunchKernelGGL((sg_deconv_fwd_pix_kernel<32, 16, 8>), dim3(B), dim3(256), 0, st, s->h3, kt1, s->w + L.c1, 1,
                     s->d1);
  if ((rc = hip_check(hipGetLastError()))) return rc;
  hipLaunchKernelGGL((sg_deconv_fwd2_kernel<16, 8, 16>), dim3(B), dim3(256), 0, st, s->d1, kt2, s->w + L.c2, 1, B,
                     s->d2);
  if ((rc = hip_check(hipGetLastError()))) return rc;
  hipLaunchKernelGGL((sg_deconv_fwd2_kernel<8, 1, 32>), dim3(B * 4), dim3(256), 0, st, s->d2, kt3, s->w + L.c3, 0, B,
                     out);
  return hip_check(hipGetLastError());
}

static int sg_backward_impl(rwpsf_sg* s, int B, const float* target, float* loss, hipStream_t st) {
  const Layout& L = s->L;
  int rc;
  const size_t ny = (size_t)B * 4096;
  const int lb = 256;
  hipLaunchKernelGGL(sg_mse_kernel, dim3(lb), dim3(256), 0, st, s->y, target, ny, s->gy, s->loss_partial);
  if ((rc = hip_check(hipGetLastError()))) return rc;
  if (loss) {
    hipLaunchKernelGGL(sg_sum_kernel, dim3(1), dim3(64), 0, st, s->loss_partial, lb, 1.0 / (double)ny, loss);
    if ((rc = hip_check(hipGetLastError()))) return rc;
  }
  const int chunk = (B + kMaxChunks - 1) / kMaxChunks;   // samples per partial sum
  const int chunks = (B + chunk - 1) / chunk;
  struct Conv { float *in, *gin, *gout; int Ci, Co, H; size_t K, c; bool relu_in; };
  const Conv convs[3] = {{s->d2, s->gd2, s->gy, 8, 1, 32, L.K3, L.c3, true},
                         {s->d1, s->gd1, s->gd2, 16, 8, 16, L.K2, L.c2, true},
                         {s->h3, s->g3, s->gd1, 32, 16, 8, L.K1, L.c1, true}};
  for (const Conv& c : convs) {
    const int np = c.Ci * c.Co * 16;
    const int lds = (c.Ci * c.H * c.H + c.Co * 4 * c.H * c.H + np + c.Co) * 4;
    hipLaunchKernelGGL(sg_deconv_bwd_weight_kernel, dim3(chunks), dim3(256), lds, st, c.in, c.gout, B, chunk, c.Ci,
                       c.Co, c.H, s->partial);
    if ((rc = hip_check(hipGetLastError()))) return rc;
    hipLaunchKernelGGL(sg_reduce_partials_kernel, dim3((np + c.Co + 255) / 256), dim3(256), 0, st, s->partial, chunks,
                       np + c.Co, s->g + c.K);   // K and its bias are adjacent in the layout
    if ((rc = hip_check(hipGetLastError()))) return rc;
    const int HO = 2 * c.H;
    hipLaunchKernelGGL(sg_deconv_bwd_data_kernel, dim3(B), dim3(256), (c.Co * HO * HO + c.Ci * c.Co * 16) * 4, st,
                       c.gout, s->w + c.K, c.Ci, c.Co, c.H, c.gin);
    if ((rc = hip_check(hipGetLastError()))) return rc;
    const size_t n = (size_t)B * c.Ci * c.H * c.H;
    hipLaunchKernelGGL(sg_relu_mask_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, c.gin, c.in, n);
    if ((rc = hip_check(hipGetLastError()))) return rc;
  }
  // dense layers: g3 = dL/d(pre3) already masked
  struct Dense { float *hin, *gin, *gout; int in, out; size_t W, b; const float* hmask; };
  const Dense dense[3] = {{s->h2, s->g2, s->g3, 1024, 2048, L.W3, L.b3, s->h2},
                          {s->h1, s->g1, s->g2, 256, 1024, L.W2, L.b2, s->h1},
                          {s->x, s->gx, s->g1, 22, 256, L.W1, L.b1, nullptr}};
  for (const Dense& d : dense) {
    // dW = hin^T gout  (in x out, K = B), db = column sums, gin = gout W^T
    if ((rc = hip_check(sg_gemm<true, false>(d.hin, d.in, d.gout, d.out, s->g + d.W, d.out, d.in, d.out, B, nullptr, 0, 3, st)))) return rc;
    hipLaunchKernelGGL(sg_colsum_kernel, dim3((d.out + 255) / 256), dim3(256), 0, st, d.gout, B, d.out, s->g + d.b);
    if ((rc = hip_check(hipGetLastError()))) return rc;
    if (d.hmask) {
      if ((rc = hip_check(sg_gemm<false, true>(d.gout, d.out, s->w + d.W, d.out, d.gin, d.in, B, d.in, d.out, nullptr, 0, 3, st)))) return rc;
      const size_t n = (size_t)B * d.in;
      hipLaunchKernelGGL(sg_relu_mask_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, d.gin, d.hmask, n);
      if ((rc = hip_check(hipGetLastError()))) return rc;
    }
  }
  return RWPSF_OK;
}

}  // namespace rw

extern "C" {

size_t rwpsf_sg_param_count(void) { return layout().total; }

int rwpsf_sg_create(int max_batch, rwpsf_sg** out) {
  using namespace rw;
  if (!out || max_batch < 1 || max_batch > (1 << 20)) return RWPSF_ERR_INVALID_ARG;
  *out = nullptr;
  int dev_count = 0;
  if (hipGetDeviceCount(&dev_count) != hipSuccess || dev_count < 1) return RWPSF_ERR_NO_DEVICE;
  rwpsf_sg* s = new (std::nothrow) rwpsf_sg();
  if (!s) return RWPSF_ERR_OOM;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return RWPSF_ERR_NO_DEVICE;
  }
  s->max_batch = max_batch;
  s->L = layout();
  const size_t P = s->L.total, B = (size_t)max_batch;
  const int chunks = std::min(max_batch, kMaxChunks);
  int rc;
  if ((rc = sg_alloc(s, &s->w, P)) || (rc = sg_alloc(s, &s->g, P)) || (rc = sg_alloc(s, &s->m, P)) ||
      (rc = sg_alloc(s, &s->v, P)) || (rc = sg_alloc(s, &s->x, B * 22)) || (rc = sg_alloc(s, &s->h1, B * 256)) ||
      (rc = sg_alloc(s, &s->h2, B * 1024)) || (rc = sg_alloc(s, &s->h3, B * 2048)) ||
      (rc = sg_alloc(s, &s->d1, B * 4096)) || (rc = sg_alloc(s, &s->d2, B * 8192)) ||
      (rc = sg_alloc(s, &s->y, B * 4096)) || (rc = sg_alloc(s, &s->gx, B * 22)) ||
      (rc = sg_alloc(s, &s->g1, B * 256)) || (rc = sg_alloc(s, &s->g2, B * 1024)) ||
      (rc = sg_alloc(s, &s->g3, B * 2048)) || (rc = sg_alloc(s, &s->gd1, B * 4096)) ||
      (rc = sg_alloc(s, &s->gd2, B * 8192)) || (rc = sg_alloc(s, &s->gy, B * 4096)) ||
      (rc = sg_alloc(s, &s->partial, (size_t)chunks * (32 * 16 * 16 + 16))) ||
      (rc = sg_alloc(s, &s->loss_partial, 256)) || (rc = sg_alloc(s, &s->kt, 32 * 16 * 16 + 16 * 8 * 16 + 8 * 16)) ||
      (rc = sg_alloc(s, &s->wsplit, 2 * (256 * 1024 + 1024 * 2048)))) {
    delete s;
    return rc;
  }
  const int fast_lds = 2 * 4 * FBM * FLD * (int)sizeof(__bf16);
  if ((rc = hip_check(hipFuncSetAttribute((const void*)sg_gemm_fast_kernel<1>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, fast_lds))) ||
      (rc = hip_check(hipFuncSetAttribute((const void*)sg_gemm_fast_kernel<3>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, fast_lds)))) {
    delete s;
    return rc;
  }
  if ((rc = hip_check(hipMemset(s->m, 0, P * sizeof(float)))) || (rc = hip_check(hipMemset(s->v, 0, P * sizeof(float)))) ||
      (rc = hip_check(hipMemset(s->w, 0, P * sizeof(float)))) || (rc = hip_check(hipDeviceSynchronize()))) {
    delete s;
    return rc;
  }
  *out = s;
  return RWPSF_OK;
}

void rwpsf_sg_destroy(rwpsf_sg* s) {   // teardown: HIP failures are ignored
  if (!s) return;
  (void)hipDeviceSynchronize();
  delete s;
}

int rwpsf_sg_set_state(rwpsf_sg* s, const float* w, const float* m, const float* v, int64_t step) {
  if (!s || !w) return RWPSF_ERR_INVALID_ARG;
  const size_t bytes = s->L.total * sizeof(float);
  int rc;
  if ((rc = rw::hip_check(hipMemcpy(s->w, w, bytes, hipMemcpyHostToDevice)))) return rc;
  if (m && (rc = rw::hip_check(hipMemcpy(s->m, m, bytes, hipMemcpyHostToDevice)))) return rc;
  if (v && (rc = rw::hip_check(hipMemcpy(s->v, v, bytes, hipMemcpyHostToDevice)))) return rc;
  s->step = step;
  return RWPSF_OK;
}

int rwpsf_sg_get_state(const rwpsf_sg* s, float* w, float* m, float* v, float* g, int64_t* step) {
  if (!s) return RWPSF_ERR_INVALID_ARG;
  const size_t bytes = s->L.total * sizeof(float);
  int rc;
  if ((rc = rw::hip_check(hipDeviceSynchronize()))) return rc;
  if (w && (rc = rw::hip_check(hipMemcpy(w, s->w, bytes, hipMemcpyDeviceToHost)))) return rc;
  if (m && (rc = rw::hip_check(hipMemcpy(m, s->m, bytes, hipMemcpyDeviceToHost)))) return rc;
  if (v && (rc = rw::hip_check(hipMemcpy(v, s->v, bytes, hipMemcpyDeviceToHost)))) return rc;
  if (g && (rc = rw::hip_check(hipMemcpy(g, s->g, bytes, hipMemcpyDeviceToHost)))) return rc;
  if (step) *step = s->step;
  return RWPSF_OK;
}

int rwpsf_sg_forward(rwpsf_sg* s, int B, const float* coef, const float* z, float* out, int precision,
                     void* stream) {
  if (!s || B < 1 || B > s->max_batch || !coef || !z || !out) return RWPSF_ERR_INVALID_ARG;
  if (precision != RWPSF_SG_BF16X3 && precision != RWPSF_SG_BF16) return RWPSF_ERR_INVALID_ARG;
  return rw::sg_forward_impl(s, B, coef, z, out, precision == RWPSF_SG_BF16X3 ? 3 : 1, (hipStream_t)stream);
}

int rwpsf_sg_gradient(rwpsf_sg* s, int B, const float* coef, const float* z, const float* target, float* loss,
                      void* stream) {
  if (!s || B < 1 || B > s->max_batch || !coef || !z || !target) return RWPSF_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  int rc = rw::sg_forward_impl(s, B, coef, z, s->y, 3, st);
  if (rc) return rc;
  return rw::sg_backward_impl(s, B, target, loss, st);
}

int rwpsf_sg_adam(rwpsf_sg* s, float lr, float beta1, float beta2, float eps, void* stream) {
  if (!s || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return RWPSF_ERR_INVALID_ARG;
  s->step += 1;
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, (double)s->step)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, (double)s->step)));
  const size_t n = s->L.total;
  hipLaunchKernelGGL(rw::sg_adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, s->w,
                     s->g, s->m, s->v, n, lr, beta1, beta2, eps, c1, c2);
  return rw::hip_check(hipGetLastError());
}

}  // extern "C"
