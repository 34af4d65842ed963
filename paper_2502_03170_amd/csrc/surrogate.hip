// Learned surrogate of the PSF engine: (21 Noll coefficients, z) -> 64 x 64 intensity.
//
//   x  = (c / 0.05, z / 1000 nm)                                   22 features
//   h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2), h3 = relu(h2 W3 + b3)   1024 each
//   convolution branch:
//     d1 = relu(T(h3 as 16x8x8; K1) + c1)  16 x 16 x 16
//     d2 = relu(T(d1; K2) + c2)            8 x 32 x 32
//     yd = T(d2; K3) + c3                  64 x 64
//   basis branch: a = h3 Wa + ba (256), yb = a Wb + bb (64 x 64)
//   y = yd + yb
// T: stride-2 transposed convolution, 4 x 4 kernel, 1 pixel padding,
//   out[co, oy, ox] = sum_{ci,ky,kx} in[ci, iy, ix] K[ci, co, ky, kx], oy = 2 iy - 1 + ky.
//
// Dense layers run on the BF16 matrix cores (v_mfma_f32_32x32x16_bf16, FP32
// accumulate).  In the accurate mode every operand is split x = hi + lo with hi,
// lo in BF16 and the product is hi*hi + hi*lo + lo*hi (relative error ~1e-5); the
// fast mode uses hi*hi only.  The forward transposed convolutions run in one fused
// kernel per sample: the first two as implicit GEMMs on v_mfma_f32_16x16x32_bf16 (same
// splitting), the last (one output channel) in FP32, activations in LDS.  The backward
// kernels stage a sample in LDS (FP32).  Weight gradients of the convolutions
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
                                                      const float* __restrict__ bias, int relu, int accumulate) {
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
      float v = acc[r] + (bias ? bias[n] : 0.f) + (accumulate ? C[(size_t)m * ldc + n] : 0.f);
      if (relu) v = fmaxf(v, 0.f);
      C[(size_t)m * ldc + n] = v;
    }
  }
}

// h1 = relu(x W1 + b1) for the 22-feature input layer, in FP32 on the vector units: with
// K = 22 the layer is bound by writing h1, and a matrix-core tile would spend more on
// staging and splitting than on its products.  Thread t owns columns 4t .. 4t + 3 with
// their 22 weights in registers and walks kDense1Rows rows (x of a row is the same for
// the whole workgroup, staged in LDS); bias first, then k in order.
constexpr int kDense1Rows = 64;
__global__ void __launch_bounds__(256) sg_dense1_kernel(const float* __restrict__ x, const float* __restrict__ W1,
                                                        const float* __restrict__ b1, int B, float* __restrict__ h1) {
  const int n = 4 * threadIdx.x;
  float4 w[22];
#pragma unroll
  for (int k = 0; k < 22; ++k) w[k] = *reinterpret_cast<const float4*>(W1 + k * 1024 + n);
  const float4 bias = make_float4(b1[n], b1[n + 1], b1[n + 2], b1[n + 3]);
  const int r0 = blockIdx.x * kDense1Rows, r1 = min(B, r0 + kDense1Rows);
  // the workgroup's rows of x, staged once (every lane then reads the same word: a broadcast)
  __shared__ float xs[kDense1Rows * 22];
  for (int i = threadIdx.x; i < (r1 - r0) * 22; i += 256) xs[i] = x[(size_t)r0 * 22 + i];
  __syncthreads();
  for (int m = r0; m < r1; ++m) {
    const float* xm = xs + (m - r0) * 22;
    float4 acc = bias;
#pragma unroll
    for (int k = 0; k < 22; ++k) {
      const float xv = xm[k];
      acc.x = fmaf(xv, w[k].x, acc.x);
      acc.y = fmaf(xv, w[k].y, acc.y);
      acc.z = fmaf(xv, w[k].z, acc.z);
      acc.w = fmaf(xv, w[k].w, acc.w);
    }
    *reinterpret_cast<float4*>(h1 + (size_t)m * 1024 + n) =
        make_float4(fmaxf(acc.x, 0.f), fmaxf(acc.y, 0.f), fmaxf(acc.z, 0.f), fmaxf(acc.w, 0.f));
  }
}

template <bool TA, bool TB>
static hipError_t sg_gemm(const float* A, int lda, const float* B, int ldb, float* C, int ldc, int M, int N,
                          int K, const float* bias, int relu, int nsplit, hipStream_t st, int accumulate = 0) {
  const dim3 grid(((M + SBM - 1) / SBM) * ((N + SBN - 1) / SBN));
  if (nsplit > 1)
    hipLaunchKernelGGL((sg_gemm_kernel<TA, TB, 3>), grid, dim3(256), 0, st, A, lda, B, ldb, C, ldc, M, N, K,
                       bias, relu, accumulate);
  else
    hipLaunchKernelGGL((sg_gemm_kernel<TA, TB, 1>), grid, dim3(256), 0, st, A, lda, B, ldb, C, ldc, M, N, K,
                       bias, relu, accumulate);
  return hipGetLastError();
}

// ---------------------------------------------------------------- dense GEMM, aligned fast path
// C[M][N] = (relu)(A B + bias) for K % 32 == 0 and N % 128 == 0 (the 1024-wide layers
// and the basis branch).  A is FP32 [M][K], split into BF16 hi / lo while it is staged;
// B is given pre-split as k-contiguous BF16 planes Bt_hi / Bt_lo [N][K].  Workgroup
// 128 x 128, 4 waves of 64 x 64 (2 x 2 MFMA blocks of 32 x 32 x 16), k-stage 32, two LDS
// stages; each lane reads its 8 consecutive k of an operand with one 16-byte LDS read.
constexpr int FBM = 128, FBN = 128, FBK = 32, FLD = FBK + 8;   // LDS row: 40 bf16 (80 B)
static_assert(4 * 64 * (64 + 4) * 4 <= 2 * 4 * FBM * FLD * 2, "the epilogue tiles fit in the stage buffers");
constexpr int kGroupM = 8;                                      // row blocks per band (XCD order)
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
                                                              const float* __restrict__ bias, int relu,
                                                              int Kc, int accumulate) {
  constexpr int PL = FBM * FLD;             // one bf16 plane of a tile
  constexpr int STAGE = 4 * PL;             // A hi, A lo, B hi, B lo
  extern __shared__ __bf16 shb[];
  const int tiles_n = N / FBN;
  int tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
  {
    // Workgroups go to the 8 XCDs round robin, and each XCD has its own L2.  When the row
    // blocks divide evenly, XCD x takes a contiguous eighth of them and walks it in bands
    // of kGroupM row blocks, column tile by column tile, so that the workgroups resident
    // on one XCD share A row blocks and B column tiles in its L2 (with the plain order the
    // 8 column tiles of a row block would sit on 8 XCDs and A would be fetched 8 times).
    const int rb = gridDim.x / tiles_n;
    if (rb % (8 * kGroupM) == 0) {
      const int xcd = blockIdx.x & 7, local = blockIdx.x >> 3;
      const int band = local / (kGroupM * tiles_n), w = local % (kGroupM * tiles_n);
      tm = xcd * (rb >> 3) + band * kGroupM + w % kGroupM;
      tn = w / kGroupM;
    }
  }
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int row0 = tm * FBM, col0 = tn * FBN;
  // split K: slice blockIdx.y covers k in [kbase, kbase + Kc) and, when there are several
  // slices, writes its raw partial product to slice blockIdx.y of C (reduced afterwards)
  const int kbase = blockIdx.y * Kc;
  if (gridDim.y > 1) C += (size_t)blockIdx.y * M * N;
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
      ra[i] = *reinterpret_cast<const float4*>(A + (size_t)gr * K + kbase + k0 + kq);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int idx = tid + 256 * i, c = idx >> 2, k8 = 8 * (idx & 3);
      rbh[i] = *reinterpret_cast<const uint4*>(Bhi + (size_t)(col0 + c) * K + kbase + k0 + k8);
      if (NSPLIT > 1) rbl[i] = *reinterpret_cast<const uint4*>(Blo + (size_t)(col0 + c) * K + kbase + k0 + k8);
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
  const int KT = Kc / FBK;
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
  // Two stages of global loads in flight: a stage's MFMAs take far less time than a
  // load's latency, so stage kt + 2 is requested while stage kt is multiplied and stage
  // kt + 1 (already in registers) is written to the other LDS buffer.  KT >= 2; the last
  // two stages are peeled, so that no branch surrounds the loads and stores.
  Staged g1 = load(FBK);
  store(shb, load(0));
  __syncthreads();
  for (int kt = 0; kt < KT - 2; ++kt) {
    const Staged g2 = load((kt + 2) * FBK);
    mma(shb + (kt & 1) * STAGE);
    store(shb + ((kt + 1) & 1) * STAGE, g1);
    __syncthreads();
    g1 = g2;
  }
  mma(shb + (KT & 1) * STAGE);
  store(shb + ((KT - 1) & 1) * STAGE, g1);
  __syncthreads();
  mma(shb + ((KT - 1) & 1) * STAGE);
  // Epilogue through LDS (the stage buffers are free now): each wave writes its 64 x 64
  // tile row-major, then stores whole 16-byte row pieces, a quarter of the store
  // instructions of one value per lane per accumulator register.
  __syncthreads();
  constexpr int TLD = 64 + 4;   // floats per LDS row of a wave's tile
  float* tw = reinterpret_cast<float*>(shb) + wave * 64 * TLD;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r)
        tw[(32 * i + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3)) * TLD + 32 * j + (lane & 31)] = acc[i][j][r];
  __syncthreads();
  const bool raw = gridDim.y > 1;
  const int c4 = lane & 15, n = col0 + wn + 4 * c4;
  float4 bn = make_float4(0.f, 0.f, 0.f, 0.f);
  if (bias && !raw) bn = make_float4(bias[n], bias[n + 1], bias[n + 2], bias[n + 3]);   // (bias is 4-byte aligned)
#pragma unroll 4
  for (int it = 0; it < 16; ++it) {
    const int row = 4 * it + (lane >> 4), m = row0 + wm + row;
    if (m < M) {
      float4 v = *reinterpret_cast<const float4*>(tw + row * TLD + 4 * c4);
      float4* dst = reinterpret_cast<float4*>(C + (size_t)m * N + n);
      if (!raw) {
        const float4 prev = accumulate ? *dst : make_float4(0.f, 0.f, 0.f, 0.f);
        v = make_float4(v.x + bn.x + prev.x, v.y + bn.y + prev.y, v.z + bn.z + prev.z, v.w + bn.w + prev.w);
        if (relu) v = make_float4(fmaxf(v.x, 0.f), fmaxf(v.y, 0.f), fmaxf(v.z, 0.f), fmaxf(v.w, 0.f));
      }
      *dst = v;
    }
  }
}

// C = (relu)(sum over slices of ws[s] (in slice order) + bias (+ C)) after a split-K product
__global__ void sg_splitk_reduce_kernel(const float* __restrict__ ws, int slices, size_t MN, int N,
                                        const float* __restrict__ bias, int relu, int accumulate,
                                        float* __restrict__ C) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= MN) return;
  float v = 0.f;
  for (int s = 0; s < slices; ++s) v += ws[(size_t)s * MN + i];
  if (bias) v += bias[i % N];
  if (accumulate) v += C[i];
  C[i] = relu ? fmaxf(v, 0.f) : v;
}

// W [n] FP32 -> hi / lo BF16 in the same order (the transposed operand of C = A W^T)
__global__ void sg_split_kernel(const float* __restrict__ W, size_t n, __bf16* __restrict__ hi,
                                __bf16* __restrict__ lo) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float w = W[i];
  const __bf16 h = (__bf16)w;
  hi[i] = h;
  lo[i] = (__bf16)(w - (float)h);
}

// C = (relu)(A B + bias (+ C)) with B given as BF16 planes Bt [N][K].  A product with few
// row tiles is split over K (up to 16 slices, each at least 128 deep) into the workspace
// ws (ws_floats floats) and reduced in slice order, so the result does not depend on the
// launch.
static hipError_t sg_gemm_fast(const float* A, const __bf16* Bh, const __bf16* Bl, float* C, int M, int N, int K,
                               const float* bias, int relu, int nsplit, hipStream_t st, int accumulate = 0,
                               float* ws = nullptr, size_t ws_floats = 0, int target_wg = 0) {
  const int tiles = ((M + FBM - 1) / FBM) * (N / FBN);
  int slices = 1;
  while (ws && slices < 16 && tiles * slices * 2 <= target_wg && K % (2 * slices * FBK) == 0 &&
         K / (2 * slices) >= 128 && (size_t)2 * slices * M * N <= ws_floats)
    slices *= 2;
  const dim3 grid(tiles, slices);
  if (K / slices < 2 * FBK) return hipErrorInvalidValue;   // the pipeline needs two k-stages
  const int lds = 2 * 4 * FBM * FLD * (int)sizeof(__bf16);
  float* out = slices > 1 ? ws : C;
  if (nsplit > 1)
    hipLaunchKernelGGL(sg_gemm_fast_kernel<3>, grid, dim3(256), lds, st, A, Bh, Bl, out, M, N, K, bias, relu,
                       K / slices, accumulate);
  else
    hipLaunchKernelGGL(sg_gemm_fast_kernel<1>, grid, dim3(256), lds, st, A, Bh, Bl, out, M, N, K, bias, relu,
                       K / slices, accumulate);
  if (slices > 1) {
    const size_t MN = (size_t)M * N;
    hipLaunchKernelGGL(sg_splitk_reduce_kernel, dim3((unsigned)((MN + 255) / 256)), dim3(256), 0, st, ws, slices, MN,
                       N, bias, relu, accumulate, C);
  }
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

// Error model of the surrogate: log rel-L2 ~ w . phi(c, z) with the features
// phi = (1, (c_1 / 0.05)^2 .. (c_21 / 0.05)^2, (z / 1000 nm)^2, |z| / 1000 nm).
constexpr int kGateFeatures = 24;
__device__ __forceinline__ float sg_gate_feature(const float* __restrict__ c, float z, int f) {
  if (f == 0) return 1.f;
  if (f <= 21) {
    const float u = c[f - 1] * (1.f / 0.05f);
    return u * u;
  }
  const float t = z * (1.f / 1000.f);
  return f == 22 ? t * t : fabsf(t);
}

__global__ void sg_gate_features_kernel(const float* __restrict__ coef, const float* __restrict__ z, int B,
                                        float* __restrict__ phi) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B * kGateFeatures) return;
  const int b = i / kGateFeatures, f = i % kGateFeatures;
  phi[i] = sg_gate_feature(coef + (size_t)b * 21, z[b], f);
}

__global__ void sg_gate_predict_kernel(const float* __restrict__ coef, const float* __restrict__ z, int B,
                                       const float* __restrict__ w, float* __restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  float s = 0.f;
#pragma unroll
  for (int f = 0; f < kGateFeatures; ++f) s = fmaf(w[f], sg_gate_feature(coef + (size_t)b * 21, z[b], f), s);
  out[b] = s;
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

// column sums of g [rows][cols] (bias gradients), two levels in a fixed order: chunk
// blockIdx.y sums its rows in order into part[chunk][col]; sg_colsum_final_kernel sums the
// chunks in order
__global__ void sg_colsum_kernel(const float* __restrict__ g, int rows, int cols, int rows_per_chunk,
                                 double* __restrict__ part) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  const int r0 = blockIdx.y * rows_per_chunk, r1 = min(rows, r0 + rows_per_chunk);
  double s = 0.0;
  for (int r = r0; r < r1; ++r) s += g[(size_t)r * cols + c];
  part[(size_t)blockIdx.y * cols + c] = s;
}

__global__ void sg_colsum_final_kernel(const double* __restrict__ part, int chunks, int cols,
                                       float* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  double s = 0.0;
  for (int k = 0; k < chunks; ++k) s += part[(size_t)k * cols + c];
  out[c] = (float)s;
}

constexpr int kColChunks = 64;   // row chunks of the column sums (partials: kColChunks x 4096 doubles)

static hipError_t sg_colsum(const float* g, int rows, int cols, float* out, double* part, hipStream_t st) {
  const int chunks = std::min(kColChunks, std::max(1, rows / 16));
  const int per = (rows + chunks - 1) / chunks;
  const int used = (rows + per - 1) / per;
  hipLaunchKernelGGL(sg_colsum_kernel, dim3((cols + 255) / 256, used), dim3(256), 0, st, g, rows, cols, per, part);
  hipLaunchKernelGGL(sg_colsum_final_kernel, dim3((cols + 255) / 256), dim3(256), 0, st, part, used, cols, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------- transposed convolution
// ---------------------------------------------------------------- fused decoder on the matrix cores
// The three transposed convolutions of one sample in one workgroup, activations kept in
// LDS.  Output pixel (2Y + py, 2X + px) of a stride-2, 4 x 4, pad-1 transposed convolution
// takes input rows Y + dy and kernel rows ky with (dy, ky) = (0, 1), (-1, 3) for py = 0 and
// (+1, 0), (0, 2) for py = 1 (the same along x), so each output parity class is a plain
// GEMM over the input pixels: M = pixels, K = (tap, input channel), N = output channels.
//   layer 1 (C0 -> C1 = 16, 8x8 -> 16x16): one GEMM per class (py, px), K = 4 C0, N = 16;
//   layer 2 (C1 -> C2 = 8, 16x16 -> 32x32): one GEMM per row class py with both column
//     classes side by side in N = 2 C2 = 16 (K = 6 C1 over the input columns X-1, X, X+1;
//     the tap a column class does not use has a zero weight);
//   layer 3 (C2 -> 1, 32x32 -> 64x64): N = 1 is a matrix-vector product, done in FP32 on
//     the vector units (a thread owns 2 x 2 input pixels and their 4 x 4 outputs).
// Layers 1 and 2 run v_mfma_f32_16x16x32_bf16: A lane l holds row l % 16 and eight
// consecutive k of group l / 16, B lane l holds column l % 16 and the same eight k, C
// register r of lane l holds row 4 (l / 16) + r, column l % 16.  Activations sit in LDS
// channel-last with a zero border, so the eight k of a lane are eight consecutive
// channels of one source pixel (two 16-byte reads), with no bounds tests.  Weights are
// pre-arranged as B fragments ([class][k-step][lane][8] BF16 hi / lo) and held in
// registers for all samples of the workgroup.  The inputs of the two matrix-core layers
// are split into BF16 hi / lo once, when they are written to LDS (each value feeds up to
// 16 fragments).
constexpr int DC0 = 16, DC1 = 16, DC2 = 8;          // decoder channels (layer inputs)
// inputs of the matrix-core layers are held as BF16 hi / lo planes (split once, when
// written), DXb BF16 per pixel (16-byte aligned, padded); the last layer's input in FP32
constexpr int DX0b = DC0 + 8, DX1b = DC1 + 8, DX2 = DC2;
constexpr int DL0b = 10 * 10 * DX0b, DL1b = 18 * 18 * DX1b, DL2 = 34 * 34 * DX2;   // elements per plane
constexpr int DK1 = 4 * DC0 / 32, DK2 = 6 * DC1 / 32;    // k-steps of the layer-1 / layer-2 GEMMs
constexpr int kDecLdsBytes = 2 * (DL0b + DL1b) * 2 + DL2 * 4;
static_assert(DC1 == 16 && 2 * DC2 == 16 && DC0 % 8 == 0 && DC1 % 8 == 0, "decoder tile shapes");
typedef float f4v_t __attribute__((ext_vector_type(4)));

// B fragments: layer 1 [4 classes][DK1][64][8], layer 2 [2 row classes][DK2][64][8], hi and lo
__global__ void sg_dec_wprep_kernel(const float* __restrict__ K1, const float* __restrict__ K2,
                                    __bf16* __restrict__ f1h, __bf16* __restrict__ f1l,
                                    __bf16* __restrict__ f2h, __bf16* __restrict__ f2l) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n1 = 4 * DK1 * 64 * 8, n2 = 2 * DK2 * 64 * 8;
  if (i < n1) {
    const int q = i % 8, l = (i / 8) % 64, s = (i / 512) % DK1, p = i / (512 * DK1);
    const int py = p >> 1, px = p & 1, co = l % 16, k = 32 * s + 8 * (l / 16) + q;
    const int tap = k / DC0, ci = k % DC0, a = tap >> 1, c = tap & 1;
    const int ky = py ? 2 * a : 1 + 2 * a, kx = px ? 2 * c : 1 + 2 * c;
    const float w = K1[((ci * DC1 + co) * 4 + ky) * 4 + kx];
    const __bf16 h = (__bf16)w;
    f1h[i] = h;
    f1l[i] = (__bf16)(w - (float)h);
  } else if (i < n1 + n2) {
    const int j = i - n1;
    const int q = j % 8, l = (j / 8) % 64, s = (j / 512) % DK2, py = j / (512 * DK2);
    const int n = l % 16, px = n / DC2, co = n % DC2, k = 32 * s + 8 * (l / 16) + q;
    const int t6 = k / DC1, ci = k % DC1, a = t6 / 3, c3 = t6 % 3;
    const int ky = py ? 2 * a : 1 + 2 * a;
    // column tap c3 reads input column X + c3 - 1: px = 0 uses kx = 3, 1 (c3 = 0, 1),
    // px = 1 uses kx = 2, 0 (c3 = 1, 2)
    const int kx = px == 0 ? (c3 == 0 ? 3 : c3 == 1 ? 1 : -1) : (c3 == 0 ? -1 : c3 == 1 ? 2 : 0);
    const float w = kx < 0 ? 0.f : K2[((ci * DC2 + co) * 4 + ky) * 4 + kx];
    const __bf16 h = (__bf16)w;
    f2h[j] = h;
    f2l[j] = (__bf16)(w - (float)h);
  }
}

// h3 [B][DC0][8][8] (relu applied) -> y [B][64][64] += T(T(T(h3))); d1 [B][DC1][16][16] and d2
// [B][DC2][32][32] (post-relu) are also written when the pointers are not null (training).
// Persistent: workgroup g serves samples g, g + gridDim.x, ...
template <int NSPLIT>
__global__ void __launch_bounds__(256, 2) sg_decoder_kernel(const float* __restrict__ h3, int B,
                                                            const bf8_t* __restrict__ f1h,
                                                            const bf8_t* __restrict__ f1l,
                                                            const bf8_t* __restrict__ f2h,
                                                            const bf8_t* __restrict__ f2l,
                                                            const float* __restrict__ c1,
                                                            const float* __restrict__ c2,
                                                            const float* __restrict__ K3,
                                                            const float* __restrict__ c3,
                                                            float* __restrict__ y, float* __restrict__ d1g,
                                                            float* __restrict__ d2g) {
  extern __shared__ float dls[];
  __bf16* X0h = reinterpret_cast<__bf16*>(dls);   // [10][10][DX0b] hi, then lo
  __bf16* X0l = X0h + DL0b;
  __bf16* X1h = X0l + DL0b;                       // [18][18][DX1b] hi, then lo
  __bf16* X1l = X1h + DL1b;
  float* X2 = reinterpret_cast<float*>(X1l + DL1b);   // [34][34][DX2] FP32
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, r16 = lane & 15;
  for (int i = tid; i < kDecLdsBytes / 4; i += 256) dls[i] = 0.f;   // zero borders (interiors are rewritten)
  // B fragments of this wave: layer-1 class p = w, layer-2 row class py2 = w / 2
  bf8_t w1h[DK1], w1l[DK1], w2h[DK2], w2l[DK2];
#pragma unroll
  for (int s = 0; s < DK1; ++s) {
    w1h[s] = f1h[(w * DK1 + s) * 64 + lane];
    if (NSPLIT > 1) w1l[s] = f1l[(w * DK1 + s) * 64 + lane];
  }
  const int py2 = w >> 1;
#pragma unroll
  for (int s = 0; s < DK2; ++s) {
    w2h[s] = f2h[(py2 * DK2 + s) * 64 + lane];
    if (NSPLIT > 1) w2l[s] = f2l[(py2 * DK2 + s) * 64 + lane];
  }
  const float bias1 = c1[r16];
  const float bias2 = c2[r16 % DC2];
  const float bias3 = c3[0];
  // staged h3 of the next sample: DC0 * 64 floats, 8 per thread as two float4
  constexpr int NV = DC0 * 64 / 4 / 256;
  float4 hv[NV];
  auto fetch = [&](int b) {
#pragma unroll
    for (int v = 0; v < NV; ++v)
      hv[v] = b < B ? *reinterpret_cast<const float4*>(h3 + (size_t)b * DC0 * 64 + 4 * (tid + 256 * v))
                    : make_float4(0.f, 0.f, 0.f, 0.f);
  };
  fetch(blockIdx.x);
  __syncthreads();   // borders zeroed before any interior write
  for (int b = blockIdx.x; b < B; b += gridDim.x) {
    // this sample's basis-branch output under the thread's 4 x 4 outputs of layer 3,
    // requested now so that its latency passes under layers 1 and 2
    float* yo = y + (size_t)b * 4096 + (4 * (tid >> 4)) * 64 + 4 * (tid & 15);
    float4 yprev[4];
#pragma unroll
    for (int oy = 0; oy < 4; ++oy) yprev[oy] = *reinterpret_cast<const float4*>(yo + oy * 64);
    // ---- stage h3 [ci][Y][X] -> X0 [Y+1][X+1][ci]
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int e = 4 * (tid + 256 * v), ci = e / 64, pix = e % 64;
      const float xs[4] = {hv[v].x, hv[v].y, hv[v].z, hv[v].w};
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int Y = (pix + t) / 8, X = (pix + t) % 8, at = ((Y + 1) * 10 + X + 1) * DX0b + ci;
        const __bf16 h = (__bf16)xs[t];
        X0h[at] = h;
        X0l[at] = (__bf16)(xs[t] - (float)h);
      }
    }
    fetch(b + gridDim.x);
    __syncthreads();
    // ---- layer 1: wave w = class (py, px); the four M-tiles of 16 pixels (Y, X) of the
    // 8 x 8 input, their accumulator chains interleaved
    {
      const int py = w >> 1, px = w & 1;
      f4v_t acc[4];
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) acc[mt] = f4v_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < DK1; ++s) {
        const int k0 = 32 * s + 8 * g, tap = k0 / DC0, ci = k0 % DC0, a = tap >> 1, c = tap & 1;
        const int dy = py ? 1 - a : -a, dx = px ? 1 - c : -c;
        bf8_t ah[4], al[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
          const int m = 16 * mt + r16, Y = m >> 3, X = m & 7;
          const int at = ((Y + dy + 1) * 10 + X + dx + 1) * DX0b + ci;
          ah[mt] = *reinterpret_cast<const bf8_t*>(X0h + at);
          al[mt] = NSPLIT > 1 ? *reinterpret_cast<const bf8_t*>(X0l + at) : ah[mt];
        }
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[mt], w1h[s], acc[mt], 0, 0, 0);
        if (NSPLIT > 1) {
#pragma unroll
          for (int mt = 0; mt < 4; ++mt)
            acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[mt], w1l[s], acc[mt], 0, 0, 0);
#pragma unroll
          for (int mt = 0; mt < 4; ++mt)
            acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[mt], w1h[s], acc[mt], 0, 0, 0);
        }
      }
      // C: rows 4 g + i (pixels), column r16 (output channel)
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int mm = 16 * mt + 4 * g + i, YY = mm >> 3, XX = mm & 7;
          const int at = ((2 * YY + py + 1) * 18 + 2 * XX + px + 1) * DX1b + r16;
          const float v = fmaxf(acc[mt][i] + bias1, 0.f);
          const __bf16 h = (__bf16)v;
          X1h[at] = h;
          X1l[at] = (__bf16)(v - (float)h);
        }
    }
    __syncthreads();
    if (d1g) {   // training: d1 [co][16][16]
      float* o = d1g + (size_t)b * DC1 * 256;
      for (int e = tid; e < DC1 * 256; e += 256) {
        const int co = e / 256, pix = e % 256, at = ((pix / 16 + 1) * 18 + pix % 16 + 1) * DX1b + co;
        o[e] = (float)X1h[at] + (float)X1l[at];   // the value to 2^-16 relative (its sign exactly)
      }
    }
    // ---- layer 2: wave w = row class py2, M-tiles 8 (w & 1) .. + 7 of the 16 x 16 input,
    // in groups of L2G tiles whose accumulator chains are interleaved (a chain's next
    // product waits for the previous one; the group's other chains fill the gap)
    {
      constexpr int L2G = 4;
#pragma unroll 1
      for (int t0 = 0; t0 < 8; t0 += L2G) {
        f4v_t acc[L2G];
#pragma unroll
        for (int u = 0; u < L2G; ++u) acc[u] = f4v_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < DK2; ++s) {
          const int k0 = 32 * s + 8 * g, t6 = k0 / DC1, ci = k0 % DC1, a = t6 / 3, c3 = t6 % 3;
          const int dy = py2 ? 1 - a : -a, dx = c3 - 1;
          bf8_t ah[L2G], al[L2G];
#pragma unroll
          for (int u = 0; u < L2G; ++u) {
            const int m = 16 * (8 * (w & 1) + t0 + u) + r16, Y = m >> 4, X = m & 15;
            const int at = ((Y + dy + 1) * 18 + X + dx + 1) * DX1b + ci;
            ah[u] = *reinterpret_cast<const bf8_t*>(X1h + at);
            al[u] = NSPLIT > 1 ? *reinterpret_cast<const bf8_t*>(X1l + at) : ah[u];
          }
#pragma unroll
          for (int u = 0; u < L2G; ++u) acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[u], w2h[s], acc[u], 0, 0, 0);
          if (NSPLIT > 1) {
#pragma unroll
            for (int u = 0; u < L2G; ++u)
              acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[u], w2l[s], acc[u], 0, 0, 0);
#pragma unroll
            for (int u = 0; u < L2G; ++u)
              acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[u], w2h[s], acc[u], 0, 0, 0);
          }
        }
        const int px = r16 / DC2, co = r16 % DC2;
#pragma unroll
        for (int u = 0; u < L2G; ++u)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int mm = 16 * (8 * (w & 1) + t0 + u) + 4 * g + i, YY = mm >> 4, XX = mm & 15;
            X2[((2 * YY + py2 + 1) * 34 + 2 * XX + px + 1) * DX2 + co] = fmaxf(acc[u][i] + bias2, 0.f);
          }
      }
    }
    __syncthreads();
    if (d2g) {   // training: d2 [co][32][32]
      float* o = d2g + (size_t)b * DC2 * 1024;
      for (int e = tid; e < DC2 * 1024; e += 256) {
        const int co = e / 1024, pix = e % 1024;
        o[e] = X2[((pix / 32 + 1) * 34 + pix % 32 + 1) * DX2 + co];
      }
    }
    // ---- layer 3 (FP32): thread owns input pixels (2 Yb + u, 2 Xb + v), u, v in {0, 1},
    // reads the 4 x 4 neighbourhood rows 2 Yb - 1 .. 2 Yb + 2 and writes the 4 x 4 outputs
    {
      const int Yb = tid >> 4, Xb = tid & 15;
      float out[4][4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) out[i][j] = bias3;
#pragma unroll
      for (int hc = 0; hc < DC2; hc += 4) {
        float4 nb[4][4];   // channels hc .. hc + 3 at padded rows 2 Yb .. 2 Yb + 3, cols 2 Xb .. 2 Xb + 3
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            nb[i][j] = *reinterpret_cast<const float4*>(X2 + ((2 * Yb + i) * 34 + 2 * Xb + j) * DX2 + hc);
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
          const int ci = hc + cc;
#pragma unroll
          for (int oy = 0; oy < 4; ++oy)      // output row 4 Yb + oy = 2 (2 Yb + u) + py
#pragma unroll
            for (int ox = 0; ox < 4; ++ox) {
              const int u = oy >> 1, py = oy & 1, v = ox >> 1, px = ox & 1;
#pragma unroll
              for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                  const int dy = py ? 1 - a : -a, dx = px ? 1 - c : -c;
                  const int ky = py ? 2 * a : 1 + 2 * a, kx = px ? 2 * c : 1 + 2 * c;
                  // input pixel (2 Yb + u + dy, 2 Xb + v + dx) sits at nb[u + dy + 1][v + dx + 1]
                  const float4 q = nb[u + dy + 1][v + dx + 1];
                  const float xv = cc == 0 ? q.x : cc == 1 ? q.y : cc == 2 ? q.z : q.w;
                  out[oy][ox] = fmaf(xv, K3[ci * 16 + ky * 4 + kx], out[oy][ox]);
                }
            }
        }
      }
      // y holds the basis branch already: add the convolution branch to it
#pragma unroll
      for (int oy = 0; oy < 4; ++oy) {
        const float4 prev = yprev[oy];
        *reinterpret_cast<float4*>(yo + oy * 64) =
            make_float4(prev.x + out[oy][0], prev.y + out[oy][1], prev.z + out[oy][2], prev.w + out[oy][3]);
      }
    }
    // the next iteration's staging writes X0 only; X1 / X2 are rewritten after its barriers
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
constexpr int kBasis = 256;   // rank of the linear crop basis
struct Layout {
  size_t W1, b1, W2, b2, W3, b3, K1, c1, K2, c2, K3, c3, Wa, ba, Wb, bb, total;
};
Layout layout() {
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t n) { size_t r = o; o += n; return r; };
  L.W1 = take(22 * 1024); L.b1 = take(1024);
  L.W2 = take(1024 * 1024); L.b2 = take(1024);
  L.W3 = take(1024 * 1024); L.b3 = take(1024);
  L.K1 = take(16 * 16 * 16); L.c1 = take(16);
  L.K2 = take(16 * 8 * 16); L.c2 = take(8);
  L.K3 = take(8 * 1 * 16); L.c3 = take(1);
  L.Wa = take(1024 * kBasis); L.ba = take(kBasis);
  L.Wb = take(kBasis * 4096); L.bb = take(4096);
  L.total = o;
  return L;
}
constexpr int kMaxChunks = 256;   // partial sums of the convolution weight gradients per step
constexpr size_t kSplitKFloats = (size_t)16 << 20;   // split-K workspace of the training products
}  // namespace

struct rwpsf_sg {
  int device = 0, max_batch = 0;
  Layout L{};
  std::vector<void*> allocations;
  float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;   // [L.total]
  float *x = nullptr, *h1 = nullptr, *h2 = nullptr, *h3 = nullptr, *d1 = nullptr, *d2 = nullptr, *y = nullptr;
  float *gx = nullptr, *g1 = nullptr, *g2 = nullptr, *g3 = nullptr, *gd1 = nullptr, *gd2 = nullptr, *gy = nullptr;
  float *a = nullptr, *ga = nullptr;   // basis coefficients [B][kBasis] and their gradient
  float* partial = nullptr;   // conv weight partials
  __bf16* decw = nullptr;     // B fragments of the decoder's matrix-core layers (hi / lo)
  int num_cus = 0;
  __bf16* wsplit = nullptr;   // BF16 hi / lo planes of W2, W3, Wa, Wb, [N][K]
  __bf16* wsplit_t = nullptr; // the same weights split in their own order (operands of g W^T)
  float* ws = nullptr;        // split-K partial products
  double* colpart = nullptr;  // column-sum partials
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

// keep: also write d1 and d2 (the backward pass needs them)
static int sg_forward_impl(rwpsf_sg* s, int B, const float* coef, const float* z, float* out, int nsplit,
                           bool keep, hipStream_t st) {
  const Layout& L = s->L;
  int rc;
  hipLaunchKernelGGL(sg_features_kernel, dim3((B * 22 + 255) / 256), dim3(256), 0, st, coef, z, B, s->x);
  if ((rc = hip_check(hipGetLastError()))) return rc;
  // (W1 is the first parameter block, so its rows are 16-byte aligned)
  hipLaunchKernelGGL(sg_dense1_kernel, dim3((B + kDense1Rows - 1) / kDense1Rows), dim3(256), 0, st, s->x,
                     s->w + L.W1, s->w + L.b1, B, s->h1);
  if ((rc = hip_check(hipGetLastError()))) return rc;
  // the wide layers on the aligned fast path, with the weights split to BF16 planes
  __bf16* w2h = s->wsplit;
  __bf16* w2l = w2h + 1024 * 1024;
  __bf16* w3h = w2l + 1024 * 1024;
  __bf16* w3l = w3h + 1024 * 1024;
  __bf16* wah = w3l + 1024 * 1024;
  __bf16* wal = wah + 1024 * kBasis;
  __bf16* wbh = wal + 1024 * kBasis;
  __bf16* wbl = wbh + kBasis * 4096;
  hipLaunchKernelGGL(sg_wsplit_kernel, dim3(1024 * 1024 / 256), dim3(256), 0, st, s->w + L.W2, 1024, 1024, w2h, w2l);
  hipLaunchKernelGGL(sg_wsplit_kernel, dim3(1024 * 1024 / 256), dim3(256), 0, st, s->w + L.W3, 1024, 1024, w3h, w3l);
  hipLaunchKernelGGL(sg_wsplit_kernel, dim3(1024 * kBasis / 256), dim3(256), 0, st, s->w + L.Wa, 1024, kBasis, wah,
                     wal);
  hipLaunchKernelGGL(sg_wsplit_kernel, dim3(kBasis * 4096 / 256), dim3(256), 0, st, s->w + L.Wb, kBasis, 4096, wbh,
                     wbl);
  if ((rc = hip_check(hipGetLastError()))) return rc;
  if ((rc = hip_check(sg_gemm_fast(s->h1, w2h, w2l, s->h2, B, 1024, 1024, s->w + L.b2, 1, nsplit, st)))) return rc;
  if ((rc = hip_check(sg_gemm_fast(s->h2, w3h, w3l, s->h3, B, 1024, 1024, s->w + L.b3, 1, nsplit, st)))) return rc;
  // basis branch (linear): a = h3 Wa + ba, out = a Wb + bb; the decoder then adds its output
  if ((rc = hip_check(sg_gemm_fast(s->h3, wah, wal, s->a, B, kBasis, 1024, s->w + L.ba, 0, nsplit, st)))) return rc;
  if ((rc = hip_check(sg_gemm_fast(s->a, wbh, wbl, out, B, 4096, kBasis, s->w + L.bb, 0, nsplit, st)))) return rc;
  // decoder: B fragments of the two matrix-core layers, then one persistent launch
  __bf16* f1h = s->decw;
  __bf16* f1l = f1h + 4 * DK1 * 64 * 8;
  __bf16* f2h = f1l + 4 * DK1 * 64 * 8;
  __bf16* f2l = f2h + 2 * DK2 * 64 * 8;
  const int nprep = (4 * DK1 + 2 * DK2) * 64 * 8;
  hipLaunchKernelGGL(sg_dec_wprep_kernel, dim3((nprep + 255) / 256), dim3(256), 0, st, s->w + L.K1, s->w + L.K2,
                     f1h, f1l, f2h, f2l);
  if ((rc = hip_check(hipGetLastError()))) return rc;
  const int grid = std::min(B, 2 * s->num_cus);
  const bf8_t* F1h = reinterpret_cast<const bf8_t*>(f1h);
  const bf8_t* F1l = reinterpret_cast<const bf8_t*>(f1l);
  const bf8_t* F2h = reinterpret_cast<const bf8_t*>(f2h);
  const bf8_t* F2l = reinterpret_cast<const bf8_t*>(f2l);
  float* d1 = keep ? s->d1 : nullptr;
  float* d2 = keep ? s->d2 : nullptr;
  if (nsplit > 1)
    hipLaunchKernelGGL(sg_decoder_kernel<3>, dim3(grid), dim3(256), kDecLdsBytes, st, s->h3, B, F1h, F1l, F2h, F2l,
                       s->w + L.c1, s->w + L.c2, s->w + L.K3, s->w + L.c3, out, d1, d2);
  else
    hipLaunchKernelGGL(sg_decoder_kernel<1>, dim3(grid), dim3(256), kDecLdsBytes, st, s->h3, B, F1h, F1l, F2h, F2l,
                       s->w + L.c1, s->w + L.c2, s->w + L.K3, s->w + L.c3, out, d1, d2);
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
                         {s->h3, s->g3, s->gd1, 16, 16, 8, L.K1, L.c1, true}};
  // weights split to BF16 in their own order: B operands of the products g W^T
  __bf16* w3h = s->wsplit_t;
  __bf16* w3l = w3h + 1024 * 1024;
  __bf16* w2h = w3l + 1024 * 1024;
  __bf16* w2l = w2h + 1024 * 1024;
  __bf16* wah = w2l + 1024 * 1024;
  __bf16* wal = wah + 1024 * kBasis;
  __bf16* wbh = wal + 1024 * kBasis;
  __bf16* wbl = wbh + kBasis * 4096;
  const struct { size_t off, n; __bf16 *h, *l; } splits[4] = {{L.W3, 1024 * 1024, w3h, w3l},
                                                              {L.W2, 1024 * 1024, w2h, w2l},
                                                              {L.Wa, 1024 * (size_t)kBasis, wah, wal},
                                                              {L.Wb, (size_t)kBasis * 4096, wbh, wbl}};
  for (const auto& sp : splits)
    hipLaunchKernelGGL(sg_split_kernel, dim3((unsigned)((sp.n + 255) / 256)), dim3(256), 0, st, s->w + sp.off, sp.n,
                       sp.h, sp.l);
  if ((rc = hip_check(hipGetLastError()))) return rc;
  const int twg = 2 * s->num_cus;
  // basis branch first: dWb = a^T gy, dbb, ga = gy Wb^T, dWa = h3^T ga, dba; its gradient of
  // h3 joins the convolution branch's before the relu mask
  if ((rc = hip_check(sg_gemm<true, false>(s->a, kBasis, s->gy, 4096, s->g + L.Wb, 4096, kBasis, 4096, B, nullptr, 0,
                                           3, st)))) return rc;
  if ((rc = hip_check(sg_colsum(s->gy, B, 4096, s->g + L.bb, s->colpart, st)))) return rc;
  if ((rc = hip_check(sg_gemm_fast(s->gy, wbh, wbl, s->ga, B, kBasis, 4096, nullptr, 0, 3, st, 0, s->ws,
                                   kSplitKFloats, twg)))) return rc;
  if ((rc = hip_check(sg_gemm<true, false>(s->h3, 1024, s->ga, kBasis, s->g + L.Wa, kBasis, 1024, kBasis, B, nullptr,
                                           0, 3, st)))) return rc;
  if ((rc = hip_check(sg_colsum(s->ga, B, kBasis, s->g + L.ba, s->colpart, st)))) return rc;
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
    // h3 also feeds the basis branch: g3 += ga Wa^T before the relu mask
    if (c.gin == s->g3 &&
        (rc = hip_check(sg_gemm_fast(s->ga, wah, wal, s->g3, B, 1024, kBasis, nullptr, 0, 3, st, 1, s->ws,
                                     kSplitKFloats, twg)))) return rc;
    const size_t n = (size_t)B * c.Ci * c.H * c.H;
    hipLaunchKernelGGL(sg_relu_mask_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, c.gin, c.in, n);
    if ((rc = hip_check(hipGetLastError()))) return rc;
  }
  // dense layers: g3 = dL/d(pre3) already masked
  struct Dense { float *hin, *gin, *gout; int in, out; size_t W, b; const float* hmask; const __bf16 *th, *tl; };
  const Dense dense[3] = {{s->h2, s->g2, s->g3, 1024, 1024, L.W3, L.b3, s->h2, w3h, w3l},
                          {s->h1, s->g1, s->g2, 1024, 1024, L.W2, L.b2, s->h1, w2h, w2l},
                          {s->x, s->gx, s->g1, 22, 1024, L.W1, L.b1, nullptr, nullptr, nullptr}};
  for (const Dense& d : dense) {
    // dW = hin^T gout  (in x out, K = B), db = column sums, gin = gout W^T
    if ((rc = hip_check(sg_gemm<true, false>(d.hin, d.in, d.gout, d.out, s->g + d.W, d.out, d.in, d.out, B, nullptr, 0, 3, st)))) return rc;
    if ((rc = hip_check(sg_colsum(d.gout, B, d.out, s->g + d.b, s->colpart, st)))) return rc;
    if (d.hmask) {
      if ((rc = hip_check(sg_gemm_fast(d.gout, d.th, d.tl, d.gin, B, d.in, d.out, nullptr, 0, 3, st, 0, s->ws,
                                       kSplitKFloats, twg)))) return rc;
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
      (rc = sg_alloc(s, &s->v, P)) || (rc = sg_alloc(s, &s->x, B * 22)) || (rc = sg_alloc(s, &s->h1, B * 1024)) ||
      (rc = sg_alloc(s, &s->h2, B * 1024)) || (rc = sg_alloc(s, &s->h3, B * 1024)) ||
      (rc = sg_alloc(s, &s->d1, B * 4096)) || (rc = sg_alloc(s, &s->d2, B * 8192)) ||
      (rc = sg_alloc(s, &s->y, B * 4096)) || (rc = sg_alloc(s, &s->gx, B * 22)) ||
      (rc = sg_alloc(s, &s->g1, B * 1024)) || (rc = sg_alloc(s, &s->g2, B * 1024)) ||
      (rc = sg_alloc(s, &s->g3, B * 1024)) || (rc = sg_alloc(s, &s->gd1, B * 4096)) ||
      (rc = sg_alloc(s, &s->gd2, B * 8192)) || (rc = sg_alloc(s, &s->gy, B * 4096)) ||
      (rc = sg_alloc(s, &s->partial, (size_t)chunks * (16 * 16 * 16 + 16))) ||
      (rc = sg_alloc(s, &s->loss_partial, 256)) || (rc = sg_alloc(s, &s->decw, 2 * (4 * DK1 + 2 * DK2) * 64 * 8)) ||
      (rc = sg_alloc(s, &s->a, B * kBasis)) || (rc = sg_alloc(s, &s->ga, B * kBasis)) ||
      (rc = sg_alloc(s, &s->wsplit, 2 * (1024 * 1024 + 1024 * 1024 + 1024 * kBasis + kBasis * 4096))) ||
      (rc = sg_alloc(s, &s->wsplit_t, 2 * (1024 * 1024 + 1024 * 1024 + 1024 * kBasis + kBasis * 4096))) ||
      (rc = sg_alloc(s, &s->ws, kSplitKFloats)) || (rc = sg_alloc(s, &s->colpart, kColChunks * 4096))) {
    delete s;
    return rc;
  }
  if (hipDeviceGetAttribute(&s->num_cus, hipDeviceAttributeMultiprocessorCount, s->device) != hipSuccess ||
      s->num_cus < 1) {
    delete s;
    return RWPSF_ERR_NO_DEVICE;
  }
  const int fast_lds = 2 * 4 * FBM * FLD * (int)sizeof(__bf16);
  if ((rc = hip_check(hipFuncSetAttribute((const void*)sg_gemm_fast_kernel<1>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, fast_lds))) ||
      (rc = hip_check(hipFuncSetAttribute((const void*)sg_gemm_fast_kernel<3>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, fast_lds))) ||
      (rc = hip_check(hipFuncSetAttribute((const void*)sg_decoder_kernel<1>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, kDecLdsBytes))) ||
      (rc = hip_check(hipFuncSetAttribute((const void*)sg_decoder_kernel<3>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, kDecLdsBytes)))) {
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
  return rw::sg_forward_impl(s, B, coef, z, out, precision == RWPSF_SG_BF16X3 ? 3 : 1, false, (hipStream_t)stream);
}

int rwpsf_sg_gradient(rwpsf_sg* s, int B, const float* coef, const float* z, const float* target, float* loss,
                      void* stream) {
  if (!s || B < 1 || B > s->max_batch || !coef || !z || !target) return RWPSF_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  int rc = rw::sg_forward_impl(s, B, coef, z, s->y, 3, true, st);
  if (rc) return rc;
  return rw::sg_backward_impl(s, B, target, loss, st);
}

int rwpsf_sg_error_features(int B, const float* coef, const float* z, float* phi, void* stream) {
  if (B < 1 || !coef || !z || !phi) return RWPSF_ERR_INVALID_ARG;
  const long long n = (long long)B * rw::kGateFeatures;
  hipLaunchKernelGGL(rw::sg_gate_features_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, coef, z, B, phi);
  return rw::hip_check(hipGetLastError());
}

int rwpsf_sg_error_predict(int B, const float* coef, const float* z, const float* weights, float* log_err,
                           void* stream) {
  if (B < 1 || !coef || !z || !weights || !log_err) return RWPSF_ERR_INVALID_ARG;
  hipLaunchKernelGGL(rw::sg_gate_predict_kernel, dim3((B + 255) / 256), dim3(256), 0, (hipStream_t)stream, coef, z, B,
                     weights, log_err);
  return rw::hip_check(hipGetLastError());
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
