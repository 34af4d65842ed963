// Complex FP32 GEMM tile engine on the CDNA3/4 matrix cores (v_mfma_f32_32x32x2_f32).
//
// A workgroup computes a BM x BN tile of C = A * B (complex, FP32 accumulate)
// with BM/WM x BN/WN waves, each owning a WM x WN tile made of 32 x 32 MFMA
// blocks.  Complex products use four real MFMAs per block and k-pair:
//   Cr += Ar Br - Ai Bi,  Ci += Ar Bi + Ai Br
// Operands are staged in LDS as separate real and imaginary planes laid out
// k-major ([k][row] and [k][col]) so that the 32 lanes of a half-wave read 32
// consecutive words.  Two LDS stages: global loads of stage k+1 are issued
// before the MFMAs of stage k and written to LDS after them.
//
// MFMA 32x32x2 f32 lane layout (wave64): A operand lane l holds A[l%32][l/32],
// B operand lane l holds B[l/32][l%32]; accumulator register r of lane l holds
// C[(r/4)*8 + (l/32)*4 + r%4][l%32].
#pragma once

#include <hip/hip_runtime.h>

namespace rw {

typedef float f16v __attribute__((ext_vector_type(16)));

template <int BM_, int BN_, int BK_, int WM_, int WN_>
struct CgCfg {
  static constexpr int BM = BM_, BN = BN_, BK = BK_, WM = WM_, WN = WN_;
  static constexpr int WAVES_M = BM / WM, WAVES_N = BN / WN;
  static constexpr int NWAVES = WAVES_M * WAVES_N;
  static constexpr int NT = NWAVES * 64;
  static constexpr int TM = WM / 32, TN = WN / 32;
  static constexpr int LDA = BM + 4, LDB = BN + 4;
  static constexpr int A_FLOATS = 2 * BK * LDA;   // re + im planes
  static constexpr int B_FLOATS = 2 * BK * LDB;
  static constexpr int STAGE_FLOATS = A_FLOATS + B_FLOATS;
  static constexpr int LDS_BYTES = 2 * STAGE_FLOATS * 4;
  static_assert(BM % WM == 0 && BN % WN == 0 && WM % 32 == 0 && WN % 32 == 0, "tile shape");
  static_assert(BK % 2 == 0, "k-pairs");
};

// Loader of a k-major complex operand: element (k, c) at src[k * ld + c], used
// for B operands ([k][n]) and for constant A operands stored transposed ([k][m]).
// Operands are zero-padded to whole tiles (rows to a multiple of BK, columns to
// a multiple of the tile width, ld even), so every load is an unconditional,
// aligned float4 (two adjacent complex values) and the prefetch stays in flight
// while the MFMAs of the current stage run.
template <class Cfg, int BW>
struct KMajorLoader {
  static constexpr int PAIRS_PER_ROW = BW / 2;
  static constexpr int PER_THREAD = Cfg::BK * PAIRS_PER_ROW / Cfg::NT;
  static_assert(Cfg::BK * PAIRS_PER_ROW % Cfg::NT == 0, "loader shape");
  const float2* src;  // already offset to column c0
  int ld;
  float4 v[PER_THREAD];

  __device__ void load(int k0, int tid) {
#pragma unroll
    for (int i = 0; i < PER_THREAD; ++i) {
      const int idx = tid + i * Cfg::NT;
      const int kk = idx / PAIRS_PER_ROW;
      const int cc = 2 * (idx % PAIRS_PER_ROW);
      v[i] = *reinterpret_cast<const float4*>(src + (size_t)(k0 + kk) * ld + cc);
    }
  }
  __device__ void store(float* re, float* im, int ldl, int tid) const {
#pragma unroll
    for (int i = 0; i < PER_THREAD; ++i) {
      const int idx = tid + i * Cfg::NT;
      const int kk = idx / PAIRS_PER_ROW;
      const int cc = 2 * (idx % PAIRS_PER_ROW);
      *reinterpret_cast<float2*>(re + kk * ldl + cc) = make_float2(v[i].x, v[i].z);
      *reinterpret_cast<float2*>(im + kk * ldl + cc) = make_float2(v[i].y, v[i].w);
    }
  }
};

template <class Cfg>
struct CgAcc {
  f16v re[Cfg::TM][Cfg::TN];
  f16v im[Cfg::TM][Cfg::TN];
  __device__ void zero() {
#pragma unroll
    for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
      for (int j = 0; j < Cfg::TN; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) { re[i][j][r] = 0.f; im[i][j][r] = 0.f; }
  }
};

// MFMAs over one LDS stage.
template <class Cfg>
__device__ __forceinline__ void cg_stage_mma(CgAcc<Cfg>& acc, const float* a_re, const float* a_im,
                                             const float* b_re, const float* b_im, int wrow,
                                             int wcol, int lane) {
  const int h = lane >> 5, l32 = lane & 31;
#pragma unroll
  for (int kp = 0; kp < Cfg::BK / 2; ++kp) {
    const int kk = 2 * kp + h;
    float ar[Cfg::TM], ai[Cfg::TM], an[Cfg::TM], br[Cfg::TN], bi[Cfg::TN];
#pragma unroll
    for (int i = 0; i < Cfg::TM; ++i) {
      ar[i] = a_re[kk * Cfg::LDA + wrow + 32 * i + l32];
      ai[i] = a_im[kk * Cfg::LDA + wrow + 32 * i + l32];
      an[i] = -ai[i];
    }
#pragma unroll
    for (int j = 0; j < Cfg::TN; ++j) {
      br[j] = b_re[kk * Cfg::LDB + wcol + 32 * j + l32];
      bi[j] = b_im[kk * Cfg::LDB + wcol + 32 * j + l32];
    }
    // four passes over the blocks so that dependent MFMAs are TM*TN issues apart
#pragma unroll
    for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
      for (int j = 0; j < Cfg::TN; ++j)
        acc.re[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[i], br[j], acc.re[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
      for (int j = 0; j < Cfg::TN; ++j)
        acc.im[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[i], bi[j], acc.im[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
      for (int j = 0; j < Cfg::TN; ++j)
        acc.re[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(an[i], bi[j], acc.re[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
      for (int j = 0; j < Cfg::TN; ++j)
        acc.im[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[i], br[j], acc.im[i][j], 0, 0, 0);
  }
}

// K loop over [k_begin, k_end): acc += A[rows, k] * B[k, cols] with double-buffered LDS
// (both bounds multiples of BK, k_end > k_begin).
template <class Cfg, class ALoader, class BLoader>
__device__ __forceinline__ void cg_mainloop(CgAcc<Cfg>& acc, ALoader& la, BLoader& lb, int k_begin,
                                            int k_end, float* lds, int tid, int wrow, int wcol, int lane);

template <class Cfg, class ALoader, class BLoader>
__device__ __forceinline__ void cg_mainloop(CgAcc<Cfg>& acc, ALoader& la, BLoader& lb, int K,
                                            float* lds, int tid, int wrow, int wcol, int lane) {
  cg_mainloop<Cfg>(acc, la, lb, 0, K, lds, tid, wrow, wcol, lane);
}

template <class Cfg, class ALoader, class BLoader>
__device__ __forceinline__ void cg_mainloop(CgAcc<Cfg>& acc, ALoader& la, BLoader& lb, int k_begin,
                                            int k_end, float* lds, int tid, int wrow, int wcol, int lane) {
  // stage pointers by arithmetic on the __shared__ base: a pointer picked from a
  // local array loses its address space and turns the LDS reads into flat loads
  const int KT = (k_end - k_begin) / Cfg::BK;
  la.load(k_begin, tid);
  lb.load(k_begin, tid);
  la.store(lds, lds + Cfg::BK * Cfg::LDA, Cfg::LDA, tid);
  lb.store(lds + Cfg::A_FLOATS, lds + Cfg::A_FLOATS + Cfg::BK * Cfg::LDB, Cfg::LDB, tid);
  __syncthreads();
  for (int kt = 0; kt < KT; ++kt) {
    float* cur = lds + (kt & 1) * Cfg::STAGE_FLOATS;
    float* nxt = lds + ((kt + 1) & 1) * Cfg::STAGE_FLOATS;
    const bool more = kt + 1 < KT;
    if (more) {
      la.load(k_begin + (kt + 1) * Cfg::BK, tid);
      lb.load(k_begin + (kt + 1) * Cfg::BK, tid);
    }
    cg_stage_mma<Cfg>(acc, cur, cur + Cfg::BK * Cfg::LDA, cur + Cfg::A_FLOATS,
                      cur + Cfg::A_FLOATS + Cfg::BK * Cfg::LDB, wrow, wcol, lane);
    if (more) {
      la.store(nxt, nxt + Cfg::BK * Cfg::LDA, Cfg::LDA, tid);
      lb.store(nxt + Cfg::A_FLOATS, nxt + Cfg::A_FLOATS + Cfg::BK * Cfg::LDB, Cfg::LDB, tid);
    }
    __syncthreads();
  }
}

// Row/column of accumulator register r in 32 x 32 block (i, j) of this wave.
__device__ __forceinline__ int cg_row(int wrow, int i, int r, int lane) {
  return wrow + 32 * i + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
}
__device__ __forceinline__ int cg_col(int wcol, int j, int lane) { return wcol + 32 * j + (lane & 31); }

// Workgroup ids are dealt round-robin over the 8 XCDs of the chip; renumber them
// so that consecutive logical ids run on the same XCD (and share its L2).
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  const int per = nblocks / 8;
  const int rem = nblocks % 8;
  const int xcd = bid % 8, slot = bid / 8;
  if (slot >= per) return bid;   // the ragged last round keeps its id (ids >= 8*per)
  (void)rem;
  return xcd * per + slot;
}

}  // namespace rw
