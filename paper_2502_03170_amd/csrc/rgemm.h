// Real FP32 GEMM tile engine on the CDNA3/4 matrix cores (v_mfma_f32_32x32x2_f32).
//
// A workgroup computes a BM x BN tile of C = A * B with BM/WM x BN/WN waves, each
// owning a WM x WN tile made of 32 x 32 MFMA blocks.  Both operands are staged in
// LDS k-major ([k][row] and [k][col], rows padded by 4 words) so that the 32 lanes
// of a half-wave read 32 consecutive words.  Two LDS stages: the global loads of
// stage k+1 are issued before the MFMAs of stage k and written to LDS after them.
//
// MFMA 32x32x2 f32 lane layout (wave64): A operand lane l holds A[l%32][l/32],
// B operand lane l holds B[l/32][l%32]; accumulator register r of lane l holds
// C[(r/4)*8 + (l/32)*4 + r%4][l%32].
#pragma once

#include <hip/hip_runtime.h>

namespace rw {

typedef float rg16v __attribute__((ext_vector_type(16)));

template <int BM_, int BN_, int BK_, int WM_, int WN_>
struct RgCfg {
  static constexpr int BM = BM_, BN = BN_, BK = BK_, WM = WM_, WN = WN_;
  static constexpr int WAVES_M = BM / WM, WAVES_N = BN / WN;
  static constexpr int NWAVES = WAVES_M * WAVES_N;
  static constexpr int NT = NWAVES * 64;
  static constexpr int TM = WM / 32, TN = WN / 32;
  static constexpr int LDA = BM + 4, LDB = BN + 4;
  static constexpr int A_FLOATS = BK * LDA;
  static constexpr int B_FLOATS = BK * LDB;
  static constexpr int STAGE_FLOATS = A_FLOATS + B_FLOATS;
  static constexpr int LDS_BYTES = 2 * STAGE_FLOATS * 4;
  static_assert(BM % WM == 0 && BN % WN == 0 && WM % 32 == 0 && WN % 32 == 0, "tile shape");
  static_assert(BK % 2 == 0, "k-pairs");
};

// Loader of a k-major real operand: element (k, c) at src[k * ld + c].  Operands are
// zero-padded to whole tiles (rows to a multiple of BK, columns to a multiple of the
// tile width, ld a multiple of 4), so every load is an unconditional aligned float4.
template <class Cfg, int BW>
struct RKMajorLoader {
  static constexpr int QUADS_PER_ROW = BW / 4;
  static constexpr int PER_THREAD = Cfg::BK * QUADS_PER_ROW / Cfg::NT;
  static_assert(Cfg::BK * QUADS_PER_ROW % Cfg::NT == 0, "loader shape");
  const float* src;  // already offset to column c0
  int ld;
  float4 v[PER_THREAD];

  __device__ void load(int k0, int tid) {
#pragma unroll
    for (int i = 0; i < PER_THREAD; ++i) {
      const int idx = tid + i * Cfg::NT;
      const int kk = idx / QUADS_PER_ROW;
      const int cc = 4 * (idx % QUADS_PER_ROW);
      v[i] = *reinterpret_cast<const float4*>(src + (size_t)(k0 + kk) * ld + cc);
    }
  }
  __device__ void store(float* dst, int ldl, int tid) const {
#pragma unroll
    for (int i = 0; i < PER_THREAD; ++i) {
      const int idx = tid + i * Cfg::NT;
      const int kk = idx / QUADS_PER_ROW;
      const int cc = 4 * (idx % QUADS_PER_ROW);
      *reinterpret_cast<float4*>(dst + kk * ldl + cc) = v[i];
    }
  }
};

template <class Cfg>
struct RgAcc {
  rg16v c[Cfg::TM][Cfg::TN];
  __device__ void zero() {
#pragma unroll
    for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
      for (int j = 0; j < Cfg::TN; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) c[i][j][r] = 0.f;
  }
};

template <class Cfg>
__device__ __forceinline__ void rg_stage_mma(RgAcc<Cfg>& acc, const float* a, const float* b, int wrow,
                                             int wcol, int lane) {
  const int h = lane >> 5, l32 = lane & 31;
#pragma unroll
  for (int kp = 0; kp < Cfg::BK / 2; ++kp) {
    const int kk = 2 * kp + h;
    float av[Cfg::TM], bv[Cfg::TN];
#pragma unroll
    for (int i = 0; i < Cfg::TM; ++i) av[i] = a[kk * Cfg::LDA + wrow + 32 * i + l32];
#pragma unroll
    for (int j = 0; j < Cfg::TN; ++j) bv[j] = b[kk * Cfg::LDB + wcol + 32 * j + l32];
#pragma unroll
    for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
      for (int j = 0; j < Cfg::TN; ++j)
        acc.c[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i], bv[j], acc.c[i][j], 0, 0, 0);
  }
}

// K loop over [k_begin, k_end) (multiples of BK, k_end > k_begin) with double-buffered LDS.
// The loaders provide load(k0, tid) and store(lds_tile, ld, tid).
template <class Cfg, class ALoader, class BLoader>
__device__ __forceinline__ void rg_mainloop(RgAcc<Cfg>& acc, ALoader& la, BLoader& lb, int k_begin, int k_end,
                                            float* lds, int tid, int wrow, int wcol, int lane) {
  // stage pointers by arithmetic on the __shared__ base (a pointer picked from a
  // local array loses its address space and turns the LDS reads into flat loads)
  const int KT = (k_end - k_begin) / Cfg::BK;
  la.load(k_begin, tid);
  lb.load(k_begin, tid);
  la.store(lds, Cfg::LDA, tid);
  lb.store(lds + Cfg::A_FLOATS, Cfg::LDB, tid);
  __syncthreads();
  for (int kt = 0; kt < KT; ++kt) {
    float* cur = lds + (kt & 1) * Cfg::STAGE_FLOATS;
    float* nxt = lds + ((kt + 1) & 1) * Cfg::STAGE_FLOATS;
    const bool more = kt + 1 < KT;
    if (more) {
      la.load(k_begin + (kt + 1) * Cfg::BK, tid);
      lb.load(k_begin + (kt + 1) * Cfg::BK, tid);
    }
    rg_stage_mma<Cfg>(acc, cur, cur + Cfg::A_FLOATS, wrow, wcol, lane);
    if (more) {
      la.store(nxt, Cfg::LDA, tid);
      lb.store(nxt + Cfg::A_FLOATS, Cfg::LDB, tid);
    }
    __syncthreads();
  }
}

// Row/column of accumulator register r in 32 x 32 block (i, j) of this wave.
__device__ __forceinline__ int rg_row(int wrow, int i, int r, int lane) {
  return wrow + 32 * i + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
}
__device__ __forceinline__ int rg_col(int wcol, int j, int lane) { return wcol + 32 * j + (lane & 31); }

}  // namespace rw
