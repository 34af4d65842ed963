// Real FP32 GEMM tile engine on the CDNA3/4 matrix cores (v_mfma_f32_32x32x2_f32).
//
// A workgroup computes a BM x BN tile of C = A * B with BM/WM x BN/WN waves, each
// owning a WM x WN tile made of 32 x 32 MFMA blocks.  Both operands are staged in LDS
// with k contiguous ([row][k] and [col][k], rows padded to BK + 4 words so that a
// half-wave's 16-byte reads of 32 rows fall in distinct banks).  A lane half reads four
// consecutive k with one ds_read_b128 and feeds them to four MFMAs: in k-group u,
// instruction t takes k = 8u + t from lanes 0-31 and k = 8u + 4 + t from lanes 32-63,
// for A and B alike, so every k of the stage is summed once.  Two LDS stages: the
// global loads of stage k+1 are issued before the MFMAs of stage k and written to
// LDS after them; the loaders return the staged data by value, so it stays in
// registers (a loader holding it in a member array ends up in scratch memory).
//
// MFMA 32x32x2 f32 lane layout (wave64): A operand lane l holds A[l%32][k(l/32)],
// B operand lane l holds B[k(l/32)][l%32]; accumulator register r of lane l holds
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
  static constexpr int LDK = BK + 4;   // words per staged row
  static constexpr int A_FLOATS = BM * LDK;
  static constexpr int B_FLOATS = BN * LDK;
  static constexpr int STAGE_FLOATS = A_FLOATS + B_FLOATS;
  static constexpr int LDS_BYTES = 2 * STAGE_FLOATS * 4;
  static_assert(BM % WM == 0 && BN % WN == 0 && WM % 32 == 0 && WN % 32 == 0, "tile shape");
  static_assert(BK % 8 == 0, "k-groups of 8");
};

// Loader of an operand stored with k contiguous in memory: element (row, k) at
// src[row * ld + k], staged to LDS as [row][k].  Operands are zero-padded to whole tiles
// (rows to the tile height, k to a multiple of BK, ld a multiple of 4), so every load is
// an unconditional aligned float4.
template <class Cfg, int ROWS>
struct RRowLoader {
  static constexpr int QUADS = Cfg::BK / 4;
  static constexpr int TOTAL = ROWS * QUADS;
  static constexpr int PER_THREAD = (TOTAL + Cfg::NT - 1) / Cfg::NT;   // the last round may be partial
  const float* src;  // already offset to row r0
  int ld;
  struct Regs {
    float4 v[PER_THREAD];
  };

  __device__ Regs load(int k0, int tid) const {
    Regs r;
#pragma unroll
    for (int i = 0; i < PER_THREAD; ++i) {
      const int idx = tid + i * Cfg::NT;
      if (TOTAL % Cfg::NT != 0 && idx >= TOTAL) break;
      const int row = idx / QUADS, kq = 4 * (idx % QUADS);
      r.v[i] = *reinterpret_cast<const float4*>(src + (size_t)row * ld + k0 + kq);
    }
    return r;
  }
  __device__ void store(float* dst, int tid, const Regs& r) const {
#pragma unroll
    for (int i = 0; i < PER_THREAD; ++i) {
      const int idx = tid + i * Cfg::NT;
      if (TOTAL % Cfg::NT != 0 && idx >= TOTAL) break;
      const int row = idx / QUADS, kq = 4 * (idx % QUADS);
      *reinterpret_cast<float4*>(dst + row * Cfg::LDK + kq) = r.v[i];
    }
  }
};

// Loader of an operand stored k-major in memory: element (row, k) at src[k * ld + row],
// staged to LDS as [row][k].  Each thread moves a 2 (k) x 4 (rows) block: two float4
// loads along the rows, transposed in registers into four 8-byte LDS writes along k.
// Consecutive lanes take consecutive k-pairs of the same rows, so a half-wave's writes
// cover consecutive words of one LDS row (no bank conflicts).
template <class Cfg, int ROWS>
struct RColLoader {
  static constexpr int KPAIRS = Cfg::BK / 2, QUADS = ROWS / 4;
  static constexpr int TOTAL = KPAIRS * QUADS;
  static constexpr int PER_THREAD = (TOTAL + Cfg::NT - 1) / Cfg::NT;   // the last round may be partial
  const float* src;  // already offset to row r0
  int ld;
  struct Regs {
    float4 v0[PER_THREAD], v1[PER_THREAD];
  };

  __device__ Regs load(int k0, int tid) const {
    Regs r;
#pragma unroll
    for (int i = 0; i < PER_THREAD; ++i) {
      const int idx = tid + i * Cfg::NT;
      if (TOTAL % Cfg::NT != 0 && idx >= TOTAL) break;
      const int kk = 2 * (idx % KPAIRS), rq = 4 * (idx / KPAIRS);
      const float* p = src + (size_t)(k0 + kk) * ld + rq;
      r.v0[i] = *reinterpret_cast<const float4*>(p);
      r.v1[i] = *reinterpret_cast<const float4*>(p + ld);
    }
    return r;
  }
  __device__ void store(float* dst, int tid, const Regs& r) const {
    const float4* v0 = r.v0;
    const float4* v1 = r.v1;
#pragma unroll
    for (int i = 0; i < PER_THREAD; ++i) {
      const int idx = tid + i * Cfg::NT;
      if (TOTAL % Cfg::NT != 0 && idx >= TOTAL) break;
      const int kk = 2 * (idx % KPAIRS), rq = 4 * (idx / KPAIRS);
      float* d = dst + rq * Cfg::LDK + kk;
      *reinterpret_cast<float2*>(d) = make_float2(v0[i].x, v1[i].x);
      *reinterpret_cast<float2*>(d + Cfg::LDK) = make_float2(v0[i].y, v1[i].y);
      *reinterpret_cast<float2*>(d + 2 * Cfg::LDK) = make_float2(v0[i].z, v1[i].z);
      *reinterpret_cast<float2*>(d + 3 * Cfg::LDK) = make_float2(v0[i].w, v1[i].w);
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
  for (int u = 0; u < Cfg::BK / 8; ++u) {
    const int k = 8 * u + 4 * h;
    float4 av[Cfg::TM], bv[Cfg::TN];
#pragma unroll
    for (int i = 0; i < Cfg::TM; ++i)
      av[i] = *reinterpret_cast<const float4*>(a + (wrow + 32 * i + l32) * Cfg::LDK + k);
#pragma unroll
    for (int j = 0; j < Cfg::TN; ++j)
      bv[j] = *reinterpret_cast<const float4*>(b + (wcol + 32 * j + l32) * Cfg::LDK + k);
#pragma unroll
    for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
      for (int j = 0; j < Cfg::TN; ++j)
        acc.c[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i].x, bv[j].x, acc.c[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
      for (int j = 0; j < Cfg::TN; ++j)
        acc.c[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i].y, bv[j].y, acc.c[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
      for (int j = 0; j < Cfg::TN; ++j)
        acc.c[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i].z, bv[j].z, acc.c[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < Cfg::TM; ++i)
#pragma unroll
      for (int j = 0; j < Cfg::TN; ++j)
        acc.c[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i].w, bv[j].w, acc.c[i][j], 0, 0, 0);
  }
}

// K loop whose first stage (k_begin) the caller has already loaded into registers
// (ra0, rb0), so that a caller can issue those loads before other memory work.
// The last stage is peeled so that the loop body has no branch around the loads and
// stores (a conditional there leaves the staged registers in scratch memory).  ORDER
// places scheduling barriers: without them (kOrderFree) the compiler tends to sink the
// global loads of the next stage to the end of the MFMA stream, right before their
// LDS stores, and a wave then waits out the load latency once per stage.
// kOrderLoadsFirst pins the loads ahead of the MFMAs and leaves the loader's
// arithmetic free to interleave with them; kOrderFull also keeps that arithmetic and
// the stores after the MFMAs.  Which order is faster depends on the loader (measured
// per kernel).
constexpr int kOrderFree = 0, kOrderFull = 1, kOrderLoadsFirst = 2;
template <class Cfg, int ORDER, class ALoader, class BLoader>
__device__ __forceinline__ void rg_mainloop_pre(RgAcc<Cfg>& acc, const ALoader& la, const BLoader& lb,
                                                const typename ALoader::Regs& ra0,
                                                const typename BLoader::Regs& rb0, int k_begin, int k_end,
                                                float* lds, int tid, int wrow, int wcol, int lane) {
  // stage pointers by arithmetic on the __shared__ base (a pointer picked from a
  // local array loses its address space and turns the LDS reads into flat loads)
  const int KT = (k_end - k_begin) / Cfg::BK;
  la.store(lds, tid, ra0);
  lb.store(lds + Cfg::A_FLOATS, tid, rb0);
  __syncthreads();
  for (int kt = 0; kt < KT - 1; ++kt) {
    float* cur = lds + (kt & 1) * Cfg::STAGE_FLOATS;
    float* nxt = lds + ((kt + 1) & 1) * Cfg::STAGE_FLOATS;
    const auto ra = la.load(k_begin + (kt + 1) * Cfg::BK, tid);
    const auto rb = lb.load(k_begin + (kt + 1) * Cfg::BK, tid);
    if constexpr (ORDER != kOrderFree) __builtin_amdgcn_sched_barrier(0);
    rg_stage_mma<Cfg>(acc, cur, cur + Cfg::A_FLOATS, wrow, wcol, lane);
    if constexpr (ORDER == kOrderFull) __builtin_amdgcn_sched_barrier(0);
    la.store(nxt, tid, ra);
    lb.store(nxt + Cfg::A_FLOATS, tid, rb);
    __syncthreads();
  }
  float* last = lds + ((KT - 1) & 1) * Cfg::STAGE_FLOATS;
  rg_stage_mma<Cfg>(acc, last, last + Cfg::A_FLOATS, wrow, wcol, lane);
  __syncthreads();
}

// K loop over [k_begin, k_end) (multiples of BK, k_end > k_begin) with double-buffered
// LDS.  The loaders provide Regs load(k0, tid) and store(lds_tile, tid, regs).
template <class Cfg, int ORDER, class ALoader, class BLoader>
__device__ __forceinline__ void rg_mainloop(RgAcc<Cfg>& acc, const ALoader& la, const BLoader& lb, int k_begin,
                                            int k_end, float* lds, int tid, int wrow, int wcol, int lane) {
  const auto ra = la.load(k_begin, tid);
  const auto rb = lb.load(k_begin, tid);
  rg_mainloop_pre<Cfg, ORDER>(acc, la, lb, ra, rb, k_begin, k_end, lds, tid, wrow, wcol, lane);
}

// Row/column of accumulator register r in 32 x 32 block (i, j) of this wave.
__device__ __forceinline__ int rg_row(int wrow, int i, int r, int lane) {
  return wrow + 32 * i + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
}
__device__ __forceinline__ int rg_col(int wcol, int j, int lane) { return wcol + 32 * j + (lane & 31); }

}  // namespace rw
