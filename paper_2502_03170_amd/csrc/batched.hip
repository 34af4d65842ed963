// Batched emitters: the Fourier form (Sec. 3.3 eq. "cartesian vectorial" with the
// Sec. 3.4 correction factors) for thousands of emitters with individual sub-pixel
// position, axial position, Zernike vector (Sec. 3.4.2), crop size and plane count,
// in one persistent launch per tile class.
//
// Per emitter b the pupil phase is
//   Phi_b[j,l] = 2 pi sum_q c_bq Z_q(s) - k (s_x x0_b + s_y y0_b)
// formed for all emitters at once by one real GEMM on the matrix cores,
//   Phi[b][cell] = sum_k coef[k][b] basis[k][cell],  basis = (2 pi Z_1..Z_21, s_x, s_y).
// The cell-centred grids are mirror-symmetric, so each emitter's pupil is folded once
// (four parities per folded cell, written to the emitter's HBM slot) and each plane d of
// each field component c is two real-coefficient GEMMs on the matrix cores,
//   U  = A2_S (D o Pf_c)    (S x N; D = exp(i k s_z z) of each folded cell, formed as the
//                            operand is staged: FP64 phase in revolutions, hardware sin/cos)
//   E' = U B1_S             (S x S, U staged in LDS as the A operand),  E = -i E'
// and I = sum_c |E_c|^2.  A2_S / B1_S are the rows of one 96-row table that cover the
// crop (pixel i of an S-crop is table row i - S/2 + 32).  Crops are evaluated on 32- or
// 64-wide tiles (the two tile classes); the (emitter, plane) items of each class are
// dealt, emitter by emitter and longest first, to eight queues, one per XCD, and the
// class's persistent kernel takes items from the queues' atomic counters until they are
// exhausted.
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
constexpr int kMaxWgPerCu = 4;  // workgroups per CU of the persistent launch (configuration bound)
constexpr int kQueues = 32;     // 8 XCD queues for each of the four tile classes (16 .. 64 rows)

struct BatchParam {
  double zoff;      // -z_e
  double ts;        // emitter depth below the coverslip (Gibson-Lanni)
  long long off;    // voxel offset of the emitter's output
  int S, D, SP, pad;
};

struct BatchArgs {
  const BatchParam* params;  // [n] cost-sorted (slot order)
  const float2* Q;           // [3][N][N]
  const double* ksz;         // [N][N]
  const float* phi;          // [n][N*N], slot order
  const double4* gl;         // [N*N] Gibson-Lanni phase W = t_s (g1.x + i g1.y) + (g0.x + i g0.y) as
                             // (g0.x, g0.y, g1.x, g1.y), or null without the layer
  const float* A2T;          // [N][96] rows 2jf + pj: pref cos / sin (k s_x[jf] x_r)
  const float* B1T;          // [N][96] rows 2lf + pl: cos / sin (k s_y[lf] y_r)
  float2* Pf;                // [n][3][N][N] folded pupils, slot order
  const int* list;           // [n] slots grouped by XCD queue
  const long long* pre;      // [n + 1] plane prefix sums over list
  const int* qoff;           // [17] queue q owns list[qoff[q] .. qoff[q+1]); queues 8 t + x of tile class t
  unsigned long long* counter;   // [16] next item of each queue
  float* I;
  float2* E;
  int n, N;
  double pitch;
};

// Each queue's counter starts at its first item (a kernel, not a memset, so that the
// launch sequence can be captured in a graph).
__global__ void batch_reset_kernel(unsigned long long* counter, const long long* pre, const int* qoff) {
  const int x = threadIdx.x;
  if (x < kQueues) counter[x] = (unsigned long long)pre[qoff[x]];
}

// Folded pupil of every emitter (one workgroup per emitter).  The pupil and pixel grids
// are mirror-symmetric (s[N-1-j] = -s[j]); with P = Q_c exp(i Phi) at the four mirror
// cells of (jf, lf),
//   Pf_{pj,pl}[jf][lf] = i^(pj+pl) sum_{a,b} (-1)^(a pj + b pl) P[mir_a(jf)][mir_b(lf)],
// stored at Pf[c][2jf + pj][2lf + pl].
__global__ void __launch_bounds__(256) batch_fold_kernel(BatchArgs a) {
  const int slot = blockIdx.x;
  const int N = a.N, NN = N * N, nh = N / 2;
  const float* phi = a.phi + (size_t)slot * NN;
  float2* Pf = a.Pf + (size_t)slot * 3 * NN;
  const double ts = a.params[slot].ts;
  for (int cell = threadIdx.x; cell < nh * nh; cell += 256) {
    const int jf = cell / nh, lf = cell % nh, j1 = N - 1 - jf, l1 = N - 1 - lf;
    const int idx[4] = {jf * N + lf, jf * N + l1, j1 * N + lf, j1 * N + l1};
    float er[4], ei[4];
    if (a.gl) {
      // the layer's phase is formed in FP64 and reduced mod 2 pi before it joins phi;
      // its imaginary part is the evanescent decay
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double4 g = a.gl[idx[q]];
        const double wr = ts * g.z + g.x, wi = ts * g.w + g.y;
        const float amp = (float)exp(-wi);
        float sn, cs;
        sincosf((float)reduce_2pi(wr + (double)phi[idx[q]]), &sn, &cs);
        er[q] = amp * cs;
        ei[q] = amp * sn;
      }
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) sincosf(phi[idx[q]], &ei[q], &er[q]);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float pr[4], pi[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float2 v = a.Q[(size_t)c * NN + idx[q]];
        pr[q] = v.x * er[q] - v.y * ei[q];
        pi[q] = v.x * ei[q] + v.y * er[q];
      }
      float2* o = Pf + (size_t)c * NN + (size_t)(2 * jf) * N + 2 * lf;
      // (pj, pl) = (0,0): +,+,+,+   (0,1): i(+,-,+,-)   (1,0): i(+,+,-,-)   (1,1): -(+,-,-,+)
      o[0] = make_float2(pr[0] + pr[1] + pr[2] + pr[3], pi[0] + pi[1] + pi[2] + pi[3]);
      o[1] = make_float2(-(pi[0] - pi[1] + pi[2] - pi[3]), pr[0] - pr[1] + pr[2] - pr[3]);
      o[N] = make_float2(-(pi[0] + pi[1] - pi[2] - pi[3]), pr[0] + pr[1] - pr[2] - pr[3]);
      o[N + 1] = make_float2(-(pr[0] - pr[1] - pr[2] + pr[3]), -(pi[0] - pi[1] - pi[2] + pi[3]));
    }
  }
}

// MFMA 32x32x2 f32: A lane l -> A[l%32][l/32], B lane l -> B[l/32][l%32],
// C register r of lane l -> C[8(r/4) + 4(l/32) + r%4][l%32].
//
// Plane d of emitter `slot`:  U = A2 (D o Pf_c)  (real x complex),  E' = U B1
// (complex x real),  E = -i E',  I = sum_c |E_c|^2, with the defocus D[jf][lf] =
// exp(i k s_z z) of the folded cell, the same for its four mirror cells.
template <int SP, int BK>
__device__ __forceinline__ void batch_plane32(const BatchArgs& a, const BatchParam& bp, int slot, int d,
                                            float* lds, int tid) {
  constexpr int TI = SP / 32;
  constexpr int LDU = SP + 1;
  constexpr int kLdaU = 64 + 4, kLdbU = 128 + 4;   // LDS row strides of the staged A (crop rows) and B (columns)
  constexpr int kStage32 = BK * (kLdaU + 2 * kLdbU);
  const int lane = tid & 63, w = tid >> 6, h = lane >> 5, l32 = lane & 31;
  const int N = a.N, NN = N * N, S = bp.S;
  const int r0 = 32 - S / 2;
  const float2* Pf = a.Pf + (size_t)slot * 3 * NN;
  float* Ure = lds;
  float* Uim = lds + N * LDU;
  const double zrev = ((d - 0.5 * (bp.D - 1)) * a.pitch + bp.zoff) * (1.0 / kTwoPi);
  float isum64[16];   // SP = 64: this wave's 32x32 block of E, MFMA C layout
  float isum32[4];    // SP = 32: elements tid + 256 q of the 32x32 image
#pragma unroll
  for (int r = 0; r < 16; ++r) isum64[r] = 0.f;
#pragma unroll
  for (int q = 0; q < 4; ++q) isum32[q] = 0.f;
  for (int c = 0; c < 3; ++c) {
    const float2* Pc = Pf + (size_t)c * NN;
    // ---- U[m][col] = sum_k A2[r0 + m][k] (D o Pf)[k][col]: k-stages of A2 rows and of the
    // defocused folded pupil (re / im planes) staged in LDS, double-buffered; wave w owns
    // columns 32 w .. 32 w + 31
    {
      float ra[4];      // A prefetch: BK x SP floats, up to 4 per thread
      float4 rp[4];     // B prefetch: BK x N/2 float4, up to 4 per thread
      double rd[4];     // k s_z of the staged folded cell
      const int na = BK * SP, nb = BK * (N / 2);   // A floats and B float4 of one stage, up to 4 per thread
      auto load = [&](int k0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int idx = tid + 256 * i;
          if (idx < na) {
            const int kk = idx / SP, m = idx % SP;
            ra[i] = a.A2T[(k0 + kk) * kTabRows + r0 + m];
          }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int idx = tid + 256 * i;
          if (idx < nb) {
            const int kk = idx / (N / 2), c2 = idx % (N / 2);
            rp[i] = *reinterpret_cast<const float4*>(Pc + (size_t)(k0 + kk) * N + 2 * c2);
            rd[i] = a.ksz[((k0 + kk) >> 1) * N + c2];
          }
        }
      };
      auto store = [&](float* st) {
        float* sa = st;
        float* sr = st + BK * kLdaU;
        float* si = sr + BK * kLdbU;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int idx = tid + 256 * i;
          if (idx < na) {
            const int kk = idx / SP, m = idx % SP;
            sa[kk * kLdaU + m] = ra[i];
          }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int idx = tid + 256 * i;
          if (idx < nb) {
            const int kk = idx / (N / 2), c2 = idx % (N / 2);
            float2 dz;   // exp(i k s_z z): FP64 phase in revolutions, hardware sine and cosine
            sincos_rev(rd[i] * zrev, &dz.y, &dz.x);
            *reinterpret_cast<float2*>(sr + kk * kLdbU + 2 * c2) =
                make_float2(rp[i].x * dz.x - rp[i].y * dz.y, rp[i].z * dz.x - rp[i].w * dz.y);
            *reinterpret_cast<float2*>(si + kk * kLdbU + 2 * c2) =
                make_float2(rp[i].x * dz.y + rp[i].y * dz.x, rp[i].z * dz.y + rp[i].w * dz.x);
          }
        }
      };
      f16v_t ur[TI], ui[TI];
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          ur[i][r] = 0.f;
          ui[i][r] = 0.f;
        }
      const bool has_cols = 32 * w < N;
      const int KT = N / BK;
      load(0);
      store(lds);
      __syncthreads();
      for (int kt = 0; kt < KT; ++kt) {
        float* cur = lds + (kt & 1) * kStage32;
        float* nxt = lds + ((kt + 1) & 1) * kStage32;
        const bool more = kt + 1 < KT;
        if (more) load((kt + 1) * BK);
        if (has_cols) {
          const float* sa = cur;
          const float* sr = cur + BK * kLdaU;
          const float* si = sr + BK * kLdbU;
#pragma unroll
          for (int kp = 0; kp < BK / 2; ++kp) {
            const int kk = 2 * kp + h;
            const float br = sr[kk * kLdbU + 32 * w + l32], bi = si[kk * kLdbU + 32 * w + l32];
#pragma unroll
            for (int i = 0; i < TI; ++i) {
              const float av = sa[kk * kLdaU + 32 * i + l32];
              ur[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, br, ur[i], 0, 0, 0);
              ui[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bi, ui[i], 0, 0, 0);
            }
          }
        }
        if (more) store(nxt);
        __syncthreads();
      }
      // U overwrites the stage buffers: every wave has passed the last barrier above
      if (has_cols) {
        const int col = 32 * w + l32;
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int m = 32 * i + 8 * (r >> 2) + 4 * h + (r & 3);
            Ure[col * LDU + m] = ur[i][r];
            Uim[col * LDU + m] = ui[i][r];
          }
      }
    }
    __syncthreads();
    // ---- E'[m][n] = sum_col U[m][col] B1[col][r0 + n]
    f16v_t er, ei;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      er[r] = 0.f;
      ei[r] = 0.f;
    }
    const int mi = (SP == 64) ? (w >> 1) : 0, ni = (SP == 64) ? (w & 1) : 0;
    const int kp1a = (SP == 64) ? 0 : w * (N / 8);               // SP = 32: K split over the waves
    const int kp1b = (SP == 64) ? N / 2 : (w + 1) * (N / 8);     // (kp1b - kp1a) is a multiple of 4
    {
      // the y-table operand comes from global memory: chunks of 4 k-steps are loaded one
      // chunk ahead of the MFMAs that use them
      const float* bsrc = a.B1T + h * kTabRows + r0 + 32 * ni + l32;
      float bc[4], bn[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) bc[t] = bsrc[(2 * (kp1a + t)) * kTabRows];
      for (int kp = kp1a; kp < kp1b; kp += 4) {
        const bool more = kp + 4 < kp1b;
#pragma unroll
        for (int t = 0; t < 4; ++t) bn[t] = more ? bsrc[(2 * (kp + 4 + t)) * kTabRows] : 0.f;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int kk = 2 * (kp + t) + h;
          const float ar = Ure[kk * LDU + 32 * mi + l32], ai = Uim[kk * LDU + 32 * mi + l32];
          er = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, bc[t], er, 0, 0, 0);
          ei = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, bc[t], ei, 0, 0, 0);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) bc[t] = bn[t];
      }
    }
    __syncthreads();   // U is consumed
    // E = -i E' = (Im E', -Re E')
    if (SP == 64) {
      float2* Ec = a.E ? a.E + 3 * bp.off + ((size_t)(d * 3 + c) * S) * S : nullptr;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = 32 * mi + 8 * (r >> 2) + 4 * h + (r & 3), n = 32 * ni + l32;
        isum64[r] += er[r] * er[r] + ei[r] * ei[r];
        if (Ec && m < S && n < S) Ec[m * S + n] = make_float2(ei[r], -er[r]);
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
        if (Ec && m < S && n < S) Ec[m * S + n] = make_float2(si, -sr);
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
  __syncthreads();   // every wave is done with the LDS before the next item
}

// MFMA 16x16x4 f32: A lane l -> A[l%16][l/16], B lane l -> B[l/16][l%16],
// C register r of lane l -> C[4(l/16) + r][l%16].
//
// Plane d of emitter `slot` on a tile of SP rows (SP = 16, 32, 48 or 64 >= S):
//   U = A2 (D o Pf_c)  (real x complex, SP x N),  E' = U B1  (complex x real, SP x SP),
//   E = -i E',  I = sum_c |E_c|^2,
// with the defocus D[jf][lf] = exp(i k s_z z) of the folded cell, the same for its four
// mirror cells.  U: wave w owns columns 32 w .. 32 w + 31 (two 16-wide column tiles) and
// all SP / 16 row tiles; k-stages of BK folded rows are staged in LDS, double-buffered.
// E': the (SP / 16)^2 output tiles are dealt round-robin to the four waves, each over the
// whole K = N; a single tile (SP = 16) is split over K between the waves and the four
// partial sums are added through LDS.
typedef float f4_t __attribute__((ext_vector_type(4)));

template <int SP, int BK>
struct PlaneTile {
  static constexpr int MT = SP / 16;                 // row tiles
  static constexpr int T2 = MT * MT;                 // output tiles of E'
  static constexpr bool KSPLIT = T2 < 4;             // SP = 16: one tile, K split four ways
  static constexpr int TPW = KSPLIT ? 1 : (T2 + 3) / 4;   // output tiles per wave
  static constexpr int LDA = SP + 4;                 // LDS row strides of the staged operands
  static constexpr int LDB = 128 + 4;
  static constexpr int STAGE = BK * (LDA + 2 * LDB);
  static constexpr int LDU = SP + 1;                 // U: [col][m]
  static constexpr int LDS_FLOATS = (2 * STAGE > 2 * 128 * LDU) ? 2 * STAGE : 2 * 128 * LDU;
};

template <int SP, int BK>
__device__ __forceinline__ void batch_plane16(const BatchArgs& a, const BatchParam& bp, int slot, int d,
                                              float* lds, int tid) {
  using P = PlaneTile<SP, BK>;
  constexpr int MT = P::MT, TPW = P::TPW;
  const int lane = tid & 63, w = tid >> 6, g = lane >> 4, l16 = lane & 15;
  const int N = a.N, NN = N * N, S = bp.S;
  const int r0 = 32 - S / 2;
  const float2* Pf = a.Pf + (size_t)slot * 3 * NN;
  float* Ure = lds;
  float* Uim = lds + 128 * P::LDU;
  const double zrev = ((d - 0.5 * (bp.D - 1)) * a.pitch + bp.zoff) * (1.0 / kTwoPi);
  f4_t isum[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) isum[t] = f4_t{0.f, 0.f, 0.f, 0.f};
  for (int c = 0; c < 3; ++c) {
    const float2* Pc = Pf + (size_t)c * NN;
    // ---- U[m][col] = sum_k A2[r0 + m][k] (D o Pf)[k][col]
    {
      constexpr int NA = (BK * SP + 255) / 256;       // A loads per thread (the last may be partial)
      constexpr int NB = (BK * 64 + 255) / 256;       // B loads (float4 = two complex) per thread, N <= 128
      float ra[NA];
      float4 rp[NB];
      double rd[NB];
      const int nbv = BK * (N / 2);                   // float4 of B per stage
      auto load = [&](int k0) {
#pragma unroll
        for (int i = 0; i < NA; ++i) {
          const int idx = tid + 256 * i;
          if (idx < BK * SP) {
            const int kk = idx / SP, m = idx % SP;
            ra[i] = a.A2T[(k0 + kk) * kTabRows + r0 + m];
          }
        }
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          const int idx = tid + 256 * i;
          if (idx < nbv) {
            const int kk = idx / (N / 2), c2 = idx % (N / 2);
            rp[i] = *reinterpret_cast<const float4*>(Pc + (size_t)(k0 + kk) * N + 2 * c2);
            rd[i] = a.ksz[((k0 + kk) >> 1) * N + c2];
          }
        }
      };
      auto store = [&](float* st) {
        float* sa = st;
        float* sr = st + BK * P::LDA;
        float* si = sr + BK * P::LDB;
#pragma unroll
        for (int i = 0; i < NA; ++i) {
          const int idx = tid + 256 * i;
          if (idx < BK * SP) {
            const int kk = idx / SP, m = idx % SP;
            sa[kk * P::LDA + m] = ra[i];
          }
        }
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          const int idx = tid + 256 * i;
          if (idx < nbv) {
            const int kk = idx / (N / 2), c2 = idx % (N / 2);
            float2 dz;   // exp(i k s_z z): FP64 phase in revolutions, hardware sine and cosine
            sincos_rev(rd[i] * zrev, &dz.y, &dz.x);
            *reinterpret_cast<float2*>(sr + kk * P::LDB + 2 * c2) =
                make_float2(rp[i].x * dz.x - rp[i].y * dz.y, rp[i].z * dz.x - rp[i].w * dz.y);
            *reinterpret_cast<float2*>(si + kk * P::LDB + 2 * c2) =
                make_float2(rp[i].x * dz.y + rp[i].y * dz.x, rp[i].z * dz.y + rp[i].w * dz.x);
          }
        }
      };
      f4_t ur[MT][2], ui[MT][2];
#pragma unroll
      for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          ur[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};
          ui[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};
        }
      const bool has_cols = 32 * w < N;
      const int KT = N / BK;
      load(0);
      store(lds);
      __syncthreads();
      for (int kt = 0; kt < KT; ++kt) {
        float* cur = lds + (kt & 1) * P::STAGE;
        float* nxt = lds + ((kt + 1) & 1) * P::STAGE;
        const bool more = kt + 1 < KT;
        if (more) load((kt + 1) * BK);
        if (has_cols) {
          const float* sa = cur;
          const float* sr = cur + BK * P::LDA;
          const float* si = sr + BK * P::LDB;
#pragma unroll
          for (int kq = 0; kq < BK / 4; ++kq) {
            const int kk = 4 * kq + g;
            float br[2], bi[2];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
              br[j] = sr[kk * P::LDB + 32 * w + 16 * j + l16];
              bi[j] = si[kk * P::LDB + 32 * w + 16 * j + l16];
            }
#pragma unroll
            for (int i = 0; i < MT; ++i) {
              const float av = sa[kk * P::LDA + 16 * i + l16];
#pragma unroll
              for (int j = 0; j < 2; ++j) {
                ur[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, br[j], ur[i][j], 0, 0, 0);
                ui[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bi[j], ui[i][j], 0, 0, 0);
              }
            }
          }
        }
        if (more) store(nxt);
        __syncthreads();
      }
      // U overwrites the stage buffers: every wave has passed the last barrier above
      if (has_cols) {
#pragma unroll
        for (int i = 0; i < MT; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            const int col = 32 * w + 16 * j + l16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int m = 16 * i + 4 * g + r;
              Ure[col * P::LDU + m] = ur[i][j][r];
              Uim[col * P::LDU + m] = ui[i][j][r];
            }
          }
      }
    }
    __syncthreads();
    // ---- E'[m][n] = sum_col U[m][col] B1[col][r0 + n]
    float2* Ec = a.E ? a.E + 3 * bp.off + ((size_t)(d * 3 + c) * S) * S : nullptr;
    if (!P::KSPLIT) {
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
        const int tile = w + 4 * t;
        if (tile < P::T2) {
          const int mi = tile / MT, ni = tile % MT;
          f4_t er = {0.f, 0.f, 0.f, 0.f}, ei = {0.f, 0.f, 0.f, 0.f};
          // the y-table operand comes from global memory: chunks of four k-steps (16
          // columns) are loaded one chunk ahead of the MFMAs that use them (N % 16 == 0)
          const float* bsrc = a.B1T + r0 + 16 * ni + l16 + g * kTabRows;
          float bc[4], bn[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) bc[q] = bsrc[(4 * q) * kTabRows];
          for (int k0 = 0; k0 < N; k0 += 16) {
            const bool more = k0 + 16 < N;
#pragma unroll
            for (int q = 0; q < 4; ++q) bn[q] = more ? bsrc[(k0 + 16 + 4 * q) * kTabRows] : 0.f;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int col = k0 + 4 * q + g;
              const float ar = Ure[col * P::LDU + 16 * mi + l16], ai = Uim[col * P::LDU + 16 * mi + l16];
              er = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, bc[q], er, 0, 0, 0);
              ei = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, bc[q], ei, 0, 0, 0);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) bc[q] = bn[q];
          }
          // E = -i E' = (Im E', -Re E')
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int m = 16 * mi + 4 * g + r, n = 16 * ni + l16;
            isum[t][r] += er[r] * er[r] + ei[r] * ei[r];
            if (Ec && m < S && n < S) Ec[m * S + n] = make_float2(ei[r], -er[r]);
          }
        }
      }
      __syncthreads();   // U is consumed
    } else {
      // one 16 x 16 tile: wave w sums columns [w N / 4, (w + 1) N / 4), partials through LDS
      f4_t er = {0.f, 0.f, 0.f, 0.f}, ei = {0.f, 0.f, 0.f, 0.f};
      const float* bsrc = a.B1T + r0 + l16;
      const int ka = w * (N / 4), kb = (w + 1) * (N / 4);
      for (int k0 = ka; k0 < kb; k0 += 4) {
        const int col = k0 + g;
        const float bv = bsrc[col * kTabRows];
        er = __builtin_amdgcn_mfma_f32_16x16x4f32(Ure[col * P::LDU + l16], bv, er, 0, 0, 0);
        ei = __builtin_amdgcn_mfma_f32_16x16x4f32(Uim[col * P::LDU + l16], bv, ei, 0, 0, 0);
      }
      __syncthreads();   // U is consumed; the partials reuse its space
      float* part = lds + w * 2 * 256;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = 4 * g + r;
        part[m * 16 + l16] = er[r];
        part[256 + m * 16 + l16] = ei[r];
      }
      __syncthreads();
      if (tid < 256) {
        const int m = tid >> 4, n = tid & 15;
        float sr = 0.f, si = 0.f;
#pragma unroll
        for (int ww = 0; ww < 4; ++ww) {
          sr += lds[ww * 512 + m * 16 + n];
          si += lds[ww * 512 + 256 + m * 16 + n];
        }
        // thread tid keeps element (m, n) = (tid / 16, tid % 16) of the single tile
        isum[0][0] += sr * sr + si * si;
        if (Ec && m < S && n < S) Ec[m * S + n] = make_float2(si, -sr);
      }
      __syncthreads();
    }
  }
  if (a.I) {
    float* Ip = a.I + bp.off + (size_t)d * S * S;
    if (!P::KSPLIT) {
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
        const int tile = w + 4 * t;
        if (tile < P::T2) {
          const int mi = tile / MT, ni = tile % MT;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int m = 16 * mi + 4 * g + r, n = 16 * ni + l16;
            if (m < S && n < S) Ip[m * S + n] = isum[t][r];
          }
        }
      }
    } else {
      const int m = tid >> 4, n = tid & 15;
      if (m < S && n < S) Ip[m * S + n] = isum[0][0];
    }
  }
  __syncthreads();   // every wave is done with the LDS before the next item
}

// Tile classes: row tiles of 16, 32, 48, 64; class t serves queues 8 t .. 8 t + 7.
constexpr int kTileClasses = 4;
__host__ __device__ constexpr int class_rows(int t) { return 16 * (t + 1); }

// Persistent plane kernel of one tile class (one launch per class, so that each has the
// registers of its own tile shape).  Workgroup ids are dealt round-robin over the 8 XCDs,
// so workgroup b serves queue b % 8 of the class: the (emitter, plane) items of the
// emitters assigned to that queue, in order, so that the planes of one emitter run at the
// same time on one XCD and its folded pupil is read from that XCD's L2.  A workgroup exits
// when its queue is exhausted; the grid has at least 8 workgroups, one per queue.
template <int SP, int BK>
__global__ void __launch_bounds__(256, 2) batch_planes_kernel(BatchArgs a) {
  extern __shared__ float lds[];
  __shared__ long long item;
  const int tid = threadIdx.x;
  const int x = 8 * (SP / 16 - 1) + (blockIdx.x & 7);
  const int lo = a.qoff[x], hi = a.qoff[x + 1];
  const long long end = a.pre[hi];
  for (;;) {
    if (tid == 0) item = (long long)atomicAdd(&a.counter[x], 1ull);
    __syncthreads();
    const long long it = item;
    __syncthreads();
    if (it >= end) break;
    // emitter e of the queue with pre[e] <= it < pre[e + 1]
    int e0 = lo, e1 = hi - 1;
    while (e0 < e1) {
      const int mid = (e0 + e1 + 1) >> 1;
      if (a.pre[mid] <= it) e0 = mid; else e1 = mid - 1;
    }
    const int slot = a.list[e0];
    const int d = (int)(it - a.pre[e0]);
    const BatchParam bp = a.params[slot];
    if constexpr (SP == 32 || SP == 64)
      batch_plane32<SP, BK>(a, bp, slot, d, lds, tid);
    else
      batch_plane16<SP, BK>(a, bp, slot, d, lds, tid);
  }
}

// LDS of a class: the 32 x 32 tiles (SP = 32, 64) hold U of a 64-row tile (or the two
// stage buffers, if larger); the 16 x 16 tiles size it for their own rows
template <int SP, int BK>
constexpr int plane_lds_bytes() {
  return (SP == 32 || SP == 64) ? ((2 * 128 * 65 > 2 * BK * (68 + 2 * 132)) ? 2 * 128 * 65 : 2 * BK * (68 + 2 * 132)) * 4
                                : PlaneTile<SP, BK>::LDS_FLOATS * 4;
}

// every (tile class, k-stage) instantiation, indexed [class][k-stage index] (BK = 8, 16)
typedef void (*PlaneKernel)(BatchArgs);
static const PlaneKernel kPlaneKernels[kTileClasses][2] = {
    {batch_planes_kernel<16, 8>, batch_planes_kernel<16, 16>},
    {batch_planes_kernel<32, 8>, batch_planes_kernel<32, 16>},
    {batch_planes_kernel<48, 8>, batch_planes_kernel<48, 16>},
    {batch_planes_kernel<64, 8>, batch_planes_kernel<64, 16>}};
static const int kPlaneLds[kTileClasses][2] = {{plane_lds_bytes<16, 8>(), plane_lds_bytes<16, 16>()},
                                               {plane_lds_bytes<32, 8>(), plane_lds_bytes<32, 16>()},
                                               {plane_lds_bytes<48, 8>(), plane_lds_bytes<48, 16>()},
                                               {plane_lds_bytes<64, 8>(), plane_lds_bytes<64, 16>()}};

}  // namespace rw

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
namespace rw {
// each crop bucket on its own tile class, k-stages of 16, two workgroups per CU
static rwpsf_batch_config default_config() {
  rwpsf_batch_config c{};
  c.wg_per_cu = 2;
  for (int q = 0; q < 4; ++q) {
    c.tile_rows[q] = 16 * (q + 1);
    c.k_stage[q] = 16;
  }
  return c;
}
static bool config_valid(const rwpsf_batch_config& c) {
  if (c.wg_per_cu < 1 || c.wg_per_cu > kMaxWgPerCu) return false;
  for (int q = 0; q < 4; ++q) {
    if (c.tile_rows[q] % 16 != 0 || c.tile_rows[q] < 16 * (q + 1) || c.tile_rows[q] > 64) return false;
    if (c.k_stage[q] != 8 && c.k_stage[q] != 16) return false;
  }
  return true;
}
static bool config_equal(const rwpsf_batch_config& x, const rwpsf_batch_config& y) {
  return x.wg_per_cu == y.wg_per_cu && std::equal(x.tile_rows, x.tile_rows + 4, y.tile_rows) &&
         std::equal(x.k_stage, x.k_stage + 4, y.k_stage);
}
}  // namespace rw

struct rwpsf_batch {
  int device = 0;
  rwpsf_optics opt{};
  int N = 0, max_emitters = 0, num_cus = 0;
  double px = 0, pitch = 0, k = 0, s_max = 0;
  std::vector<void*> allocations;
  float2* d_Q = nullptr;
  double* d_ksz = nullptr;
  double4* d_gl = nullptr;      // [N*N] Gibson-Lanni phase tables, or null
  float* d_A2T = nullptr;       // [N][96] folded x table (prefactor included)
  float* d_B1T = nullptr;       // [N][96] folded y table
  float2* d_pf = nullptr;       // [max][3][N][N] folded pupils
  long long items = 0;          // (emitter, plane) items of the staged call
  long long class_items[4] = {0, 0, 0, 0};   // of them, in the 16-, 32-, 48- and 64-row tile classes
  int class_grid[4] = {0, 0, 0, 0};          // persistent grid of each class (0 = class not launched)
  float* d_basis = nullptr;
  float* d_phi = nullptr;
  char* d_upload = nullptr;     // params [max] then coefT [32][max_pad]
  unsigned long long* d_counter = nullptr;   // [8] queue counters
  char* h_staging = nullptr;    // pinned mirror of d_upload
  size_t upload_bytes = 0;
  int max_pad = 0;
  hipEvent_t upload_done = nullptr;
  bool upload_pending = false;
  rwpsf_batch_config cfg = rw::default_config();
  bool use_graph = false;
  hipGraphExec_t gexec = nullptr;
  struct Key {
    int n = -1;
    void* I = nullptr;
    void* E = nullptr;
    rwpsf_batch_config cfg{};
    int grid[4] = {0, 0, 0, 0};   // the captured launches: a replay must launch the same classes
    hipStream_t st = nullptr;
  } gkey;
  ~rwpsf_batch() {   // teardown: failures cannot be reported and are ignored
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (upload_done) (void)hipEventDestroy(upload_done);
    if (h_staging) (void)hipHostFree(h_staging);
    for (void* p : allocations) (void)hipFree(p);
  }
};

namespace rw {

static int batch_validate(const rwpsf_batch* b, int n, const rwpsf_emitter* e) {
  if (!b || n < 1 || n > b->max_emitters || !e) return RWPSF_ERR_INVALID_ARG;
  for (int i = 0; i < n; ++i) {
    const rwpsf_emitter& x = e[i];
    if (!std::isfinite(x.x0_nm) || !std::isfinite(x.y0_nm) || !std::isfinite(x.z_nm))
      return RWPSF_ERR_INVALID_ARG;
    if (b->opt.gibson_lanni && (!std::isfinite(x.t_s_nm) || x.t_s_nm < 0.0)) return RWPSF_ERR_INVALID_ARG;
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

// Upload block: params [max] | coefT [32][max_pad] | list [max] | pre [max + 1] | qoff [17]
static size_t off_coef(const rwpsf_batch* b) { return sizeof(BatchParam) * b->max_emitters; }
static size_t off_list(const rwpsf_batch* b) { return off_coef(b) + sizeof(float) * kBasisRows * b->max_pad; }
static size_t off_pre(const rwpsf_batch* b) {
  return (off_list(b) + sizeof(int) * b->max_emitters + 7) / 8 * 8;
}
static size_t off_qoff(const rwpsf_batch* b) { return off_pre(b) + sizeof(long long) * (b->max_emitters + 1); }
static size_t upload_size(const rwpsf_batch* b) { return off_qoff(b) + sizeof(int) * (kQueues + 1); }

// Fill the pinned staging area: cost-sorted params, the coefficient matrix, and the
// (emitter, plane) queues: per tile class, eight queues, the class's emitters dealt
// longest first to its least-loaded queue.
static void batch_stage(rwpsf_batch* b, int n, const rwpsf_emitter* e) {
  std::vector<long long> off(n + 1, 0);
  for (int i = 0; i < n; ++i) off[i + 1] = off[i] + (long long)e[i].planes * e[i].crop * e[i].crop;
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  auto sp_of = [&](int i) { return b->cfg.tile_rows[(e[i].crop - 1) / 16]; };
  auto cost = [&](int i) { return (double)e[i].planes * sp_of(i) * (b->N + sp_of(i)); };
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost(x) > cost(y); });
  BatchParam* prm = (BatchParam*)b->h_staging;
  float* coefT = (float*)(b->h_staging + off_coef(b));
  for (int slot = 0; slot < n; ++slot) {
    const int i = order[slot];
    prm[slot].zoff = -e[i].z_nm;
    prm[slot].ts = b->opt.gibson_lanni ? e[i].t_s_nm : 0.0;
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
  std::vector<int> queue(n);
  double load[kQueues] = {};
  int count[kQueues] = {};
  for (int t = 0; t < kTileClasses; ++t) b->class_items[t] = 0;
  for (int slot = 0; slot < n; ++slot) {
    const int t = prm[slot].SP / 16 - 1;
    const int x = 8 * t + (int)(std::min_element(load + 8 * t, load + 8 * t + 8) - (load + 8 * t));
    queue[slot] = x;
    load[x] += cost(order[slot]);
    count[x] += 1;
    b->class_items[t] += prm[slot].D;
  }
  int* list = (int*)(b->h_staging + off_list(b));
  long long* pre = (long long*)(b->h_staging + off_pre(b));
  int* qoff = (int*)(b->h_staging + off_qoff(b));
  qoff[0] = 0;
  for (int x = 0; x < kQueues; ++x) qoff[x + 1] = qoff[x] + count[x];
  int fill[kQueues];
  for (int x = 0; x < kQueues; ++x) fill[x] = qoff[x];
  for (int slot = 0; slot < n; ++slot) list[fill[queue[slot]]++] = slot;
  pre[0] = 0;
  for (int i = 0; i < n; ++i) pre[i + 1] = pre[i] + prm[list[i]].D;
  b->items = pre[n];
  // persistent grid of each class: at least one workgroup per queue, no more than the
  // configured residency, none for an empty class
  for (int t = 0; t < kTileClasses; ++t) {
    const long long want =
        std::max<long long>(8, std::min<long long>(b->class_items[t], (long long)b->num_cus * b->cfg.wg_per_cu));
    b->class_grid[t] =
        b->class_items[t] == 0 ? 0 : (int)std::min<long long>(want, (long long)b->num_cus * kMaxWgPerCu);
  }
}

// Copy the staged parameter block to the device and record upload_done right after it,
// so that the next call may restage the pinned area while this call's kernels still run.
static int batch_upload(rwpsf_batch* b, hipStream_t st) {
  int rc;
  if ((rc = hip_check(hipMemcpyAsync(b->d_upload, b->h_staging, b->upload_bytes, hipMemcpyHostToDevice, st))) ||
      (rc = hip_check(hipEventRecord(b->upload_done, st))))
    return rc;
  b->upload_pending = true;
  return RWPSF_OK;
}

// The kernels of one call (they read the uploaded block in stream order): queue reset,
// phase GEMM, fold, one persistent launch per tile class.  This is what a graph captures.
static int batch_kernels(rwpsf_batch* b, int n, float* I, float2* E, hipStream_t st) {
  int rc;
  const long long* d_pre = (const long long*)(b->d_upload + off_pre(b));
  const int* d_qoff = (const int*)(b->d_upload + off_qoff(b));
  hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, st, b->d_counter, d_pre, d_qoff);
  if ((rc = hip_check(hipGetLastError()))) return rc;
  const float* coefT = (const float*)(b->d_upload + off_coef(b));
  const int NN = b->N * b->N;
  if ((rc = hip_check(launch_rgemm(coefT, b->max_pad, b->d_basis, NN, b->d_phi, NN, n, NN, kBasisRows, st))))
    return rc;
  BatchArgs a{};
  a.params = (const BatchParam*)b->d_upload;
  a.Q = b->d_Q;
  a.ksz = b->d_ksz;
  a.phi = b->d_phi;
  a.gl = b->d_gl;
  a.A2T = b->d_A2T;
  a.B1T = b->d_B1T;
  a.Pf = b->d_pf;
  a.list = (const int*)(b->d_upload + off_list(b));
  a.pre = d_pre;
  a.qoff = d_qoff;
  a.I = I;
  a.E = E;
  a.counter = b->d_counter;
  a.n = n;
  a.N = b->N;
  a.pitch = b->pitch;
  hipLaunchKernelGGL(batch_fold_kernel, dim3(n), dim3(256), 0, st, a);
  if ((rc = hip_check(hipGetLastError()))) return rc;
  // one launch per tile class, the tall tiles first; at least one workgroup per queue and
  // no more than the configured residency
  for (int t = kTileClasses - 1; t >= 0; --t) {
    const int grid = b->class_grid[t];
    if (grid == 0) continue;
    const int ki = b->cfg.k_stage[t] == 8 ? 0 : 1;
    hipLaunchKernelGGL(kPlaneKernels[t][ki], dim3(grid), dim3(256), kPlaneLds[t][ki], st, a);
    if ((rc = hip_check(hipGetLastError()))) return rc;
  }
  return RWPSF_OK;
}

static int batch_enqueue(rwpsf_batch* b, int n, float* I, float2* E, hipStream_t st) {
  const int rc = batch_upload(b, st);
  return rc ? rc : batch_kernels(b, n, I, E, st);
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
  rwpsf_numerics nm{RWPSF_FORM_FOURIER, n_pupil, 2, 8, RWPSF_MODEL_VECTORIAL, RWPSF_THETA_GAUSS};
  int st = validate_plan(o, &g, &nm);
  if (st != RWPSF_OK) return st;
  if (n_pupil < 32 || n_pupil > 128 || n_pupil % 32 != 0) return RWPSF_ERR_INVALID_ARG;
  if (!(pixel_nm > 0) || !std::isfinite(pixel_nm) || !(pitch_nm >= 0) || !std::isfinite(pitch_nm))
    return RWPSF_ERR_INVALID_ARG;
  if (max_emitters < 1 || max_emitters > (1 << 20)) return RWPSF_ERR_INVALID_ARG;
  int dev_count = 0;
  if (hipGetDeviceCount(&dev_count) != hipSuccess || dev_count < 1) return RWPSF_ERR_NO_DEVICE;
  rwpsf_batch* b = new (std::nothrow) rwpsf_batch();
  if (!b) return RWPSF_ERR_OOM;
  if (hipGetDevice(&b->device) != hipSuccess ||
      hipDeviceGetAttribute(&b->num_cus, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess ||
      b->num_cus < 1) {
    delete b;
    return RWPSF_ERR_NO_DEVICE;
  }
  b->opt = *o;
  b->N = n_pupil;
  b->px = pixel_nm;
  b->pitch = pitch_nm;
  b->max_emitters = max_emitters;
  b->k = kTwoPi * o->n_i / o->wavelength_nm;
  b->s_max = o->na / o->n_i;
  const int N = n_pupil;
  const size_t NN = (size_t)N * N;
  std::vector<float2> Q(3 * NN, make_float2(0.f, 0.f));
  std::vector<double> ksz(NN, 0.0);
  std::vector<double4> gl(o->gibson_lanni ? NN : 0, make_double4(0.0, 0.0, 0.0, 0.0));
  GLParams glp{};
  glp.k0 = kTwoPi / o->wavelength_nm;
  glp.n_i = o->n_i;
  glp.n_s = o->n_s;
  glp.n_g = o->n_g;
  glp.n_g_d = o->n_g_design;
  glp.n_i_d = o->n_i_design;
  glp.t_g = o->t_g_nm;
  glp.t_g_d = o->t_g_design_nm;
  glp.t_i_d = o->t_i_design_nm;
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
      std::complex<double> e[3];
      base_pupil_cell(*o, 3, ds, sx, sy, e);
      for (int c = 0; c < 3; ++c) Q[c * NN + cell] = make_float2((float)e[c].real(), (float)e[c].imag());
      ksz[cell] = b->k * std::sqrt(1.0 - (sx * sx + sy * sy));
      if (o->gibson_lanni) {
        // the phase is affine in t_s (t_i is affine in it and each layer's term is linear
        // in its thickness): store its value at t_s = 0 and its slope
        const double sin_t = std::sqrt(sx * sx + sy * sy), T = 1.0e4;
        double r0, i0, r1, i1;
        gl_opd(glp, 0.0, sin_t, &r0, &i0);
        gl_opd(glp, T, sin_t, &r1, &i1);
        gl[cell] = make_double4(r0, i0, (r1 - r0) / T, (i1 - i0) / T);
      }
    }
  // folded DFT tables: row 2jf + p holds cos (p = 0) or sin (p = 1) of k s[jf] x_r,
  // x_r = (r - 32) pixel; the x table carries the prefactor f k / 2 pi (E = -i E')
  std::vector<float> A2T((size_t)N * kTabRows), B1T((size_t)N * kTabRows);
  const double pref = o->focal_length * b->k / kTwoPi;
  for (int jf = 0; jf < N / 2; ++jf) {
    const double s = (2.0 * jf + 1.0 - N) * b->s_max / N;
    for (int r = 0; r < kTabRows; ++r) {
      const double ph = b->k * s * (r - 32) * pixel_nm;
      A2T[(size_t)(2 * jf) * kTabRows + r] = (float)(pref * std::cos(ph));
      A2T[(size_t)(2 * jf + 1) * kTabRows + r] = (float)(pref * std::sin(ph));
      B1T[(size_t)(2 * jf) * kTabRows + r] = (float)std::cos(ph);
      B1T[(size_t)(2 * jf + 1) * kTabRows + r] = (float)std::sin(ph);
    }
  }
  b->max_pad = (max_emitters + 63) / 64 * 64;
  b->upload_bytes = upload_size(b);
  int rc;
  if ((rc = balloc(b, &b->d_Q, 3 * NN)) || (rc = balloc(b, &b->d_ksz, NN)) ||
      (rc = balloc(b, &b->d_A2T, (size_t)N * kTabRows)) || (rc = balloc(b, &b->d_B1T, (size_t)N * kTabRows)) ||
      (rc = balloc(b, &b->d_pf, (size_t)max_emitters * 3 * NN)) ||
      (rc = balloc(b, &b->d_basis, (size_t)kBasisRows * NN)) ||
      (rc = balloc(b, &b->d_phi, (size_t)max_emitters * NN)) || (rc = balloc(b, &b->d_upload, b->upload_bytes)) ||
      (rc = balloc(b, &b->d_counter, kQueues)) || (o->gibson_lanni && (rc = balloc(b, &b->d_gl, NN)))) {
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
      (rc = hip_check(hipMemcpy(b->d_A2T, A2T.data(), A2T.size() * sizeof(float), hipMemcpyHostToDevice))) ||
      (rc = hip_check(hipMemcpy(b->d_B1T, B1T.data(), B1T.size() * sizeof(float), hipMemcpyHostToDevice))) ||
      (o->gibson_lanni &&
       (rc = hip_check(hipMemcpy(b->d_gl, gl.data(), gl.size() * sizeof(double4), hipMemcpyHostToDevice)))) ||
      (rc = hip_check(hipMemcpy(b->d_basis, basis.data(), basis.size() * sizeof(float), hipMemcpyHostToDevice))) ||
      (rc = hip_check(hipMemcpy(b->d_upload, b->h_staging, b->upload_bytes, hipMemcpyHostToDevice))) ||
      (rc = hip_check(hipDeviceSynchronize()))) {
    delete b;
    return rc;
  }
  for (int t = 0; t < kTileClasses; ++t)
    for (int k = 0; k < 2; ++k)
      if ((rc = hip_check(hipFuncSetAttribute((const void*)kPlaneKernels[t][k],
                                              hipFuncAttributeMaxDynamicSharedMemorySize, kPlaneLds[t][k])))) {
        delete b;
        return rc;
      }
  *out = b;
  return RWPSF_OK;
}

void rwpsf_batch_destroy(rwpsf_batch* b) {   // teardown: HIP failures are ignored
  if (!b) return;
  int cur = 0;
  const bool had = hipGetDevice(&cur) == hipSuccess;
  (void)hipSetDevice(b->device);
  (void)hipDeviceSynchronize();
  delete b;
  if (had) (void)hipSetDevice(cur);
}

int rwpsf_batch_set_graph(rwpsf_batch* b, int enable) {
  if (!b) return RWPSF_ERR_INVALID_ARG;
  b->use_graph = enable != 0;
  return RWPSF_OK;
}

int rwpsf_batch_set_config(rwpsf_batch* b, const rwpsf_batch_config* c) {
  if (!b || !c || !rw::config_valid(*c)) return RWPSF_ERR_INVALID_ARG;
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
  if (hipGetDevice(&cur) != hipSuccess || cur != b->device) return RWPSF_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  if (b->use_graph && !st) return RWPSF_ERR_INVALID_ARG;   // the legacy default stream cannot be captured
  // the previous upload must have left the pinned staging area before it is rewritten
  if (b->upload_pending && (rc = hip_check(hipEventSynchronize(b->upload_done)))) return rc;
  batch_stage(b, n, e);
  if ((rc = batch_upload(b, st))) return rc;
  if (!b->use_graph) {
    rc = batch_kernels(b, n, I, (float2*)E, st);
  } else {
    const bool same = b->gexec && b->gkey.n == n && b->gkey.I == I && b->gkey.E == E &&
                      config_equal(b->gkey.cfg, b->cfg) &&
                      std::equal(b->class_grid, b->class_grid + kTileClasses, b->gkey.grid) && b->gkey.st == st;
    if (!same) {
      if (b->gexec) {
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
      }
      hipGraph_t g = nullptr;
      if ((rc = hip_check(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal)))) return rc;
      const int erc = batch_kernels(b, n, I, (float2*)E, st);
      hipError_t ce = hipStreamEndCapture(st, &g);
      if (erc) {
        if (g) (void)hipGraphDestroy(g);
        return erc;
      }
      if ((rc = hip_check(ce))) return rc;
      ce = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if ((rc = hip_check(ce))) return rc;
      b->gkey.n = n;
      b->gkey.I = I;
      b->gkey.E = E;
      b->gkey.cfg = b->cfg;
      std::copy(b->class_grid, b->class_grid + kTileClasses, b->gkey.grid);
      b->gkey.st = st;
    }
    rc = hip_check(hipGraphLaunch(b->gexec, st));
  }
  return rc;
}

}  // extern "C"

namespace rw {

// Autotune cache: a flat JSON object
//   {"key": [wg_per_cu, tile_rows[0..3], k_stage[0..3], ms], ...}
// in the file named by RWPSF_AUTOTUNE_CACHE.  Anything that does not parse is ignored
// (and replaced on the next write).
static std::string tune_key(const rwpsf_batch* b, int n, const rwpsf_emitter* e) {
  int bucket[4] = {0, 0, 0, 0};
  long long planes = 0;
  for (int i = 0; i < n; ++i) {
    bucket[(e[i].crop - 1) / 16] += 1;
    planes += e[i].planes;
  }
  int nb = 1;
  while (nb < n) nb <<= 1;
  char buf[200];
  snprintf(buf, sizeof buf, "N%d_n%d_b%d-%d-%d-%d_meanD%lld_cus%d", b->N, nb, (int)(16.0 * bucket[0] / n),
           (int)(16.0 * bucket[1] / n), (int)(16.0 * bucket[2] / n), (int)(16.0 * bucket[3] / n), planes / n,
           b->num_cus);
  return buf;
}

typedef std::map<std::string, std::pair<rwpsf_batch_config, double>> TuneCache;

static TuneCache cache_read(const char* path) {
  TuneCache m;
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
    rwpsf_batch_config c{};
    double ms = 0;
    if (sscanf(text.c_str() + b0, "[%d , %d , %d , %d , %d , %d , %d , %d , %d , %lf]", &c.wg_per_cu, &c.tile_rows[0],
               &c.tile_rows[1], &c.tile_rows[2], &c.tile_rows[3], &c.k_stage[0], &c.k_stage[1], &c.k_stage[2],
               &c.k_stage[3], &ms) != 10)
      return {};
    if (!config_valid(c)) return {};
    m[text.substr(k0 + 1, k1 - k0 - 1)] = {c, ms};
    pos = b1 + 1;
  }
  return m;
}

static void cache_write(const char* path, const TuneCache& m) {
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return;
  fprintf(f, "{\n");
  size_t i = 0;
  for (const auto& kv : m) {
    const rwpsf_batch_config& c = kv.second.first;
    fprintf(f, "  \"%s\": [%d, %d, %d, %d, %d, %d, %d, %d, %d, %.6f]%s\n", kv.first.c_str(), c.wg_per_cu,
            c.tile_rows[0], c.tile_rows[1], c.tile_rows[2], c.tile_rows[3], c.k_stage[0], c.k_stage[1], c.k_stage[2],
            c.k_stage[3], kv.second.second, ++i < m.size() ? "," : "");
  }
  fprintf(f, "}\n");
  fclose(f);
  rename(tmp.c_str(), path);
}

// Device time of one call with configuration c: the emitters are staged on the host once,
// then one untimed and two timed enqueues, so the host staging stays outside the window.
static int tune_trial(rwpsf_batch* b, int n, const rwpsf_emitter* e, float* I, hipStream_t st,
                      const rwpsf_batch_config& c, hipEvent_t t0, hipEvent_t t1, float* ms) {
  int rc;
  if (b->upload_pending && (rc = hip_check(hipEventSynchronize(b->upload_done)))) return rc;
  b->cfg = c;
  batch_stage(b, n, e);
  if ((rc = batch_enqueue(b, n, I, nullptr, st))) return rc;
  if ((rc = hip_check(hipEventRecord(t0, st)))) return rc;
  for (int r = 0; r < 2; ++r)
    if ((rc = batch_enqueue(b, n, I, nullptr, st))) return rc;
  if ((rc = hip_check(hipEventRecord(t1, st)))) return rc;
  if ((rc = hip_check(hipEventSynchronize(t1))) || (rc = hip_check(hipEventElapsedTime(ms, t0, t1)))) return rc;
  *ms *= 0.5f;
  return RWPSF_OK;
}

}  // namespace rw

extern "C" {

int rwpsf_batch_autotune(rwpsf_batch* b, int n, const rwpsf_emitter* e, float* I, void* stream,
                         rwpsf_batch_config* best_out, double* best_ms) {
  using namespace rw;
  int rc = batch_validate(b, n, e);
  if (rc) return rc;
  if (!I) return RWPSF_ERR_INVALID_ARG;
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != b->device) return RWPSF_ERR_INVALID_ARG;
  const char* cache_path = getenv("RWPSF_AUTOTUNE_CACHE");
  std::string key;
  TuneCache cache;
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
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if ((rc = hip_check(hipEventCreate(&t0))) || (rc = hip_check(hipEventCreate(&t1)))) {
    if (t0) (void)hipEventDestroy(t0);
    return rc;
  }
  // coordinate search from the default: workgroups per CU, then for each crop bucket the
  // taller tile classes it could share (fewer, fuller launches against more padding),
  // then the k-stage of each class in use
  rwpsf_batch_config best = default_config();
  float best_t = 1e30f;
  auto consider = [&](const rwpsf_batch_config& c) {
    float ms = 0.f;
    const int r = tune_trial(b, n, e, I, st, c, t0, t1, &ms);
    if (r == RWPSF_OK && ms < best_t) {
      best_t = ms;
      best = c;
    }
    return r;
  };
  rc = consider(best);
  for (int wg = 1; wg <= 3 && !rc; ++wg) {
    if (wg == best.wg_per_cu) continue;
    rwpsf_batch_config c = best;
    c.wg_per_cu = wg;
    rc = consider(c);
  }
  bool used[4] = {false, false, false, false};
  for (int i = 0; i < n; ++i) used[(e[i].crop - 1) / 16] = true;
  for (int q = 0; q < 3 && !rc; ++q) {
    if (!used[q]) continue;
    const rwpsf_batch_config base = best;
    for (int rows = base.tile_rows[q] + 16; rows <= 64 && !rc; rows += 16) {
      rwpsf_batch_config c = base;
      c.tile_rows[q] = rows;
      rc = consider(c);
    }
  }
  for (int t = 0; t < kTileClasses && !rc; ++t) {
    bool in_use = false;
    for (int q = 0; q < 4; ++q) in_use = in_use || (used[q] && best.tile_rows[q] == class_rows(t));
    if (!in_use) continue;
    rwpsf_batch_config c = best;
    c.k_stage[t] = best.k_stage[t] == 16 ? 8 : 16;
    rc = consider(c);
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
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
