// Bessel (spherical) form of the vectorial Richards-Wolf integral on gfx950.
//
// Sec. 3.3 eq. "polar vectorial final" and eq. "I0": for an axisymmetric pupil
// p(theta) = a(theta) exp(i W(theta)) and constant polarisation (ex, ey),
//   I_n(rho, z) = int_0^theta_max p(t) g_n(t) J_n(k rho sin t) exp(i k z cos t) dt
//   g_0 = sin t (1 + cos t), g_1 = sin^2 t, g_2 = sin t (cos t - 1)
//   E = -(i f k / 2) [ ex (I0 - I2 cos 2v) - ey I2 sin 2v,
//                     -ex I2 sin 2v + ey (I0 + I2 cos 2v),
//                     -2i (ex cos v + ey sin v) I1 ]
// with v the azimuth of the pixel.  With the Fresnel products q_s(t), q_p(t) of Sec. 3.3
// kept in eq. "field Gaussian sphere", the phi integral gives the same combination with
//   g_0 = sin t (q_s + q_p cos t), g_1 = q_p sin^2 t, g_2 = sin t (q_p cos t - q_s);
// the scalar model (Sec. 3.2, eq. "polar scalar final") is E = -i f k int p sin t J_0 ... dt.
// Evaluated as
//   plan:  theta nodes t_q and weights w_q on [0, theta_max] (Gauss-Legendre, split at
//          the sample's critical angle when it lies inside; or composite Simpson; or the
//          left Riemann sum), radial samples rho_r = r drho, and the table
//          B[q][g R + r] = w_q h_g(t_q) J_{n_g}(k rho_r sin t_q) for the groups g below
//          (FP64 kernel, stored FP32);
//   call:  Phi[q][(s, z), v] = p_s(t_q) exp(i k z cos t_q) u_v(t_q)   (FP64 phase -> FP32)
//          In[(s, z), v, :, g R + r] = sum_q Phi[q][(s, z), v] B[q][g R + r]
//                                       (real GEMM on MFMA, re/im as two rows)
//          radial epilogue: the I_n from the (v, g) products, 4-point Lagrange in rho
//          (parity ghosts I_n(-rho) = (-1)^n I_n(rho)), angular combination, |E|^2.
//          A single stack of few planes runs all three steps in one launch, one
//          workgroup per radial band of a plane.
// Modes (groups g: order n_g, weight h_g; variants v: factor u_v):
//   vectorial       g = (J0, sin t (1 + cos t)), (J1, sin^2 t), (J2, sin t (cos t - 1)); u = 1
//   with Fresnel    g = (J0, sin t), (J0, sin t cos t), (J1, sin^2 t), (J2, sin t cos t),
//                   (J2, sin t); u = q_s, q_p; I_0 = [s, g0] + [p, g1], I_1 = [p, g2],
//                   I_2 = [p, g3] - [s, g4]
//   scalar          g = (J0, sin t); u = 1
#include <algorithm>
#include <cmath>
#include <complex>
#include <mutex>
#include <vector>

#include "rw_common.h"
#include "rw_plan.h"

namespace rw {

typedef float f16v_b __attribute__((ext_vector_type(16)));

// --------------------------------------------------------------------------
// Plan-time Bessel table (FP64 arithmetic).
// --------------------------------------------------------------------------
enum BesselMode { kModeVectorial = 0, kModeFresnel = 1, kModeScalar = 2 };
inline int bessel_groups(int mode) { return mode == kModeFresnel ? 5 : (mode == kModeScalar ? 1 : 3); }
inline int bessel_variants(int mode) { return mode == kModeFresnel ? 2 : 1; }

__global__ void bessel_table_kernel(float* __restrict__ out, const double* __restrict__ theta,
                                    const double* __restrict__ wt, int T, int R, int mode, double k,
                                    double drho) {
  const int G = mode == kModeFresnel ? 5 : (mode == kModeScalar ? 1 : 3);
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= G * R * T) return;
  const int q = idx / (G * R);
  const int gr = idx % (G * R);
  const int g = gr / R, r = gr % R;
  const double t = theta[q];
  const double st = sin(t), ct = cos(t);
  int n;
  double h;
  if (mode == kModeVectorial) {
    n = g;
    h = g == 0 ? st * (1.0 + ct) : (g == 1 ? st * st : st * (ct - 1.0));
  } else if (mode == kModeFresnel) {
    const int order[5] = {0, 0, 1, 2, 2};
    const double w5[5] = {st, st * ct, st * st, st * ct, st};
    n = order[g];
    h = w5[g];
  } else {
    n = 0;
    h = st;
  }
  out[(size_t)q * G * R + gr] = (float)(wt[q] * h * bessel_j(n, k * (r * drho) * st));
}

// --------------------------------------------------------------------------
// Per call: pupil x defocus on the theta nodes, Phi[q][s * nz + z] (complex64).
// --------------------------------------------------------------------------
// Only the axisymmetric Noll terms reach the Bessel form (validated): j = 1, 4, 11, 22
// (radial orders 0, 2, 4, 6) within RWPSF_MAX_ZERNIKE.
constexpr int kAxiTerms = 4;
constexpr int kAxiNoll[kAxiTerms] = {1, 4, 11, 22};
struct PhiStack {
  double t_s, zoff;
  double coef[kAxiTerms];
};
constexpr int kPhiStacks = 64;
template <int NS>
struct PhiArgsT {
  int T, nz, nstk, V, max_zernike, gibson_lanni;   // V: variants per column
  double s_max;
  GLParams gl;
  PhiStack s[NS];
};
using PhiArgs = PhiArgsT<kPhiStacks>;

// Per theta node, from the plan (FP64): sin t, cos t, the stack-independent amplitude
// (apodization x envelope x extra s_z factor) and k cos t.
struct BesselNode {
  double sin_t, cos_t, amp, kc;
};

// The plane-independent part of the pupil of stack `st` at node nd: the amplitude
// m = nd.amp x exp(-Im W) and the real phase W (Gibson-Lanni and the axisymmetric
// Zernike terms), FP64.
template <class A>
__device__ __forceinline__ void phi_node(const A& a, const PhiStack& st, const BesselNode& nd, float* m,
                                         double* w) {
  double w_re = 0.0, w_im = 0.0;
  if (a.gibson_lanni) gl_opd(a.gl, st.t_s, nd.sin_t, &w_re, &w_im);
  const double r = nd.sin_t / a.s_max;
  for (int j = 0; j < kAxiTerms; ++j)
    if (st.coef[j] != 0.0) w_re += kTwoPi * st.coef[j] * zernike_noll(kAxiNoll[j], r, 1.0, 0.0);
  *m = (float)(w_im != 0.0 ? nd.amp * exp(-w_im) : nd.amp);
  *w = w_re;
}

// Phi of one node and plane: the pupil times the defocus exp(i k z cos t) (FP64 phase,
// reduced before the FP32 sine and cosine), times q_s and q_p when V = 2.
__device__ __forceinline__ void phi_plane(float m, double ph, int V, const float* qsp, float2* out) {
  float sn, cs;
  sincosf((float)reduce_2pi(ph), &sn, &cs);
  const float pr = m * cs, pi = m * sn;
  if (V == 1) {
    out[0] = make_float2(pr, pi);
  } else {
    out[0] = make_float2(pr * qsp[0] - pi * qsp[1], pr * qsp[1] + pi * qsp[0]);
    out[1] = make_float2(pr * qsp[2] - pi * qsp[3], pr * qsp[3] + pi * qsp[2]);
  }
}

// fq: per node (Re q_s, Im q_s, Re q_p, Im q_p) when V = 2.  One thread per (node,
// stack, group of kPhiZ planes): the plane-independent part (apodization, envelope,
// Gibson-Lanni, Zernike phase; FP64 transcendentals) is formed once per thread, then
// only the defocus phase per plane.  phi: this launch's first column; ld: the row
// stride of the Phi matrix in complex entries.
constexpr int kPhiZ = 4;
__global__ void bessel_phi_kernel(PhiArgs a, const BesselNode* __restrict__ node,
                                  const double* __restrict__ z, const double* __restrict__ fq,
                                  float2* __restrict__ phi, int ld) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int nzg = (a.nz + kPhiZ - 1) / kPhiZ;
  const int per_q = a.nstk * nzg;
  if (idx >= a.T * per_q) return;
  const int q = idx / per_q, rem = idx % per_q;
  const int si = rem / nzg, z0 = (rem % nzg) * kPhiZ;
  const PhiStack& st = a.s[si];
  const BesselNode nd = node[q];
  float m;
  double w_re;
  phi_node(a, st, nd, &m, &w_re);
  const double kc = nd.kc;
  float qsp[4] = {0.f, 0.f, 0.f, 0.f};
  if (a.V == 2)
    for (int i = 0; i < 4; ++i) qsp[i] = (float)fq[4 * q + i];
  const int z1 = min(z0 + kPhiZ, a.nz);
  float2* out = phi + (size_t)q * ld + ((size_t)si * a.nz + z0) * a.V;
  for (int zi = z0; zi < z1; ++zi, out += a.V) phi_plane(m, w_re + kc * (z[zi] + st.zoff), a.V, qsp, out);
}

// --------------------------------------------------------------------------
// Real FP32 GEMM on the matrix cores for the theta contraction:
//   C[row][col] = sum_q A[q][row] B[q][col]
// rows = (stack, plane, re/im) read from Phi viewed as real [T][2 S nz],
// cols = (n, r) from the Bessel table [T][3R].  Output In[row][col].
// Workgroup 64 x 128, 4 waves of 32 x 64, k-stage 16, LDS double buffer.
// --------------------------------------------------------------------------
constexpr int RBM = 64, RBN = 128, RBK = 16, RWM = 32, RWN = 64;
constexpr int RLDA = RBM + 4, RLDB = RBN + 4;
constexpr int RSTAGE = RBK * RLDA + RBK * RLDB;

__global__ void __launch_bounds__(256) bessel_contract_kernel(const float* __restrict__ A, int lda,
                                                               const float* __restrict__ B, int ldb,
                                                               float* __restrict__ C, int ldc, int M,
                                                               int N, int K) {
  __shared__ float lds[2 * RSTAGE];
  const int tiles_n = (N + RBN - 1) / RBN;
  const int tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wrow = (wave / 2) * RWM, wcol = (wave % 2) * RWN;
  const int row0 = tm * RBM, col0 = tn * RBN;
  f16v_b acc[2];
  for (int j = 0; j < 2; ++j)
    for (int r = 0; r < 16; ++r) acc[j][r] = 0.f;

  // loads: A tile RBK x RBM (1024 floats, 4 per thread), B tile RBK x RBN (2048, 8 per thread)
  float ra[4], rb[8];
  auto gload = [&](int k0) {
    for (int i = 0; i < 4; ++i) {
      const int e = tid + i * 256;
      const int kk = e / RBM, c = e % RBM;
      const int k = k0 + kk, gc = row0 + c;
      ra[i] = (k < K && gc < M) ? A[(size_t)k * lda + gc] : 0.f;
    }
    for (int i = 0; i < 8; ++i) {
      const int e = tid + i * 256;
      const int kk = e / RBN, c = e % RBN;
      const int k = k0 + kk, gc = col0 + c;
      rb[i] = (k < K && gc < N) ? B[(size_t)k * ldb + gc] : 0.f;
    }
  };
  auto sstore = [&](float* st) {
    for (int i = 0; i < 4; ++i) {
      const int e = tid + i * 256;
      st[(e / RBM) * RLDA + (e % RBM)] = ra[i];
    }
    for (int i = 0; i < 8; ++i) {
      const int e = tid + i * 256;
      st[RBK * RLDA + (e / RBN) * RLDB + (e % RBN)] = rb[i];
    }
  };
  const int KT = (K + RBK - 1) / RBK;
  gload(0);
  sstore(lds);
  __syncthreads();
  const int h = lane >> 5, l32 = lane & 31;
  for (int kt = 0; kt < KT; ++kt) {
    float* cur = lds + (kt & 1) * RSTAGE;
    float* nxt = lds + ((kt + 1) & 1) * RSTAGE;
    const bool more = kt + 1 < KT;
    if (more) gload((kt + 1) * RBK);
#pragma unroll
    for (int kp = 0; kp < RBK / 2; ++kp) {
      const int kk = 2 * kp + h;
      const float a = cur[kk * RLDA + wrow + l32];
      const float b0 = cur[RBK * RLDA + kk * RLDB + wcol + l32];
      const float b1 = cur[RBK * RLDA + kk * RLDB + wcol + 32 + l32];
      acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b0, acc[0], 0, 0, 0);
      acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b1, acc[1], 0, 0, 0);
    }
    if (more) sstore(nxt);
    __syncthreads();
  }
  for (int j = 0; j < 2; ++j) {
    const int col = col0 + wcol + 32 * j + l32;
    for (int r = 0; r < 16; ++r) {
      const int row = row0 + wrow + (r >> 2) * 8 + h * 4 + (r & 3);
      if (row < M && col < N) C[(size_t)row * ldc + col] = acc[j][r];
    }
  }
}

// C[M x N] (row stride ldc) = A^T B with A [K][lda], B [K][ldb]; also the batched
// per-emitter phase GEMM.
hipError_t launch_rgemm(const float* A, int lda, const float* B, int ldb, float* C, int ldc, int M,
                        int N, int K, hipStream_t st) {
  const int blocks = ((M + RBM - 1) / RBM) * ((N + RBN - 1) / RBN);
  hipLaunchKernelGGL(bessel_contract_kernel, dim3(blocks), dim3(256), 0, st, A, lda, B, ldb, C, ldc, M,
                     N, K);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// Radial epilogue: one workgroup per (stack, plane).  The GEMM rows of this plane,
// (variant, re/im) x [G][R], are combined into I_n and staged in LDS as
// [re/im][NI][R] (NI = 3 integrals, or 1 for the scalar model).
// --------------------------------------------------------------------------
constexpr int kEpiStacks = 256;   // stacks per contraction and epilogue launch
// Workgroups per plane in the epilogue: a call with few planes splits each plane into 4
// runs of pixels, so that more CUs work on it (one stack: 40 -> 31-34 us per call); a call
// with many planes keeps one workgroup per plane (4 per plane made the 256-stack call's
// epilogue 246 -> 303 us).  The split does not change any result.
constexpr int kEpiSplitFew = 4, kEpiFewPlanes = 1024;
struct EpiArgs {
  int nx, ny, nz, R, nstk, s_base, mode, split;   // split: workgroups per plane
  float dx, dy, inv_drho;
  float exr, exi, eyr, eyi;   // polarisation times -(i f k / 2); scalar: exr + i exi = -i f k
  float x0[kEpiStacks], y0[kEpiStacks];
};
static_assert(sizeof(EpiArgs) <= 4000, "kernel arguments are passed by value (4 KB limit)");

__global__ void __launch_bounds__(256) bessel_epilogue_kernel(EpiArgs a, const float* __restrict__ In,
                                                              float2* __restrict__ E,
                                                              float* __restrict__ I) {
  extern __shared__ float sh[];  // [2][NI][R]
  // a.split workgroups per plane, each a contiguous run of its pixels
  const int part = blockIdx.x % a.split, pl = blockIdx.x / a.split;
  const int si = pl / a.nz, zi = pl % a.nz;
  const int R = a.R;
  const int G = a.mode == kModeFresnel ? 5 : (a.mode == kModeScalar ? 1 : 3);
  const int V = a.mode == kModeFresnel ? 2 : 1;
  const int NI = a.mode == kModeScalar ? 1 : 3;
  const float* src = In + ((size_t)si * a.nz + zi) * V * 2 * G * R;
  for (int i = threadIdx.x; i < 2 * NI * R; i += blockDim.x) {
    const int ri = i / (NI * R), n = (i / R) % NI, r = i % R;
    float v;
    if (a.mode == kModeFresnel) {
      const float* rs = src + (size_t)ri * G * R;         // variant q_s
      const float* rp = src + (size_t)(2 + ri) * G * R;   // variant q_p
      v = n == 0 ? rs[r] + rp[R + r] : (n == 1 ? rp[2 * R + r] : rp[3 * R + r] - rs[4 * R + r]);
    } else {
      v = src[(size_t)ri * G * R + n * R + r];
    }
    sh[i] = v;
  }
  __syncthreads();
  const float* re = sh;
  const float* im = sh + NI * R;
  const size_t plane = (size_t)a.nx * a.ny;
  const size_t gs = (size_t)(a.s_base + si);
  float2* Eb = E ? E + (gs * a.nz + zi) * NI * plane : nullptr;
  float* Ib = I ? I + (gs * a.nz + zi) * plane : nullptr;
  const float x0 = a.x0[si], y0 = a.y0[si];
  const int run = ((int)plane + a.split - 1) / a.split;
  const int pbeg = part * run, pend = min((int)plane, pbeg + run);
  if (a.mode == kModeScalar) {
    for (int pix = pbeg + threadIdx.x; pix < pend; pix += blockDim.x) {
      const int i = pix / a.ny, j = pix % a.ny;
      const float x = (float)(i - a.nx / 2) * a.dx - x0;
      const float y = (float)(j - a.ny / 2) * a.dy - y0;
      const float t = sqrtf(x * x + y * y) * a.inv_drho;
      const int r0 = min((int)t, R - 3);
      const float f = t - (float)r0;
      const float wm = -f * (f - 1.f) * (f - 2.f) * (1.f / 6.f);
      const float w0 = (f + 1.f) * (f - 1.f) * (f - 2.f) * 0.5f;
      const float w1 = -(f + 1.f) * f * (f - 2.f) * 0.5f;
      const float w2 = (f + 1.f) * f * (f - 1.f) * (1.f / 6.f);
      const int rm = r0 == 0 ? 1 : r0 - 1;   // I_0 is even in rho
      const float vr = wm * re[rm] + w0 * re[r0] + w1 * re[r0 + 1] + w2 * re[r0 + 2];
      const float vi = wm * im[rm] + w0 * im[r0] + w1 * im[r0 + 1] + w2 * im[r0 + 2];
      const float er = a.exr * vr - a.exi * vi, ei = a.exr * vi + a.exi * vr;
      if (Eb) Eb[pix] = make_float2(er, ei);
      if (Ib) Ib[pix] = er * er + ei * ei;
    }
    return;
  }
  for (int pix = pbeg + threadIdx.x; pix < pend; pix += blockDim.x) {
    const int i = pix / a.ny, j = pix % a.ny;
    const float x = (float)(i - a.nx / 2) * a.dx - x0;
    const float y = (float)(j - a.ny / 2) * a.dy - y0;
    const float rho = sqrtf(x * x + y * y);
    const float t = rho * a.inv_drho;
    int r0 = (int)t;
    r0 = min(r0, R - 3);
    const float f = t - (float)r0;
    // 4-point Lagrange weights on nodes -1, 0, 1, 2 (relative to r0)
    const float wm = -f * (f - 1.f) * (f - 2.f) * (1.f / 6.f);
    const float w0 = (f + 1.f) * (f - 1.f) * (f - 2.f) * 0.5f;
    const float w1 = -(f + 1.f) * f * (f - 2.f) * 0.5f;
    const float w2 = (f + 1.f) * f * (f - 1.f) * (1.f / 6.f);
    float vr[3], vi[3];
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      const float* pr = re + n * R;
      const float* pi = im + n * R;
      float gr, gi;
      if (r0 == 0) {  // ghost at -drho: I_n(-rho) = (-1)^n I_n(rho)
        const float sg = (n == 1) ? -1.f : 1.f;
        gr = sg * pr[1];
        gi = sg * pi[1];
      } else {
        gr = pr[r0 - 1];
        gi = pi[r0 - 1];
      }
      vr[n] = wm * gr + w0 * pr[r0] + w1 * pr[r0 + 1] + w2 * pr[r0 + 2];
      vi[n] = wm * gi + w0 * pi[r0] + w1 * pi[r0 + 1] + w2 * pi[r0 + 2];
    }
    float c1 = 1.f, s1 = 0.f;
    if (rho > 0.f) {
      c1 = x / rho;
      s1 = y / rho;
    }
    const float c2 = c1 * c1 - s1 * s1, s2 = 2.f * s1 * c1;
    // A = I0 - I2 c2, Bv = I2 s2, Cv = I0 + I2 c2
    const float Ar = vr[0] - vr[2] * c2, Ai = vi[0] - vi[2] * c2;
    const float Br = vr[2] * s2, Bi = vi[2] * s2;
    const float Cr = vr[0] + vr[2] * c2, Ci = vi[0] + vi[2] * c2;
    // Ex = ex A - ey B ; Ey = -ex B + ey C ; Ez = -2i (ex c1 + ey s1) I1
    const float exr = a.exr, exi = a.exi, eyr = a.eyr, eyi = a.eyi;
    const float Exr = exr * Ar - exi * Ai - (eyr * Br - eyi * Bi);
    const float Exi = exr * Ai + exi * Ar - (eyr * Bi + eyi * Br);
    const float Eyr = -(exr * Br - exi * Bi) + (eyr * Cr - eyi * Ci);
    const float Eyi = -(exr * Bi + exi * Br) + (eyr * Ci + eyi * Cr);
    const float pr_ = exr * c1 + eyr * s1, pi_ = exi * c1 + eyi * s1;  // ex c1 + ey s1
    const float qr = pr_ * vr[1] - pi_ * vi[1], qi = pr_ * vi[1] + pi_ * vr[1];
    const float Ezr = 2.f * qi, Ezi = -2.f * qr;  // -2i q
    if (Eb) {
      Eb[pix] = make_float2(Exr, Exi);
      Eb[plane + pix] = make_float2(Eyr, Eyi);
      Eb[2 * plane + pix] = make_float2(Ezr, Ezi);
    }
    if (Ib) Ib[pix] = Exr * Exr + Exi * Exi + Eyr * Eyr + Eyi * Eyi + Ezr * Ezr + Ezi * Ezi;
  }
}

// --------------------------------------------------------------------------
// Calls of one stack: phase, contraction and radial epilogue in one launch.  With a few
// dozen planes the three-launch path is bound by its contraction (the GEMM then has a
// dozen workgroups, each walking the whole theta range), so here one workgroup serves
// one radial band of one plane.  It forms Phi of its plane on every
// node into LDS, contracts it with the Bessel-table columns of the radial samples its
// pixels' stencils reach (vector FMAs; the node range split between thread groups, eight
// table loads in flight per thread, the partial sums added in a fixed order), then walks
// the plane and writes the pixels whose stencil base sample r0 lies in the band.  The
// host sets the band edges so that the bands cost about the same (contraction samples
// against pixels).
// --------------------------------------------------------------------------
// Measured on the 65 x 65 x 33 stack: one stack 29.9 -> 21.7 us per call; two stacks
// 30.9 us either way, three or more slower than the three launches, so only a single
// stack of at most 64 planes takes this path (at least 8 bands per plane).
constexpr int kFusedStacks = 1;      // a call of at most this many stacks ...
constexpr int kFusedPlanes = 64;     // ... and planes takes the fused path
constexpr int kFusedBands = 64;      // bands per plane, at most
constexpr int kFusedLdsBytes = 64 * 1024;
struct FusedArgs {
  PhiArgsT<kFusedStacks> phi;
  int nx, ny, R, P;   // P: bands per plane
  float dx, dy, inv_drho;
  float exr, exi, eyr, eyi;
  float x0[kFusedStacks], y0[kFusedStacks];
  int edge[kFusedBands + 1];   // band b: pixels with r0 in [edge[b], edge[b + 1])
};
static_assert(sizeof(BesselNode) == 4 * sizeof(double), "the plan stores four doubles per node");
static_assert(sizeof(FusedArgs) <= 4000, "kernel arguments are passed by value (4 KB limit)");

template <int MODE>
struct FusedTerms {
  static constexpr int NI = MODE == kModeScalar ? 1 : 3;
  static constexpr int G = MODE == kModeFresnel ? 5 : (MODE == kModeScalar ? 1 : 3);
  static constexpr int V = MODE == kModeFresnel ? 2 : 1;
};

// LDS floats of one fused workgroup: Phi [T][V] complex, partial sums [2][max(256,
// items)], the band's integrals [2][items] (items = NI x samples).
__host__ __device__ inline int fused_lds_floats(int T, int V, int items) {
  return 2 * T * V + 2 * (items > 256 ? items : 256) + 2 * items;
}

template <int MODE>
__global__ void __launch_bounds__(256) bessel_fused_kernel(FusedArgs a, const BesselNode* __restrict__ node,
                                                           const double* __restrict__ z,
                                                           const double* __restrict__ fq,
                                                           const float* __restrict__ btab,
                                                           float2* __restrict__ E, float* __restrict__ I) {
  using FT = FusedTerms<MODE>;
  constexpr int NI = FT::NI, G = FT::G, V = FT::V;
  extern __shared__ float sh[];
  const int tid = threadIdx.x;
  const int band = blockIdx.x % a.P, pl = blockIdx.x / a.P;
  const int nz = a.phi.nz, T = a.phi.T, R = a.R;
  const int si = pl / nz, zi = pl % nz;
  const PhiStack& st = a.phi.s[si];
  // ---- Phi of this plane on every node
  float2* ph = reinterpret_cast<float2*>(sh);
  for (int q = tid; q < T; q += 256) {
    const BesselNode nd = node[q];
    float m;
    double w;
    phi_node(a.phi, st, nd, &m, &w);
    float qsp[4] = {0.f, 0.f, 0.f, 0.f};
    if (V == 2)
      for (int k = 0; k < 4; ++k) qsp[k] = (float)fq[4 * q + k];
    phi_plane(m, w + nd.kc * (z[zi] + st.zoff), V, qsp, ph + (size_t)q * V);
  }
  // ---- the band's radial samples: stencils r0 - 1 .. r0 + 2 of r0 in [e0, e1); the
  // ghost of r0 = 0 reads sample 1, which the band then holds (e1 >= 1)
  const int e0 = a.edge[band], e1 = a.edge[band + 1];
  const int ra = max(e0 - 1, 0), rb = min(e1 + 2, R);
  const int ns = rb - ra, items = NI * ns;
  const int stride = max(256, items);
  float* part = sh + 2 * T * V;
  float* inl = part + 2 * stride;   // [re/im][NI][ns]
  __syncthreads();
  const int groups = items >= 256 ? 1 : 256 / items;
  for (int u = tid; u < items * groups; u += 256) {
    const int g = u / items, it = u % items;
    const int n = it / ns, r = ra + it % ns;
    const int q0 = (int)((long long)g * T / groups), q1 = (int)((long long)(g + 1) * T / groups);
    // I_n = [v1, table group g1] + sg2 [v2, g2]; with Fresnel factors I_0 = [s, 0] +
    // [p, 1], I_1 = [p, 2], I_2 = [p, 3] - [s, 4], otherwise I_n = [0, n]
    int v1 = 0, o1 = n * R, v2 = 0, o2 = 0;
    float sg2 = 0.f;
    if (MODE == kModeFresnel) {
      v1 = n == 0 ? 0 : 1;
      o1 = (n == 0 ? 0 : n + 1) * R;
      v2 = n == 0 ? 1 : 0;
      o2 = (n == 0 ? 1 : 4) * R;
      sg2 = n == 0 ? 1.f : (n == 2 ? -1.f : 0.f);
    }
    float sr = 0.f, si_ = 0.f;
    const float* bcol = btab + r;
    for (int q = q0; q < q1; q += 8) {
      float b1[8], b2[8];
#pragma unroll
      for (int u8 = 0; u8 < 8; ++u8) {
        const size_t row = (size_t)min(q + u8, q1 - 1) * G * R;
        b1[u8] = bcol[row + o1];
        b2[u8] = MODE == kModeFresnel ? bcol[row + o2] : 0.f;
      }
#pragma unroll
      for (int u8 = 0; u8 < 8; ++u8) {
        if (q + u8 < q1) {
          const float2* pq = ph + (size_t)(q + u8) * V;
          const float2 p1 = pq[v1];
          sr += p1.x * b1[u8];
          si_ += p1.y * b1[u8];
          if (MODE == kModeFresnel) {
            const float2 p2 = pq[v2];
            sr += sg2 * (p2.x * b2[u8]);
            si_ += sg2 * (p2.y * b2[u8]);
          }
        }
      }
    }
    part[g * items + it] = sr;
    part[stride + g * items + it] = si_;
  }
  __syncthreads();
  for (int it = tid; it < items; it += 256) {
    float sr = 0.f, si_ = 0.f;
    for (int g = 0; g < groups; ++g) {
      sr += part[g * items + it];
      si_ += part[stride + g * items + it];
    }
    inl[it] = sr;
    inl[items + it] = si_;
  }
  // ---- the band's pixels (same interpolation and angular combination as the epilogue
  // kernel, samples indexed from ra)
  const float* re = inl - ra;
  const float* im = inl + items - ra;
  const int plane = a.nx * a.ny;
  const size_t gp = (size_t)si * nz + zi;
  float2* Eb = E ? E + gp * NI * plane : nullptr;
  float* Ib = I ? I + gp * plane : nullptr;
  const float x0 = a.x0[si], y0 = a.y0[si];
  __syncthreads();
  for (int pix = tid; pix < plane; pix += 256) {
    const int i = pix / a.ny, j = pix % a.ny;
    const float x = (float)(i - a.nx / 2) * a.dx - x0;
    const float y = (float)(j - a.ny / 2) * a.dy - y0;
    const float rho = sqrtf(x * x + y * y);
    const float t = rho * a.inv_drho;
    const int r0 = min((int)t, R - 3);
    if (r0 < e0 || r0 >= e1) continue;
    const float f = t - (float)r0;
    const float wm = -f * (f - 1.f) * (f - 2.f) * (1.f / 6.f);
    const float w0 = (f + 1.f) * (f - 1.f) * (f - 2.f) * 0.5f;
    const float w1 = -(f + 1.f) * f * (f - 2.f) * 0.5f;
    const float w2 = (f + 1.f) * f * (f - 1.f) * (1.f / 6.f);
    if (MODE == kModeScalar) {
      const int rm = r0 == 0 ? 1 : r0 - 1;   // I_0 is even in rho
      const float vr = wm * re[rm] + w0 * re[r0] + w1 * re[r0 + 1] + w2 * re[r0 + 2];
      const float vi = wm * im[rm] + w0 * im[r0] + w1 * im[r0 + 1] + w2 * im[r0 + 2];
      const float er = a.exr * vr - a.exi * vi, ei = a.exr * vi + a.exi * vr;
      if (Eb) Eb[pix] = make_float2(er, ei);
      if (Ib) Ib[pix] = er * er + ei * ei;
      continue;
    }
    float vr[3], vi[3];
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      const float* pr = re + n * ns;
      const float* pi = im + n * ns;
      float gr, gi;
      if (r0 == 0) {  // ghost at -drho: I_n(-rho) = (-1)^n I_n(rho)
        const float sg = (n == 1) ? -1.f : 1.f;
        gr = sg * pr[1];
        gi = sg * pi[1];
      } else {
        gr = pr[r0 - 1];
        gi = pi[r0 - 1];
      }
      vr[n] = wm * gr + w0 * pr[r0] + w1 * pr[r0 + 1] + w2 * pr[r0 + 2];
      vi[n] = wm * gi + w0 * pi[r0] + w1 * pi[r0 + 1] + w2 * pi[r0 + 2];
    }
    float c1 = 1.f, s1 = 0.f;
    if (rho > 0.f) {
      c1 = x / rho;
      s1 = y / rho;
    }
    const float c2 = c1 * c1 - s1 * s1, s2 = 2.f * s1 * c1;
    const float Ar = vr[0] - vr[2] * c2, Ai = vi[0] - vi[2] * c2;
    const float Br = vr[2] * s2, Bi = vi[2] * s2;
    const float Cr = vr[0] + vr[2] * c2, Ci = vi[0] + vi[2] * c2;
    const float exr = a.exr, exi = a.exi, eyr = a.eyr, eyi = a.eyi;
    const float Exr = exr * Ar - exi * Ai - (eyr * Br - eyi * Bi);
    const float Exi = exr * Ai + exi * Ar - (eyr * Bi + eyi * Br);
    const float Eyr = -(exr * Br - exi * Bi) + (eyr * Cr - eyi * Ci);
    const float Eyi = -(exr * Bi + exi * Br) + (eyr * Ci + eyi * Cr);
    const float pr_ = exr * c1 + eyr * s1, pi_ = exi * c1 + eyi * s1;
    const float qr = pr_ * vr[1] - pi_ * vi[1], qi = pr_ * vi[1] + pi_ * vr[1];
    const float Ezr = 2.f * qi, Ezi = -2.f * qr;
    if (Eb) {
      Eb[pix] = make_float2(Exr, Exi);
      Eb[plane + pix] = make_float2(Eyr, Eyi);
      Eb[2 * plane + pix] = make_float2(Ezr, Ezi);
    }
    if (Ib) Ib[pix] = Exr * Exr + Exi * Exi + Eyr * Eyr + Eyi * Eyi + Ezr * Ezr + Ezi * Ezi;
  }
}

// --------------------------------------------------------------------------
// Plan and dispatch
// --------------------------------------------------------------------------
// Cost of the fused path per stencil base sample r0 = 0 .. R - 3, accumulated: per
// radial sample the contraction (one table read, one Phi read and two FMAs per term and
// node), per pixel its interpolation, angular combination and stores (the pixels of the
// unshifted grid; a shifted stack only moves the balance).
static void fused_plan_cost(rwpsf_plan* p) {
  const int R = p->num.n_rho, T = p->n_theta_total, nr = R - 2;
  const int terms = p->bessel_mode == kModeFresnel ? 5 : (p->bessel_mode == kModeScalar ? 1 : 3);
  constexpr double kPixelCost = 120.0;
  std::vector<double> cost(nr, 4.0 * terms * T);
  const float inv = (float)(1.0 / p->drho), dx = (float)p->grid.dx_nm, dy = (float)p->grid.dy_nm;
  for (int i = 0; i < p->grid.nx; ++i)
    for (int j = 0; j < p->grid.ny; ++j) {
      const float x = (float)(i - p->grid.nx / 2) * dx, y = (float)(j - p->grid.ny / 2) * dy;
      cost[std::min((int)(std::sqrt(x * x + y * y) * inv), R - 3)] += kPixelCost;
    }
  p->fused_cum.assign(nr + 1, 0.0);
  for (int r = 0; r < nr; ++r) p->fused_cum[r + 1] = p->fused_cum[r] + cost[r];
}

int bessel_scratch_init(int dev, float** out);

int bessel_plan_init(rwpsf_plan* p) {
  const int R = p->num.n_rho;
  if (6 * R * (int)sizeof(float) > 160 * 1024) return RWPSF_ERR_UNSUPPORTED;  // epilogue stages 6R floats
  p->bessel_mode = p->num.model == RWPSF_MODEL_SCALAR ? kModeScalar : (p->opt.fresnel ? kModeFresnel : kModeVectorial);
  const int G = bessel_groups(p->bessel_mode), V = bessel_variants(p->bessel_mode);
  std::vector<double> th, wt;
  const double tmax = p->theta_max;
  double tc = -1.0;
  if (p->opt.gibson_lanni && p->opt.n_s < p->opt.na && p->num.theta_rule == RWPSF_THETA_GAUSS)
    tc = std::asin(p->opt.n_s / p->opt.n_i);
  auto add_rule = [&](int n, double a, double b) {
    std::vector<double> x(n), w(n);
    gauss_legendre(n, a, b, x.data(), w.data());
    th.insert(th.end(), x.begin(), x.end());
    wt.insert(wt.end(), w.begin(), w.end());
  };
  if (tc > 0.0) {
    // sqrt(n_s^2 - n_i^2 sin^2 t) has a square-root branch point at the critical angle
    // t_c; on each side t = t_c -+ d u^2 makes the integrand smooth in u, so the
    // Gauss-Legendre rule in u keeps its exponential convergence.
    int n1 = (int)std::lround(p->num.n_theta * tc / tmax);
    n1 = std::max(2, std::min(p->num.n_theta - 2, n1));
    const int n2 = p->num.n_theta - n1;
    std::vector<double> u(std::max(n1, n2)), wu(std::max(n1, n2));
    gauss_legendre(n1, 0.0, 1.0, u.data(), wu.data());
    for (int i = 0; i < n1; ++i) {        // [0, t_c]: t = t_c - t_c (1 - u)^2
      const double v = 1.0 - u[i];
      th.push_back(tc - tc * v * v);
      wt.push_back(wu[i] * 2.0 * tc * v);
    }
    gauss_legendre(n2, 0.0, 1.0, u.data(), wu.data());
    for (int i = 0; i < n2; ++i) {        // [t_c, t_max]: t = t_c + (t_max - t_c) u^2
      th.push_back(tc + (tmax - tc) * u[i] * u[i]);
      wt.push_back(wu[i] * 2.0 * (tmax - tc) * u[i]);
    }
  } else if (p->num.theta_rule == RWPSF_THETA_SIMPSON) {
    // composite Simpson on n (odd) equally spaced nodes: h/3 (1, 4, 2, 4, ..., 4, 1)
    const int n = p->num.n_theta;
    const double h = tmax / (n - 1);
    for (int i = 0; i < n; ++i) {
      th.push_back(i * h);
      wt.push_back(h / 3.0 * ((i == 0 || i == n - 1) ? 1.0 : (i % 2 ? 4.0 : 2.0)));
    }
  } else if (p->num.theta_rule == RWPSF_THETA_RIEMANN) {
    // left Riemann sum: nodes i h, i < n, h = theta_max / n
    const int n = p->num.n_theta;
    const double h = tmax / n;
    for (int i = 0; i < n; ++i) {
      th.push_back(i * h);
      wt.push_back(h);
    }
  } else {
    add_rule(p->num.n_theta, 0.0, tmax);
  }
  const int T = (int)th.size();
  p->n_theta_total = T;
  // radial samples cover the farthest pixel plus a one-pixel emitter shift
  const double hx = (p->grid.nx / 2) * p->grid.dx_nm + p->grid.dx_nm;
  const double hy = (p->grid.ny / 2) * p->grid.dy_nm + p->grid.dy_nm;
  p->drho = std::sqrt(hx * hx + hy * hy) / (R - 3);
  fused_plan_cost(p);
  int st;
  if ((st = dev_alloc(p, &p->d_theta, T))) return st;
  if ((st = dev_alloc(p, &p->d_wtheta, T))) return st;
  if ((st = dev_alloc(p, &p->d_btab, (size_t)G * R * T))) return st;
  if ((st = dev_alloc(p, &p->d_z, (size_t)p->grid.nz))) return st;
  p->bessel_stacks = kEpiStacks;
  if ((st = bessel_scratch_init(p->device, &p->scratch))) return st;
  if ((st = dev_alloc(p, &p->d_phi, (size_t)T * p->bessel_stacks * p->grid.nz * V))) return st;
  if ((st = dev_alloc(p, (float**)&p->d_In, (size_t)p->bessel_stacks * p->grid.nz * V * 2 * G * R))) return st;
  if (V == 2) {
    // Fresnel products per node, FP64 (Re q_s, Im q_s, Re q_p, Im q_p)
    std::vector<double> fq(4 * (size_t)T);
    for (int q = 0; q < T; ++q) {
      std::complex<double> qs, qp;
      fresnel_q(p->opt, std::sin(th[q]), &qs, &qp);
      fq[4 * q] = qs.real();
      fq[4 * q + 1] = qs.imag();
      fq[4 * q + 2] = qp.real();
      fq[4 * q + 3] = qp.imag();
    }
    if ((st = dev_alloc(p, &p->d_fq, fq.size()))) return st;
    if ((st = hip_check(hipMemcpy(p->d_fq, fq.data(), fq.size() * sizeof(double), hipMemcpyHostToDevice))))
      return st;
  }
  if ((st = hip_check(hipMemcpy(p->d_theta, th.data(), T * sizeof(double), hipMemcpyHostToDevice)))) return st;
  {
    std::vector<BesselNode> nodes(T);
    for (int q = 0; q < T; ++q) {
      const double sn = std::sin(th[q]), cs = std::cos(th[q]);
      double amp = 1.0;
      if (p->opt.apodization) amp *= std::sqrt(cs);
      if (p->opt.s_env > 0.0) amp *= std::exp(-(sn * sn) / (p->opt.s_env * p->opt.s_env));
      if (p->opt.extra_sz) amp *= cs;
      nodes[q] = BesselNode{sn, cs, amp, p->k * cs};
    }
    if ((st = dev_alloc(p, &p->d_node, 4 * (size_t)T))) return st;
    if ((st = hip_check(hipMemcpy(p->d_node, nodes.data(), T * sizeof(BesselNode), hipMemcpyHostToDevice))))
      return st;
  }
  if ((st = hip_check(hipMemcpy(p->d_wtheta, wt.data(), T * sizeof(double), hipMemcpyHostToDevice)))) return st;
  if ((st = hip_check(hipMemcpy(p->d_z, p->z.data(), p->z.size() * sizeof(double), hipMemcpyHostToDevice)))) return st;
  const int total = G * R * T;
  hipLaunchKernelGGL(bessel_table_kernel, dim3((total + 255) / 256), dim3(256), 0, 0, p->d_btab,
                     p->d_theta, p->d_wtheta, T, R, p->bessel_mode, p->k, p->drho);
  if ((st = hip_check(hipGetLastError()))) return st;
  // the limit belongs to the kernel, not to this plan: allow the whole LDS, so that a later
  // plan with fewer radial samples cannot lower it below what this plan launches with
  if ((st = hip_check(hipFuncSetAttribute((const void*)bessel_epilogue_kernel,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024))))
    return st;
  const void* fused[3] = {(const void*)bessel_fused_kernel<kModeVectorial>,
                          (const void*)bessel_fused_kernel<kModeFresnel>, (const void*)bessel_fused_kernel<kModeScalar>};
  for (const void* k : fused)
    if ((st = hip_check(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, kFusedLdsBytes))))
      return st;
  return hip_check(hipDeviceSynchronize());
}

// Pupil x defocus on the theta nodes for stacks s[0..nb), nb <= kPhiStacks, into the Phi
// matrix at phi (its first column for these stacks), row stride ld complex entries.
template <int NS>
static void fill_phi_args(const rwpsf_plan* p, const rwpsf_stack* s, int nb, PhiArgsT<NS>& pa) {
  pa.T = p->n_theta_total;
  pa.nz = p->grid.nz;
  pa.nstk = nb;
  pa.V = bessel_variants(p->bessel_mode);
  pa.gibson_lanni = p->opt.gibson_lanni;
  pa.s_max = p->s_max;
  pa.gl = p->gl;
  int maxz = 0;
  for (int i = 0; i < nb; ++i) {
    const rwpsf_stack& x = s[i];
    pa.s[i].t_s = x.t_s_nm;
    pa.s[i].zoff = x.z_offset_nm;
    for (int q = 0; q < kAxiTerms; ++q)
      pa.s[i].coef[q] = kAxiNoll[q] <= x.n_zernike ? x.zernike_waves[kAxiNoll[q] - 1] : 0.0;
    maxz = std::max(maxz, x.n_zernike);
  }
  pa.max_zernike = maxz;
}

static int bessel_phi(rwpsf_plan* p, const rwpsf_stack* s, int nb, float2* phi, int ld, hipStream_t st) {
  const int T = p->n_theta_total, nz = p->grid.nz;
  PhiArgs pa{};
  fill_phi_args(p, s, nb, pa);
  const int total = T * nb * ((nz + kPhiZ - 1) / kPhiZ);
  const int tr = p->time_begin(RWPSF_KERNEL_BESSEL_PHI, st);
  hipLaunchKernelGGL(bessel_phi_kernel, dim3((total + 255) / 256), dim3(256), 0, st, pa, reinterpret_cast<const BesselNode*>(p->d_node),
                     p->d_z, p->d_fq, phi, ld);
  const int rc = hip_check(hipGetLastError());
  p->time_end(tr, st);
  return rc;
}

// Phi of stacks s[0..nb) (in launches of up to kPhiStacks) into the Phi matrix of nb
// stacks.
static int bessel_phi_all(rwpsf_plan* p, const rwpsf_stack* s, int nb, float2* phi, hipStream_t st) {
  const int V = bessel_variants(p->bessel_mode), nz = p->grid.nz;
  for (int c0 = 0; c0 < nb; c0 += kPhiStacks) {
    const int rc = bessel_phi(p, s + c0, std::min(kPhiStacks, nb - c0), phi + (size_t)c0 * nz * V, nb * nz * V, st);
    if (rc) return rc;
  }
  return RWPSF_OK;
}

// Polarisation factors of the angular combination with the prefactor folded in:
// vectorial -(i f k / 2) (ex, ey); scalar (-i f k, 0).
static void bessel_pol(const rwpsf_plan* p, float out[4]) {
  const std::complex<double> pref(0.0, -0.5 * p->opt.focal_length * p->k);
  std::complex<double> ex = pref * std::complex<double>(p->opt.ex_re, p->opt.ex_im);
  std::complex<double> ey = pref * std::complex<double>(p->opt.ey_re, p->opt.ey_im);
  if (p->bessel_mode == kModeScalar) {   // E = -i f k I_0, unit incident amplitude
    ex = std::complex<double>(0.0, -p->opt.focal_length * p->k);
    ey = 0.0;
  }
  out[0] = (float)ex.real();
  out[1] = (float)ex.imag();
  out[2] = (float)ey.real();
  out[3] = (float)ey.imag();
}

// The fused launch of a call of n stacks: P bands per plane (about two workgroups per CU
// in all) at equal shares of the plan's cost estimate, strictly increasing.  False when
// the call is too large for it or its LDS does not fit.
struct FusedPlan {
  int P, ns_max;
  int edge[kFusedBands + 1];
};
static bool fused_plan(const rwpsf_plan* p, int n, FusedPlan* f) {
  const int nz = p->grid.nz, R = p->num.n_rho, nr = R - 2, T = p->n_theta_total;
  if (n < 1 || n > kFusedStacks || n * nz > kFusedPlanes) return false;
  const int P = std::max(1, std::min(std::min(kFusedBands, nr), 512 / (n * nz)));
  const std::vector<double>& cum = p->fused_cum;
  f->P = P;
  f->edge[0] = 0;
  f->edge[P] = nr;
  int r = 0;
  for (int b = 1; b < P; ++b) {
    const double target = cum[nr] * b / P;
    while (r < nr && cum[r] < target) ++r;
    f->edge[b] = std::min(std::max(r, f->edge[b - 1] + 1), nr - (P - b));
  }
  f->ns_max = 0;
  for (int b = 0; b < P; ++b)
    f->ns_max = std::max(f->ns_max, std::min(f->edge[b + 1] + 2, R) - std::max(f->edge[b] - 1, 0));
  const int NI = p->bessel_mode == kModeScalar ? 1 : 3;
  return (size_t)fused_lds_floats(T, bessel_variants(p->bessel_mode), NI * f->ns_max) * sizeof(float) <=
         (size_t)kFusedLdsBytes;
}

static int bessel_fused(rwpsf_plan* p, int n, const rwpsf_stack* s, float2* E, float* I, const FusedPlan& f,
                        hipStream_t st) {
  const int mode = p->bessel_mode, NI = mode == kModeScalar ? 1 : 3;
  FusedArgs a{};
  fill_phi_args(p, s, n, a.phi);
  a.nx = p->grid.nx;
  a.ny = p->grid.ny;
  a.R = p->num.n_rho;
  a.P = f.P;
  a.dx = (float)p->grid.dx_nm;
  a.dy = (float)p->grid.dy_nm;
  a.inv_drho = (float)(1.0 / p->drho);
  float pol[4];
  bessel_pol(p, pol);
  a.exr = pol[0];
  a.exi = pol[1];
  a.eyr = pol[2];
  a.eyi = pol[3];
  for (int i = 0; i < n; ++i) {
    a.x0[i] = (float)s[i].x0_nm;
    a.y0[i] = (float)s[i].y0_nm;
  }
  for (int b = 0; b <= f.P; ++b) a.edge[b] = f.edge[b];
  const size_t lds = (size_t)fused_lds_floats(p->n_theta_total, bessel_variants(mode), NI * f.ns_max) * sizeof(float);
  const dim3 grid(n * p->grid.nz * f.P);
  const int tr = p->time_begin(RWPSF_KERNEL_BESSEL_FUSED, st);
  if (mode == kModeFresnel)
    hipLaunchKernelGGL(bessel_fused_kernel<kModeFresnel>, grid, dim3(256), lds, st, a, reinterpret_cast<const BesselNode*>(p->d_node), p->d_z, p->d_fq,
                       p->d_btab, E, I);
  else if (mode == kModeScalar)
    hipLaunchKernelGGL(bessel_fused_kernel<kModeScalar>, grid, dim3(256), lds, st, a, reinterpret_cast<const BesselNode*>(p->d_node), p->d_z, p->d_fq,
                       p->d_btab, E, I);
  else
    hipLaunchKernelGGL(bessel_fused_kernel<kModeVectorial>, grid, dim3(256), lds, st, a, reinterpret_cast<const BesselNode*>(p->d_node), p->d_z,
                       p->d_fq, p->d_btab, E, I);
  const int rc = hip_check(hipGetLastError());
  p->time_end(tr, st);
  return rc;
}

// Stacks s[0..n) in chunks of up to `chunk` (<= kEpiStacks) stacks, with Phi and I_n of a
// chunk in the workspaces phi ([T][chunk nz V] complex) and In ([chunk nz V][2][G][R]
// float): one contraction and one epilogue launch per chunk.  A call of one stack of few
// planes takes the fused launch instead (no workspace).
static int bessel_compute_ws(rwpsf_plan* p, int n, const rwpsf_stack* s, float2* E, float* I, float2* phi,
                             float* In, int chunk, hipStream_t st) {
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != p->device) return RWPSF_ERR_INVALID_ARG;
  if (6 * p->num.n_rho * 4 > 160 * 1024) return RWPSF_ERR_UNSUPPORTED;
  FusedPlan fp;
  if (fused_plan(p, n, &fp)) return bessel_fused(p, n, s, E, I, fp, st);
  const int T = p->n_theta_total, R = p->num.n_rho, nz = p->grid.nz;
  const int mode = p->bessel_mode, G = bessel_groups(mode), V = bessel_variants(mode);
  float pol[4];
  bessel_pol(p, pol);
  for (int b0 = 0; b0 < n; b0 += chunk) {
    const int nb = std::min(chunk, n - b0);
    int rc = bessel_phi_all(p, s + b0, nb, phi, st);
    if (rc) return rc;
    const int cols = nb * nz;
    const int M = 2 * cols * V, N = G * R;
    const int blocks = ((M + RBM - 1) / RBM) * ((N + RBN - 1) / RBN);
    int tr = p->time_begin(RWPSF_KERNEL_BESSEL_CONTRACT, st);
    hipLaunchKernelGGL(bessel_contract_kernel, dim3(blocks), dim3(256), 0, st, (const float*)phi, M,
                       (const float*)p->d_btab, N, In, N, M, N, T);
    if ((rc = hip_check(hipGetLastError()))) return rc;
    p->time_end(tr, st);
    EpiArgs ea{};
    ea.nx = p->grid.nx;
    ea.ny = p->grid.ny;
    ea.nz = nz;
    ea.R = R;
    ea.nstk = nb;
    ea.s_base = b0;
    ea.mode = mode;
    ea.dx = (float)p->grid.dx_nm;
    ea.dy = (float)p->grid.dy_nm;
    ea.inv_drho = (float)(1.0 / p->drho);
    ea.exr = pol[0];
    ea.exi = pol[1];
    ea.eyr = pol[2];
    ea.eyi = pol[3];
    for (int i = 0; i < nb; ++i) {
      ea.x0[i] = (float)s[b0 + i].x0_nm;
      ea.y0[i] = (float)s[b0 + i].y0_nm;
    }
    tr = p->time_begin(RWPSF_KERNEL_BESSEL_EPILOGUE, st);
    ea.split = nb * nz < kEpiFewPlanes ? kEpiSplitFew : 1;
    hipLaunchKernelGGL(bessel_epilogue_kernel, dim3(nb * nz * ea.split), dim3(256), 6 * R * sizeof(float), st, ea,
                       (const float*)In, E, I);
    if ((rc = hip_check(hipGetLastError()))) return rc;
    p->time_end(tr, st);
  }
  return RWPSF_OK;
}

int bessel_compute(rwpsf_plan* p, int n, const rwpsf_stack* s, float2* E, float* I, hipStream_t st) {
  return bessel_compute_ws(p, n, s, E, I, p->d_phi, (float*)p->d_In, kEpiStacks, st);
}

// --------------------------------------------------------------------------
// Allocation-free evaluation.  Phi and I_n of each chunk of stacks live in `scratch`, a
// fixed array in the library's device image (each device that loads the library holds
// its own copy until the process ends), so the call allocates nothing.  The host takes
// the array's device address once per device with hipGetSymbolAddress, with that device
// current (at the first Bessel plan created on it) and passes only that address on.
// Every call on one device shares the array: calls that overlap on a device race.
// --------------------------------------------------------------------------
constexpr size_t kScratchFloats = RWPSF_NOALLOC_SCRATCH_BYTES / sizeof(float);
constexpr size_t kScratchAlign = 64;   // floats (256 bytes) between Phi and I_n
constexpr int kScratchDevices = 64;
static __device__ __align__(256) float scratch[kScratchFloats];

static std::mutex g_scratch_mutex;
static float* g_scratch_ptr[kScratchDevices] = {};

// Device address of `scratch` on the current device `dev` (looked up once per device).
int bessel_scratch_init(int dev, float** out) {
  *out = nullptr;
  if (dev < 0 || dev >= kScratchDevices) return RWPSF_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_check(e);
    if (!ptr) return RWPSF_ERR_HIP;
    g_scratch_ptr[dev] = (float*)ptr;
  }
  *out = g_scratch_ptr[dev];
  return RWPSF_OK;
}

// Scratch floats one stack of this plan needs (Phi, then I_n), without the alignment gap.
static size_t bessel_scratch_per_stack(const rwpsf_plan* p) {
  const size_t V = bessel_variants(p->bessel_mode), G = bessel_groups(p->bessel_mode);
  const size_t nz = p->grid.nz, T = p->n_theta_total, R = p->num.n_rho;
  return 2 * T * nz * V + nz * V * 2 * G * R;
}

int bessel_compute_noalloc(rwpsf_plan* p, int n, const rwpsf_stack* s, float2* E, float* I, hipStream_t st) {
  if (!p->scratch) return RWPSF_ERR_HIP;   // the plan could not resolve the array's address
  const size_t per = bessel_scratch_per_stack(p);
  if (per + kScratchAlign > kScratchFloats) return RWPSF_ERR_SCRATCH_LIMIT;
  const int chunk = (int)std::min<size_t>(kEpiStacks, (kScratchFloats - kScratchAlign) / per);
  const size_t V = bessel_variants(p->bessel_mode);
  const size_t phi_floats = 2 * (size_t)p->n_theta_total * chunk * p->grid.nz * V;
  const size_t in_off = (phi_floats + kScratchAlign - 1) / kScratchAlign * kScratchAlign;
  return bessel_compute_ws(p, n, s, E, I, (float2*)p->scratch, p->scratch + in_off, chunk, st);
}

// --------------------------------------------------------------------------
// Adjoint of the Bessel form.  For a real loss L(I) with g = dL/dI:
//   G_E = 2 g E;  G_In[n](r) = sum over the pixels whose radial stencil reaches r of
//   weight(r) conj(C_cn) G_E,c  (the transpose of the Lagrange interpolation and of
//   the angular combination); G_Phi = G_In B^T (the transpose of the contraction);
//   X_s[q] = sum_{z,v} conj(G_Phi) Phi;  dL/dtheta = sum_q Re(i dW/dtheta(t_q) X_s[q])
//   with dW/dc_j = 2 pi Z_j, dW/dt_s = d W_GL / d t_s, dW/dz_offset = k cos t.
// --------------------------------------------------------------------------
struct AdjRadArgs {
  int nx, ny, nz, R, mode, s_base, M;   // M: rows of G_In^T (2 nb nz V)
  float dx, dy, inv_drho, drho;
  float exr, exi, eyr, eyi;
  float x0[kPhiStacks], y0[kPhiStacks];
};

// Projections P_n = sum_c conj(C_cn) G_E,c of one pixel (the transpose of the angular
// combination), G_E = 2 (dL/dI) E; p[0..5] = (P_0, P_1, P_2) as re, im.
__device__ __forceinline__ void adjb_project(const AdjRadArgs& a, bool scalar, const float2* Eb, size_t plane,
                                             float g2, int pix, float x, float y, float rho, float p[6]) {
  // computed into scalars and stored once, so that p stays in registers
  float p0, p1, p2 = 0.f, p3 = 0.f, p4 = 0.f, p5 = 0.f;
  if (scalar) {
    const float2 e = Eb[pix];
    const float gr = g2 * e.x, gi = g2 * e.y;
    p0 = a.exr * gr + a.exi * gi;    // conj(pref) G
    p1 = a.exr * gi - a.exi * gr;
  } else {
    const float2 ex = Eb[pix], ey = Eb[plane + pix], ez = Eb[2 * plane + pix];
    const float gxr = g2 * ex.x, gxi = g2 * ex.y, gyr = g2 * ey.x, gyi = g2 * ey.y;
    const float gzr = g2 * ez.x, gzi = g2 * ez.y;
    float c1 = 1.f, s1 = 0.f;
    if (rho > 0.f) {
      c1 = x / rho;
      s1 = y / rho;
    }
    const float c2 = c1 * c1 - s1 * s1, s2 = 2.f * s1 * c1;
    // P0 = conj(ex) Gx + conj(ey) Gy
    p0 = a.exr * gxr + a.exi * gxi + a.eyr * gyr + a.eyi * gyi;
    p1 = a.exr * gxi - a.exi * gxr + a.eyr * gyi - a.eyi * gyr;
    // P1 = 2i conj(ex c1 + ey s1) Gz
    const float qr = a.exr * c1 + a.eyr * s1, qi = a.exi * c1 + a.eyi * s1;
    p2 = -2.f * (qr * gzi - qi * gzr);
    p3 = 2.f * (qr * gzr + qi * gzi);
    // P2 = conj(-(ex c2 + ey s2)) Gx + conj(-ex s2 + ey c2) Gy
    const float ur = -(a.exr * c2 + a.eyr * s2), ui = -(a.exi * c2 + a.eyi * s2);
    const float vr = -a.exr * s2 + a.eyr * c2, vi = -a.exi * s2 + a.eyi * c2;
    p4 = ur * gxr + ui * gxi + vr * gyr + vi * gyi;
    p5 = ur * gxi - ui * gxr + vr * gyi - vi * gyr;
  }
  p[0] = p0;
  p[1] = p1;
  p[2] = p2;
  p[3] = p3;
  p[4] = p4;
  p[5] = p5;
}

// One workgroup per (stack, plane).  Every pixel adds w_k P_n to the four radial samples
// of its stencil (node -1 mirrored onto node 1 with the parity (-1)^n), the transpose of
// the forward interpolation.  The sums are kept in LDS as 64-bit integers in units of
// 2^-36 of the plane's largest |P|: integer addition is associative, so the atomics give
// a bitwise repeatable result whatever their order, and the quantisation error (2^-37 of
// the largest term per term) is far below FP32 rounding.  Writes
// G_In^T[g R + r][2 ((s nz + z) V + v) + re/im].
__global__ void __launch_bounds__(256) adjb_radial_kernel(AdjRadArgs a, const float2* __restrict__ E,
                                                          const float* __restrict__ dLdI,
                                                          float* __restrict__ GInT) {
  extern __shared__ long long accq[];        // [R][6]
  __shared__ float red[256];
  const int si = blockIdx.x / a.nz, zi = blockIdx.x % a.nz;
  const int R = a.R, tid = threadIdx.x;
  const bool scalar = a.mode == kModeScalar;
  const int NI = scalar ? 1 : 3;
  const int P = a.nx * a.ny;
  const size_t plane = (size_t)P;
  const size_t gsz = (size_t)(a.s_base + si) * a.nz + zi;
  const float2* Eb = E + gsz * NI * plane;
  const float* Lb = dLdI + gsz * plane;
  const float x0 = a.x0[si], y0 = a.y0[si];
  for (int i = tid; i < 6 * R; i += blockDim.x) accq[i] = 0;
  // largest |P| of the plane (a max does not depend on the order)
  float mx = 0.f;
  for (int pix = tid; pix < P; pix += blockDim.x) {
    const int i = pix / a.ny, j = pix % a.ny;
    const float x = (float)(i - a.nx / 2) * a.dx - x0, y = (float)(j - a.ny / 2) * a.dy - y0;
    float p[6];
    adjb_project(a, scalar, Eb, plane, 2.f * Lb[pix], pix, x, y, sqrtf(x * x + y * y), p);
#pragma unroll
    for (int e = 0; e < 6; ++e) mx = fmaxf(mx, fabsf(p[e]));
  }
  red[tid] = mx;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) red[tid] = fmaxf(red[tid], red[tid + h]);
    __syncthreads();
  }
  mx = red[0];
  const double scale = mx > 0.f ? ldexp(1.0, 36 - ilogbf(mx)) : 0.0;
  if (mx > 0.f) {
    for (int pix = tid; pix < P; pix += blockDim.x) {
      const int i = pix / a.ny, j = pix % a.ny;
      const float x = (float)(i - a.nx / 2) * a.dx - x0, y = (float)(j - a.ny / 2) * a.dy - y0;
      const float rho = sqrtf(x * x + y * y);
      const float t = rho * a.inv_drho;
      const int r0 = min((int)t, R - 3);
      const float f = t - (float)r0;
      const float w[4] = {-f * (f - 1.f) * (f - 2.f) * (1.f / 6.f), (f + 1.f) * (f - 1.f) * (f - 2.f) * 0.5f,
                          -(f + 1.f) * f * (f - 2.f) * 0.5f, (f + 1.f) * f * (f - 1.f) * (1.f / 6.f)};
      float p[6];
      adjb_project(a, scalar, Eb, plane, 2.f * Lb[pix], pix, x, y, rho, p);
      // fully unrolled, so that w, p and the signs stay in registers
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const bool ghost = r0 - 1 + k < 0;   // node -1: I_n(-rho) = (-1)^n I_n(rho)
        long long* d = accq + 6 * (ghost ? 1 : r0 - 1 + k);
#pragma unroll
        for (int e = 0; e < 6; ++e) {
          const float sg = (ghost && (e == 2 || e == 3)) ? -1.f : 1.f;
          const long long v = llrint((double)(sg * w[k] * p[e]) * scale);
          if (v) atomicAdd(reinterpret_cast<unsigned long long*>(d + e), (unsigned long long)v);
        }
      }
    }
  }
  __syncthreads();
  const double inv = mx > 0.f ? 1.0 / scale : 0.0;
  const int V = a.mode == kModeFresnel ? 2 : 1;
  const int col = (si * a.nz + zi) * V;
  for (int r = tid; r < R; r += blockDim.x) {
    float g[6];
#pragma unroll
    for (int e = 0; e < 6; ++e) g[e] = (float)((double)accq[6 * r + e] * inv);
    auto put = [&](int v, int gg, float re, float im) {
      float* d = GInT + (size_t)(gg * R + r) * a.M + 2 * (col + v);
      d[0] = re;
      d[1] = im;
    };
    if (a.mode == kModeFresnel) {
      put(0, 0, g[0], g[1]);
      put(1, 1, g[0], g[1]);
      put(1, 2, g[2], g[3]);
      put(1, 3, g[4], g[5]);
      put(0, 4, -g[4], -g[5]);
      put(1, 0, 0.f, 0.f);
      put(0, 1, 0.f, 0.f);
      put(0, 2, 0.f, 0.f);
      put(0, 3, 0.f, 0.f);
      put(1, 4, 0.f, 0.f);
    } else {
#pragma unroll
      for (int n = 0; n < 3; ++n)
        if (n < NI) put(0, n, g[2 * n], g[2 * n + 1]);
    }
  }
}

// X_s[q] = sum_{z,v} conj(G_Phi[(s,z,v)][q]) Phi[q][(s,z),v], FP64 accumulation.
__global__ void adjb_x_kernel(const float* __restrict__ GPhi, const float2* __restrict__ phi,
                              double2* __restrict__ X, int nb, int nz, int V, int T) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nb * T) return;
  const int s = idx / T, q = idx % T;
  const int ld = nb * nz * V;
  double xr = 0.0, xi = 0.0;
  for (int z = 0; z < nz; ++z)
    for (int v = 0; v < V; ++v) {
      const int col = (s * nz + z) * V + v;
      const double gr = GPhi[(size_t)(2 * col) * T + q], gi = GPhi[(size_t)(2 * col + 1) * T + q];
      const float2 ph = phi[(size_t)q * ld + col];
      xr += gr * ph.x + gi * ph.y;
      xi += gr * ph.y - gi * ph.x;
    }
  X[idx] = make_double2(xr, xi);
}

// Per stack (one 64-lane workgroup each): dL/dt_s, dL/dz_offset and the stack's share of
// dL/dc_j.  Lane l sums the nodes q = l, l + 64, ... in order, then a fixed tree joins
// the lanes: bitwise repeatable.
// node[q] = (k cos t, Re dW/dt_s, Im dW/dt_s, 2 pi Z_1, 2 pi Z_4, 2 pi Z_11, 2 pi Z_22).
__global__ void __launch_bounds__(64) adjb_stack_kernel(const double2* __restrict__ X, const double* __restrict__ node,
                                                        int T, int s_base, float* __restrict__ dts,
                                                        float* __restrict__ dz, double* __restrict__ dcp) {
  __shared__ double red[6][64];
  const int s = blockIdx.x, l = threadIdx.x;
  double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};   // t_s, z, c_1, c_4, c_11, c_22
  for (int q = l; q < T; q += 64) {
    const double2 x = X[(size_t)s * T + q];
    const double* nd = node + 7 * (size_t)q;
    v[1] -= nd[0] * x.y;                   // Re(i w X) = -w Im X for real w
    v[0] -= nd[1] * x.y + nd[2] * x.x;     // Re(i (a + ib) X)
    for (int j = 0; j < 4; ++j) v[2 + j] -= nd[3 + j] * x.y;
  }
  for (int e = 0; e < 6; ++e) red[e][l] = v[e];
  __syncthreads();
  for (int h = 32; h > 0; h >>= 1) {
    if (l < h)
      for (int e = 0; e < 6; ++e) red[e][l] += red[e][l + h];
    __syncthreads();
  }
  if (l == 0) {
    const int gs = s_base + s;
    if (dts) dts[gs] = (float)red[0][0];
    if (dz) dz[gs] = (float)red[1][0];
    for (int j = 0; j < 4; ++j) dcp[4 * (size_t)gs + j] = red[2 + j][0];
  }
}

__global__ void adjb_coef_kernel(const double* __restrict__ dcp, int n, float* __restrict__ dc) {
  const int j = threadIdx.x;
  if (j >= 4) return;
  double acc = 0.0;
  for (int s = 0; s < n; ++s) acc += dcp[4 * (size_t)s + j];
  dc[j] = (float)acc;
}

__global__ void adjb_transpose_kernel(const float* __restrict__ in, float* __restrict__ out, int rows, int cols) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  const int r = idx / cols, c = idx % cols;
  out[(size_t)c * rows + r] = in[idx];
}

// Tables and workspace of the adjoint, built on first use.
static int bessel_adjoint_prepare(rwpsf_plan* p) {
  if (p->d_btabT) return RWPSF_OK;
  const int T = p->n_theta_total, R = p->num.n_rho, nz = p->grid.nz;
  const int G = bessel_groups(p->bessel_mode), V = bessel_variants(p->bessel_mode);
  // per-sample sums [R][6] 64-bit integers in LDS
  if ((size_t)R * 6 * sizeof(long long) > 150 * 1024) return RWPSF_ERR_UNSUPPORTED;
  std::vector<double> th(T);
  int st;
  if ((st = hip_check(hipMemcpy(th.data(), p->d_theta, T * sizeof(double), hipMemcpyDeviceToHost)))) return st;
  std::vector<double> node(7 * (size_t)T);
  const int noll[4] = {1, 4, 11, 22};
  for (int q = 0; q < T; ++q) {
    const double sn = std::sin(th[q]), cs = std::cos(th[q]);
    node[7 * q] = p->k * cs;
    double a = 0.0, b = 0.0;
    if (p->opt.gibson_lanni) {
      // t_i = t_s + n_i (-t_s / n_s - ...): dW/dt_s = k0 (root(n_s) + (1 - n_i / n_s) root(n_i))
      const double inv2 = (p->opt.n_i * sn) * (p->opt.n_i * sn);
      const std::complex<double> rs = std::sqrt(std::complex<double>(p->opt.n_s * p->opt.n_s - inv2, 0.0));
      const std::complex<double> ri = std::sqrt(std::complex<double>(p->opt.n_i * p->opt.n_i - inv2, 0.0));
      const std::complex<double> d = (kTwoPi / p->opt.wavelength_nm) * (rs + (1.0 - p->opt.n_i / p->opt.n_s) * ri);
      a = d.real();
      b = d.imag();
    }
    node[7 * q + 1] = a;
    node[7 * q + 2] = b;
    for (int j = 0; j < 4; ++j) node[7 * q + 3 + j] = kTwoPi * zernike_noll(noll[j], sn / p->s_max, 1.0, 0.0);
  }
  const size_t M = 2 * (size_t)kPhiStacks * nz * V;
  if ((st = dev_alloc(p, &p->d_btabT, (size_t)G * R * T))) return st;
  if ((st = dev_alloc(p, &p->d_GInT, (size_t)G * R * M))) return st;
  if ((st = dev_alloc(p, &p->d_GPhi, M * T))) return st;
  if ((st = dev_alloc(p, &p->d_adjX, (size_t)kPhiStacks * T))) return st;
  if ((st = dev_alloc(p, &p->d_adjnode, node.size()))) return st;
  if ((st = dev_alloc(p, &p->d_dcp, 4 * (size_t)RWPSF_MAX_STACKS_PER_CALL))) return st;

  if ((st = hip_check(hipMemcpy(p->d_adjnode, node.data(), node.size() * sizeof(double), hipMemcpyHostToDevice))))
    return st;
  // the limits are per kernel, not per plan: allow the whole LDS so plans of any size can launch
  if ((st = hip_check(hipFuncSetAttribute((const void*)adjb_radial_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                          150 * 1024))))
    return st;
  const int total = G * R * T;
  hipLaunchKernelGGL(adjb_transpose_kernel, dim3((total + 255) / 256), dim3(256), 0, 0, p->d_btab, p->d_btabT, T,
                     G * R);
  if ((st = hip_check(hipGetLastError()))) return st;
  return hip_check(hipDeviceSynchronize());
}

int bessel_adjoint(rwpsf_plan* p, int n, const rwpsf_stack* s, const float2* E, const float* dLdI, float* dc,
                   float* dts, float* dz, hipStream_t st) {
  int rc = bessel_adjoint_prepare(p);
  if (rc) return rc;
  const int T = p->n_theta_total, R = p->num.n_rho, nz = p->grid.nz;
  const int mode = p->bessel_mode, G = bessel_groups(mode), V = bessel_variants(mode);
  float pol[4];
  bessel_pol(p, pol);
  for (int b0 = 0; b0 < n; b0 += kPhiStacks) {
    const int nb = std::min(kPhiStacks, n - b0);
    if ((rc = bessel_phi(p, s + b0, nb, p->d_phi, nb * nz * V, st))) return rc;
    const int M = 2 * nb * nz * V;
    AdjRadArgs ra{};
    ra.nx = p->grid.nx;
    ra.ny = p->grid.ny;
    ra.nz = nz;
    ra.R = R;
    ra.mode = mode;
    ra.s_base = b0;
    ra.M = M;
    ra.dx = (float)p->grid.dx_nm;
    ra.dy = (float)p->grid.dy_nm;
    ra.inv_drho = (float)(1.0 / p->drho);
    ra.drho = (float)p->drho;
    ra.exr = pol[0];
    ra.exi = pol[1];
    ra.eyr = pol[2];
    ra.eyi = pol[3];
    for (int i = 0; i < nb; ++i) {
      ra.x0[i] = (float)s[b0 + i].x0_nm;
      ra.y0[i] = (float)s[b0 + i].y0_nm;
    }
    int tr = p->time_begin(RWPSF_KERNEL_ADJB_RADIAL, st);
    hipLaunchKernelGGL(adjb_radial_kernel, dim3(nb * nz), dim3(256), (size_t)R * 6 * sizeof(long long), st, ra, E,
                       dLdI, p->d_GInT);
    if ((rc = hip_check(hipGetLastError()))) return rc;
    p->time_end(tr, st);
    // G_Phi[m][q] = sum_k G_In^T[k][m] B^T[k][q]
    const int K = G * R;
    const int blocks = ((M + RBM - 1) / RBM) * ((T + RBN - 1) / RBN);
    tr = p->time_begin(RWPSF_KERNEL_ADJB_CONTRACT, st);
    hipLaunchKernelGGL(bessel_contract_kernel, dim3(blocks), dim3(256), 0, st, (const float*)p->d_GInT, M,
                       (const float*)p->d_btabT, T, p->d_GPhi, T, M, T, K);
    if ((rc = hip_check(hipGetLastError()))) return rc;
    p->time_end(tr, st);
    tr = p->time_begin(RWPSF_KERNEL_ADJB_REDUCE, st);
    hipLaunchKernelGGL(adjb_x_kernel, dim3((nb * T + 255) / 256), dim3(256), 0, st, (const float*)p->d_GPhi,
                       (const float2*)p->d_phi, p->d_adjX, nb, nz, V, T);
    if ((rc = hip_check(hipGetLastError()))) return rc;
    hipLaunchKernelGGL(adjb_stack_kernel, dim3(nb), dim3(64), 0, st, (const double2*)p->d_adjX,
                       (const double*)p->d_adjnode, T, b0, dts, dz, p->d_dcp);
    if ((rc = hip_check(hipGetLastError()))) return rc;
    p->time_end(tr, st);
  }
  if (dc) {
    hipLaunchKernelGGL(adjb_coef_kernel, dim3(1), dim3(64), 0, st, (const double*)p->d_dcp, n, dc);
    if ((rc = hip_check(hipGetLastError()))) return rc;
  }
  return RWPSF_OK;
}

}  // namespace rw
