// Chirp-z (Bluestein) evaluation of the Fourier form, the paper's own algorithm for the
// Cartesian integral (Sec. 3.3, the discussion of the chirp-Z transform that follows eq.
// "cartesian vectorial"): each 1-D transform of the separable sum
//   T[j][n] = sum_l P~[j][l] e^{i k s_l y_n},   E_c[m][n] = C sum_j e^{i k s_j x_m} T[j][n]
// has equispaced inputs and outputs, k s_l y_n = beta (l - l0)(n - n0) with
// beta = k (2 s_max / N) dy, l0 = (N-1)/2, n0 = ny/2, so with l n = (l^2 + n^2 - (n-l)^2)/2
//   T[n] = post[n] sum_l (P~[l] pre[l]) c[n - l],
//   pre[l] = e^{i beta (l^2/2 - l n0)},  post[n] = e^{i beta (n^2/2 - l0 n + l0 n0)},
//   c[m] = e^{-i beta m^2 / 2},
// a linear convolution evaluated by FFTs of length L >= N + ny - 1 (power of two):
//   T = post . IFFT( FFT(a) . FFT(c) ),  IFFT(x) = conj(FFT(conj(x))) / L.
// The same holds along x with alpha = k (2 s_max / N) dx and the prefactor C in post.
// The result is the same discrete sum as the matrix-DFT evaluation (the oracle's
// separable form); only the rounding differs.
//
// FFTs run in LDS, one per wave and without workgroup barriers: a Stockham auto-sort
// transform of radix-8 passes and one final radix-4 or radix-2 pass (butterfly j reads
// j + r L/R, writes (j / Ns) Ns R + j mod Ns + r Ns after the twiddle
// W^{(j mod Ns) r L / (Ns R)}, W = e^{-2 pi i / L}).
//   K1 czt_rows_kernel  4 pupil rows per workgroup (one per wave), the three components
//                       in turn sharing the row's defocus factors -> T [s][z][c][N][ny]
//   K2 czt_cols_kernel  CB output columns per workgroup: T staged in LDS with coalesced
//                       row loads, one column FFT pair per wave at a time, E written by
//                       rows from LDS and I = sum_c |E_c|^2 accumulated in LDS.
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "rw_common.h"
#include "rw_fourier.h"
#include "rw_plan.h"

namespace rw {

constexpr int kCztMaxL = 2048;   // longest transform (N + max(nx, ny) - 1 <= 2048)
constexpr int kCztMaxN = 1024;   // pupil cells per axis

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }   // a * (-i)

template <int R>
__device__ __forceinline__ void dft_small(float2* v) {
  if (R == 2) {
    const float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if (R == 4) {
    const float2 b0 = cadd(v[0], v[2]), b2 = csub(v[0], v[2]);
    const float2 b1 = cadd(v[1], v[3]), b3 = mul_mi(csub(v[1], v[3]));
    v[0] = cadd(b0, b1);
    v[1] = cadd(b2, b3);
    v[2] = csub(b0, b1);
    v[3] = csub(b2, b3);
  } else {   // R == 8: two radix-2 halves with W8 twiddles, then two 4-point DFTs
    const float r = 0.70710678118654752f;
    float2 t0 = cadd(v[0], v[4]), t4 = csub(v[0], v[4]);
    float2 t1 = cadd(v[1], v[5]), t5 = csub(v[1], v[5]);
    float2 t2 = cadd(v[2], v[6]), t6 = csub(v[2], v[6]);
    float2 t3 = cadd(v[3], v[7]), t7 = csub(v[3], v[7]);
    t5 = make_float2(r * (t5.x + t5.y), r * (t5.y - t5.x));    // * e^{-i pi/4}
    t6 = mul_mi(t6);                                           // * e^{-i pi/2}
    t7 = make_float2(r * (t7.y - t7.x), -r * (t7.x + t7.y));   // * e^{-3 i pi/4}
    float2 e[4] = {t0, t1, t2, t3}, o[4] = {t4, t5, t6, t7};
    dft_small<4>(e);
    dft_small<4>(o);
    v[0] = e[0];
    v[1] = o[0];
    v[2] = e[1];
    v[3] = o[1];
    v[4] = e[2];
    v[5] = o[2];
    v[6] = e[3];
    v[7] = o[3];
  }
}

// Each wave owns its FFT buffer: a wave's LDS operations are carried out in program
// order, so between the read and write phases of a pass only the compiler has to be kept
// from reordering (a wavefront-scope fence), not the other waves.
__device__ __forceinline__ void wave_lds_order() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_wave_barrier();
}

// FFT buffers hold entry i at i + i / 8 (one pad slot per 8 entries), so that the
// stride-8 writes of the first passes fall in distinct banks.
__device__ __forceinline__ int pidx(int i) { return i + (i >> 3); }
template <int L>
constexpr int padded(void) { return L + L / 8; }

// e^{-2 pi i q / L} for integer q, from the hardware sine / cosine of the exact fraction
// q / L in revolutions (max error ~1.3e-7), and its powers 2..R-1 by complex products.
template <int R, int L>
__device__ __forceinline__ void twiddles_pow(int q, float2* w) {
  const float u = (float)(q & (L - 1)) * (1.f / L);
  w[1] = make_float2(__builtin_amdgcn_cosf(u), -__builtin_amdgcn_sinf(u));
#pragma unroll
  for (int r = 2; r < R; ++r) w[r] = cmul(w[r - 1], w[1]);
}

// One Stockham pass of radix R over the wave's buffer.
template <int R, int L>
__device__ __forceinline__ void fft_pass(float2* buf, int Ns, int lane) {
  constexpr int nb = L / R;
  constexpr int MAXB = (nb + 63) / 64;   // butterflies per lane
  float2 v[MAXB][R];
#pragma unroll
  for (int t = 0; t < MAXB; ++t) {
    const int j = lane + 64 * t;
    if (j < nb)
#pragma unroll
      for (int r = 0; r < R; ++r) v[t][r] = buf[pidx(j + r * nb)];
  }
  wave_lds_order();
#pragma unroll
  for (int t = 0; t < MAXB; ++t) {
    const int j = lane + 64 * t;
    if (j < nb) {
      const int k = j % Ns, step = L / (Ns * R);
      if (Ns > 1) {
        float2 w[R];
        twiddles_pow<R, L>(k * step, w);
#pragma unroll
        for (int r = 1; r < R; ++r) v[t][r] = cmul(v[t][r], w[r]);
      }
      dft_small<R>(v[t]);
      const int d = (j / Ns) * Ns * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[pidx(d + r * Ns)] = v[t][r];
    }
  }
  wave_lds_order();
}

constexpr int log2i(int v) { return v <= 1 ? 0 : 1 + log2i(v / 2); }

// Forward FFT (e^{-2 pi i f m / L}) of the wave's buffer; L = 8^p8 * rem, rem in {1, 2, 4}.
template <int L>
__device__ __forceinline__ void fft(float2* buf, int lane) {
  constexpr int p8 = log2i(L) / 3, rem = 1 << (log2i(L) % 3);
  int Ns = 1;
#pragma unroll
  for (int p = 0; p < p8; ++p) {
    fft_pass<8, L>(buf, Ns, lane);
    Ns *= 8;
  }
  if (rem == 4) fft_pass<4, L>(buf, Ns, lane);
  if (rem == 2) fft_pass<2, L>(buf, Ns, lane);
}

// The convolution of one row or column for L = 512 . 2^e (e = 0, 1, 2: radix-8 passes
// at Ns = 1, 8, 64, then for 1024 and 2048 one radix-2 or radix-4 pass at Ns = 512) with
// the values in registers between the two transforms.  Lane j holds x[j + 64 u],
// u = 0 .. L/64 - 1: the first pass's butterfly j + 64 t reads exactly these
// (u = t + r L/512), and the last pass's butterfly j + 64 t writes them (d = j + 64 t,
// outputs d + r Ns, so u = t + r Ns/64).  The first pass therefore starts from registers,
// the last leaves its outputs in them, and the spectrum product and the conjugation of
// the inverse transform happen in registers: 2 LDS round trips fewer per transform, and
// no fill or read-back of the buffer.
template <int L>
constexpr int czt_reg_last_radix() { return L == 512 ? 8 : (L == 1024 ? 2 : 4); }
template <int L>
constexpr bool czt_reg_ok() { return L == 512 || L == 1024 || L == 2048; }

template <int L>
__device__ __forceinline__ void czt_first_reg(float2* buf, float2 (&v)[L / 64], int lane) {
  constexpr int T1 = L / 8 / 64;
#pragma unroll
  for (int t = 0; t < T1; ++t) {
    float2 b[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) b[r] = v[t + r * T1];
    dft_small<8>(b);
    const int j = lane + 64 * t;
#pragma unroll
    for (int r = 0; r < 8; ++r) buf[pidx(8 * j + r)] = b[r];
  }
  wave_lds_order();
}
template <int L>
__device__ __forceinline__ void czt_last_reg(float2* buf, float2 (&v)[L / 64], int lane) {
  constexpr int R = czt_reg_last_radix<L>(), NS = L / R, T2 = NS / 64;
#pragma unroll
  for (int t = 0; t < T2; ++t)
#pragma unroll
    for (int r = 0; r < R; ++r) v[t + r * T2] = buf[pidx(lane + 64 * t + r * NS)];
  wave_lds_order();
#pragma unroll
  for (int t = 0; t < T2; ++t) {
    float2 b[R], w[R];
#pragma unroll
    for (int r = 0; r < R; ++r) b[r] = v[t + r * T2];
    twiddles_pow<R, L>(lane + 64 * t, w);   // k = j, step 1
#pragma unroll
    for (int r = 1; r < R; ++r) b[r] = cmul(b[r], w[r]);
    dft_small<R>(b);
#pragma unroll
    for (int r = 0; r < R; ++r) v[t + r * T2] = b[r];
  }
}
template <int L>
__device__ __forceinline__ void czt_fft_reg(float2* buf, float2 (&v)[L / 64], int lane) {
  czt_first_reg<L>(buf, v, lane);
  fft_pass<8, L>(buf, 8, lane);
  if (L > 512) fft_pass<8, L>(buf, 64, lane);
  czt_last_reg<L>(buf, v, lane);
}
// v: in x (already multiplied by the pre-chirp), out conj(FFT(conj(FFT(x) chat)))
template <int L>
__device__ __forceinline__ void czt_pair_reg(float2* buf, float2 (&v)[L / 64], const float2* __restrict__ chat,
                                             int lane) {
  // at L = 512 the lane's spectrum factors are requested before the first transform (16
  // registers); the longer transforms have no registers to spare and read them after it
  constexpr int CH = L == 512 ? L / 64 : 1;
  float2 ch[CH];
  if constexpr (L == 512)
#pragma unroll
    for (int u = 0; u < CH; ++u) ch[u] = chat[lane + 64 * u];
  czt_fft_reg<L>(buf, v, lane);
#pragma unroll
  for (int u = 0; u < L / 64; ++u) {
    const float2 t = cmul(v[u], L == 512 ? ch[u % CH] : chat[lane + 64 * u]);
    v[u] = make_float2(t.x, -t.y);
  }
  czt_fft_reg<L>(buf, v, lane);
}

struct CztRowArgs {
  const float2* P;       // [nstk][nc][np][np] base pupils
  const double* ksz;     // [np][np]
  const double* z;       // plan planes
  const float2* pre;     // [N]
  const float2* post;    // [ny]
  const float2* chat;    // [L] FFT of the chirp, divided by L
  float2* T;             // [nstk][nzs][nc][N][ny]
  double zoff[kPupilStacks];
  int n, np, ny, nstk, z0, nzs, nc;   // nc: channels (3 vectorial, 1 scalar)
};

template <int L>
__global__ void __launch_bounds__(256) czt_rows_kernel(CztRowArgs a) {
  extern __shared__ float2 cbuf[];
  const int rblocks = (a.n + 3) / 4;
  int id = blockIdx.x;
  const int rb = id % rblocks; id /= rblocks;
  const int zi = id % a.nzs;
  const int s = id / a.nzs;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = 4 * rb + wave;
  const bool live = j < a.n;   // a wave past the last row still takes part in the barriers
  float2* buf = cbuf + wave * padded<L>();
  const size_t npp = (size_t)a.np * a.np;
  const double zrev = (a.z[a.z0 + zi] + a.zoff[s]) * (1.0 / kTwoPi);
  // defocus factors of this row, shared by the channels (N < L)
  constexpr int MAXT = L / 64;
  float2 dz[MAXT];
#pragma unroll
  for (int t = 0; t < MAXT; ++t) {
    const int l = lane + 64 * t;
    dz[t] = make_float2(0.f, 0.f);
    if (live && l < a.n) {
      float sn, cs;
      sincos_rev(a.ksz[(size_t)j * a.np + l] * zrev, &sn, &cs);
      dz[t] = cmul(make_float2(cs, sn), a.pre[l]);
    }
  }
  if constexpr (czt_reg_ok<L>()) {
    for (int c = 0; c < a.nc; ++c) {
      const float2* Pr = a.P + ((size_t)s * a.nc + c) * npp + (size_t)(live ? j : 0) * a.np;
      float2 v[MAXT];
#pragma unroll
      for (int u = 0; u < MAXT; ++u) {
        const int l = lane + 64 * u;
        v[u] = (live && l < a.n) ? cmul(Pr[l], dz[u]) : make_float2(0.f, 0.f);
      }
      czt_pair_reg<L>(buf, v, a.chat, lane);
      if (live) {
        float2* Tr = a.T + (((size_t)s * a.nzs + zi) * a.nc + c) * (size_t)a.n * a.ny + (size_t)j * a.ny;
#pragma unroll
        for (int u = 0; u < MAXT; ++u) {
          const int n = lane + 64 * u;
          if (n < a.ny) Tr[n] = cmul(make_float2(v[u].x, -v[u].y), a.post[n]);
        }
      }
    }
    return;
  }
  for (int c = 0; c < a.nc; ++c) {
    const float2* Pr = a.P + ((size_t)s * a.nc + c) * npp + (size_t)(live ? j : 0) * a.np;
#pragma unroll
    for (int t = 0; t < MAXT; ++t) {
      const int l = lane + 64 * t;
      if (l < a.n) buf[pidx(l)] = live ? cmul(Pr[l], dz[t]) : make_float2(0.f, 0.f);
    }
    for (int l = a.n + lane; l < L; l += 64) buf[pidx(l)] = make_float2(0.f, 0.f);
    wave_lds_order();
    fft<L>(buf, lane);
    for (int f = lane; f < L; f += 64) {
      const float2 v = cmul(buf[pidx(f)], a.chat[f]);
      buf[pidx(f)] = make_float2(v.x, -v.y);   // conj, for the inverse transform
    }
    wave_lds_order();
    fft<L>(buf, lane);
    if (live) {
      float2* Tr = a.T + (((size_t)s * a.nzs + zi) * a.nc + c) * (size_t)a.n * a.ny + (size_t)j * a.ny;
      for (int n = lane; n < a.ny; n += 64) {
        const float2 b = buf[pidx(n)];
        Tr[n] = cmul(make_float2(b.x, -b.y), a.post[n]);
      }
    }
    wave_lds_order();
  }
}

struct CztColArgs {
  const float2* T;       // [nstk][nzs][nc][N][ny]
  const float2* pre;     // [N]
  const float2* post;    // [nx], prefactor C included
  const float2* chat;    // [L]
  float2* E;             // [stacks][nz][nc][nx][ny] or null
  float* I;              // [stacks][nz][nx][ny] or null
  int n, nx, ny, nz, cb, nstk, s_base, z0, nzs, nc;
};

template <int L>
__global__ void __launch_bounds__(256) czt_cols_kernel(CztColArgs a) {
  extern __shared__ float2 cbuf[];
  const int CB = a.cb;
  const int cblocks = (a.ny + CB - 1) / CB;
  int id = blockIdx.x;
  const int cbk = id % cblocks; id /= cblocks;
  const int zi = id % a.nzs;
  const int s = id / a.nzs;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n0 = cbk * CB;
  float2* stage = cbuf;                    // [CB][N]: the block's T columns
  float2* outs = stage + CB * a.n;         // [CB][nx]: transformed columns
  float2* buf = outs + CB * a.nx + wave * padded<L>();
  float* isum = reinterpret_cast<float*>(outs + CB * a.nx + 4 * padded<L>());   // [nx * CB] sum_c |E_c|^2
  const size_t gstk = (size_t)(a.s_base + s), gz = (size_t)(a.z0 + zi);
  const size_t plane = (size_t)a.nx * a.ny;
  for (int idx = tid; idx < a.nx * CB; idx += 256) isum[idx] = 0.f;
  for (int c = 0; c < a.nc; ++c) {
    const float2* Tc = a.T + (((size_t)s * a.nzs + zi) * a.nc + c) * (size_t)a.n * a.ny;
    for (int idx = tid; idx < a.n * CB; idx += 256) {
      const int j = idx / CB, cc = idx % CB;
      stage[cc * a.n + j] = (n0 + cc < a.ny) ? Tc[(size_t)j * a.ny + n0 + cc] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    if constexpr (czt_reg_ok<L>()) {
      constexpr int U = L / 64;
      for (int q = 0; q < CB / 4; ++q) {
        const int cc = 4 * q + wave;
        float2 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int j = lane + 64 * u;
          v[u] = j < a.n ? cmul(stage[cc * a.n + j], a.pre[j]) : make_float2(0.f, 0.f);
        }
        czt_pair_reg<L>(buf, v, a.chat, lane);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int m = lane + 64 * u;
          if (m < a.nx) outs[cc * a.nx + m] = cmul(make_float2(v[u].x, -v[u].y), a.post[m]);
        }
      }
    } else
    for (int r = 0; r < CB / 4; ++r) {
      const int cc = 4 * r + wave;
      for (int j = lane; j < L; j += 64)
        buf[pidx(j)] = j < a.n ? cmul(stage[cc * a.n + j], a.pre[j]) : make_float2(0.f, 0.f);
      wave_lds_order();
      fft<L>(buf, lane);
      for (int f = lane; f < L; f += 64) {
        const float2 v = cmul(buf[pidx(f)], a.chat[f]);
        buf[pidx(f)] = make_float2(v.x, -v.y);
      }
      wave_lds_order();
      fft<L>(buf, lane);
      for (int m = lane; m < a.nx; m += 64) {
        const float2 b = buf[pidx(m)];
        outs[cc * a.nx + m] = cmul(make_float2(b.x, -b.y), a.post[m]);
      }
      wave_lds_order();
    }
    __syncthreads();   // every wave's columns are in outs
    // rows of E from LDS: CB consecutive columns per row
    float2* Ec = a.E ? a.E + ((gstk * a.nz + gz) * a.nc + c) * plane : nullptr;
    for (int idx = tid; idx < a.nx * CB; idx += 256) {   // each thread keeps its own entries
      const int m = idx / CB, cc = idx % CB;
      const float2 v = outs[cc * a.nx + m];
      isum[idx] += v.x * v.x + v.y * v.y;
      if (Ec && n0 + cc < a.ny) Ec[(size_t)m * a.ny + n0 + cc] = v;
    }
    __syncthreads();
  }
  if (a.I) {
    float* Ip = a.I + (gstk * a.nz + gz) * plane;
    for (int idx = tid; idx < a.nx * CB; idx += 256) {
      const int m = idx / CB, cc = idx % CB;
      if (n0 + cc < a.ny) Ip[(size_t)m * a.ny + n0 + cc] = isum[idx];
    }
  }
}

// --------------------------------------------------------------------------
// Plan tables (FP64 on the host) and dispatch
// --------------------------------------------------------------------------
// LDS of the column kernel: T columns, transformed columns, 4 FFT buffers, |E|^2 sums
static size_t czt_cols_lds(int cb, int N, int nx, int L) {
  return (size_t)(cb * N + cb * nx + 4 * (L + L / 8)) * sizeof(float2) + (size_t)nx * cb * sizeof(float);
}

// The limit belongs to the kernel, not to a plan: the column kernel's LDS depends on the
// plan, so it is allowed the whole LDS (a later plan must not lower it).
template <int L>
static hipError_t czt_attributes() {
  const hipError_t e =
      hipFuncSetAttribute((const void*)czt_cols_kernel<L>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)czt_rows_kernel<L>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             4 * padded<L>() * (int)sizeof(float2));
}

static int pow2_at_least(int v) {
  int L = 64;
  while (L < v) L *= 2;
  return L;
}

// One axis of the transform: inputs l = 0..N-1 at (l - (N-1)/2) * step_s, outputs
// n = 0..M-1 at (n - M/2) * step_x, phase k s x = beta (l - l0)(n - n0).
static void chirp_tables(int N, int M, int L, double beta, std::complex<double> scale, std::vector<float2>& pre,
                         std::vector<float2>& post, std::vector<float2>& chat) {
  const double l0 = 0.5 * (N - 1), n0 = (double)(M / 2);
  auto e = [](double ph) { return std::complex<double>(std::cos(ph), std::sin(ph)); };
  auto f2 = [](std::complex<double> v) { return make_float2((float)v.real(), (float)v.imag()); };
  pre.resize(N);
  post.resize(M);
  chat.resize(L);
  for (int l = 0; l < N; ++l) pre[l] = f2(e(beta * (0.5 * l * (double)l - l * n0)));
  for (int n = 0; n < M; ++n) post[n] = f2(scale * e(beta * (0.5 * n * (double)n - l0 * n + l0 * n0)));
  std::vector<std::complex<double>> cv(L, 0.0);
  for (int m = -(N - 1); m < M; ++m) cv[(m % L + L) % L] = e(-0.5 * beta * m * (double)m);
  for (int f = 0; f < L; ++f) {
    std::complex<double> acc = 0.0;
    for (int m = 0; m < L; ++m) {
      if (cv[m] == 0.0) continue;
      const long long km = (long long)f * m % L;
      acc += cv[m] * e(-kTwoPi * (double)km / L);
    }
    chat[f] = f2(acc / (double)L);
  }
}

int czt_plan_init(rwpsf_plan* p) {
  const int N = p->num.n_pupil, nx = p->grid.nx, ny = p->grid.ny;
  const int Ly = pow2_at_least(N + ny - 1), Lx = pow2_at_least(N + nx - 1);
  if (N > kCztMaxN || Ly > kCztMaxL || Lx > kCztMaxL) return RWPSF_ERR_UNSUPPORTED;
  const double step_s = 2.0 * p->s_max / N, k = p->k;
  const std::complex<double> C(0.0, -p->opt.focal_length * k / kTwoPi);
  std::vector<float2> pre_y, post_y, chat_y, pre_x, post_x, chat_x;
  chirp_tables(N, ny, Ly, k * step_s * p->grid.dy_nm, 1.0, pre_y, post_y, chat_y);
  chirp_tables(N, nx, Lx, k * step_s * p->grid.dx_nm, C, pre_x, post_x, chat_x);
  p->czt_Ly = Ly;
  p->czt_Lx = Lx;
  // columns per workgroup of the column pass: as many as fit 2 workgroups per CU, down to 4
  int cb = 16;
  while (cb > 4 && czt_cols_lds(cb, N, nx, Lx) > 80 * 1024) cb /= 2;
  if (czt_cols_lds(cb, N, nx, Lx) > 160 * 1024) return RWPSF_ERR_UNSUPPORTED;
  p->czt_cb = cb;
  const size_t tables = (size_t)N + ny + Ly + N + nx + Lx;
  int st;
  if ((st = dev_alloc(p, &p->d_czt, tables))) return st;
  float2* d = p->d_czt;
  const std::vector<float2>* parts[6] = {&pre_y, &post_y, &chat_y, &pre_x, &post_x, &chat_x};
  float2** dst[6] = {&p->czt_pre_y, &p->czt_post_y, &p->czt_chat_y, &p->czt_pre_x, &p->czt_post_x, &p->czt_chat_x};
  for (int i = 0; i < 6; ++i) {
    *dst[i] = d;
    if ((st = hip_check(hipMemcpy(d, parts[i]->data(), parts[i]->size() * sizeof(float2), hipMemcpyHostToDevice))))
      return st;
    d += parts[i]->size();
  }
  // plane workspace [stack-planes][3][N][ny], capped at 512 MiB
  const size_t plane_bytes = 3 * (size_t)N * ny * sizeof(float2);
  const size_t want = (size_t)kPupilStacks * p->grid.nz;
  p->czt_planes = std::max<size_t>(1, std::min(want, (size_t)(512u << 20) / plane_bytes));
  if ((st = dev_alloc(p, &p->d_czt_T, p->czt_planes * 3 * (size_t)N * ny))) return st;
  for (int L : {Ly, Lx}) {
    hipError_t e;
    switch (L) {
      case 64: e = czt_attributes<64>(); break;
      case 128: e = czt_attributes<128>(); break;
      case 256: e = czt_attributes<256>(); break;
      case 512: e = czt_attributes<512>(); break;
      case 1024: e = czt_attributes<1024>(); break;
      default: e = czt_attributes<2048>(); break;
    }
    if ((st = hip_check(e))) return st;
  }
  return hip_check(hipGetLastError());
}

template <int L>
static void launch_rows(const CztRowArgs& a, int blocks, hipStream_t st) {
  hipLaunchKernelGGL(czt_rows_kernel<L>, dim3(blocks), dim3(256), 4 * padded<L>() * sizeof(float2), st, a);
}
template <int L>
static void launch_cols(const CztColArgs& a, int blocks, size_t lds, hipStream_t st) {
  hipLaunchKernelGGL(czt_cols_kernel<L>, dim3(blocks), dim3(256), lds, st, a);
}
static int czt_slab(rwpsf_plan* p, int s_local, int ns, const double* zoff, int s_global, int z0, int nzs, float2* E,
                    float* I, hipStream_t st) {
  const int N = p->num.n_pupil, nx = p->grid.nx, ny = p->grid.ny;
  CztRowArgs ra{};
  ra.P = p->d_P + (size_t)s_local * p->nc * p->np * p->np;
  ra.ksz = p->d_ksz;
  ra.z = p->d_z;
  ra.pre = p->czt_pre_y;
  ra.post = p->czt_post_y;
  ra.chat = p->czt_chat_y;
  ra.T = p->d_czt_T;
  for (int i = 0; i < ns; ++i) ra.zoff[i] = zoff[i];
  ra.n = N;
  ra.np = p->np;
  ra.ny = ny;
  ra.nstk = ns;
  ra.z0 = z0;
  ra.nzs = nzs;
  ra.nc = p->nc;
  int tr = p->time_begin(RWPSF_KERNEL_CZT_ROWS, st);
  const int rblocks = ns * nzs * ((N + 3) / 4);
#define RW_ROWS(LL) launch_rows<LL>(ra, rblocks, st)
  switch (p->czt_Ly) {
    case 64: RW_ROWS(64); break;
    case 128: RW_ROWS(128); break;
    case 256: RW_ROWS(256); break;
    case 512: RW_ROWS(512); break;
    case 1024: RW_ROWS(1024); break;
    default: RW_ROWS(2048); break;
  }
#undef RW_ROWS
  int rc = hip_check(hipGetLastError());
  if (rc) return rc;
  p->time_end(tr, st);
  CztColArgs ca{};
  ca.T = p->d_czt_T;
  ca.pre = p->czt_pre_x;
  ca.post = p->czt_post_x;
  ca.chat = p->czt_chat_x;
  ca.E = E;
  ca.I = I;
  ca.n = N;
  ca.nx = nx;
  ca.ny = ny;
  ca.nz = p->grid.nz;
  ca.cb = p->czt_cb;
  ca.nc = p->nc;
  ca.nstk = ns;
  ca.s_base = s_global;
  ca.z0 = z0;
  ca.nzs = nzs;
  const size_t lds = czt_cols_lds(ca.cb, N, nx, p->czt_Lx);
  const int cblocks = ns * nzs * ((ny + ca.cb - 1) / ca.cb);
  tr = p->time_begin(RWPSF_KERNEL_CZT_COLS, st);
#define RW_COLS(LL) launch_cols<LL>(ca, cblocks, lds, st)
  switch (p->czt_Lx) {
    case 64: RW_COLS(64); break;
    case 128: RW_COLS(128); break;
    case 256: RW_COLS(256); break;
    case 512: RW_COLS(512); break;
    case 1024: RW_COLS(1024); break;
    default: RW_COLS(2048); break;
  }
#undef RW_COLS
  if ((rc = hip_check(hipGetLastError()))) return rc;
  p->time_end(tr, st);
  return RWPSF_OK;
}

int czt_compute(rwpsf_plan* p, int n, const rwpsf_stack* s, float2* E, float* I, hipStream_t st) {
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != p->device) return RWPSF_ERR_INVALID_ARG;
  const int nz = p->grid.nz;
  for (int b0 = 0; b0 < n; b0 += kPupilStacks) {
    const int nb = std::min(kPupilStacks, n - b0);
    int rc = fourier_build_pupils(p, s + b0, nb, st);
    if (rc) return rc;
    double zoff[kPupilStacks];
    for (int i = 0; i < nb; ++i) zoff[i] = s[b0 + i].z_offset_nm;
    const size_t cap = p->czt_planes;
    if ((size_t)nz <= cap) {
      const int stk_per = (int)std::min<size_t>(nb, cap / nz);
      for (int s0 = 0; s0 < nb; s0 += stk_per) {
        const int ns = std::min(stk_per, nb - s0);
        if ((rc = czt_slab(p, s0, ns, zoff + s0, b0 + s0, 0, nz, E, I, st))) return rc;
      }
    } else {
      for (int i = 0; i < nb; ++i)
        for (int z0 = 0; z0 < nz; z0 += (int)cap) {
          const int nzs = (int)std::min<size_t>(cap, nz - z0);
          if ((rc = czt_slab(p, i, 1, zoff + i, b0 + i, z0, nzs, E, I, st))) return rc;
        }
    }
  }
  return RWPSF_OK;
}

}  // namespace rw
