// Kernel argument blocks and launchers of the Fourier form (internal).
#pragma once

#include "rw_common.h"

namespace rw {

constexpr int kPupilStacks = 8;  // stacks per pupil launch (by-value arguments stay < 4 KB)
constexpr int kGemmStacks = 64;  // stacks per GEMM launch (folded pupils of up to 8 pupil launches): fewer
                                 // kernel prologues and tails, and small outputs need many stacks per
                                 // launch to fill the GPU

struct PupilStack {
  double t_s, x0, y0;
  double coef[RWPSF_MAX_ZERNIKE];
  const float* w0;
};

// Channels: nc = 3 (vectorial model, x, y, z) or 1 (scalar model); every per-channel
// array below holds nc channels.
template <int NS>
struct PupilArgsT {
  int n, np, nstk, max_zernike, gibson_lanni, nc;   // n: pupil cells per axis, np: padded stride
  double s_max, k;
  GLParams gl;
  PupilStack s[NS];
};
using PupilArgs = PupilArgsT<kPupilStacks>;
static_assert(sizeof(PupilArgs) <= 4000, "kernel arguments are passed by value (4 KB limit)");

// Device operands are zero-padded: np = n rounded up to 64, nxp = nx rounded up
// to 128, nyp = ny rounded up to 128, and the folded pupil axis nh = ceil(n/2) to
// nhp = nh rounded up to 32 (so 2 nhp = np).

struct Gemm1Args {
  const float2* Pf;    // [nstk][nc][2 nhp][2 nhp]
  const double* kszf;  // [nhp][nhp] k s_z on the folded cells
  const double* z;     // plan planes
  const float* B1;     // [nyp][2 nhp] cos / sin (k s_y[lf] y_n), k contiguous
  float2* T;           // [nstk][nzs][nc][2 nhp][nyp]
  double zoff[kGemmStacks];
  int n, nhp, nyp, nstk, z0, nzs, nc;   // n: pupil cells per axis
};

struct Gemm2Args {
  const float* A2;     // [nxp][2 nhp] pref cos / sin (k s_x[jf] x_m), k contiguous
  const float2* T;     // [nstk][nzs][nc][2 nhp][nyp]
  float2* E;           // [stacks][nz][nc][nx][ny] or null
  float* I;            // [stacks][nz][nx][ny] or null
  int nhp, nxp, nyp, nx, ny, nz, nstk, s_base, z0, nzs, nc;
};

inline int round_up(int v, int m) { return (v + m - 1) / m * m; }
constexpr int kPadPupil = 64, kPadX = 128, kPadY = 128, kFoldPad = 32, kPadSmall = 64;
// padding of an output axis of n pixels: 64 for n <= 64, else a multiple of 128
inline int pad_axis(int n) { return n <= kPadSmall ? kPadSmall : round_up(n, kPadX); }

hipError_t launch_zernike_table(float* out, int n, int nj, hipStream_t st);
hipError_t launch_pupil_build(const PupilArgs& a, const float2* Q, const float* ztab, float2* P,
                              hipStream_t st);
// Pf [nstk][nc][2 nhp][2 nhp] of the stacks of a (its np field is the stride of Q)
hipError_t launch_pupil_build_folded(const PupilArgs& a, const float2* Q, const float* ztab, float2* Pf, int nhp,
                                     hipStream_t st);
hipError_t launch_gemm_pupil(const Gemm1Args& a, hipStream_t st);
hipError_t launch_gemm_image(const Gemm2Args& a, hipStream_t st);
hipError_t fourier_kernel_attributes();

}  // namespace rw
