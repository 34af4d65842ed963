/*
 * rwpsf.h -- C ABI of the MI355X (gfx950) vectorial Richards-Wolf PSF engine.
 *
 * The library evaluates the focal field E = (Ex, Ey, Ez) and the intensity
 * |E|^2 of a high-NA objective over a z-stack (Liu et al., arXiv 2502.03170):
 *
 *   E(rho) = -(i f k / 2 pi) Iint_Omega a(s) exp(i W(s)) e_inf(s) exp(i k s.rho) dOmega
 *
 * (Sec. 3.1 eq. "initial vectorial" with the correction factors of Sec. 3.4,
 * eq. "vectorial general with correction"), in either of the two
 * parameterisations the paper proves equivalent:
 *
 *   RWPSF_FORM_FOURIER -- Cartesian form, Sec. 3.3 eq. "cartesian vectorial":
 *       the pupil on a cell-centred N x N grid, one 2-D discrete transform
 *       per z-plane (a separable matrix DFT on the matrix cores).
 *   RWPSF_FORM_BESSEL  -- spherical form, Sec. 3.3 eq. "polar vectorial final"
 *       and eq. "I0": three 1-D theta integrals of J0/J1/J2 kernels by
 *       Gauss-Legendre quadrature, sampled on a radial grid and interpolated
 *       onto the pixels.  Needs an axisymmetric pupil (Sec. 3.4.2, Sec. 4.1).
 *
 * Conventions (all calls):
 *   - lengths in nanometres, Zernike coefficients in waves (Noll index 1..K,
 *     orthonormal on the unit pupil disk), phase maps in radians;
 *   - k = 2 pi n_i / lambda, s_max = NA / n_i (Sec. 3.1);
 *   - pixel (i, j) sits at x = (i - nx/2) dx, y = (j - ny/2) dy (integer
 *     division), the emitter at (x0, y0), the defocus of plane p is
 *     z[p] + z_offset (observation plane minus emitter plane);
 *   - outputs follow the paper's (z, channel, x, y) order (Sec. 4.1), y
 *     fastest: E as interleaved complex64 [stack][z][C][nx][ny] with C = 3
 *     channels for the vectorial model and C = 1 for the scalar model, I as
 *     float [stack][z][nx][ny] (the sum of |E_c|^2 over the channels);
 *   - status codes: 0 = RWPSF_OK, negative = error (rwpsf_status_string).
 *     Argument errors are reported before anything is enqueued; kernel
 *     faults surface at the caller's next synchronisation.  No call blocks
 *     the host on the GPU unless stated.
 *   - `stream` arguments are hipStream_t values passed as void* (NULL = the
 *     default stream).  A plan may be used on one stream at a time.
 *   - Device pointers are owned by the caller; a plan owns its tables and
 *     workspace on the device that was current when it was created.
 */
#ifndef RWPSF_H
#define RWPSF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RWPSF_ABI_VERSION 3

enum rwpsf_status_code {
  RWPSF_OK = 0,
  RWPSF_ERR_INVALID_ARG = -1,      /* sizes <= 0, NA >= n_i, non-finite values, NULL where required */
  RWPSF_ERR_NOT_AXISYMMETRIC = -2, /* Bessel form given m != 0 Zernike terms or a phase map */
  RWPSF_ERR_UNSUPPORTED = -3,      /* option not implemented for this form */
  RWPSF_ERR_OOM = -4,              /* device or host allocation failed */
  RWPSF_ERR_HIP = -5,              /* a HIP runtime call failed; rwpsf_last_hip_error() has the code */
  RWPSF_ERR_NO_DEVICE = -6,        /* no usable gfx950 device */
  RWPSF_ERR_SCRATCH_LIMIT = -7     /* rwpsf_compute_noalloc: one stack needs more than its fixed scratch */
};

/* RWPSF_FORM_CHIRPZ evaluates the same discrete Cartesian sum as RWPSF_FORM_FOURIER
   with the chirp-z (Bluestein) transform of Sec. 3.3: per z-plane and component, one
   FFT convolution along y for every pupil row and one along x for every output column
   (FFT lengths: powers of two >= N + ny - 1 and N + nx - 1, at least 64 and at most
   2048; N <= 1024; rwpsf_plan_create returns RWPSF_ERR_UNSUPPORTED when four output
   columns of the x pass, 4 (N + nx) complex values plus four transform buffers and the
   intensity sums, exceed the 160 KB of LDS of one workgroup).
   It needs fewer flops than the matrix DFT for large pupils; the result agrees with
   RWPSF_FORM_FOURIER to FP32 rounding.  The adjoint is not available for it. */
enum rwpsf_form { RWPSF_FORM_BESSEL = 0, RWPSF_FORM_FOURIER = 1, RWPSF_FORM_CHIRPZ = 2 };

/* Propagation model (Sec. 3.2 and 3.3): the vectorial model rotates the incident
   polarisation onto the Gaussian sphere (eq. "field Gaussian sphere") and gives three
   channels; the scalar model takes the far field equal to a unit incident amplitude
   (eq. "cartesian scalar", eq. "polar scalar final") and gives one channel.  The
   polarisation fields and the Fresnel factors do not enter the scalar model. */
enum rwpsf_model { RWPSF_MODEL_VECTORIAL = 0, RWPSF_MODEL_SCALAR = 1 };

/* Theta quadrature of the Bessel form.  GAUSS: n_theta Gauss-Legendre nodes on
   [0, theta_max], split at the sample's critical angle when Gibson-Lanni puts one
   inside the aperture.  SIMPSON: composite Simpson's rule on n_theta equally spaced
   nodes including both ends (n_theta odd, >= 3), the rule of Sec. 4.1.  RIEMANN: left
   Riemann sum, nodes i h (i < n_theta), h = theta_max / n_theta, the first-order rule
   of Sec. 5.2.2.  SIMPSON and RIEMANN do not split the range. */
enum rwpsf_theta_rule { RWPSF_THETA_GAUSS = 0, RWPSF_THETA_SIMPSON = 1, RWPSF_THETA_RIEMANN = 2 };

/* Physical parameters (Sec. 3.1, 3.3, 3.4). */
typedef struct rwpsf_optics {
  double na;             /* numerical aperture, 0 < na < n_i */
  double wavelength_nm;  /* vacuum wavelength */
  double n_i;            /* immersion index (the propagation medium of the integral) */
  double focal_length;   /* f of eq. "initial vectorial"; scales E only (1 = unit) */
  double ex_re, ex_im;   /* incident polarisation e_inc = (ex, ey, 0), eq. "field Gaussian sphere" */
  double ey_re, ey_im;
  int apodization;       /* 1: a(s) *= sqrt(cos theta) (Sec. 3.4.3) */
  double s_env;          /* > 0: a(s) *= exp(-sin^2 theta / s_env^2) (Sec. 3.4.4); 0 = off */
  int gibson_lanni;      /* 1: add the stratified-layer OPD of Sec. 3.4.1 */
  double n_s, n_g, n_g_design, n_i_design;        /* sample, glass (actual, design), immersion design */
  double t_g_nm, t_g_design_nm, t_i_design_nm;    /* thicknesses; t_i from eq. "gibson lanni t_i" */
  int fresnel;           /* 1: the far field carries the products q_s, q_p of the Fresnel
                            transmission coefficients (Sec. 3.3) of the interfaces sample
                            (n_s) -> coverslip (n_g) -> immersion (n_i); each ray keeps
                            n_m sin t_m = n_i sin t, and beyond a critical angle n_m cos t_m
                            is taken on the positive imaginary branch.  Vectorial model only
                            (RWPSF_ERR_UNSUPPORTED with the scalar model). */
  int extra_sz;          /* 1: a(s) *= s_z = cos theta, the factor that turns the scalar
                            integral into the Fourier transform of the flat disk (the Airy
                            comparison of Sec. 5.2.2); 0 = off */
} rwpsf_optics;

/* Output sampling.  z_nm (host, nz values) is copied at plan creation. */
typedef struct rwpsf_grid {
  int nx, ny;
  double dx_nm, dy_nm;
  int nz;
  const double* z_nm;
} rwpsf_grid;

/* Numerical parameters. */
typedef struct rwpsf_numerics {
  int form;     /* rwpsf_form */
  int n_pupil;  /* Fourier: pupil cells per axis, 2..1024 */
  int n_theta;  /* Bessel: Gauss-Legendre nodes on [0, theta_max], 2..4096 */
  int n_rho;    /* Bessel: radial samples, 8..65536 */
  int model;    /* rwpsf_model (0 = vectorial) */
  int theta_rule; /* Bessel: rwpsf_theta_rule (0 = Gauss-Legendre) */
} rwpsf_numerics;

/* One stack of a compute call: emitter and aberration (Sec. 3.4.1, 3.4.2). */
typedef struct rwpsf_stack {
  double t_s_nm;               /* emitter depth below the coverslip (Gibson-Lanni only) */
  double x0_nm, y0_nm;         /* lateral emitter position */
  double z_offset_nm;          /* added to every plane's z */
  int n_zernike;               /* 0..RWPSF_MAX_ZERNIKE */
  const double* zernike_waves; /* host, n_zernike Noll coefficients (j = 1..n_zernike) */
  const float* phase_map;      /* device [n_pupil][n_pupil] radians (W0 of eq. "Zernike
                                  aberrations"), pupil cell (j, l) <-> (s_x, s_y); NULL = none.
                                  Fourier form only. */
} rwpsf_stack;

#define RWPSF_MAX_ZERNIKE 36
#define RWPSF_MAX_STACKS_PER_CALL 4096

typedef struct rwpsf_plan rwpsf_plan;

/* ABI version of the loaded library (RWPSF_ABI_VERSION it was built with). */
int rwpsf_abi_version(void);

/* Static string for a status code; never NULL. */
const char* rwpsf_status_string(int status);

/* HIP error code behind the most recent RWPSF_ERR_HIP on this thread (0 if none). */
int rwpsf_last_hip_error(void);

/* Host-only validation of a plan description; makes no HIP call. */
int rwpsf_validate(const rwpsf_optics* optics, const rwpsf_grid* grid, const rwpsf_numerics* num);

/* Host-only validation of stacks against a plan description (form-specific rules,
   e.g. the Bessel form rejects m != 0 Zernike terms and phase maps). */
int rwpsf_validate_stacks(const rwpsf_optics* optics, const rwpsf_grid* grid,
                          const rwpsf_numerics* num, int n_stacks, const rwpsf_stack* stacks);

/* Build a plan on the current device: copies the description, evaluates the
   FP64 tables (pupil geometry, Zernike basis, DFT matrices or Gauss-Legendre
   rule and Bessel table) and uploads them.  Synchronous.  *out is NULL on error. */
int rwpsf_plan_create(const rwpsf_optics* optics, const rwpsf_grid* grid,
                      const rwpsf_numerics* num, rwpsf_plan** out);

/* Release a plan and its device memory (synchronises its device). NULL is a no-op. */
void rwpsf_plan_destroy(rwpsf_plan* plan);

/* Device bytes held by the plan (tables + workspace). */
size_t rwpsf_plan_device_bytes(const rwpsf_plan* plan);

/* Plain forward evaluation of n_stacks stacks (1..RWPSF_MAX_STACKS_PER_CALL).
   E_out: device complex64 [n_stacks][nz][C][nx][ny] (C = 3 vectorial, 1 scalar) or NULL;
   I_out: device float [n_stacks][nz][nx][ny] or NULL (not both NULL).
   Enqueued on `stream`; returns after the enqueue. */
int rwpsf_compute(rwpsf_plan* plan, int n_stacks, const rwpsf_stack* stacks,
                  void* E_out, float* I_out, void* stream);

/* Allocation-free variant of rwpsf_compute, for callers that cannot allocate device
   memory during the call (code under HIP graph capture, tight serving loops, harnesses
   that forbid hipMalloc).  Same arguments, outputs and results as rwpsf_compute; Bessel
   form only (RWPSF_ERR_UNSUPPORTED otherwise).  The per-call workspace (the pupil x
   defocus matrix on the theta nodes and the radial integrals I_n) lives in one fixed
   device array of RWPSF_NOALLOC_SCRATCH_BYTES inside the library, which every device the
   library runs on holds until the process ends; the call allocates and frees nothing.
   Stacks go through the array in chunks; a plan whose single stack needs more than the
   array (per stack: 8 T nz V + 8 nz V G n_rho bytes, T theta nodes, V = 2 with the
   Fresnel factors else 1, G = 5 with them, 1 scalar, else 3) gets RWPSF_ERR_SCRATCH_LIMIT
   before anything is enqueued.  All calls on one device share the array and a call
   leaves its contents behind: calls that may overlap on one device (different streams,
   or host threads) race and must be serialised by the caller. */
#define RWPSF_NOALLOC_SCRATCH_BYTES ((size_t)16 << 20)
int rwpsf_compute_noalloc(rwpsf_plan* plan, int n_stacks, const rwpsf_stack* stacks,
                          void* E_out, float* I_out, void* stream);

/* Adjoint of the Fourier form (the paper differentiates through PyTorch autograd,
   Sec. 4.1; this is the hand-written transposed chain).  Given the fields E_in
   (device complex64 [n_stacks][nz][3][nx][ny], as written by rwpsf_compute for the
   same plan and stacks) and dL_dI (device float [n_stacks][nz][nx][ny]) of a real
   loss L(I), writes the gradient with respect to a phase perturbation shared by
   all stacks:
     dL_dc  : device float [n_zernike], dL/dc_q for Noll q = 1..n_zernike (waves)
              (may be NULL when n_zernike = 0);
     dL_dW0 : device float [n_pupil][n_pupil], dL/dW0 on the pupil cells (radians),
              0 outside the disk; may be NULL.
   Outputs are overwritten, never accumulated.  Fourier form, vectorial model, with
   nx, ny multiples of 16 (RWPSF_ERR_UNSUPPORTED otherwise).  Every reduction runs in a fixed order,
   so repeated calls give bitwise-identical results.  The first call allocates the adjoint's
   tables, and a call with more stacks than any before it grows the partial-sum workspace
   (device allocations; earlier buffers stay owned by the plan until it is destroyed). */
int rwpsf_adjoint(rwpsf_plan* plan, int n_stacks, const rwpsf_stack* stacks, const void* E_in,
                  const float* dL_dI, int n_zernike, float* dL_dc, float* dL_dW0, void* stream);

/* Adjoint of the Bessel form (hand-written; the paper differentiates through PyTorch
   autograd, Sec. 4.1).  The phase of stack b is W_b(t) = W_GL(t; t_s,b) + 2 pi sum_j c_j
   Z_j(sin t / s_max) over the axisymmetric Noll terms j = 1, 4, 11, 22, and its planes sit
   at z + z_offset_b (Sec. 3.4.1, 3.4.2).  Given E_in (device complex64
   [n_stacks][nz][C][nx][ny], as written by rwpsf_compute for the same plan and stacks) and
   dL_dI (device float [n_stacks][nz][nx][ny]) of a real loss L(I), writes
     dL_dc  : device float [4], dL/dc_j for j = 1, 4, 11, 22 (waves) for a change of c_j
              applied to every stack (the sum over stacks); may be NULL;
     dL_dts : device float [n_stacks], dL/dt_s per stack (per nm; 0 without the
              Gibson-Lanni layer, where W does not depend on t_s); may be NULL;
     dL_dz  : device float [n_stacks], dL/dz_offset per stack (per nm); may be NULL.
   Outputs are overwritten, never accumulated.  Bessel form, any model and theta rule
   (RWPSF_ERR_UNSUPPORTED for the other forms, or for n_rho > 3200, whose per-sample
   sums no longer fit one workgroup's LDS).  The gradient is that of the computed
   discrete model (theta rule, radial interpolation).  Every reduction runs in a fixed
   order, so repeated calls give bitwise-identical results.  The first call on a plan
   allocates the adjoint's tables and workspace and synchronises the device. */
int rwpsf_adjoint_bessel(rwpsf_plan* plan, int n_stacks, const rwpsf_stack* stacks, const void* E_in,
                         const float* dL_dI, float* dL_dc, float* dL_dts, float* dL_dz, void* stream);

/* ---- batched emitters ----------------------------------------------------------
   Thousands of emitters, each with its own sub-pixel position, axial position,
   Zernike vector, crop size and plane count, evaluated by the Fourier form in one
   persistent launch (optionally replayed from a captured hipGraph).  Optics as in
   rwpsf_optics, vectorial model (the Gibson-Lanni layer, the Fresnel factors and the
   extra s_z factor included; with the layer each emitter carries its own depth t_s).
   Emitter b gets
   crop x crop pixels at pitch pixel_nm, pixel (i, j) at ((i - crop/2) p, (j - crop/2) p)
   relative to the crop centre, and `planes` planes at z_d = (d - (planes-1)/2) *
   plane_pitch_nm, d = 0..planes-1; its defocus is z_d - z_nm.  Outputs are packed in
   input order: emitter b starts at voxel offset o_b = sum_{b'<b} planes_b' crop_b'^2
   (rwpsf_batch_offsets) with layout I[o_b + (d crop + i) crop + j] (float) and
   E[3 o_b + ((d 3 + c) crop + i) crop + j] (complex64). */
#define RWPSF_BATCH_MAX_CROP 64
#define RWPSF_BATCH_MAX_ZERNIKE 21

typedef struct rwpsf_emitter {
  double x0_nm, y0_nm;     /* lateral position relative to the crop centre, |x0|,|y0| <= 4 pixels */
  double z_nm;             /* axial position of the emitter */
  int crop;                /* 1..RWPSF_BATCH_MAX_CROP */
  int planes;              /* 1..4096 */
  double zernike_waves[RWPSF_BATCH_MAX_ZERNIKE];   /* Noll 1..21, waves */
  double t_s_nm;           /* depth below the coverslip, >= 0 (read only with the Gibson-Lanni layer) */
} rwpsf_emitter;

typedef struct rwpsf_batch rwpsf_batch;

/* Tables and workspace for up to max_emitters emitters on the current device.
   n_pupil: 32, 64, 96 or 128.  Synchronous. */
int rwpsf_batch_create(const rwpsf_optics* optics, int n_pupil, double pixel_nm,
                       double plane_pitch_nm, int max_emitters, rwpsf_batch** out);
void rwpsf_batch_destroy(rwpsf_batch* batch);

/* Host-only: packed voxel offsets (n+1 values, offsets[n] = total voxels). */
int rwpsf_batch_offsets(int n, const rwpsf_emitter* emitters, int64_t* offsets);

/* Evaluate n emitters (host array, validated and copied before return).  I_out:
   device float [total voxels] or NULL; E_out: device complex64 [3 total voxels] or
   NULL (not both NULL).  The emitters are staged in a pinned host area and copied to the
   device at the start of the call's work on `stream`; with graphs enabled the kernels
   (queue reset, phase GEMM, fold, persistent plane kernels) are captured once per (n,
   outputs, configuration, launched tile classes, stream) and replayed after the copy;
   graph mode needs a created stream (not NULL).  Before the staging area is rewritten
   the call waits for the previous call's copy (not for its kernels). */
int rwpsf_batch_compute(rwpsf_batch* batch, int n, const rwpsf_emitter* emitters, float* I_out,
                        void* E_out, void* stream);
int rwpsf_batch_set_graph(rwpsf_batch* batch, int enable);

/* Launch configuration.  Crops fall into four buckets by size (1-16, 17-32, 33-48 and
   49-64 pixels); the crops of bucket q are evaluated on tiles of tile_rows[q] rows (16,
   32, 48 or 64, at least 16 (q + 1)); the tile class of r rows stages its pupil GEMM in
   k-stages of k_stage[r / 16 - 1] folded pupil rows (8 or 16); the persistent grid of
   each class has wg_per_cu workgroups per CU (1..4).  The 32- and 64-row classes run
   32 x 32 x 2 matrix-core tiles, the 16- and 48-row classes 16 x 16 x 4 ones.  The
   default puts each bucket on its own class with k-stages of 16 and two workgroups per
   CU. */
typedef struct rwpsf_batch_config {
  int wg_per_cu;
  int tile_rows[4];
  int k_stage[4];
} rwpsf_batch_config;
int rwpsf_batch_set_config(rwpsf_batch* batch, const rwpsf_batch_config* cfg);
int rwpsf_batch_get_config(const rwpsf_batch* batch, rwpsf_batch_config* cfg);

/* Time each candidate configuration on these emitters (outputs written to I_out)
   and keep the fastest.  Synchronises the stream.  best_ms may be NULL.  If the
   environment variable RWPSF_AUTOTUNE_CACHE names a file, a configuration stored there
   for the same key (pupil size, batch-size bucket, crop mix, mean plane count, CU
   count) is used without timing, and new results are added to it; a file that does
   not parse is ignored and rewritten. */
int rwpsf_batch_autotune(rwpsf_batch* batch, int n, const rwpsf_emitter* emitters, float* I_out,
                         void* stream, rwpsf_batch_config* best, double* best_ms);

/* ---- learned surrogate ----------------------------------------------------------
   A network (3.44M parameters) from 21 Noll coefficients (waves) and a defocus z (nm)
   to a 64 x 64 intensity crop, trained on crops this engine generates (the paper
   motivates PSF models as generators of training data for networks, Sec. 6):
     x = (c / 0.05, z / 1000); dense layers 22 -> 1024 -> 1024 -> 1024 (h3), relu;
     convolution branch: h3 read as 16 x 8 x 8, three stride-2 transposed convolutions
       (4 x 4 kernel, padding 1) 16 -> 16 -> 8 -> 1 channels, relu after the first two;
     basis branch: a = h3 Wa + ba (256 coefficients, linear), a Wb + bb (a learned basis
       of 256 crops plus a mean crop);
     output = convolution branch + basis branch.
   Parameters are one flat FP32 array in the order W1 [22][1024], b1, W2 [1024][1024], b2,
   W3 [1024][1024], b3, K1 [16][16][4][4], c1, K2 [16][8][4][4], c2, K3 [8][1][4][4], c3,
   Wa [1024][256], ba, Wb [256][4096], bb (rwpsf_sg_param_count values).  Dense layers
   and the first two transposed convolutions run on the BF16 matrix cores (the
   convolutions as implicit GEMMs per output parity class); the last convolution runs in
   FP32.  With RWPSF_SG_BF16X3 each matrix-core operand is split into two BF16 parts and
   three products are summed (FP32-level accuracy, about 1e-6 relative); with
   RWPSF_SG_BF16 only the leading parts are multiplied (about 1e-2 relative).  All device
   arrays are caller-owned except the parameters, gradients and Adam moments, which the
   handle owns.  Gradient reductions run in a fixed order. */
enum rwpsf_sg_precision { RWPSF_SG_BF16X3 = 0, RWPSF_SG_BF16 = 1 };
typedef struct rwpsf_sg rwpsf_sg;
size_t rwpsf_sg_param_count(void);
/* Workspace for batches up to max_batch; parameters and moments start at zero. */
int rwpsf_sg_create(int max_batch, rwpsf_sg** out);
void rwpsf_sg_destroy(rwpsf_sg* sg);
/* Host arrays of rwpsf_sg_param_count floats; m, v may be NULL (left unchanged / not read). */
int rwpsf_sg_set_state(rwpsf_sg* sg, const float* params, const float* adam_m, const float* adam_v,
                       int64_t step);
int rwpsf_sg_get_state(const rwpsf_sg* sg, float* params, float* adam_m, float* adam_v, float* grads,
                       int64_t* step);
/* out = net(coef, z): coef device float [B][21], z device float [B], out device float [B][64][64]. */
int rwpsf_sg_forward(rwpsf_sg* sg, int B, const float* coef, const float* z, float* out, int precision,
                     void* stream);
/* Gradient of the mean squared error to target (device float [B][64][64]) into the handle's
   gradient buffer (accurate precision); loss: device float [1] or NULL. */
int rwpsf_sg_gradient(rwpsf_sg* sg, int B, const float* coef, const float* z, const float* target,
                      float* loss, void* stream);
/* One Adam step (Kingma & Ba, bias-corrected) on the FP32 parameters with the stored gradient. */
int rwpsf_sg_adam(rwpsf_sg* sg, float lr, float beta1, float beta2, float eps, void* stream);
/* Error model of the surrogate's fallback gate: the predicted log rel-L2 of a crop against
   the plain path is w . phi(c, z), phi = (1, (c_1/0.05)^2 .. (c_21/0.05)^2, (z/1000)^2,
   |z|/1000) (RWPSF_SG_GATE_FEATURES values; c in waves, z in nm).  The weights are fitted
   by the caller on crops judged by the plain path.  rwpsf_sg_error_features writes phi
   (device float [B][24]); rwpsf_sg_error_predict writes w . phi (device float [B]) for
   device weights w [24].  coef device float [B][21], z device float [B]. */
#define RWPSF_SG_GATE_FEATURES 24
int rwpsf_sg_error_features(int B, const float* coef, const float* z, float* phi, void* stream);
int rwpsf_sg_error_predict(int B, const float* coef, const float* z, const float* weights, float* log_err,
                           void* stream);

/* ---- per-kernel timing, for benchmarking -------------------------------------
   When enabled, every kernel the plan launches is bracketed by HIP events on
   the call's stream.  rwpsf_plan_timing waits for the recorded events, folds them
   into per-kernel totals and returns the total milliseconds and launch count of
   one kernel since timing was last enabled. */
enum rwpsf_kernel_id {
  RWPSF_KERNEL_PUPIL_BUILD = 0,       /* Fourier: base pupil with FP64 phases */
  RWPSF_KERNEL_GEMM_PUPIL = 1,        /* Fourier: (pupil x defocus) x Ay^T */
  RWPSF_KERNEL_GEMM_IMAGE = 2,        /* Fourier: Ax x T, fields and |E|^2 */
  RWPSF_KERNEL_BESSEL_PHI = 3,        /* Bessel: pupil x defocus on the theta nodes */
  RWPSF_KERNEL_BESSEL_CONTRACT = 4,   /* Bessel: theta contraction on the matrix cores */
  RWPSF_KERNEL_BESSEL_EPILOGUE = 5,   /* Bessel: radial interpolation, fields and |E|^2 */
  RWPSF_KERNEL_ADJ_H = 6,             /* adjoint: (2 dL/dI E) conj(Ay) */
  RWPSF_KERNEL_ADJ_G = 7,             /* adjoint: Ax'^H H with Im(G conj(P~)) accumulation */
  RWPSF_KERNEL_ADJ_REDUCE = 8,        /* adjoint: fixed-order reductions to dL/dW0, dL/dc */
  RWPSF_KERNEL_CZT_ROWS = 9,          /* chirp-z: pupil rows (defocus, FFT convolution along y) */
  RWPSF_KERNEL_CZT_COLS = 10,         /* chirp-z: output columns (FFT convolution along x), |E|^2 */
  RWPSF_KERNEL_ADJB_RADIAL = 11,      /* Bessel adjoint: pixels -> radial samples (transposed interpolation) */
  RWPSF_KERNEL_ADJB_CONTRACT = 12,    /* Bessel adjoint: transposed theta contraction on the matrix cores */
  RWPSF_KERNEL_ADJB_REDUCE = 13,      /* Bessel adjoint: fixed-order reductions to the parameter gradients */
  RWPSF_KERNEL_BESSEL_FUSED = 14,     /* Bessel, calls of few planes: phase, contraction and epilogue in one launch */
  RWPSF_KERNEL_COUNT = 16
};
int rwpsf_plan_set_timing(rwpsf_plan* plan, int enable);   /* also resets the totals */
int rwpsf_plan_timing(rwpsf_plan* plan, int kernel, double* total_ms, int64_t* launches);

/* ---- host-only reference routines used to build the plan tables ----------
   Exported so that the tables can be checked on a machine without a GPU. */

/* n-point Gauss-Legendre rule on [a, b] (Newton iteration on the three-term
   Legendre recurrence).  x, w: host arrays of n doubles. */
int rwpsf_gauss_legendre(int n, double a, double b, double* x, double* w);

/* Bessel function of the first kind J_order(x), order 0..8, x >= 0, evaluated as the
   periodic trapezoid rule on Bessel's integral (1/pi) int_0^pi cos(n t - x sin t) dt.
   x, out: host arrays of `count` doubles. */
int rwpsf_bessel_j(int order, int count, const double* x, double* out);

/* Orthonormal Noll Zernike polynomial Z_j(r, phi), j >= 1. Host arrays of `count`. */
int rwpsf_zernike(int j, int count, const double* r, const double* phi, double* out);

#ifdef __cplusplus
}
#endif

#endif /* RWPSF_H */
