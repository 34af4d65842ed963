"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module holds configuration constants and random draws only -- none of the
method's arithmetic.  Every generator takes a seed and returns plain NumPy
arrays / Python numbers; both sides build their own structures from them.

Workloads (sizes follow the paper's optics at NA 1.4 oil immersion; the paper
publishes no dataset, so every input is synthetic):

* ``bessel_plain``   -- unaberrated vectorial focus, NA 1.4, n_i 1.518, 532 nm,
                        circular polarisation, 65 x 65 px at 20 nm, 33 planes over
                        +-1 um, 200 theta nodes, 256 radial samples.
* ``fourier_plain``  -- NA 1.4, 600 nm, 256 x 256 pupil, Gibson-Lanni
                        (n_s 1.33, emitter depth U[0, 5] um) + Noll 4..21
                        coefficients N(0, 0.05) waves, 128 x 128 px at 20 nm, 64
                        planes; planes are z' - t_s with z' over +-1 um.
* ``batched``        -- emitters with sub-pixel x0, y0 ~ U(+-0.5 px), z_e ~
                        U(+-800 nm), Noll 4..21 ~ N(0, 0.04) waves, crops S ~
                        U{24..64}, planes D ~ U{1..41}, 100 nm pixels, 50 nm plane
                        pitch, 128 x 128 pupil.
* ``adjoint``        -- 64 stacks of 64 x 64 x 21 at 100 nm, 256 x 256 pupil.
* ``surrogate``      -- (Noll 4..21 ~ N(0, 0.05) waves, z ~ U(+-1 um)) -> 64 x 64
                        crops at 100 nm from a 128 x 128 pupil.
"""
from __future__ import annotations

import math

import numpy as np

CIRCULAR = (1.0 / math.sqrt(2.0), 1.0j / math.sqrt(2.0))
X_LINEAR = (1.0 + 0.0j, 0.0j)

BESSEL_OPTICS = dict(na=1.4, wavelength=532.0, n_i=1.518)
FOURIER_OPTICS = dict(na=1.4, wavelength=600.0, n_i=1.518)
# design/actual glass and immersion values (coverslip 170 um, n_g = 1.5)
GIBSON_LANNI = dict(n_s=1.33, n_g=1.5, n_g_design=1.5, n_i_design=1.518, t_g=170e3,
                    t_g_design=170e3, t_i_design=150e3)


def bessel_plain(n_stacks: int = 1, seed: int = 101):
    """Bessel-form workload; extra stacks get a focal offset U(+-100 nm)."""
    rng = np.random.default_rng(seed)
    offsets = np.zeros(n_stacks)
    if n_stacks > 1:
        offsets = rng.uniform(-100.0, 100.0, n_stacks)
    z = np.linspace(-1000.0, 1000.0, 33)
    return dict(optics=dict(BESSEL_OPTICS), e_inc=CIRCULAR, nx=65, ny=65, dx=20.0, dy=20.0,
                z=z, z_offsets=offsets, n_theta=200, n_rho=256)


def fourier_plain(n_stacks: int = 16, seed: int = 202, n_pupil: int = 256, nx: int = 128,
                  nz: int = 64, dx: float = 20.0):
    """Fourier-form workload: per-stack emitter depth and Zernike draw."""
    rng = np.random.default_rng(seed)
    t_s = rng.uniform(0.0, 5000.0, n_stacks)
    coeffs = np.zeros((n_stacks, 21))
    coeffs[:, 3:21] = rng.normal(0.0, 0.05, (n_stacks, 18))
    zp = np.linspace(-1000.0, 1000.0, nz)
    z = zp[None, :] - t_s[:, None]
    return dict(optics=dict(FOURIER_OPTICS), e_inc=CIRCULAR, gl=dict(GIBSON_LANNI), n_pupil=n_pupil,
                nx=nx, ny=nx, dx=dx, dy=dx, t_s=t_s, zernike=coeffs, z=z)


def batched(n_emitters: int = 4096, seed: int = 303, s_min: int = 24, s_max: int = 64,
            d_min: int = 1, d_max: int = 41, n_pupil: int = 128):
    rng = np.random.default_rng(seed)
    px = 100.0
    x0 = rng.uniform(-0.5, 0.5, n_emitters) * px
    y0 = rng.uniform(-0.5, 0.5, n_emitters) * px
    z_e = rng.uniform(-800.0, 800.0, n_emitters)
    coeffs = np.zeros((n_emitters, 21))
    coeffs[:, 3:21] = rng.normal(0.0, 0.04, (n_emitters, 18))
    S = rng.integers(s_min, s_max + 1, n_emitters)
    D = rng.integers(d_min, d_max + 1, n_emitters)
    return dict(optics=dict(FOURIER_OPTICS), e_inc=CIRCULAR, n_pupil=n_pupil, dx=px, dz=50.0,
                x0=x0, y0=y0, z_e=z_e, zernike=coeffs, S=S.astype(np.int32), D=D.astype(np.int32))


def smooth_phase_map(n: int, rms: float, seed: int, n_modes: int = 12):
    """Random smooth map: a few low-frequency cosine modes, scaled to the given RMS."""
    rng = np.random.default_rng(seed)
    u = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(u, u, indexing="ij")
    m = np.zeros((n, n))
    for _ in range(n_modes):
        fx, fy = rng.integers(0, 4, 2)
        ph = rng.uniform(0, 2 * math.pi)
        m += rng.normal() * np.cos(2 * math.pi * (fx * X + fy * Y) + ph)
    m -= m.mean()
    return m * (rms / math.sqrt(np.mean(m * m)))


def adjoint(n_stacks: int = 64, seed_truth: int = 404, seed_noise: int = 405, n_pupil: int = 256,
            nx: int = 64, nz: int = 21):
    rng = np.random.default_rng(seed_truth)
    c_true = np.zeros(21)
    c_true[3:21] = rng.normal(0.0, 0.05, 18)
    c_eval = np.zeros(21)
    c_eval[3:21] = rng.normal(0.0, 0.02, 18)
    w0 = smooth_phase_map(n_pupil, 0.1, seed_truth + 1000)
    rng2 = np.random.default_rng(seed_noise)
    photons = np.exp(rng2.uniform(math.log(1e3), math.log(1e5), n_stacks))
    return dict(optics=dict(FOURIER_OPTICS), e_inc=CIRCULAR, n_pupil=n_pupil, nx=nx, ny=nx,
                dx=100.0, dy=100.0, z=np.linspace(-1000.0, 1000.0, nz), c_true=c_true,
                c_eval=c_eval, w0_eval=w0, photons=photons, noise_seed=seed_noise)


def poisson(rate, seed: int):
    return np.random.default_rng(seed).poisson(np.clip(rate, 0, None)).astype(np.float64)


def surrogate(n: int, seed: int, sigma: float = 0.05, z_half: float = 1000.0):
    rng = np.random.default_rng(seed)
    coeffs = np.zeros((n, 21))
    coeffs[:, 3:21] = rng.normal(0.0, sigma, (n, 18))
    z = rng.uniform(-z_half, z_half, n)
    return dict(optics=dict(FOURIER_OPTICS), e_inc=CIRCULAR, n_pupil=128, nx=64, dx=100.0,
                zernike=coeffs, z=z)
