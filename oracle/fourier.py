"""Cartesian (Fourier) parameterisation of the Richards-Wolf integral, FP64 oracle.

Test infrastructure only.  Follows eq. "cartesian vectorial" (Sec. 3.3) with the
correction factors of eq. "vectorial general with correction" (Sec. 3.4): the
solid-angle element is ds_x ds_y / s_z, the integral runs over the disk
s_x^2 + s_y^2 <= s_max^2, and the prefactor is -i f k / (2 pi).

The continuum integral is discretised on a cell-centred N x N grid with cell
area ds^2 (the discrete sum that a chirp-z transform or a matrix DFT of the same
pupil reaches), so

    E_c(x, y, z) = -(i f k / 2 pi) * sum_{j,l in disk} P_c[j,l] exp(i k s_z z)
                   * exp(i k (s_x[j] (x - x0) + s_y[l] (y - y0)))

with the base pupil P_c = ds^2 * a * exp(iW) * e_inf,c / s_z.
"""
from __future__ import annotations

import math

import numpy as np

from . import optics as O


def pupil_geometry(n: int, opt: O.Optics):
    sx, sy, mask, ds = O.cartesian_pupil_grid(n, opt.s_max)
    s2 = sx * sx + sy * sy
    sin_t = np.sqrt(s2)
    cos_t = np.sqrt(np.clip(1.0 - s2, 0.0, None))
    phi = np.arctan2(sy, sx)          # 0 at the centre cell of an odd grid
    return dict(sx=sx, sy=sy, sz=cos_t, sin_t=sin_t, cos_t=cos_t, phi=phi,
                r=sin_t / opt.s_max, mask=mask, ds=ds, n=n)


def pupil_phase(geom, opt: O.Optics, zernike=None, phase_map=None, t_s: float = 0.0,
                gl_compensated: bool = False):
    """Total phase W = W_GL + 2 pi sum_j c_j Z_j + W0 (complex if evanescent)."""
    w = np.zeros(geom["sx"].shape, dtype=np.complex128)
    if opt.gl is not None:
        w = w + O.gibson_lanni_opd(geom["sin_t"], opt, t_s, compensated=gl_compensated)
    if zernike is not None:
        for j, c in enumerate(np.asarray(zernike, dtype=np.float64), start=1):
            if c != 0.0:
                w = w + 2.0 * math.pi * c * O.zernike_noll(j, geom["r"], geom["phi"])
    if phase_map is not None:
        w = w + np.asarray(phase_map, dtype=np.float64)
    return w


def base_pupil(geom, opt: O.Optics, phase=None, scalar: bool = False, extra_cos: bool = False):
    """P_c[j, l] = ds^2 * a * exp(iW) * e_inf,c / s_z on the disk, 0 outside.

    ``scalar`` uses e_inf = e_inc as one channel of amplitude 1 (Sec. 3.2; the scalar
    model has no Fresnel factors); the vectorial far field carries the Fresnel
    products q_s, q_p of ``opt.fresnel_media`` (1 when empty);
    ``extra_cos`` multiplies by s_z, which turns the integrand into the
    Fourier transform of the flat disk (the Airy comparison of Sec. 5.2.2).
    """
    mask = geom["mask"]
    cos_t, sin_t = geom["cos_t"], geom["sin_t"]
    a = O.amplitude(cos_t, sin_t, opt)
    if phase is None:
        phase = np.zeros_like(a, dtype=np.complex128)
    common = geom["ds"] ** 2 * a * np.exp(1j * phase) / np.where(mask, cos_t, 1.0)
    if extra_cos:
        common = common * cos_t
    common = np.where(mask, common, 0.0)
    if scalar:
        return common[None].astype(np.complex128)
    sin_p = np.where(sin_t > 0, geom["sy"] / np.where(sin_t > 0, sin_t, 1.0), 0.0)
    cos_p = np.where(sin_t > 0, geom["sx"] / np.where(sin_t > 0, sin_t, 1.0), 1.0)
    ex, ey = opt.e_inc
    qs, qp = O.fresnel_q(sin_t, opt)
    e_far = O.far_field(ex, ey, cos_t, sin_t, cos_p, sin_p, qs, qp)
    return e_far * common[None]


def prefactor(opt: O.Optics) -> complex:
    return -1j * opt.f * opt.k / (2.0 * math.pi)


def field_direct(P, geom, opt: O.Optics, points, x0: float = 0.0, y0: float = 0.0, chunk: int = 64):
    """Brute-force double sum at arbitrary points (K, 3) = (x, y, z) -> (C, K).

    One complex exponential of the full phase k(s_x x + s_y y + s_z z) per
    pupil cell and point; no factorisation.
    """
    pts = np.atleast_2d(np.asarray(points, dtype=np.float64))
    m = geom["mask"]
    sx, sy, sz = geom["sx"][m], geom["sy"][m], geom["sz"][m]
    Pm = P[:, m]
    k = opt.k
    out = np.empty((P.shape[0], pts.shape[0]), dtype=np.complex128)
    for a in range(0, pts.shape[0], chunk):
        p = pts[a:a + chunk]
        ph = k * (np.outer(p[:, 0] - x0, sx) + np.outer(p[:, 1] - y0, sy) + np.outer(p[:, 2], sz))
        out[:, a:a + chunk] = Pm @ np.exp(1j * ph).T
    return prefactor(opt) * out


def field_separable(P, geom, opt: O.Optics, nx: int, ny: int, dx: float, dy: float, z,
                    x0: float = 0.0, y0: float = 0.0):
    """Whole stack through the factorisation exp(ik(s_x x + s_y y)) = exp(ik s_x x) exp(ik s_y y).

    E_c[z] = C * Ax @ (P_c * exp(i k s_z z)) @ Ay^T with Ax[m, j] = exp(i k s_x[j] (x_m - x0)).
    Returns complex128 of shape (Z, C, nx, ny), the paper's (z, channel, x, y) order.
    """
    k = opt.k
    sxv = geom["sx"][:, 0]
    syv = geom["sy"][0, :]
    xs = O.output_axis(nx, dx, x0)
    ys = O.output_axis(ny, dy, y0)
    Ax = np.exp(1j * k * np.outer(xs, sxv))
    Ay = np.exp(1j * k * np.outer(ys, syv))
    z = np.atleast_1d(np.asarray(z, dtype=np.float64))
    out = np.empty((z.size, P.shape[0], nx, ny), dtype=np.complex128)
    sz = np.where(geom["mask"], geom["sz"], 0.0)
    for iz, zz in enumerate(z):
        D = np.exp(1j * k * sz * zz)
        for c in range(P.shape[0]):
            out[iz, c] = Ax @ (P[c] * D) @ Ay.T
    return prefactor(opt) * out


def intensity(E):
    """|E|^2 summed over the channel axis (axis 1 of a (z, c, x, y) stack)."""
    return np.sum(E.real ** 2 + E.imag ** 2, axis=1)
