"""Spherical (Bessel) parameterisation of the Richards-Wolf integral, FP64 oracle.

Test infrastructure only.

* ``field_polar``  -- the polar double integral, eq. "polar vectorial" (Sec. 3.3)
  with the correction factors of eq. "vectorial general with correction":
  d Omega = sin t dt dp, Gauss-Legendre in theta, trapezoid in phi (spectrally
  exact for the periodic phi integrand), evaluated point by point with the full
  plane-wave phase k s . rho -- no Bessel identity is used.
* ``field_bessel`` -- the 1-D form, eq. "polar vectorial final" with the three
  integrals of eq. "I0", J_n from SciPy; valid for an axisymmetric pupil.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special

from . import optics as O


def _axisymmetric_phase(sin_t, opt: O.Optics, zernike=None, t_s: float = 0.0,
                        gl_compensated: bool = False):
    """W(theta) for an axisymmetric pupil: Gibson-Lanni and m = 0 Zernike terms."""
    w = np.zeros(np.shape(sin_t), dtype=np.complex128)
    if opt.gl is not None:
        w = w + O.gibson_lanni_opd(sin_t, opt, t_s, compensated=gl_compensated)
    if zernike is not None:
        r = np.asarray(sin_t) / opt.s_max
        for j, c in enumerate(np.asarray(zernike, dtype=np.float64), start=1):
            if c == 0.0:
                continue
            n, m = O.noll_to_nm(j)
            if m != 0:
                raise ValueError("the Bessel form needs an axisymmetric pupil (m = 0 Zernike only)")
            w = w + 2.0 * math.pi * c * O.zernike_noll(j, r, 0.0)
    return w


def theta_rule(opt: O.Optics, n_theta: int, substitute: bool = True, rule: str = "gauss"):
    """Quadrature nodes/weights on [0, theta_max].

    ``rule`` = "simpson": composite Simpson's rule on n_theta (odd) equally spaced
    nodes including both ends, step h = theta_max / (n_theta - 1) (the rule of
    Sec. 4.1); "riemann": the left Riemann sum, nodes i h for i < n_theta,
    h = theta_max / n_theta (the first-order rule of Sec. 5.2.2).  Neither splits
    the range.  "gauss":
    without a sample layer: n_theta Gauss-Legendre nodes.  With Gibson-Lanni and a
    critical angle t_c inside the aperture, sqrt(n_s^2 - n_i^2 sin^2 t) has a
    square-root branch point at t_c; the range is split there and, with
    ``substitute``, each side is mapped by t = t_c - t_c (1 - u)^2 resp.
    t = t_c + (t_max - t_c) u^2 (an exact change of variables that makes the
    integrand smooth in u), with n_theta GL nodes in u on each side.
    """
    tmax = opt.theta_max
    if rule == "simpson":
        if n_theta < 3 or n_theta % 2 == 0:
            raise ValueError("Simpson's rule needs an odd number of nodes >= 3")
        h = tmax / (n_theta - 1)
        w = np.full(n_theta, 2.0)
        w[1::2] = 4.0
        w[0] = w[-1] = 1.0
        return h * np.arange(n_theta), w * (h / 3.0)
    if rule == "riemann":
        h = tmax / n_theta
        return h * np.arange(n_theta), np.full(n_theta, h)
    if rule != "gauss":
        raise ValueError(rule)
    if opt.gl is None or opt.gl.n_s >= opt.na:
        return O.gauss_legendre(n_theta, 0.0, tmax)
    tc = math.asin(opt.gl.n_s / opt.n_i)
    if not substitute:
        a, wa = O.gauss_legendre(n_theta, 0.0, tc)
        b, wb = O.gauss_legendre(n_theta, tc, tmax)
        return np.concatenate([a, b]), np.concatenate([wa, wb])
    u, wu = O.gauss_legendre(n_theta, 0.0, 1.0)
    v = 1.0 - u
    t1, w1 = tc - tc * v * v, wu * 2.0 * tc * v
    t2, w2 = tc + (tmax - tc) * u * u, wu * 2.0 * (tmax - tc) * u
    return np.concatenate([t1, t2]), np.concatenate([w1, w2])


def bessel_integrals(rho, z, opt: O.Optics, n_theta: int = 256, zernike=None, t_s: float = 0.0,
                     gl_compensated: bool = False, scalar: bool = False, extra_cos: bool = False,
                     rule: str = "gauss"):
    """I_0, I_1, I_2 (eq. "I0") without the polarisation factor e_inc^a.

    Shapes: rho (R,), z (Z,) -> each (Z, R) complex128.  The pupil factor
    p(theta) = a(theta) exp(i W(theta)) multiplies every integrand.  With
    ``scalar`` only I_0 with weight sin t is returned (eq. "polar scalar final").

    With Fresnel media the angular weights follow from integrating eq. "field
    Gaussian sphere" over phi with q_s, q_p kept: sin t (q_s + q_p cos t) for I_0,
    q_p sin^2 t for I_1 and sin t (q_p cos t - q_s) for I_2 (q_s = q_p = 1 gives the
    printed weights).
    """
    t, w = theta_rule(opt, n_theta, rule=rule)
    sin_t, cos_t = np.sin(t), np.cos(t)
    p = O.amplitude(cos_t, sin_t, opt) * np.exp(1j * _axisymmetric_phase(sin_t, opt, zernike, t_s,
                                                                       gl_compensated))
    if extra_cos:
        p = p * cos_t
    k = opt.k
    rho = np.atleast_1d(np.asarray(rho, dtype=np.float64))
    z = np.atleast_1d(np.asarray(z, dtype=np.float64))
    arg = k * np.outer(rho, sin_t)                      # (R, T)
    defocus = np.exp(1j * k * np.outer(z, cos_t))       # (Z, T)
    if scalar:
        g = [sin_t]
    else:
        qs, qp = O.fresnel_q(sin_t, opt)
        g = [sin_t * (qs + qp * cos_t), qp * sin_t ** 2, sin_t * (qp * cos_t - qs)]
    out = []
    for n, gn in enumerate(g):
        kern = special.jv(n, arg) * (w * gn * p)[None, :]   # (R, T)
        out.append(defocus @ kern.T)                         # (Z, R)
    return out


def field_bessel(opt: O.Optics, nx: int, ny: int, dx: float, dy: float, z, x0: float = 0.0,
                 y0: float = 0.0, n_theta: int = 256, zernike=None, t_s: float = 0.0,
                 gl_compensated: bool = False, rule: str = "gauss", scalar: bool = False,
                 extra_cos: bool = False):
    """Field at exact pixel radii: vectorial (Z, 3, nx, ny) from eq. "polar vectorial
    final", or with ``scalar`` (Z, 1, nx, ny) from eq. "polar scalar final"."""
    xs = O.output_axis(nx, dx, x0)
    ys = O.output_axis(ny, dy, y0)
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    rho = np.hypot(X, Y).ravel()
    varphi = np.arctan2(Y, X).ravel()            # 0 on the axis
    if scalar:
        (I0,) = bessel_integrals(rho, z, opt, n_theta, zernike, t_s, gl_compensated, scalar=True,
                                 extra_cos=extra_cos, rule=rule)
        return (-1j * opt.f * opt.k * I0).reshape(I0.shape[0], 1, nx, ny)
    I0, I1, I2 = bessel_integrals(rho, z, opt, n_theta, zernike, t_s, gl_compensated,
                                  extra_cos=extra_cos, rule=rule)
    ex, ey = opt.e_inc
    c1, s1 = np.cos(varphi), np.sin(varphi)
    c2, s2 = np.cos(2 * varphi), np.sin(2 * varphi)
    Ex = ex * (I0 - I2 * c2) - ey * I2 * s2
    Ey = -ex * I2 * s2 + ey * (I0 + I2 * c2)
    Ez = -2j * ex * I1 * c1 - 2j * ey * I1 * s1
    E = np.stack([Ex, Ey, Ez], axis=1)           # (Z, 3, R)
    pref = -1j * opt.f * opt.k / 2.0
    return pref * E.reshape(E.shape[0], 3, nx, ny)


def field_polar(opt: O.Optics, points, x0: float = 0.0, y0: float = 0.0, n_theta: int = 256,
                n_phi: int = 96, zernike=None, phase_fn=None, t_s: float = 0.0,
                gl_compensated: bool = False, scalar: bool = False, extra_cos: bool = False,
                chunk: int = 32):
    """Polar double integral at points (K, 3) -> (C, K), C = 3 (vectorial) or 1 (scalar).

    ``zernike`` may hold any Noll terms (the polar integral needs no symmetry);
    ``phase_fn(theta, phi)`` adds an arbitrary pupil phase (e.g. a vortex).
    """
    t, w = theta_rule(opt, n_theta)
    p = 2.0 * math.pi * np.arange(n_phi) / n_phi
    T, P = np.meshgrid(t, p, indexing="ij")
    Wt = np.repeat(w[:, None], n_phi, axis=1) * (2.0 * math.pi / n_phi)
    sin_t, cos_t = np.sin(T), np.cos(T)
    cos_p, sin_p = np.cos(P), np.sin(P)
    phase = np.zeros(T.shape, dtype=np.complex128)
    if opt.gl is not None:
        phase = phase + O.gibson_lanni_opd(sin_t, opt, t_s, compensated=gl_compensated)
    if zernike is not None:
        r = sin_t / opt.s_max
        for j, c in enumerate(np.asarray(zernike, dtype=np.float64), start=1):
            if c != 0.0:
                phase = phase + 2.0 * math.pi * c * O.zernike_noll(j, r, P)
    if phase_fn is not None:
        phase = phase + phase_fn(T, P)
    amp = O.amplitude(cos_t, sin_t, opt) * np.exp(1j * phase) * Wt * sin_t
    if extra_cos:
        amp = amp * cos_t
    if scalar:
        field = amp[None]
    else:
        ex, ey = opt.e_inc
        qs, qp = O.fresnel_q(sin_t, opt)
        field = O.far_field(ex, ey, cos_t, sin_t, cos_p, sin_p, qs, qp) * amp[None]
    field = field.reshape(field.shape[0], -1)
    sx, sy, sz = (sin_t * cos_p).ravel(), (sin_t * sin_p).ravel(), cos_t.ravel()
    pts = np.atleast_2d(np.asarray(points, dtype=np.float64))
    k = opt.k
    out = np.empty((field.shape[0], pts.shape[0]), dtype=np.complex128)
    for a in range(0, pts.shape[0], chunk):
        q = pts[a:a + chunk]
        ph = k * (np.outer(q[:, 0] - x0, sx) + np.outer(q[:, 1] - y0, sy) + np.outer(q[:, 2], sz))
        out[:, a:a + chunk] = field @ np.exp(1j * ph).T
    return (-1j * opt.f * opt.k / (2.0 * math.pi)) * out
