"""Pins of the Gaussian envelope a(s) *= exp(-sin^2 t / s_env^2) (Sec. 3.4.4).

Closed forms, independent of the oracle's code:

* Scalar model, apodization off, the extra factor s_z of the accuracy benchmark and
  z = 0: with u = sin t (du = cos t dt) the spherical integral becomes the Hankel
  transform of a Gaussian,
      E(rho) = -i f k int_0^{s_max} exp(-u^2 / s_env^2) J0(k rho u) u du
             = -i f k (s_env^2 / 2) exp(-(k rho s_env)^2 / 4) + tail,
  |tail| <= f k (s_env^2 / 2) exp(-s_max^2 / s_env^2) (|J0| <= 1).  The Cartesian
  form reaches the same value as the 2-D Fourier transform of the Gaussian.
* Vectorial model with apodization: by Plancherel on the Cartesian form the
  focal-plane energy is f^2 int |e_inf|^2 a^2 / s_z^2 ds_x ds_y
      = 2 pi f^2 int_0^{t_max} exp(-2 sin^2 t / s_env^2) sin t dt
      = 2 pi f^2 [D(g) - D(g c_m) exp(-g^2 (1 - c_m^2))] / g,
  g = sqrt(2) / s_env, c_m = cos t_max, D = Dawson's integral (substitute c = cos t).
  The squared envelope enters, so a slip between exp(-x) and exp(-x^2) fails it.
"""
import math

import numpy as np
import pytest
from scipy.special import dawsn

from oracle import bessel as B
from oracle import fourier as F
from oracle import optics as O


def _opt(**kw):
    d = dict(na=1.4, wavelength=532.0, n_i=1.518)
    d.update(kw)
    return O.Optics(**d)


def _closed_form(opt, rho, edge=None):
    """Closed form and the bound on the Gaussian's tail beyond radius ``edge`` (s_max)."""
    s = opt.s_env
    edge = opt.s_max if edge is None else edge
    ref = -1j * opt.f * opt.k * s * s / 2 * np.exp(-(opt.k * rho * s) ** 2 / 4)
    tail = opt.f * opt.k * s * s / 2 * math.exp(-edge ** 2 / s ** 2)
    return ref, tail


@pytest.mark.parametrize("s_env", [0.15, 0.2])
def test_envelope_hankel_closed_form_bessel_form(s_env):
    opt = _opt(apodization=False, s_env=s_env)
    rho = np.linspace(0.0, 900.0, 61)
    (I0,) = B.bessel_integrals(rho, [0.0], opt, 256, scalar=True, extra_cos=True)
    E = -1j * opt.f * opt.k * I0[0]
    ref, tail = _closed_form(opt, rho)
    assert np.max(np.abs(E - ref)) < tail + 1e-12 * abs(ref[0])


@pytest.mark.parametrize("s_env", [0.15, 0.2])
def test_envelope_hankel_closed_form_polar_double_integral(s_env):
    opt = _opt(apodization=False, s_env=s_env)
    pts = np.array([[0.0, 0.0, 0.0], [60.0, 0.0, 0.0], [-90.0, 140.0, 0.0], [300.0, -250.0, 0.0]])
    E = B.field_polar(opt, pts, n_theta=128, n_phi=64, scalar=True, extra_cos=True)[0]
    ref, tail = _closed_form(opt, np.hypot(pts[:, 0], pts[:, 1]))
    assert np.max(np.abs(E - ref)) < tail + 1e-12 * abs(ref[0])


@pytest.mark.parametrize("s_env", [0.15, 0.2])
def test_envelope_fourier_transform_of_gaussian_cartesian_form(s_env):
    # the midpoint sum of a Gaussian that vanishes at the disk edge is spectrally accurate;
    # the cell-centred mask differs from the disk only in cells within ds / sqrt(2) of the
    # circle, so the truncation is bounded by the Gaussian's mass beyond s_max - ds
    opt = _opt(apodization=False, s_env=s_env)
    g = F.pupil_geometry(96, opt)
    P = F.base_pupil(g, opt, scalar=True, extra_cos=True)
    E = F.field_separable(P, g, opt, 31, 31, 25.0, 25.0, [0.0])[0, 0]
    xs = O.output_axis(31, 25.0)
    ref, tail = _closed_form(opt, np.hypot(xs[:, None], xs[None, :]), edge=opt.s_max - g["ds"])
    assert np.max(np.abs(E - ref)) < tail + 1e-12 * abs(ref[15, 15])


@pytest.mark.parametrize("s_env", [0.2, 0.5])
def test_envelope_vectorial_energy_closed_form(s_env):
    opt = _opt(s_env=s_env)   # sqrt(cos) apodization on, circular polarisation
    g2 = 2.0 / s_env ** 2
    gg, cm = math.sqrt(g2), math.cos(opt.theta_max)
    target = 2 * math.pi * opt.f ** 2 * (dawsn(gg) - dawsn(gg * cm) * math.exp(-g2 * (1 - cm * cm))) / gg
    errs = []
    for n in (64, 256, 1024):
        geo = F.pupil_geometry(n, opt)
        P = F.base_pupil(geo, opt)
        errs.append(abs(opt.f ** 2 * np.sum(np.abs(P) ** 2) / geo["ds"] ** 2 / target - 1))
    if s_env == 0.2:
        # the integrand is ~1e-18 at the disk edge: the sum is spectrally accurate
        assert errs[-1] < 1e-12, errs
    else:
        assert errs[-1] < 2e-3 and errs[-1] < errs[0], errs


def test_envelope_off_and_wide_limit():
    # s_env = 0 switches the factor off; a very wide envelope tends to no envelope
    c, s = np.linspace(0.4, 1.0, 7), np.sqrt(1 - np.linspace(0.4, 1.0, 7) ** 2)
    np.testing.assert_array_equal(O.amplitude(c, s, _opt(s_env=0.0)), np.sqrt(c))
    np.testing.assert_allclose(O.amplitude(c, s, _opt(s_env=1e4)), np.sqrt(c), rtol=1e-8)
