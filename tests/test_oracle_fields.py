"""Pins of the oracle's focal fields against closed forms, exact identities and brute force.

None of these compares the oracle with itself: each check is a value or a
property that the paper or the mathematics fixes independently of the code.
"""
import math

import numpy as np
import pytest
from scipy.special import j1

from oracle import bessel as B
from oracle import fourier as F
from oracle import optics as O

X_LIN = (1.0 + 0j, 0j)
CIRC = (1 / math.sqrt(2), 1j / math.sqrt(2))


def _opt(**kw):
    d = dict(na=1.4, wavelength=532.0, n_i=1.518)
    d.update(kw)
    return O.Optics(**d)


# ----------------------------------------------------------------- Airy (Sec. 5.2.2)
def test_airy_closed_form_spherical_scalar():
    # scalar spherical form with the extra cos(theta): exactly -(i f k s_max^2 / 2) 2 J1(v)/v
    opt = _opt(apodization=False)
    rho = np.linspace(0.5, 900.0, 64)
    (I0,) = B.bessel_integrals(rho, [0.0], opt, 128, scalar=True, extra_cos=True)
    E = -1j * opt.f * opt.k * I0[0]
    v = opt.k * opt.s_max * rho
    ref = -1j * opt.f * opt.k * opt.s_max ** 2 / 2 * 2 * j1(v) / v
    assert np.max(np.abs(E - ref)) < 1e-12 * np.max(np.abs(ref))


def test_airy_polar_double_integral_scalar():
    opt = _opt(apodization=False)
    pts = np.array([[0.0, 0.0, 0.0], [130.0, 0.0, 0.0], [-90.0, 200.0, 0.0], [400.0, 300.0, 0.0]])
    E = B.field_polar(opt, pts, n_theta=96, n_phi=64, scalar=True, extra_cos=True)[0]
    v = opt.k * opt.s_max * np.hypot(pts[:, 0], pts[:, 1])
    airy = np.where(v > 0, 2 * j1(np.where(v > 0, v, 1)) / np.where(v > 0, v, 1), 1.0)
    ref = -1j * opt.f * opt.k * opt.s_max ** 2 / 2 * airy
    assert np.max(np.abs(E - ref)) < 1e-12 * abs(ref[0])


def test_airy_cartesian_converges_between_first_and_second_order():
    opt = _opt(apodization=False)
    xs = O.output_axis(41, 20.0)
    v = opt.k * opt.s_max * np.abs(xs)
    ref = -1j * opt.f * opt.k * opt.s_max ** 2 / 2 * np.where(v > 0, 2 * j1(np.where(v > 0, v, 1)) / np.where(v > 0, v, 1), 1.0)
    errs, hs = [], []
    for n in (32, 64, 128, 256, 512):
        g = F.pupil_geometry(n, opt)
        P = F.base_pupil(g, opt, scalar=True, extra_cos=True)
        E = F.field_separable(P, g, opt, 41, 1, 20.0, 20.0, [0.0])[0, 0, :, 0]
        errs.append(np.linalg.norm(E - ref) / np.linalg.norm(ref))
        hs.append(2 * opt.s_max / n)
    order = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    assert errs[-1] < 2e-4
    assert 1.0 <= order <= 2.0, order


def test_vectorial_low_na_tends_to_airy_squared():
    # x-polarised vectorial focus -> (2 J1(v)/v)^2 as NA -> 0, deviation O(NA^2)
    devs = []
    for na in (0.1, 0.05):
        opt = O.Optics(na=na, wavelength=532.0, n_i=1.0, apodization=False, e_inc=X_LIN)
        dx = 6.0 / (opt.k * opt.s_max) / 20          # 41 px spanning v in [-6, 6]
        E = B.field_bessel(opt, 41, 1, dx, 1.0, [0.0], n_theta=64)
        I = np.sum(np.abs(E[0, :, :, 0]) ** 2, axis=0)
        v = opt.k * opt.s_max * np.abs(O.output_axis(41, dx))
        airy2 = np.where(v > 0, 2 * j1(np.where(v > 0, v, 1)) / np.where(v > 0, v, 1), 1.0) ** 2
        devs.append(np.max(np.abs(I / I[20] - airy2)))
    ratio = devs[0] / devs[1]
    assert 3.0 < ratio < 5.0, ratio


# ------------------------------------------------ Fourier / Bessel equivalence (Sec. 4.1)
@pytest.mark.parametrize("e_inc", [CIRC, X_LIN])
def test_polar_double_integral_equals_bessel_form(e_inc):
    opt = _opt(e_inc=e_inc)
    zern = np.zeros(11)
    zern[3], zern[10] = 0.08, -0.05                       # m = 0 terms only
    pts = np.array([[0, 0, 0], [60, -40, 300], [200, 100, -500], [-350, 20, 800], [500, 500, 0],
                    [0, 240, -120]], float)
    Ep = B.field_polar(opt, pts, n_theta=200, n_phi=96, zernike=zern)
    Eb = np.stack([B.field_bessel(opt, 1, 1, 1.0, 1.0, [p[2]], x0=-p[0], y0=-p[1], n_theta=200,
                                  zernike=zern)[0, :, 0, 0] for p in pts], axis=1)
    assert np.linalg.norm(Ep - Eb) / np.linalg.norm(Eb) < 1e-12


def test_cartesian_converges_to_bessel_form():
    opt = _opt()
    z = [-300.0, 0.0, 400.0]
    Eb = B.field_bessel(opt, 33, 33, 20.0, 20.0, z, n_theta=200)
    errs = []
    for n in (32, 64, 128, 256):
        g = F.pupil_geometry(n, opt)
        E = F.field_separable(F.base_pupil(g, opt), g, opt, 33, 33, 20.0, 20.0, z)
        errs.append(np.linalg.norm(E - Eb) / np.linalg.norm(Eb))
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-3


# ----------------------------------------------------------------------------- Parseval
def _aberrated_pupil(n, opt, seed=3):
    g = F.pupil_geometry(n, opt)
    rng = np.random.default_rng(seed)
    zern = np.zeros(21)
    zern[3:] = rng.normal(0, 0.05, 18)
    return g, F.base_pupil(g, opt, F.pupil_phase(g, opt, zernike=zern))


def test_parseval_discrete_full_period_grid():
    # with k ds dx = 2 pi / M and M >= N the M x M output is an exact unitary DFT image
    opt = _opt()
    n, m = 24, 32
    g, P = _aberrated_pupil(n, opt)
    dx = 2 * math.pi / (opt.k * g["ds"] * m)
    for z in (0.0, 450.0, -800.0):
        E = F.field_separable(P, g, opt, m, m, dx, dx, [z])[0]
        sz = np.where(g["mask"], g["sz"], 0.0)
        Pz = P * np.exp(1j * opt.k * sz * z)
        lhs = np.sum(np.abs(E) ** 2, axis=(1, 2))
        rhs = (opt.f * opt.k / (2 * math.pi)) ** 2 * m * m * np.sum(np.abs(Pz) ** 2, axis=(1, 2))
        np.testing.assert_allclose(lhs, rhs, rtol=1e-12)


def test_parseval_continuum_energy():
    # Plancherel on the Cartesian form: total focal-plane energy -> 2 pi f^2 (1 - cos theta_max)
    opt = _opt()
    target = 2 * math.pi * opt.f ** 2 * (1 - math.cos(opt.theta_max))
    errs = []
    for n in (64, 256, 1024):
        g = F.pupil_geometry(n, opt)
        P = F.base_pupil(g, opt)
        energy = opt.f ** 2 * np.sum(np.abs(P) ** 2) / g["ds"] ** 2
        errs.append(abs(energy / target - 1))
    assert errs[-1] < 1e-2 and errs[-1] < errs[0]


# ------------------------------------------------------------------------- symmetries
def test_bessel_axisymmetry_circular():
    opt = _opt()
    E = B.field_bessel(opt, 13, 13, 20.0, 20.0, [0.0, 350.0], n_theta=120)
    I = F.intensity(E)
    c = 6
    for zi in range(2):
        assert abs(I[zi, c + 3, c + 4] - I[zi, c + 5, c]) < 1e-12 * I[zi].max()
        assert abs(I[zi, c - 4, c + 3] - I[zi, c, c - 5]) < 1e-12 * I[zi].max()


def test_fourier_quarter_turn_invariance_circular():
    opt = _opt()
    g = F.pupil_geometry(40, opt)
    E = F.field_separable(F.base_pupil(g, opt), g, opt, 17, 17, 25.0, 25.0, [0.0, 300.0])
    I = F.intensity(E)
    np.testing.assert_allclose(np.rot90(I, 1, axes=(1, 2)), I, rtol=0, atol=1e-12 * I.max())


def test_axial_mirror_unaberrated():
    opt = _opt(e_inc=X_LIN)
    g = F.pupil_geometry(32, opt)
    P = F.base_pupil(g, opt)
    I = F.intensity(F.field_separable(P, g, opt, 15, 15, 30.0, 30.0, [-420.0, 420.0]))
    np.testing.assert_allclose(I[0], I[1], rtol=0, atol=1e-12 * I.max())


def test_donut_on_axis_zero_only_for_matching_handedness():
    def vortex(t, p):
        return p

    on_axis = np.array([[0.0, 0.0, z] for z in (-500.0, 0.0, 300.0)])
    e_plus = B.field_polar(_opt(e_inc=(1 / math.sqrt(2), 1j / math.sqrt(2))), on_axis, n_theta=80,
                           n_phi=64, phase_fn=vortex)
    e_minus = B.field_polar(_opt(e_inc=(1 / math.sqrt(2), -1j / math.sqrt(2))), on_axis, n_theta=80,
                            n_phi=64, phase_fn=vortex)
    scale = np.max(np.abs(e_minus))
    assert np.max(np.abs(e_plus)) < 1e-12 * scale
    assert np.max(np.abs(e_minus[2])) > 0.1 * scale    # E_z survives for the other handedness


def test_half_moon_ex_vanishes_on_the_y_axis():
    # pi step across the y-axis with x-linear polarisation: E_x odd in x
    opt = _opt(e_inc=X_LIN)
    g = F.pupil_geometry(32, opt)
    w0 = np.where(g["sx"] > 0, math.pi, 0.0)
    P = F.base_pupil(g, opt, F.pupil_phase(g, opt, phase_map=w0))
    E = F.field_separable(P, g, opt, 15, 15, 30.0, 30.0, [0.0, 250.0])
    c = 7
    assert np.max(np.abs(E[:, 0, c, :])) < 1e-12 * np.max(np.abs(E))
    assert np.max(np.abs(E[:, 1, c, :])) > 1e-3 * np.max(np.abs(E))


# ---------------------------------------------------------------- brute force / shifts
def test_direct_double_sum_equals_separable():
    opt = O.Optics(na=1.4, wavelength=600.0, n_i=1.518, gl=O.GibsonLanni(n_s=1.33, n_i_design=1.518))
    g = F.pupil_geometry(20, opt)
    rng = np.random.default_rng(7)
    zern = np.zeros(21)
    zern[3:] = rng.normal(0, 0.05, 18)
    P = F.base_pupil(g, opt, F.pupil_phase(g, opt, zernike=zern, phase_map=rng.normal(0, 0.2, (20, 20)),
                                           t_s=1800.0))
    z = [-2500.0, -1800.0, -700.0]
    Es = F.field_separable(P, g, opt, 9, 7, 30.0, 25.0, z, x0=13.0, y0=-4.0)
    xs, ys = O.output_axis(9, 30.0), O.output_axis(7, 25.0)
    X, Y, Z = np.meshgrid(xs, ys, z, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    Ed = F.field_direct(P, g, opt, pts, x0=13.0, y0=-4.0).reshape(3, 9, 7, 3)
    np.testing.assert_allclose(np.moveaxis(Ed, 3, 0), Es, rtol=0, atol=1e-13 * np.abs(Es).max())


def test_emitter_shift_by_one_pixel_translates_the_image():
    opt = _opt()
    g, P = _aberrated_pupil(24, opt)
    E0 = F.field_separable(P, g, opt, 12, 12, 40.0, 40.0, [100.0])
    E1 = F.field_separable(P, g, opt, 12, 12, 40.0, 40.0, [100.0], x0=40.0, y0=-80.0)
    # E1(x, y) = E0(x - 40, y + 80): pixel (m, n) of E1 is pixel (m - 1, n + 2) of E0
    np.testing.assert_allclose(E1[:, :, 1:, :-2], E0[:, :, :-1, 2:], rtol=0, atol=1e-13 * np.abs(E0).max())


def test_gibson_lanni_literal_focus_is_shifted_by_depth():
    # PSF_literal(z) = PSF_compensated(z + t_s)
    opt = O.Optics(na=1.4, wavelength=600.0, n_i=1.518, gl=O.GibsonLanni(n_s=1.33, n_i_design=1.518))
    g = F.pupil_geometry(24, opt)
    t_s = 1200.0
    P_lit = F.base_pupil(g, opt, F.pupil_phase(g, opt, t_s=t_s))
    P_cmp = F.base_pupil(g, opt, F.pupil_phase(g, opt, t_s=t_s, gl_compensated=True))
    z = np.array([-1500.0, -1200.0, -600.0])
    E_lit = F.field_separable(P_lit, g, opt, 9, 9, 30.0, 30.0, z)
    E_cmp = F.field_separable(P_cmp, g, opt, 9, 9, 30.0, 30.0, z + t_s)
    np.testing.assert_allclose(E_lit, E_cmp, rtol=0, atol=1e-12 * np.abs(E_cmp).max())


def test_critical_angle_substitution_matches_brute_force_rule():
    # the substituted rule equals plain Gauss-Legendre with many nodes on each side of t_c
    opt = O.Optics(na=1.4, wavelength=532.0, n_i=1.518, gl=O.GibsonLanni(n_s=1.33, n_i_design=1.518))
    rho = np.array([0.0, 150.0, 420.0])
    z = np.array([-2200.0, -1900.0])
    sub = B.bessel_integrals(rho, z, opt, 128, t_s=2000.0)
    brute = B.bessel_integrals(rho, z, opt, 4096, t_s=2000.0)      # substitute=True path
    t, w = B.theta_rule(opt, 4096, substitute=False)
    assert abs(np.sum(w) - opt.theta_max) < 1e-13
    plain = []
    for n in (512, 4096):
        tt, ww = B.theta_rule(opt, n, substitute=False)
        f = np.exp(1j * O.gibson_lanni_opd(np.sin(tt), opt, 2000.0)) * np.sqrt(np.cos(tt)) * np.sin(tt)
        plain.append(np.sum(ww * f))
    tt, ww = B.theta_rule(opt, 64)
    f = np.exp(1j * O.gibson_lanni_opd(np.sin(tt), opt, 2000.0)) * np.sqrt(np.cos(tt)) * np.sin(tt)
    smooth = np.sum(ww * f)
    # plain GL converges as n^-3 towards the substituted value
    assert abs(plain[1] - smooth) < 1e-8 * abs(smooth)
    assert abs(plain[1] - smooth) < abs(plain[0] - smooth) / 100
    for a, b in zip(sub, brute):
        assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(b))
