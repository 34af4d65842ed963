"""Pins of the oracle's scalar propagators, its Simpson / Riemann theta rules and its
Fresnel transmission factors, against closed forms, conservation laws and exact
identities (Sec. 3.2, Sec. 3.3, Sec. 4.1, Sec. 5.2.2).
"""
import math

import numpy as np
import pytest
from scipy.special import j1

from oracle import bessel as B
from oracle import fourier as F
from oracle import optics as O

CIRC = (1 / math.sqrt(2), 1j / math.sqrt(2))


def _opt(**kw):
    d = dict(na=1.4, wavelength=532.0, n_i=1.518)
    d.update(kw)
    return O.Optics(**d)


def _airy_line(opt, n_px=41, dx=20.0):
    v = opt.k * opt.s_max * np.abs(O.output_axis(n_px, dx))
    safe = np.where(v > 0, v, 1.0)
    return -1j * opt.f * opt.k * opt.s_max ** 2 / 2 * np.where(v > 0, 2 * j1(safe) / safe, 1.0)


# ------------------------------------------------------------------ theta rules
def test_simpson_exact_on_cubics_riemann_closed_form_error():
    opt = _opt()
    b = opt.theta_max
    t, w = B.theta_rule(opt, 9, rule="simpson")
    assert t[0] == 0.0 and abs(t[-1] - b) < 1e-15
    for p in range(4):
        assert abs(np.sum(w * t ** p) - b ** (p + 1) / (p + 1)) < 1e-14
    assert abs(np.sum(w * t ** 4) - b ** 5 / 5) > 1e-8       # degree 4 is not exact
    n = 10
    t, w = B.theta_rule(opt, n, rule="riemann")
    h = b / n
    # left Riemann sum of t: exactly b^2/2 - b h / 2 (first-order error)
    assert abs(np.sum(w * t) - (b * b / 2 - b * h / 2)) < 1e-14
    with pytest.raises(ValueError):
        B.theta_rule(opt, 8, rule="simpson")


def _order(hs, errs):
    return np.polyfit(np.log(hs), np.log(errs), 1)[0]


def test_accuracy_benchmark_orders_against_airy():
    # Sec. 5.2.2: scalar spherical propagator with the extra s_z factor against
    # 2 J1(v)/v; Riemann converges at first order, Simpson at fourth order.
    opt = _opt(apodization=False)
    ref = _airy_line(opt)
    rho = np.abs(O.output_axis(41, 20.0))
    res = {}
    for rule, ns in (("riemann", (16, 32, 64, 128, 256)), ("simpson", (9, 17, 33, 65))):
        errs, hs = [], []
        for n in ns:
            (I0,) = B.bessel_integrals(rho, [0.0], opt, n, scalar=True, extra_cos=True, rule=rule)
            E = -1j * opt.f * opt.k * I0[0]
            errs.append(np.linalg.norm(E - ref) / np.linalg.norm(ref))
            hs.append(opt.theta_max / (n if rule == "riemann" else n - 1))
        res[rule] = (_order(hs, errs), errs[-1])
    assert 0.9 < res["riemann"][0] < 1.1, res
    assert 3.7 < res["simpson"][0] < 4.3, res
    assert res["simpson"][1] < 1e-6, res


def test_scalar_bessel_equals_scalar_polar_double_integral():
    opt = _opt()
    zern = np.zeros(11)
    zern[3], zern[10] = 0.1, -0.04
    pts = np.array([[0, 0, 0], [60, -40, 300], [200, 100, -500], [-350, 20, 800]], float)
    Ep = B.field_polar(opt, pts, n_theta=128, n_phi=96, zernike=zern, scalar=True)[0]
    Eb = np.array([B.field_bessel(opt, 1, 1, 1.0, 1.0, [p[2]], x0=-p[0], y0=-p[1], n_theta=128,
                                  zernike=zern, scalar=True)[0, 0, 0, 0] for p in pts])
    assert np.linalg.norm(Ep - Eb) / np.linalg.norm(Eb) < 1e-12


def test_scalar_cartesian_converges_to_scalar_bessel():
    opt = _opt()
    z = [-300.0, 0.0, 400.0]
    Eb = B.field_bessel(opt, 33, 33, 20.0, 20.0, z, n_theta=200, scalar=True)
    errs = []
    for n in (32, 64, 128, 256):
        g = F.pupil_geometry(n, opt)
        E = F.field_separable(F.base_pupil(g, opt, scalar=True), g, opt, 33, 33, 20.0, 20.0, z)
        errs.append(np.linalg.norm(E - Eb) / np.linalg.norm(Eb))
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-3


# ------------------------------------------------------------------ Fresnel factors
def _single(n1, n2):
    return _opt(na=min(n1, n2) * 0.99, n_i=n2, fresnel_media=(n1,))


@pytest.mark.parametrize("n1,n2", [(1.33, 1.518), (1.518, 1.33), (1.0, 1.5)])
def test_fresnel_single_interface_conserves_energy(n1, n2):
    # r and t of each polarisation satisfy |r|^2 + (n2 cos t2 / n1 cos t1) |t|^2 = 1
    opt = _single(n1, n2)
    sin2 = np.linspace(0.0, 0.98 * min(n1, n2) / n2, 40)       # angle in medium 2
    qs, qp = O.fresnel_q(sin2, opt)
    sin1 = n2 * sin2 / n1
    c1, c2 = np.sqrt(1 - sin1 ** 2), np.sqrt(1 - sin2 ** 2)
    rs = (n1 * c1 - n2 * c2) / (n1 * c1 + n2 * c2)
    rp = (n2 * c1 - n1 * c2) / (n2 * c1 + n1 * c2)
    ratio = (n2 * c2) / (n1 * c1)
    np.testing.assert_allclose(np.abs(rs) ** 2 + ratio * np.abs(qs) ** 2, 1.0, atol=1e-13)
    np.testing.assert_allclose(np.abs(rp) ** 2 + ratio * np.abs(qp) ** 2, 1.0, atol=1e-13)


def test_fresnel_normal_incidence_and_brewster():
    n1, n2 = 1.33, 1.518
    opt = _single(n1, n2)
    qs, qp = O.fresnel_q(np.array([0.0]), opt)
    assert abs(qs[0] - 2 * n1 / (n1 + n2)) < 1e-15 and abs(qp[0] - 2 * n1 / (n1 + n2)) < 1e-15
    # Brewster: tan t1 = n2 / n1, no p reflection, so t_p = n1 / n2
    t1 = math.atan(n2 / n1)
    sin2 = n1 * math.sin(t1) / n2
    _, qp = O.fresnel_q(np.array([sin2]), opt)
    assert abs(qp[0] - n1 / n2) < 1e-14


def test_fresnel_equal_media_transmit_fully_and_compose():
    opt = _opt(fresnel_media=(1.518, 1.518))
    s = np.linspace(0, opt.s_max, 17)
    qs, qp = O.fresnel_q(s, opt)
    np.testing.assert_allclose(qs, 1.0, atol=1e-15)
    np.testing.assert_allclose(qp, 1.0, atol=1e-15)
    # an intermediate layer of the immersion index changes nothing
    a = O.fresnel_q(s, _opt(na=1.3, fresnel_media=(1.33, 1.518)))
    b = O.fresnel_q(s, _opt(na=1.3, fresnel_media=(1.33,)))
    np.testing.assert_allclose(a[0], b[0], atol=1e-15)
    np.testing.assert_allclose(a[1], b[1], atol=1e-15)


@pytest.mark.parametrize("na", [1.2, 1.45])
def test_fresnel_polar_double_integral_equals_bessel_form(na):
    # the q-weighted I_n of the 1-D form against the phi integral of eq. "field Gaussian
    # sphere" with q_s, q_p (NA 1.45 reaches beyond the sample's critical angle: complex q)
    opt = _opt(na=na, e_inc=CIRC, fresnel_media=(1.33, 1.52))
    pts = np.array([[0, 0, 0], [60, -40, 300], [200, 100, -500], [-350, 20, 800], [500, 500, 0]], float)
    Ep = B.field_polar(opt, pts, n_theta=160, n_phi=96)
    Eb = np.stack([B.field_bessel(opt, 1, 1, 1.0, 1.0, [p[2]], x0=-p[0], y0=-p[1],
                                  n_theta=160)[0, :, 0, 0] for p in pts], axis=1)
    assert np.linalg.norm(Ep - Eb) / np.linalg.norm(Eb) < 1e-12


def test_fresnel_cartesian_converges_to_bessel_form():
    opt = _opt(na=1.2, fresnel_media=(1.33, 1.52))
    z = [-300.0, 0.0, 400.0]
    Eb = B.field_bessel(opt, 33, 33, 20.0, 20.0, z, n_theta=200)
    errs = []
    for n in (32, 64, 128, 256):
        g = F.pupil_geometry(n, opt)
        E = F.field_separable(F.base_pupil(g, opt), g, opt, 33, 33, 20.0, 20.0, z)
        errs.append(np.linalg.norm(E - Eb) / np.linalg.norm(Eb))
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-3
    # and the factors matter: the field without them differs by far more than that
    g = F.pupil_geometry(256, opt)
    plain = _opt(na=1.2)
    E0 = F.field_separable(F.base_pupil(g, plain), g, plain, 33, 33, 20.0, 20.0, z)
    assert np.linalg.norm(E0 - Eb) / np.linalg.norm(Eb) > 10 * errs[-1]
