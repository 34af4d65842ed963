"""Pins of the oracle's optical building blocks against closed forms and textbook facts."""
import math

import numpy as np
import pytest

from oracle import optics as O


def test_gauss_legendre_exact_on_polynomials():
    # n-point rule on [a, b] integrates t^p exactly up to p = 2n - 1
    a, b = 0.0, 1.1739
    t, w = O.gauss_legendre(6, a, b)
    assert abs(w.sum() - (b - a)) < 1e-14
    for p in range(0, 12):
        exact = (b ** (p + 1) - a ** (p + 1)) / (p + 1)
        assert abs(np.sum(w * t ** p) - exact) < 1e-13 * max(1.0, exact)
    # degree 2n is no longer exact
    exact = b ** 13 / 13
    assert abs(np.sum(w * t ** 12) - exact) > 1e-10 * exact


# Noll (1976) table: (j, n, m) with m > 0 cosine, m < 0 sine
NOLL_NM = [(1, 0, 0), (2, 1, 1), (3, 1, -1), (4, 2, 0), (5, 2, -2), (6, 2, 2), (7, 3, -1),
           (8, 3, 1), (9, 3, -3), (10, 3, 3), (11, 4, 0), (12, 4, 2), (13, 4, -2), (14, 4, 4),
           (15, 4, -4), (16, 5, 1), (17, 5, -1), (18, 5, 3), (19, 5, -3), (20, 5, 5), (21, 5, -5),
           (22, 6, 0)]


@pytest.mark.parametrize("j,n,m", NOLL_NM)
def test_noll_index_table(j, n, m):
    assert O.noll_to_nm(j) == (n, m)


def test_zernike_low_order_closed_forms():
    rng = np.random.default_rng(0)
    r = rng.uniform(0, 1, 200)
    p = rng.uniform(0, 2 * math.pi, 200)
    s3, s6, s8 = math.sqrt(3), math.sqrt(6), math.sqrt(8)
    closed = {
        1: np.ones_like(r),
        2: 2 * r * np.cos(p),
        3: 2 * r * np.sin(p),
        4: s3 * (2 * r ** 2 - 1),
        5: s6 * r ** 2 * np.sin(2 * p),
        6: s6 * r ** 2 * np.cos(2 * p),
        7: s8 * (3 * r ** 3 - 2 * r) * np.sin(p),
        8: s8 * (3 * r ** 3 - 2 * r) * np.cos(p),
        9: s8 * r ** 3 * np.sin(3 * p),
        10: s8 * r ** 3 * np.cos(3 * p),
        11: math.sqrt(5) * (6 * r ** 4 - 6 * r ** 2 + 1),
        22: math.sqrt(7) * (20 * r ** 6 - 30 * r ** 4 + 12 * r ** 2 - 1),
    }
    for j, ref in closed.items():
        np.testing.assert_allclose(O.zernike_noll(j, r, p), ref, rtol=0, atol=1e-13)


def test_zernike_orthonormal_on_disk():
    # polar product rule: GL in r (exact for the polynomial radial parts), trapezoid in phi
    r, wr = O.gauss_legendre(16, 0.0, 1.0)
    nphi = 64
    p = 2 * math.pi * np.arange(nphi) / nphi
    R, P = np.meshgrid(r, p, indexing="ij")
    W = (wr[:, None] * R) * (2 * math.pi / nphi) / math.pi     # area-normalised
    Z = np.stack([O.zernike_noll(j, R, P) for j in range(1, 23)])
    G = np.einsum("aij,bij,ij->ab", Z, Z, W)
    assert np.max(np.abs(G - np.eye(22))) < 1e-12


def test_far_field_reduces_to_incident_on_axis():
    # low-NA limit theta = 0 with q_s = q_p = 1: e_inf = e_inc for every phi
    ex, ey = 0.3 - 0.2j, 0.7 + 0.4j
    for phi in np.linspace(0, 2 * math.pi, 7):
        e = O.far_field(ex, ey, 1.0, 0.0, math.cos(phi), math.sin(phi))
        np.testing.assert_allclose(e, [ex, ey, 0.0], atol=1e-15)


def test_far_field_preserves_norm():
    # with q_s = q_p = 1 the basis change is a rotation: |e_inf| = |e_inc|
    rng = np.random.default_rng(1)
    t = rng.uniform(0, 1.2, 100)
    p = rng.uniform(0, 2 * math.pi, 100)
    ex, ey = 0.6 + 0.1j, -0.2 + 0.75j
    e = O.far_field(ex, ey, np.cos(t), np.sin(t), np.cos(p), np.sin(p))
    np.testing.assert_allclose(np.sum(np.abs(e) ** 2, axis=0), abs(ex) ** 2 + abs(ey) ** 2, rtol=1e-14)


def test_far_field_meridional_example():
    # x-polarised light in the x-z plane (phi = 0) is tilted by theta: (cos t, 0, -sin t)
    t = 0.8
    e = O.far_field(1.0, 0.0, math.cos(t), math.sin(t), 1.0, 0.0)
    np.testing.assert_allclose(e, [math.cos(t), 0.0, -math.sin(t)], atol=1e-15)
    # y-polarised light in the x-z plane is s-polarised: unchanged
    e = O.far_field(0.0, 1.0, math.cos(t), math.sin(t), 1.0, 0.0)
    np.testing.assert_allclose(e, [0.0, 1.0, 0.0], atol=1e-15)


def _gl_optics(n_s=1.33):
    return O.Optics(na=1.4, wavelength=600.0, n_i=1.518,
                    gl=O.GibsonLanni(n_s=n_s, n_i_design=1.518))


def test_gibson_lanni_literal_minus_compensated_is_a_defocus():
    opt = _gl_optics()
    sin_t = np.linspace(0, opt.s_max, 50)
    t_s = 2300.0
    w_lit = O.gibson_lanni_opd(sin_t, opt, t_s)
    w_cmp = O.gibson_lanni_opd(sin_t, opt, t_s, compensated=True)
    np.testing.assert_allclose(w_lit - w_cmp, opt.k * t_s * np.sqrt(1 - sin_t ** 2), rtol=1e-13)


def test_gibson_lanni_closed_form_and_index_match():
    opt = _gl_optics()
    sin_t = np.linspace(0, 0.85, 40)          # below the critical angle of n_s = 1.33
    t_s = 1700.0
    k0 = 2 * math.pi / opt.wavelength
    n_s, n_i = 1.33, 1.518
    w_cmp = O.gibson_lanni_opd(sin_t, opt, t_s, compensated=True)
    ref = k0 * t_s * (np.sqrt(n_s ** 2 - n_i ** 2 * sin_t ** 2) - n_i ** 2 / n_s * np.sqrt(1 - sin_t ** 2))
    np.testing.assert_allclose(w_cmp.real, ref, rtol=1e-12, atol=1e-9)
    # index-matched sample: no aberration left at the paraxial focus
    opt2 = _gl_optics(n_s=1.518)
    w = O.gibson_lanni_opd(sin_t, opt2, t_s, compensated=True)
    assert np.max(np.abs(w)) < 1e-8


def test_gibson_lanni_evanescent_branch_decays():
    opt = _gl_optics()
    sin_c = 1.33 / 1.518
    sin_t = np.linspace(sin_c + 1e-3, opt.s_max, 20)
    w1 = O.gibson_lanni_opd(sin_t, opt, 1000.0)
    w2 = O.gibson_lanni_opd(sin_t, opt, 3000.0)
    assert np.all(w1.imag > 0) and np.all(w2.imag > w1.imag)
    assert np.all(np.abs(np.exp(1j * w2)) < 1.0)
