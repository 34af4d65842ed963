"""Pins of the Bessel-form gradient oracle: central finite differences of the forward
oracle (the definition of the derivative), the global-phase invariance, and the linear
dependence of the Gibson-Lanni phase on the depth."""
import math

import numpy as np
import pytest

from oracle import adjoint_bessel as AB
from oracle import optics as O
from oracle.adjoint import mse_loss

CIRC = (1 / math.sqrt(2), 1j / math.sqrt(2))
NX, DX = 17, 40.0
Z = np.array([-400.0, 0.0, 350.0])


def _opt(gl=True, fresnel=False):
    g = O.GibsonLanni(n_s=1.33, n_i_design=1.518) if gl else None
    return O.Optics(na=1.4, wavelength=600.0, n_i=1.518, e_inc=CIRC, gl=g,
                    fresnel_media=(1.33, 1.5) if fresnel else ())


def _case(opt, scalar=False, rule="gauss", n_theta=64):
    coeffs = np.zeros(22)
    coeffs[3], coeffs[10], coeffs[21] = 0.06, -0.04, 0.02
    stacks = [(800.0, 5.0, -8.0, -800.0), (2500.0, -12.0, 3.0, -2400.0)]
    _, I0 = AB.forward(opt, NX, NX, DX, DX, Z, coeffs, stacks, n_theta, rule, scalar)
    # scales make s_b I of order one; the target is made at perturbed parameters with
    # noise, so that no gradient component is zero
    s0 = 1.0 / np.max(I0)
    scale = [s0, 1.3 * s0]
    c2 = coeffs.copy()
    c2[3] += 0.03
    _, I1 = AB.forward(opt, NX, NX, DX, DX, Z, c2, stacks, n_theta, rule, scalar)
    rng = np.random.default_rng(9)
    Y = np.array(scale)[:, None, None, None] * I1 * (1 + 0.2 * rng.standard_normal(I1.shape))
    _, g = mse_loss(I0, Y, scale)
    grads = AB.gradient(opt, NX, NX, DX, DX, Z, coeffs, stacks, g, n_theta, rule, scalar)
    return coeffs, stacks, Y, scale, grads


@pytest.mark.parametrize("kind", ["vectorial", "fresnel", "scalar"])
def test_gradient_matches_central_differences(kind):
    opt = _opt(fresnel=kind == "fresnel")
    scalar = kind == "scalar"
    coeffs, stacks, Y, scale, (dc, dts, dzo) = _case(opt, scalar)
    fd = lambda which, h: AB.finite_difference(opt, NX, NX, DX, DX, Z, coeffs, stacks, Y, scale, which, h,
                                                64, "gauss", scalar)
    for i, j in enumerate((4, 11, 22)):
        ref = fd(("c", j), 1e-5)
        assert abs(dc[i + 1] - ref) <= 1e-6 * abs(ref), (j, dc[i + 1], ref)
    for b in range(2):
        ref = fd(("ts", b), 1e-2)
        assert abs(dts[b] - ref) <= 1e-6 * abs(ref), (b, dts[b], ref)
        ref = fd(("zo", b), 1e-2)
        assert abs(dzo[b] - ref) <= 1e-6 * abs(ref), (b, dzo[b], ref)


def test_piston_gradient_vanishes_and_simpson_rule():
    opt = _opt()
    _, _, _, _, (dc, dts, dzo) = _case(opt, rule="simpson", n_theta=65)
    scale = np.max(np.abs(dc[1:]))
    assert scale > 0 and abs(dc[0]) < 1e-10 * scale


def test_depth_gradient_zero_without_sample_layer():
    opt = _opt(gl=False)
    _, _, _, _, (dc, dts, dzo) = _case(opt)
    assert np.all(dts == 0.0)
    assert np.all(np.abs(dzo) > 0)


def test_gibson_lanni_phase_is_linear_in_depth():
    opt = _opt()
    s = np.linspace(0, opt.s_max, 41)
    d = AB.gl_opd_dts(s, opt)
    w1 = O.gibson_lanni_opd(s, opt, 1000.0)
    w2 = O.gibson_lanni_opd(s, opt, 3500.0)
    np.testing.assert_allclose((w2 - w1) / 2500.0, d, rtol=1e-10, atol=1e-12)
