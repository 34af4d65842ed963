"""Pins of the FP64 gradient oracle: central finite differences, global-phase invariants,
and the dot-product test of the transposed DFT chain."""
import math

import numpy as np

from oracle import adjoint as OA
from oracle import fourier as OF
from oracle import optics as O


def _setup(n=24, nx=9, nz=3, n_stacks=2, seed=0):
    opt = O.Optics(na=1.4, wavelength=600.0, n_i=1.518)
    g = OF.pupil_geometry(n, opt)
    rng = np.random.default_rng(seed)
    coeffs = np.zeros(11)
    coeffs[3:] = rng.normal(0, 0.05, 8)
    w0 = rng.normal(0, 0.2, (n, n))
    stacks = [(rng.uniform(-40, 40), rng.uniform(-40, 40), rng.uniform(-200, 200)) for _ in range(n_stacks)]
    z = np.linspace(-400, 400, nz)
    _, I = OA.forward(g, opt, coeffs, w0, stacks, nx, nx, 60.0, 60.0, z)
    Y = rng.poisson(500.0 * I / I.max()).astype(float)
    scale = 500.0 / I.max() * np.array([1.0, 1.3])[:n_stacks]
    return opt, g, coeffs, w0, stacks, z, Y, scale, nx


def test_gradient_matches_central_differences():
    opt, g, coeffs, w0, stacks, z, Y, scale, nx = _setup()
    _, I = OA.forward(g, opt, coeffs, w0, stacks, nx, nx, 60.0, 60.0, z)
    _, dLdI = OA.mse_loss(I, Y, scale)
    dc, dw = OA.gradient(g, opt, coeffs, w0, stacks, nx, nx, 60.0, 60.0, z, dLdI)
    for q in (1, 3, 4, 7, 10):
        fd = OA.finite_difference(g, opt, coeffs, w0, stacks, nx, nx, 60.0, 60.0, z, Y, scale, ("c", q), 1e-6)
        assert abs(fd - dc[q]) < 1e-6 * max(1.0, abs(dc).max()), (q, fd, dc[q])
    cells = [(12, 12), (5, 14), (18, 7), (11, 3)]
    for cell in cells:
        fd = OA.finite_difference(g, opt, coeffs, w0, stacks, nx, nx, 60.0, 60.0, z, Y, scale, ("w", cell), 1e-6)
        assert abs(fd - dw[cell]) < 1e-6 * max(1.0, np.abs(dw).max()), (cell, fd, dw[cell])


def test_gradient_global_phase_invariants():
    # |E|^2 ignores a global phase: zero piston gradient, zero sum of dL/dW0, zero outside the disk
    opt, g, coeffs, w0, stacks, z, Y, scale, nx = _setup(seed=1)
    _, I = OA.forward(g, opt, coeffs, w0, stacks, nx, nx, 60.0, 60.0, z)
    _, dLdI = OA.mse_loss(I, Y, scale)
    dc, dw = OA.gradient(g, opt, coeffs, w0, stacks, nx, nx, 60.0, 60.0, z, dLdI)
    scale_ref = np.abs(dw).max() * dw.size
    assert abs(dc[0]) < 1e-12 * scale_ref
    assert abs(np.sum(dw)) < 1e-12 * scale_ref
    assert np.all(dw[~g["mask"]] == 0.0)


def test_transposed_chain_dot_product():
    # <F p, e> = <p, F^H e> for F p = Ax' p Ay^T and F^H e = Ax'^H e conj(Ay)
    opt = O.Optics(na=1.4, wavelength=600.0, n_i=1.518)
    g = OF.pupil_geometry(20, opt)
    Ax, Ay = OA._tables(g, opt, 11, 13, 45.0, 45.0)
    rng = np.random.default_rng(2)
    p = rng.normal(size=(20, 20)) + 1j * rng.normal(size=(20, 20))
    e = rng.normal(size=(11, 13)) + 1j * rng.normal(size=(11, 13))
    lhs = np.vdot(Ax @ p @ Ay.T, e)
    rhs = np.vdot(p, Ax.conj().T @ e @ Ay.conj())
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_gradient_forward_matches_fourier_oracle():
    # the forward used for gradients is the pinned Cartesian form
    opt, g, coeffs, w0, stacks, z, Y, scale, nx = _setup(seed=3)
    E, _ = OA.forward(g, opt, coeffs, w0, stacks, nx, nx, 60.0, 60.0, z)
    x0, y0, zo = stacks[1]
    P = OF.base_pupil(g, opt, OF.pupil_phase(g, opt, zernike=coeffs, phase_map=w0))
    ref = OF.field_separable(P, g, opt, nx, nx, 60.0, 60.0, z + zo, x0=x0, y0=y0)
    np.testing.assert_allclose(E[1], ref, rtol=0, atol=1e-13 * np.abs(ref).max())
