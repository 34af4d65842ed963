"""Gradient of a stack loss through the Cartesian form, FP64 oracle (test infrastructure only).

The forward model is the discrete Cartesian form of ``oracle.fourier`` (Sec. 3.3
eq. "cartesian vectorial" with the Sec. 3.4 correction factors): for stack b,
plane z and component c,

    E = Ax' (P~) Ay^T,  P~[j,l] = Q_c[j,l] exp(i Phi_b[j,l]) exp(i k s_z z),
    Ax'[m,j] = C exp(i k s_x[j] x_m),  Ay[n,l] = exp(i k s_y[l] y_n),  C = -i f k / 2 pi,
    Phi_b = 2 pi sum_q c_q Z_q + W0 - k (s_x x0_b + s_y y0_b),
    I = sum_c |E_c|^2.

For a real loss L(I) with g = dL/dI (per voxel), dL = sum g 2 Re(conj(E) dE), and
dE = Ax' (i P~ dPhi) Ay^T, so

    dL/dPhi[j,l] = sum_{b,z,c} Im( G[j,l] conj(P~[j,l]) ),
    G = Ax'^H (2 g E) conj(Ay)          (the transposed chain)
    dL/dW0 = dL/dPhi,   dL/dc_q = 2 pi sum_{j,l} dL/dPhi[j,l] Z_q[j,l].

The coefficients c and the map W0 are shared by all stacks (a pupil mask seen
through many emitters); each stack has its own lateral position and defocus.
"""
from __future__ import annotations

import math

import numpy as np

from . import fourier as OF
from . import optics as O


def _tables(geom, opt, nx, ny, dx, dy):
    k = opt.k
    xs = O.output_axis(nx, dx)
    ys = O.output_axis(ny, dy)
    Ax = OF.prefactor(opt) * np.exp(1j * k * np.outer(xs, geom["sx"][:, 0]))
    Ay = np.exp(1j * k * np.outer(ys, geom["sy"][0, :]))
    return Ax, Ay


def phase(geom, opt, coeffs, w0, x0=0.0, y0=0.0):
    ph = np.zeros(geom["sx"].shape)
    for q, c in enumerate(np.asarray(coeffs, dtype=np.float64), start=1):
        if c != 0.0:
            ph = ph + 2 * math.pi * c * O.zernike_noll(q, geom["r"], geom["phi"])
    if w0 is not None:
        ph = ph + np.asarray(w0, dtype=np.float64)
    return ph - opt.k * (geom["sx"] * x0 + geom["sy"] * y0)


def forward(geom, opt, coeffs, w0, stacks, nx, ny, dx, dy, z):
    """Fields (B, Z, 3, nx, ny) and intensity (B, Z, nx, ny); stacks = [(x0, y0, z_offset)]."""
    base = OF.base_pupil(geom, opt)                      # Q_c = ds^2 a e_inf,c / s_z
    Ax, Ay = _tables(geom, opt, nx, ny, dx, dy)
    sz = np.where(geom["mask"], geom["sz"], 0.0)
    z = np.asarray(z, dtype=np.float64)
    E = np.empty((len(stacks), z.size, 3, nx, ny), dtype=np.complex128)
    for b, (x0, y0, zo) in enumerate(stacks):
        P = base * np.exp(1j * phase(geom, opt, coeffs, w0, x0, y0))[None]
        for iz, zz in enumerate(z + zo):
            D = np.exp(1j * opt.k * sz * zz)
            for c in range(3):
                E[b, iz, c] = Ax @ (P[c] * D) @ Ay.T
    return E, np.sum(np.abs(E) ** 2, axis=2)


def gradient(geom, opt, coeffs, w0, stacks, nx, ny, dx, dy, z, dL_dI, n_coeffs=None):
    """Analytic (dL/dc, dL/dW0) for a loss with per-voxel dL/dI, by the transposed chain."""
    base = OF.base_pupil(geom, opt)
    Ax, Ay = _tables(geom, opt, nx, ny, dx, dy)
    sz = np.where(geom["mask"], geom["sz"], 0.0)
    z = np.asarray(z, dtype=np.float64)
    E, _ = forward(geom, opt, coeffs, w0, stacks, nx, ny, dx, dy, z)
    dphi = np.zeros(geom["sx"].shape)
    AxH = Ax.conj().T
    AyC = Ay.conj()
    for b, (x0, y0, zo) in enumerate(stacks):
        P = base * np.exp(1j * phase(geom, opt, coeffs, w0, x0, y0))[None]
        for iz, zz in enumerate(z + zo):
            D = np.exp(1j * opt.k * sz * zz)
            for c in range(3):
                Ebar = 2.0 * dL_dI[b, iz] * E[b, iz, c]
                G = AxH @ Ebar @ AyC
                dphi += np.imag(G * np.conj(P[c] * D))
    nq = len(coeffs) if n_coeffs is None else n_coeffs
    dc = np.array([2 * math.pi * np.sum(dphi * O.zernike_noll(q, geom["r"], geom["phi"]) * geom["mask"])
                   for q in range(1, nq + 1)])
    return dc, np.where(geom["mask"], dphi, 0.0)


def mse_loss(I, Y, scale):
    """L = mean over voxels of (s_b I - Y)^2 and its dL/dI."""
    s = np.asarray(scale, dtype=np.float64).reshape(-1, *([1] * (I.ndim - 1)))
    r = s * I - Y
    nv = I.size
    return float(np.sum(r * r) / nv), 2.0 * s * r / nv


def finite_difference(geom, opt, coeffs, w0, stacks, nx, ny, dx, dy, z, Y, scale, which, h):
    """Central difference of mse_loss w.r.t. one coefficient ('c', q) or one map cell ('w', (j, l))."""
    def loss(cv, wv):
        _, I = forward(geom, opt, cv, wv, stacks, nx, ny, dx, dy, z)
        return mse_loss(I, Y, scale)[0]

    kind, idx = which
    cp, cm = np.array(coeffs, dtype=np.float64), np.array(coeffs, dtype=np.float64)
    wp, wm = np.array(w0, dtype=np.float64), np.array(w0, dtype=np.float64)
    if kind == "c":
        cp[idx] += h
        cm[idx] -= h
    else:
        wp[idx] += h
        wm[idx] -= h
    return (loss(cp, wp) - loss(cm, wm)) / (2 * h)
