"""Gradient of a stack loss through the spherical (Bessel) form, FP64 oracle.

Test infrastructure only.  The forward model is ``oracle.bessel.field_bessel`` (Sec. 3.3
eq. "polar vectorial final" with the integrals of eq. "I0", or eq. "polar scalar final"
for the scalar model, with the Sec. 3.4 correction factors).  For stack b, plane z and
pixel p at radius rho_p and azimuth v_p from the emitter:

    I_n[z, p] = sum_q Phi_b[q, z] K_n[p, q]
    Phi_b[q, z] = a(t_q) exp(i W_b(t_q)) exp(i k (z + zo_b) cos t_q)
    K_n[p, q] = w_q g_n(t_q) J_n(k rho_p sin t_q)   (g_n carries q_s, q_p with Fresnel factors)
    E_c[z, p] = sum_n C_cn(v_p) I_n[z, p]
    W_b(t) = W_GL(t; t_s,b) + 2 pi sum_j c_j Z_j(sin t / s_max)   (axisymmetric Noll terms)

For a real loss L(I) with g = dL/dI per voxel, dL = sum 2 g Re(conj(E) dE).  With the
complex-linear maps above the gradient is pulled back by their adjoints:

    G_E = 2 g E,   G_In[z, p] = sum_c conj(C_cn(v_p)) G_E,c[z, p],
    G_Phi[q, z] = sum_{n, p} conj(K_n[p, q]) G_In[z, p],
    X_b[q] = sum_z conj(G_Phi[q, z]) Phi_b[q, z],

and a parameter theta that enters as dPhi = i (dW/dtheta) Phi gives
dL/dtheta = sum_q Re(i dW/dtheta(t_q) X_b[q]), with dW/dc_j = 2 pi Z_j, dW/dt_s the
derivative of the Gibson-Lanni OPD (complex beyond a critical angle) and dW/dzo = k cos t.
The coefficients c are shared by all stacks (their gradient is summed over stacks); the
depth t_s and axial offset zo are per stack.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special

from . import bessel as OB
from . import optics as O
from .adjoint import mse_loss

AXISYMMETRIC_NOLL = (1, 4, 11, 22)


def forward(opt: O.Optics, nx, ny, dx, dy, z, coeffs, stacks, n_theta=200, rule="gauss", scalar=False):
    """Fields (B, Z, C, nx, ny) and intensity (B, Z, nx, ny); stacks = [(t_s, x0, y0, zo)]."""
    z = np.asarray(z, dtype=np.float64)
    E = np.stack([OB.field_bessel(opt, nx, ny, dx, dy, z + zo, x0=x0, y0=y0, n_theta=n_theta,
                                  zernike=coeffs, t_s=ts, rule=rule, scalar=scalar)
                  for (ts, x0, y0, zo) in stacks])
    return E, np.sum(np.abs(E) ** 2, axis=2)


def gl_opd_dts(sin_t, opt: O.Optics):
    """d W_GL / d t_s for the printed focusing relation t_i = t_s + n_i (-t_s/n_s - ...):
    k0 (sqrt(n_s^2 - n_i^2 sin^2 t) + (1 - n_i / n_s) sqrt(n_i^2 - n_i^2 sin^2 t))."""
    gl = opt.gl
    s2 = (opt.n_i * np.asarray(sin_t, dtype=np.float64)) ** 2
    root = lambda n: np.sqrt((n * n - s2).astype(np.complex128))
    k0 = 2.0 * math.pi / opt.wavelength
    return k0 * (root(gl.n_s) + (1.0 - opt.n_i / gl.n_s) * root(opt.n_i))


def gradient(opt: O.Optics, nx, ny, dx, dy, z, coeffs, stacks, dL_dI, n_theta=200, rule="gauss",
             scalar=False):
    """Analytic (dL/dc for Noll 1, 4, 11, 22; dL/dt_s per stack; dL/dzo per stack)."""
    z = np.asarray(z, dtype=np.float64)
    E, _ = forward(opt, nx, ny, dx, dy, z, coeffs, stacks, n_theta, rule, scalar)
    t, w = OB.theta_rule(opt, n_theta, rule=rule)
    sin_t, cos_t = np.sin(t), np.cos(t)
    k = opt.k
    amp = O.amplitude(cos_t, sin_t, opt)
    if scalar:
        g = [sin_t]
        pref = -1j * opt.f * k
    else:
        qs, qp = O.fresnel_q(sin_t, opt)
        g = [sin_t * (qs + qp * cos_t), qp * sin_t ** 2, sin_t * (qp * cos_t - qs)]
        pref = -1j * opt.f * k / 2.0
    zern_t = {j: O.zernike_noll(j, sin_t / opt.s_max, 0.0) for j in AXISYMMETRIC_NOLL}
    dwdts = gl_opd_dts(sin_t, opt) if opt.gl is not None else np.zeros_like(sin_t)
    dc = np.zeros(len(AXISYMMETRIC_NOLL))
    dts = np.zeros(len(stacks))
    dzo = np.zeros(len(stacks))
    for b, (ts, x0, y0, zo) in enumerate(stacks):
        xs = O.output_axis(nx, dx, x0)
        ys = O.output_axis(ny, dy, y0)
        X, Y = np.meshgrid(xs, ys, indexing="ij")
        rho = np.hypot(X, Y).ravel()
        v = np.arctan2(Y, X).ravel()
        c1, s1, c2, s2 = np.cos(v), np.sin(v), np.cos(2 * v), np.sin(2 * v)
        # pupil x defocus on the nodes, as in the forward model
        W = OB._axisymmetric_phase(sin_t, opt, coeffs, ts)
        Phi = (amp * np.exp(1j * W))[:, None] * np.exp(1j * k * np.outer(cos_t, z + zo))   # (T, Z)
        K = [special.jv(n, k * np.outer(rho, sin_t)) * (w * gn)[None, :] for n, gn in enumerate(g)]
        GE = 2.0 * dL_dI[b][:, None] * E[b]                                            # (Z, C, nx, ny)
        GE = GE.reshape(GE.shape[0], GE.shape[1], -1)
        if scalar:
            GIn = [np.conj(pref) * GE[:, 0]]
        else:
            ex, ey = pref * opt.e_inc[0], pref * opt.e_inc[1]
            Cx = (ex, 0.0, -(ex * c2 + ey * s2))
            Cy = (ey, 0.0, -ex * s2 + ey * c2)
            Cz = (0.0, -2j * (ex * c1 + ey * s1), 0.0)
            GIn = [np.conj(Cx[n]) * GE[:, 0] + np.conj(Cy[n]) * GE[:, 1] + np.conj(Cz[n]) * GE[:, 2]
                   for n in range(3)]
        GPhi = sum(np.conj(K[n]).T @ GIn[n].T for n in range(len(g)))                  # (T, Z)
        Xb = np.sum(np.conj(GPhi) * Phi, axis=1)                                        # (T,)
        for i, j in enumerate(AXISYMMETRIC_NOLL):
            dc[i] += np.sum(np.real(1j * 2 * math.pi * zern_t[j] * Xb))
        dts[b] = np.sum(np.real(1j * dwdts * Xb))
        dzo[b] = np.sum(np.real(1j * k * cos_t * Xb))
    return dc, dts, dzo


def finite_difference(opt: O.Optics, nx, ny, dx, dy, z, coeffs, stacks, Y, scale, which, h,
                      n_theta=200, rule="gauss", scalar=False):
    """Central difference of mse_loss w.r.t. ('c', Noll j), ('ts', b) or ('zo', b)."""
    def loss(cv, sv):
        _, I = forward(opt, nx, ny, dx, dy, z, cv, sv, n_theta, rule, scalar)
        return mse_loss(I, Y, scale)[0]

    kind, idx = which
    cp = np.array(coeffs, dtype=np.float64)
    cm = np.array(coeffs, dtype=np.float64)
    sp = [list(s) for s in stacks]
    sm = [list(s) for s in stacks]
    if kind == "c":
        cp[idx - 1] += h
        cm[idx - 1] -= h
    else:
        col = 0 if kind == "ts" else 3
        sp[idx][col] += h
        sm[idx][col] -= h
    return (loss(cp, sp) - loss(cm, sm)) / (2 * h)
