"""Writes the stored expected values of tests/golden/ from the FP64 oracle only.

    python tests/golden/make_golden.py

* airy_line.txt     -- Sec. 5.2.2: the scalar spherical field with the extra s_z factor
                       (Simpson's rule, 65 nodes) on a 41-pixel line at 20 nm, NA 1.4,
                       532 nm, n_i 1.518, no apodization, next to the closed form
                       -(i f k s_max^2 / 2) 2 J1(v)/v of the paper's Airy comparison.
* fresnel_q.txt     -- Sec. 3.3: the Fresnel products q_s, q_p for sample 1.33 ->
                       coverslip 1.52 -> immersion 1.518 at 9 immersion angles (beyond the
                       sample's critical angle they are complex).
* psf_vectorial.txt -- Sec. 3.3 eq. "cartesian vectorial": the vectorial field of a 16 x 16
                       pupil (NA 1.2, 532 nm, n_i 1.518, circular, apodization, Noll 4 and 11)
                       on 9 x 9 pixels at 40 nm and two planes, component by component.
Each file holds one value per line (real and imaginary parts), preceded by '#' comments.
"""
import math
import os
import sys

import numpy as np
from scipy.special import j1

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import bessel as OB  # noqa: E402
from oracle import fourier as OF  # noqa: E402
from oracle import optics as O  # noqa: E402


def airy_line():
    opt = O.Optics(na=1.4, wavelength=532.0, n_i=1.518, apodization=False)
    rho = np.abs(O.output_axis(41, 20.0))
    (I0,) = OB.bessel_integrals(rho, [0.0], opt, 65, scalar=True, extra_cos=True, rule="simpson")
    E = -1j * opt.f * opt.k * I0[0]
    v = opt.k * opt.s_max * rho
    safe = np.where(v > 0, v, 1.0)
    ref = -1j * opt.f * opt.k * opt.s_max ** 2 / 2 * np.where(v > 0, 2 * j1(safe) / safe, 1.0)
    return E, ref


def fresnel_q():
    opt = O.Optics(na=1.45, wavelength=532.0, n_i=1.518, fresnel_media=(1.33, 1.52))
    s = np.linspace(0.0, opt.s_max, 9)
    return O.fresnel_q(s, opt)


def psf_vectorial():
    opt = O.Optics(na=1.2, wavelength=532.0, n_i=1.518)
    g = OF.pupil_geometry(16, opt)
    zern = np.zeros(11)
    zern[3], zern[10] = 0.07, -0.03
    P = OF.base_pupil(g, opt, OF.pupil_phase(g, opt, zernike=zern))
    return OF.field_separable(P, g, opt, 9, 9, 40.0, 40.0, [-250.0, 300.0])


def write(name, header, arrays):
    with open(os.path.join(HERE, name), "w") as f:
        for line in header:
            f.write(f"# {line}\n")
        for a in arrays:
            for v in np.asarray(a).ravel():
                f.write(f"{v.real:.17e} {v.imag:.17e}\n")


if __name__ == "__main__":
    E, ref = airy_line()
    write("airy_line.txt", ["Sec. 5.2.2: 41 oracle values (Simpson, 65 nodes), then 41 closed-form values"], [E, ref])
    qs, qp = fresnel_q()
    write("fresnel_q.txt", ["Sec. 3.3: q_s at 9 angles, then q_p"], [qs, qp])
    write("psf_vectorial.txt", ["Sec. 3.3: E[z][c][x][y], 2 x 3 x 9 x 9"], [psf_vectorial()])
