"""Builds the oracle's and the HIP path's inputs from one workload description."""
from __future__ import annotations

import numpy as np

from oracle import fourier as OF
from oracle import optics as O


def oracle_optics(w, e_inc=None, gl=True):
    o = w["optics"]
    g = None
    if gl and w.get("gl"):
        d = w["gl"]
        g = O.GibsonLanni(n_s=d["n_s"], n_g=d["n_g"], n_g_design=d["n_g_design"],
                          n_i_design=d["n_i_design"], t_g=d["t_g"], t_g_design=d["t_g_design"],
                          t_i_design=d["t_i_design"])
    return O.Optics(na=o["na"], wavelength=o["wavelength"], n_i=o["n_i"],
                    e_inc=e_inc if e_inc is not None else w["e_inc"], gl=g)


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def oracle_fourier_stack(opt, n_pupil, nx, ny, dx, dy, z, zernike=None, phase_map=None, t_s=0.0,
                         x0=0.0, y0=0.0):
    g = OF.pupil_geometry(n_pupil, opt)
    P = OF.base_pupil(g, opt, OF.pupil_phase(g, opt, zernike=zernike, phase_map=phase_map, t_s=t_s))
    return OF.field_separable(P, g, opt, nx, ny, dx, dy, z, x0=x0, y0=y0)
