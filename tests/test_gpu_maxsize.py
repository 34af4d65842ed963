"""The largest sizes the interfaces accept, against the FP64 oracle on sampled planes: the
1024 x 1024 pupil of the matrix-DFT form with more planes than its plane workspace holds
(so the planes of one stack run in several slabs), and one batched emitter with the
largest crop and plane count."""
import numpy as np
import pytest

import workloads as W
from oracle import fourier as OF
from oracle import optics as O
from tests.helpers import oracle_fourier_stack, oracle_optics, rel_l2

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _np(t):
    return t.detach().cpu().numpy()


def test_fourier_largest_pupil_in_plane_slabs(lib):
    import torch
    rw = lib
    n, nx, nz = 1024, 256, 200   # 3 x 1024 x 256 x 8 B per plane: the 1 GiB workspace holds 170 planes
    z = np.linspace(-1500.0, 1500.0, nz)
    p = rw.Plan(form=rw.FORM_FOURIER, na=1.4, wavelength=600.0, n_i=1.518, nx=nx, ny=nx, dx=25.0, dy=25.0, z=z,
                e_inc=W.CIRCULAR, n_pupil=n)
    zern = [0, 0, 0, 0.03, -0.02, 0.01]
    E, I = p.compute([dict(zernike=zern, x0=7.0)])
    torch.cuda.synchronize()
    opt = O.Optics(na=1.4, wavelength=600.0, n_i=1.518, e_inc=W.CIRCULAR)
    for zi in (0, 169, 170, 199):
        ref = oracle_fourier_stack(opt, n, nx, nx, 25.0, 25.0, [z[zi]], zernike=zern, x0=7.0)
        assert rel_l2(_np(E[0, zi]), ref[0]) < TOL, zi
        assert rel_l2(_np(I[0, zi]), OF.intensity(ref)[0]) < TOL, zi


def test_batched_largest_crop_and_plane_count(lib):
    import torch
    rw = lib
    w = W.batched(n_emitters=2, seed=34)
    o = w["optics"]
    b = rw.Batch(na=o["na"], wavelength=o["wavelength"], n_i=o["n_i"], pixel=w["dx"], plane_pitch=2.0,
                 max_emitters=2, n_pupil=w["n_pupil"], e_inc=w["e_inc"])
    em = rw.make_emitters(w["x0"][:2], w["y0"][:2], w["z_e"][:2], [64, 24], [4096, 1], w["zernike"][:2])
    off = rw.batch_offsets(em)
    I = torch.zeros(off[-1], dtype=torch.float32, device="cuda")
    b.compute(em, I=I)
    torch.cuda.synchronize()
    got = I[:off[1]].cpu().numpy().reshape(4096, 64, 64)
    opt = oracle_optics(w, gl=False)
    for d in (0, 2047, 4095):
        zd = (d - 0.5 * 4095) * 2.0 - w["z_e"][0]
        ref = oracle_fourier_stack(opt, w["n_pupil"], 64, 64, w["dx"], w["dx"], [zd], zernike=w["zernike"][0],
                                   x0=w["x0"][0], y0=w["y0"][0])
        assert rel_l2(got[d], OF.intensity(ref)[0]) < TOL, d
