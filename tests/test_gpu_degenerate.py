"""Degenerate and extreme sizes on the GPU against the FP64 oracle: the smallest pupil
(2 x 2), one-pixel and one-row images, a single plane, the fewest theta nodes and radial
samples, many stacks per call across the internal chunk boundaries, and the largest
chirp-z transform length."""
import numpy as np
import pytest

import workloads as W
from oracle import bessel as OB
from oracle import fourier as OF
from oracle import optics as O
from tests.helpers import rel_l2

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _np(t):
    return t.detach().cpu().numpy()


def _cart(rw, form, n_pupil, nx, ny, z, model=0, **kw):
    return rw.Plan(form=form, na=1.2, wavelength=532.0, n_i=1.518, nx=nx, ny=ny, dx=30.0, dy=25.0, z=z,
                   e_inc=W.CIRCULAR, n_pupil=n_pupil, model=model, **kw)


def _oracle_cart(n_pupil, nx, ny, z, scalar=False, zern=None, x0=0.0, y0=0.0):
    opt = O.Optics(na=1.2, wavelength=532.0, n_i=1.518, e_inc=W.CIRCULAR)
    g = OF.pupil_geometry(n_pupil, opt)
    P = OF.base_pupil(g, opt, OF.pupil_phase(g, opt, zernike=zern), scalar=scalar)
    return OF.field_separable(P, g, opt, nx, ny, 30.0, 25.0, z, x0=x0, y0=y0)


@pytest.mark.parametrize("form", ["fourier", "chirpz"])
@pytest.mark.parametrize("n_pupil,nx,ny", [(2, 1, 1), (3, 5, 1), (2, 1, 7), (5, 2, 3)])
@pytest.mark.parametrize("scalar", [False, True])
def test_cartesian_tiny_grids(lib, form, n_pupil, nx, ny, scalar):
    import torch
    rw = lib
    f = rw.FORM_FOURIER if form == "fourier" else rw.FORM_CHIRPZ
    z = [250.0]
    p = _cart(rw, f, n_pupil, nx, ny, z, model=rw.MODEL_SCALAR if scalar else rw.MODEL_VECTORIAL)
    zern = [0.0, 0.0, 0.0, 0.1, 0.05]
    E, I = p.compute([dict(zernike=zern, x0=3.0, y0=-4.0)])
    torch.cuda.synchronize()
    ref = _oracle_cart(n_pupil, nx, ny, z, scalar, zern, 3.0, -4.0)
    assert rel_l2(_np(E[0]), ref) < TOL
    assert rel_l2(_np(I[0]), OF.intensity(ref)) < TOL


def test_fourier_many_stacks_across_chunks(lib):
    # 37 stacks: two full 16-stack GEMM groups and a ragged one, pupils built 8 at a time
    import torch
    rw = lib
    z = [-300.0, 200.0]
    p = _cart(rw, rw.FORM_FOURIER, 24, 9, 11, z)
    rng = np.random.default_rng(12)
    zs = [[0.0, 0.0, 0.0] + list(rng.normal(0, 0.05, 3)) for _ in range(37)]
    offs = rng.uniform(-300, 300, 37)
    st = [dict(zernike=zs[b], z_offset=float(offs[b])) for b in range(37)]
    E, I = p.compute(st)
    torch.cuda.synchronize()
    for b in (0, 7, 8, 15, 16, 31, 32, 36):
        ref = _oracle_cart(24, 9, 11, np.array(z) + offs[b], zern=zs[b])
        assert rel_l2(_np(E[b]), ref) < TOL, b
        assert rel_l2(_np(I[b]), OF.intensity(ref)) < TOL, b


@pytest.mark.parametrize("rule,n_theta", [(0, 2), (1, 3), (2, 2)])
def test_bessel_fewest_nodes_and_samples(lib, rule, n_theta):
    import torch
    rw = lib
    z = [0.0, 300.0]
    p = rw.Plan(form=rw.FORM_BESSEL, na=1.2, wavelength=532.0, n_i=1.518, nx=3, ny=2, dx=30.0, dy=30.0, z=z,
                e_inc=W.CIRCULAR, n_theta=n_theta, n_rho=8, theta_rule=rule)
    E, I = p.compute([dict(x0=5.0)])
    torch.cuda.synchronize()
    opt = O.Optics(na=1.2, wavelength=532.0, n_i=1.518, e_inc=W.CIRCULAR)
    name = {0: "gauss", 1: "simpson", 2: "riemann"}[rule]
    ref = OB.field_bessel(opt, 3, 2, 30.0, 30.0, z, x0=5.0, n_theta=n_theta, rule=name)
    # 8 radial samples over a 3 x 2 image (17 nm apart): the 4-point radial interpolation
    # error (k s_max drho = 0.24 rad per sample) dominates the comparison here
    assert rel_l2(_np(E[0]), ref) < 1e-3
    assert rel_l2(_np(I[0]), OF.intensity(ref)) < 1e-3


def test_chirpz_longest_transform(lib):
    # N + max(nx, ny) - 1 = 2048: the largest FFT length along both axes (one plane)
    import torch
    rw = lib
    z = [400.0]
    p = _cart(rw, rw.FORM_CHIRPZ, 1024, 1025, 16, z)
    E, I = p.compute([dict(zernike=[0, 0, 0, 0.05])])
    torch.cuda.synchronize()
    ref = _oracle_cart(1024, 1025, 16, z, zern=[0, 0, 0, 0.05])
    assert rel_l2(_np(E[0]), ref) < TOL


@pytest.mark.parametrize("nx,ny,n_rho,n_theta,mode", [(3, 2, 8, 2, "vectorial"), (9, 9, 8, 64, "scalar"),
                                                      (41, 1, 256, 4096, "vectorial"),
                                                      (17, 23, 256, 4096, "fresnel")])
def test_bessel_single_launch_edges_match_chunked_path(lib, nx, ny, n_rho, n_theta, mode):
    """The single-stack launch at its edges: the fewest radial samples (8, so at most six
    bands), two nodes, one-pixel rows, 4096 nodes (the Fresnel case does not fit its LDS
    and takes the three launches) -- against the same stack twice in one call (the three
    launches), and that call against the oracle where 256 radial samples make the radial
    interpolation exact to FP32."""
    import torch
    rw = lib
    z = [-250.0, 0.0, 400.0]
    fres = (W.GIBSON_LANNI["n_s"], W.GIBSON_LANNI["n_g"]) if mode == "fresnel" else None
    p = rw.Plan(form=rw.FORM_BESSEL, na=1.3, wavelength=532.0, n_i=1.518, nx=nx, ny=ny, dx=30.0, dy=30.0, z=z,
                e_inc=W.X_LINEAR, n_theta=n_theta, n_rho=n_rho,
                model=rw.MODEL_SCALAR if mode == "scalar" else rw.MODEL_VECTORIAL, fresnel=fres)
    s = dict(x0=7.0, y0=-4.0, z_offset=30.0, zernike=[0, 0, 0, 0.04])
    E1, I1 = p.compute([s])
    E2, I2 = p.compute([s, s])
    torch.cuda.synchronize()
    # the two paths sum the nodes in different orders in FP32: about sqrt(T) ulp apart
    # (measured 1.04e-6 at 4096 nodes)
    cross = 1e-6 if n_theta <= 256 else 1e-5
    for b in range(2):
        assert rel_l2(_np(E1[0]), _np(E2[b])) < cross
        assert rel_l2(_np(I1[0]), _np(I2[b])) < cross
    if n_rho == 8:
        return   # the radial interpolation error dominates there (the test above bounds it)
    opt = O.Optics(na=1.3, wavelength=532.0, n_i=1.518, e_inc=W.X_LINEAR, fresnel_media=fres or ())
    ref = OB.field_bessel(opt, nx, ny, 30.0, 30.0, np.array(z) + 30.0, x0=7.0, y0=-4.0, n_theta=n_theta,
                          zernike=[0, 0, 0, 0.04], scalar=mode == "scalar")
    assert rel_l2(_np(E2[0]), ref) < TOL
    assert rel_l2(_np(I2[0]), OF.intensity(ref)) < TOL
