"""Parity of the HIP path with the FP64 oracle (rel-L2 <= 1e-5 for FP32 fields and intensity)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import bessel as OB
from oracle import fourier as OF
from oracle import optics as O
from tests.helpers import oracle_fourier_stack, oracle_optics, rel_l2

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _np(t):
    return t.detach().cpu().numpy()


# ----------------------------------------------------------------------------- Fourier
def _fourier_plan(rw, w, n_pupil, nx, ny, dx, z, gl=True):
    o = w["optics"]
    return rw.Plan(form=rw.FORM_FOURIER, na=o["na"], wavelength=o["wavelength"], n_i=o["n_i"], nx=nx,
                   ny=ny, dx=dx, dy=dx, z=z, e_inc=w["e_inc"], gibson_lanni=w["gl"] if gl else None,
                   n_pupil=n_pupil)


@pytest.mark.parametrize("n_pupil,nx,ny", [(40, 33, 29), (37, 20, 70), (130, 65, 131), (48, 200, 150), (40, 90, 40)])
def test_fourier_small_all_corrections(lib, n_pupil, nx, ny):
    import torch
    rw = lib
    w = W.fourier_plain(n_stacks=3, seed=11)
    zp = np.linspace(-600.0, 900.0, 5)
    rng = np.random.default_rng(2)
    maps = [rng.normal(0, 0.3, (n_pupil, n_pupil)) for _ in range(3)]
    plan = _fourier_plan(rw, w, n_pupil, nx, ny, 25.0, zp)
    stacks = []
    for b in range(3):
        stacks.append(dict(t_s=w["t_s"][b] / 3, x0=[0.0, 13.0, -31.0][b], y0=[0.0, -7.0, 44.0][b],
                           z_offset=-w["t_s"][b] / 3, zernike=w["zernike"][b],
                           phase_map=torch.tensor(maps[b], dtype=torch.float32, device="cuda")))
    E, I = plan.compute(stacks)
    torch.cuda.synchronize()
    opt = oracle_optics(w)
    for b in range(3):
        ref = oracle_fourier_stack(opt, n_pupil, nx, ny, 25.0, 25.0, zp - w["t_s"][b] / 3,
                                   zernike=w["zernike"][b], phase_map=maps[b].astype(np.float32),
                                   t_s=w["t_s"][b] / 3, x0=stacks[b]["x0"], y0=stacks[b]["y0"])
        assert rel_l2(_np(E[b]), ref) < TOL
        assert rel_l2(_np(I[b]), OF.intensity(ref)) < TOL


def test_fourier_many_stacks_span_chunks(lib):
    """70 stacks in one call: more than one chunk of the stacks-per-launch limit and more
    than one pupil launch per chunk; sampled stacks against the oracle, and each stack's
    intensity against the same stack computed alone."""
    import torch
    rw = lib
    w = W.fourier_plain(n_stacks=1, seed=13)
    zp = np.linspace(-500.0, 500.0, 3)
    plan = _fourier_plan(rw, w, 32, 24, 24, 40.0, zp, gl=False)
    rng = np.random.default_rng(14)
    coef = rng.normal(0.0, 0.05, (70, 21))
    stacks = [dict(zernike=coef[b], x0=float(rng.uniform(-30, 30)), z_offset=float(rng.uniform(-100, 100)))
              for b in range(70)]
    E, I = plan.compute(stacks)
    torch.cuda.synchronize()
    opt = oracle_optics(w, gl=False)
    for b in (0, 7, 8, 63, 64, 69):
        ref = oracle_fourier_stack(opt, 32, 24, 24, 40.0, 40.0, zp + stacks[b]["z_offset"], zernike=coef[b],
                                   x0=stacks[b]["x0"])
        assert rel_l2(_np(E[b]), ref) < TOL, b
        assert rel_l2(_np(I[b]), OF.intensity(ref)) < TOL, b
    for b in (5, 66):
        _, I1 = plan.compute([stacks[b]], fields=False)
        torch.cuda.synchronize()
        assert rel_l2(_np(I1[0]), _np(I[b])) < 1e-6, b


def test_fourier_outputs_optional_and_single_plane(lib):
    import torch
    rw = lib
    w = W.fourier_plain(n_stacks=1, seed=12)
    plan = _fourier_plan(rw, w, 64, 17, 17, 30.0, [150.0], gl=False)
    st = [dict(zernike=w["zernike"][0])]
    E, _ = plan.compute(st, intensity=False)
    _, I = plan.compute(st, fields=False)
    torch.cuda.synchronize()
    ref = oracle_fourier_stack(oracle_optics(w, gl=False), 64, 17, 17, 30.0, 30.0, [150.0],
                               zernike=w["zernike"][0])
    assert rel_l2(_np(E[0]), ref) < TOL
    assert rel_l2(_np(I[0]), OF.intensity(ref)) < TOL


def test_fourier_full_config_batch16(lib):
    """256 x 256 pupil -> 128 x 128 x 64, 16 stacks in one call (the benchmark launch)."""
    import torch
    rw = lib
    w = W.fourier_plain()
    zp = np.linspace(-1000.0, 1000.0, 64)
    plan = _fourier_plan(rw, w, 256, 128, 128, 20.0, zp)
    stacks = [dict(t_s=w["t_s"][b], z_offset=-w["t_s"][b], zernike=w["zernike"][b]) for b in range(16)]
    E, I = plan.compute(stacks)
    torch.cuda.synchronize()
    E = _np(E)
    I = _np(I)
    opt = oracle_optics(w)
    # two whole stacks through the separable oracle
    for b in (0, 9):
        ref = oracle_fourier_stack(opt, 256, 128, 128, 20.0, 20.0, w["z"][b], zernike=w["zernike"][b],
                                   t_s=w["t_s"][b])
        assert rel_l2(E[b], ref) < TOL
        assert rel_l2(I[b], OF.intensity(ref)) < TOL
    # every stack: 64 seeded voxels by the brute-force double sum
    rng = np.random.default_rng(99)
    g = OF.pupil_geometry(256, opt)
    xs = O.output_axis(128, 20.0)
    for b in range(16):
        P = OF.base_pupil(g, opt, OF.pupil_phase(g, opt, zernike=w["zernike"][b], t_s=w["t_s"][b]))
        iz, ix, iy = rng.integers(0, 64, 64), rng.integers(0, 128, 64), rng.integers(0, 128, 64)
        pts = np.stack([xs[ix], xs[iy], w["z"][b][iz]], 1)
        ref = OF.field_direct(P, g, opt, pts)                 # (3, 64)
        got = E[b][iz, :, ix, iy].T
        assert rel_l2(got, ref) < TOL


# ------------------------------------------------------------------------------ Bessel
def _bessel_plan(rw, w, nx=65, z=None, n_theta=200, n_rho=256, e_inc=None, gl=None, dx=20.0):
    o = w["optics"]
    return rw.Plan(form=rw.FORM_BESSEL, na=o["na"], wavelength=o["wavelength"], n_i=o["n_i"], nx=nx,
                   ny=nx, dx=dx, dy=dx, z=w["z"] if z is None else z,
                   e_inc=e_inc if e_inc is not None else w["e_inc"], gibson_lanni=gl,
                   n_theta=n_theta, n_rho=n_rho)


def test_bessel_full_config(lib):
    """65 x 65 x 33, GL-200 theta rule, 256 radial samples, vs the oracle at exact radii."""
    import torch
    rw = lib
    w = W.bessel_plain()
    plan = _bessel_plan(rw, w)
    E, I = plan.compute([dict()])
    torch.cuda.synchronize()
    opt = O.Optics(na=1.4, wavelength=532.0, n_i=1.518, e_inc=w["e_inc"])
    ref = OB.field_bessel(opt, 65, 65, 20.0, 20.0, w["z"], n_theta=256)
    assert rel_l2(_np(E[0]), ref) < TOL
    assert rel_l2(_np(I[0]), OF.intensity(ref)) < TOL


@pytest.mark.parametrize("e_inc", [W.CIRCULAR, W.X_LINEAR])
def test_bessel_batch_offsets_shifts_and_axisymmetric_aberration(lib, e_inc):
    import torch
    rw = lib
    w = W.bessel_plain(n_stacks=11, seed=101)
    z = np.linspace(-700.0, 500.0, 7)
    plan = _bessel_plan(rw, w, nx=40, z=z, e_inc=e_inc)
    rng = np.random.default_rng(4)
    stacks = []
    for b in range(11):
        c = np.zeros(11)
        c[3], c[10] = rng.normal(0, 0.05), rng.normal(0, 0.05)
        stacks.append(dict(z_offset=w["z_offsets"][b], x0=rng.uniform(-10, 10), y0=rng.uniform(-10, 10),
                           zernike=c))
    E, I = plan.compute(stacks)
    torch.cuda.synchronize()
    opt = O.Optics(na=1.4, wavelength=532.0, n_i=1.518, e_inc=e_inc)
    for b in range(11):
        s = stacks[b]
        ref = OB.field_bessel(opt, 40, 40, 20.0, 20.0, z + s["z_offset"], x0=s["x0"], y0=s["y0"],
                              n_theta=256, zernike=s["zernike"])
        assert rel_l2(_np(E[b]), ref) < TOL
        assert rel_l2(_np(I[b]), OF.intensity(ref)) < TOL


def test_bessel_gibson_lanni_critical_angle_split(lib):
    import torch
    rw = lib
    w = W.bessel_plain()
    gl = dict(W.GIBSON_LANNI)
    z = np.linspace(-2500.0, -1500.0, 5)
    plan = _bessel_plan(rw, w, nx=33, z=z, gl=gl, n_theta=200)
    E, I = plan.compute([dict(t_s=2000.0)])
    torch.cuda.synchronize()
    g = O.GibsonLanni(n_s=gl["n_s"], n_g=gl["n_g"], n_g_design=gl["n_g_design"],
                      n_i_design=gl["n_i_design"], t_g=gl["t_g"], t_g_design=gl["t_g_design"],
                      t_i_design=gl["t_i_design"])
    opt = O.Optics(na=1.4, wavelength=532.0, n_i=1.518, e_inc=w["e_inc"], gl=g)
    ref = OB.field_bessel(opt, 33, 33, 20.0, 20.0, z, n_theta=256, t_s=2000.0)
    assert rel_l2(_np(E[0]), ref) < TOL


def test_bessel_matches_fourier_on_gpu_as_pupil_grows(lib):
    """The paper's equivalence claim, on the GPU: Cartesian -> spherical as N grows."""
    import torch
    rw = lib
    w = W.bessel_plain()
    z = np.array([-400.0, 0.0, 300.0])
    pb = _bessel_plan(rw, w, nx=33, z=z)
    _, Ib = pb.compute([dict()], fields=False)
    errs = []
    for n in (64, 128, 256):
        o = w["optics"]
        pf = rw.Plan(form=rw.FORM_FOURIER, na=o["na"], wavelength=o["wavelength"], n_i=o["n_i"], nx=33,
                     ny=33, dx=20.0, dy=20.0, z=z, e_inc=w["e_inc"], n_pupil=n)
        _, If = pf.compute([dict()], fields=False)
        torch.cuda.synchronize()
        errs.append(rel_l2(_np(If[0]), _np(Ib[0])))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 2e-3


def test_fourier_small_tile_launch_matches_large_tile_launch(lib):
    """A launch that would underfill the GPU with large tiles (one plane of one stack) takes
    the small-tile kernels: the same planes computed inside the 16-stack, 64-plane launch
    (large tiles) must agree with it to FP32 rounding of a different summation tiling."""
    import torch
    rw = lib
    w = W.fourier_plain()
    zp = np.linspace(-1000.0, 1000.0, 64)
    stacks = [dict(t_s=w["t_s"][b], z_offset=-w["t_s"][b], zernike=w["zernike"][b]) for b in range(16)]
    E, I = _fourier_plan(rw, w, 256, 128, 128, 20.0, zp).compute(stacks)
    torch.cuda.synchronize()
    for b, zi in ((0, 0), (5, 31), (15, 63)):
        one = _fourier_plan(rw, w, 256, 128, 128, 20.0, [zp[zi]])
        E1, I1 = one.compute([stacks[b]])
        torch.cuda.synchronize()
        assert rel_l2(_np(E1[0, 0]), _np(E[b, zi])) < 2e-6, (b, zi)
        assert rel_l2(_np(I1[0, 0]), _np(I[b, zi])) < 2e-6, (b, zi)
