"""The allocation-free entry point (rwpsf_compute_noalloc) against rwpsf_compute.

The variant runs the same Bessel-form kernels with its workspace in a fixed device
array, so its outputs must equal rwpsf_compute's bit for bit (and both meet the FP64
oracle at rel-L2 <= 1e-5).  Two calls in a row, the second smaller, check that what the
first call leaves in the shared array does not leak into the second.
"""
import numpy as np
import pytest

import workloads as W
from oracle import bessel as OB
from oracle import fourier as OF
from oracle import optics as O
from tests.helpers import rel_l2

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _plan(rw, w, nx, z, n_theta=200, n_rho=256, fresnel=None):
    o = w["optics"]
    return rw.Plan(form=rw.FORM_BESSEL, na=o["na"], wavelength=o["wavelength"], n_i=o["n_i"], nx=nx, ny=nx,
                   dx=20.0, dy=20.0, z=z, e_inc=w["e_inc"], n_theta=n_theta, n_rho=n_rho, fresnel=fresnel)


def _stacks(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        c = np.zeros(11)
        c[3], c[10] = rng.normal(0, 0.05), rng.normal(0, 0.05)
        out.append(dict(z_offset=rng.uniform(-100, 100), x0=rng.uniform(-10, 10), y0=rng.uniform(-10, 10),
                        zernike=c))
    return out


def _both(rw, plan, stacks):
    import torch
    E0, I0 = plan.compute(stacks)
    E1, I1 = plan.compute(stacks, noalloc=True)
    torch.cuda.synchronize()
    return E0.cpu().numpy(), I0.cpu().numpy(), E1.cpu().numpy(), I1.cpu().numpy()


def test_noalloc_equals_compute_two_calls(lib):
    rw = lib
    w = W.bessel_plain()
    plan = _plan(rw, w, 65, w["z"])
    first = _stacks(9, 1)
    E0, I0, E1, I1 = _both(rw, plan, first)
    assert np.array_equal(E0, E1) and np.array_equal(I0, I1)
    opt = O.Optics(na=1.4, wavelength=532.0, n_i=1.518, e_inc=w["e_inc"])
    s = first[4]
    ref = OB.field_bessel(opt, 65, 65, 20.0, 20.0, w["z"] + s["z_offset"], x0=s["x0"], y0=s["y0"],
                          n_theta=256, zernike=s["zernike"])
    assert rel_l2(E1[4], ref) < TOL and rel_l2(I1[4], OF.intensity(ref)) < TOL
    second = _stacks(2, 2)                    # smaller call after a larger one
    E0, I0, E1, I1 = _both(rw, plan, second)
    assert np.array_equal(E0, E1) and np.array_equal(I0, I1)
    plan.close()


def test_noalloc_chunks_through_the_scratch(lib):
    """A plan whose stacks need several passes through the fixed array (99 planes: 21 stacks
    per chunk), then a smaller call, both against rwpsf_compute; one stack against the oracle."""
    import torch
    rw = lib
    w = W.bessel_plain()
    z = np.linspace(-1000.0, 1000.0, 99)
    plan = _plan(rw, w, 33, z)
    stacks = _stacks(50, 3)
    E0, I0, E1, I1 = _both(rw, plan, stacks)
    assert np.array_equal(E0, E1) and np.array_equal(I0, I1)
    opt = O.Optics(na=1.4, wavelength=532.0, n_i=1.518, e_inc=w["e_inc"])
    s = stacks[37]
    ref = OB.field_bessel(opt, 33, 33, 20.0, 20.0, z + s["z_offset"], x0=s["x0"], y0=s["y0"], n_theta=256,
                          zernike=s["zernike"])
    assert rel_l2(E1[37], ref) < TOL
    _, I_small = plan.compute(stacks[:5], fields=False, noalloc=True)
    torch.cuda.synchronize()
    assert np.array_equal(I_small.cpu().numpy(), I0[:5])
    plan.close()


def test_noalloc_fresnel_intensity_only(lib):
    """Fresnel mode (two pupil variants, five table groups), intensity output only."""
    import torch
    rw = lib
    w = W.bessel_plain()
    z = np.linspace(-800.0, 800.0, 13)
    plan = _plan(rw, w, 41, z, fresnel=(1.33, 1.5))
    stacks = _stacks(6, 4)
    _, I0 = plan.compute(stacks, fields=False)
    _, I1 = plan.compute(stacks, fields=False, noalloc=True)
    torch.cuda.synchronize()
    assert np.array_equal(I0.cpu().numpy(), I1.cpu().numpy())
    plan.close()


def test_noalloc_rejects_what_does_not_fit_and_other_forms(lib):
    import torch
    rw = lib
    w = W.bessel_plain()
    # one stack: 200 planes x 3 groups x 4096 radial samples x 2 floats = 19.7 MB > 16 MiB
    z = np.linspace(-1000.0, 1000.0, 200)
    plan = _plan(rw, w, 17, z, n_rho=4096)
    with pytest.raises(rw.RwpsfError) as ei:
        plan.compute([dict()], noalloc=True)
    assert ei.value.status == rw.ERR_SCRATCH_LIMIT
    plan.close()
    o = W.fourier_plain(n_stacks=1)["optics"]
    fp = rw.Plan(form=rw.FORM_FOURIER, na=o["na"], wavelength=o["wavelength"], n_i=o["n_i"], nx=16, ny=16,
                 dx=30.0, dy=30.0, z=[0.0], n_pupil=32)
    with pytest.raises(rw.RwpsfError) as ei:
        fp.compute([dict()], noalloc=True)
    assert ei.value.status == -3
    torch.cuda.synchronize()
    fp.close()
