"""The Gaussian envelope a(s) *= exp(-sin^2 t / s_env^2) (Sec. 3.4.4) on the GPU in every
form against the FP64 oracle (rel-L2 <= 1e-5), and the scalar Bessel form against the
envelope's closed form (the Hankel transform of a Gaussian)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import bessel as OB
from oracle import fourier as OF
from oracle import optics as O
from tests.helpers import oracle_optics, rel_l2

pytestmark = pytest.mark.gpu
TOL = 1e-5
S_ENV = 0.5   # NA/n_i = 0.92: the envelope falls to exp(-3.4) at the aperture edge


def _np(t):
    return t.detach().cpu().numpy()


def _with(opt, **kw):
    d = dict(opt.__dict__)
    d.update(kw)
    return O.Optics(**d)


@pytest.mark.parametrize("form", ["fourier", "chirpz"])
@pytest.mark.parametrize("model", ["vectorial", "scalar"])
@pytest.mark.parametrize("n_pupil,nx,ny", [(40, 33, 29), (130, 65, 131)])
def test_cartesian_forms_with_envelope(lib, form, model, n_pupil, nx, ny):
    import torch
    rw = lib
    w = W.fourier_plain(n_stacks=2, seed=15)
    o = w["optics"]
    zp = np.linspace(-600.0, 900.0, 4)
    scalar = model == "scalar"
    plan = rw.Plan(form=rw.FORM_FOURIER if form == "fourier" else rw.FORM_CHIRPZ, na=o["na"],
                   wavelength=o["wavelength"], n_i=o["n_i"], nx=nx, ny=ny, dx=25.0, dy=25.0, z=zp,
                   e_inc=w["e_inc"], gibson_lanni=w["gl"], n_pupil=n_pupil, s_env=S_ENV,
                   model=rw.MODEL_SCALAR if scalar else rw.MODEL_VECTORIAL)
    rng = np.random.default_rng(8)
    maps = [rng.normal(0, 0.3, (n_pupil, n_pupil)).astype(np.float32) for _ in range(2)]
    stacks = [dict(t_s=w["t_s"][b] / 3, x0=[9.0, -31.0][b], y0=[-7.0, 44.0][b], z_offset=-w["t_s"][b] / 3,
                   zernike=w["zernike"][b], phase_map=torch.tensor(maps[b], device="cuda"))
              for b in range(2)]
    E, I = plan.compute(stacks)
    torch.cuda.synchronize()
    opt = _with(oracle_optics(w), s_env=S_ENV)
    g = OF.pupil_geometry(n_pupil, opt)
    for b, s in enumerate(stacks):
        ph = OF.pupil_phase(g, opt, zernike=w["zernike"][b], phase_map=maps[b], t_s=s["t_s"])
        ref = OF.field_separable(OF.base_pupil(g, opt, ph, scalar=scalar), g, opt, nx, ny, 25.0, 25.0,
                                 zp + s["z_offset"], x0=s["x0"], y0=s["y0"])
        assert rel_l2(_np(E[b]), ref) < TOL, b
        assert rel_l2(_np(I[b]), OF.intensity(ref)) < TOL, b


@pytest.mark.parametrize("model", ["vectorial", "scalar"])
@pytest.mark.parametrize("rule,n_theta", [(0, 200), (1, 201)])
def test_bessel_form_with_envelope(lib, model, rule, n_theta):
    import torch
    rw = lib
    w = W.bessel_plain(n_stacks=2, seed=103)
    o = w["optics"]
    z = np.linspace(-700.0, 500.0, 5)
    scalar = model == "scalar"
    plan = rw.Plan(form=rw.FORM_BESSEL, na=o["na"], wavelength=o["wavelength"], n_i=o["n_i"], nx=40, ny=40,
                   dx=20.0, dy=20.0, z=z, e_inc=w["e_inc"], n_theta=n_theta, n_rho=256, s_env=S_ENV,
                   model=rw.MODEL_SCALAR if scalar else rw.MODEL_VECTORIAL, theta_rule=rule)
    rng = np.random.default_rng(9)
    stacks = []
    for b in range(2):
        c = np.zeros(11)
        c[3], c[10] = rng.normal(0, 0.05), rng.normal(0, 0.05)
        stacks.append(dict(z_offset=w["z_offsets"][b], x0=rng.uniform(-10, 10), y0=rng.uniform(-10, 10),
                           zernike=c))
    E, I = plan.compute(stacks)
    torch.cuda.synchronize()
    opt = O.Optics(na=o["na"], wavelength=o["wavelength"], n_i=o["n_i"], e_inc=w["e_inc"], s_env=S_ENV)
    for b, s in enumerate(stacks):
        ref = OB.field_bessel(opt, 40, 40, 20.0, 20.0, z + s["z_offset"], x0=s["x0"], y0=s["y0"],
                              n_theta=n_theta, zernike=s["zernike"], rule="gauss" if rule == 0 else "simpson",
                              scalar=scalar)
        assert rel_l2(_np(E[b]), ref) < TOL, b
        assert rel_l2(_np(I[b]), OF.intensity(ref)) < TOL, b


def test_bessel_scalar_envelope_matches_hankel_closed_form(lib):
    """Scalar spherical form, extra s_z, no apodization, z = 0: E(rho) = -i f k (s^2/2)
    exp(-(k rho s)^2 / 4) up to exp(-s_max^2 / s^2) = 6e-10 of the peak at s = 0.2."""
    import torch
    rw = lib
    na, lam, ni, s = 1.4, 532.0, 1.518, 0.2
    plan = rw.Plan(form=rw.FORM_BESSEL, na=na, wavelength=lam, n_i=ni, nx=41, ny=41, dx=15.0, dy=15.0,
                   z=[0.0], apodization=False, s_env=s, model=rw.MODEL_SCALAR, extra_sz=True, n_theta=200,
                   n_rho=256)
    E, _ = plan.compute([dict()], intensity=False)
    torch.cuda.synchronize()
    k = 2 * math.pi * ni / lam
    xs = O.output_axis(41, 15.0)
    rho = np.hypot(xs[:, None], xs[None, :])
    ref = -1j * k * s * s / 2 * np.exp(-(k * rho * s) ** 2 / 4)
    assert rel_l2(_np(E[0, 0, 0]), ref) < TOL


def test_batched_with_envelope_matches_oracle(lib):
    import torch
    rw = lib
    w = W.batched(n_emitters=6, seed=38)
    o = w["optics"]
    b = rw.Batch(na=o["na"], wavelength=o["wavelength"], n_i=o["n_i"], pixel=w["dx"], plane_pitch=w["dz"],
                 max_emitters=8, n_pupil=w["n_pupil"], e_inc=w["e_inc"], s_env=S_ENV)
    crops, planes = np.array([24, 31, 40, 64, 17, 50]), np.array([3, 2, 1, 2, 1, 2])
    em = rw.make_emitters(w["x0"][:6], w["y0"][:6], w["z_e"][:6], crops, planes, w["zernike"][:6])
    off = rw.batch_offsets(em)
    I = torch.zeros(off[-1], dtype=torch.float32, device="cuda")
    E = torch.zeros(3 * off[-1], dtype=torch.complex64, device="cuda")
    b.compute(em, I=I, E=E)
    torch.cuda.synchronize()
    opt = _with(oracle_optics(w, gl=False), s_env=S_ENV)
    g = OF.pupil_geometry(w["n_pupil"], opt)
    In, En = I.cpu().numpy(), E.cpu().numpy()
    for i in range(6):
        S, D = int(crops[i]), int(planes[i])
        z = (np.arange(D) - 0.5 * (D - 1)) * w["dz"] - w["z_e"][i]
        P = OF.base_pupil(g, opt, OF.pupil_phase(g, opt, zernike=w["zernike"][i]))
        ref = OF.field_separable(P, g, opt, S, S, w["dx"], w["dx"], z, x0=w["x0"][i], y0=w["y0"][i])
        assert rel_l2(En[3 * off[i]:3 * off[i + 1]].reshape(D, 3, S, S), ref) < TOL, i
        assert rel_l2(In[off[i]:off[i + 1]].reshape(D, S, S), OF.intensity(ref)) < TOL, i
