"""Scalar model, Simpson / Riemann theta rules, the extra s_z factor and the Fresnel
factors on the GPU against the FP64 oracle (same discrete sums, rel-L2 <= 1e-5), and
the accuracy benchmark of Sec. 5.2.2 (convergence orders against the Airy disk) run
through the GPU kernels."""
import math

import numpy as np
import pytest
from scipy.special import j1

import workloads as W
from oracle import bessel as OB
from oracle import fourier as OF
from oracle import optics as O
from tests.helpers import oracle_optics, rel_l2

pytestmark = pytest.mark.gpu
TOL = 1e-5
GL = W.GIBSON_LANNI
FRESNEL = (GL["n_s"], GL["n_g"])


def _np(t):
    return t.detach().cpu().numpy()


def _with(opt, **kw):
    d = dict(opt.__dict__)
    d.update(kw)
    return O.Optics(**d)


# --------------------------------------------------------------------- Cartesian forms
def _cart_plan(rw, form, w, n_pupil, nx, ny, dx, z, **kw):
    o = w["optics"]
    return rw.Plan(form=form, na=o["na"], wavelength=o["wavelength"], n_i=o["n_i"], nx=nx, ny=ny, dx=dx,
                   dy=dx, z=z, e_inc=w["e_inc"], gibson_lanni=w["gl"], n_pupil=n_pupil, **kw)


def _cart_case(rw, torch, form, n_pupil, nx, ny, scalar, fresnel):
    w = W.fourier_plain(n_stacks=3, seed=13)
    zp = np.linspace(-600.0, 900.0, 5)
    rng = np.random.default_rng(5)
    maps = [rng.normal(0, 0.3, (n_pupil, n_pupil)) for _ in range(3)]
    kw = dict(model=rw.MODEL_SCALAR if scalar else rw.MODEL_VECTORIAL, fresnel=FRESNEL if fresnel else None)
    plan = _cart_plan(rw, form, w, n_pupil, nx, ny, 25.0, zp, **kw)
    stacks = [dict(t_s=w["t_s"][b] / 3, x0=[0.0, 13.0, -31.0][b], y0=[0.0, -7.0, 44.0][b],
                   z_offset=-w["t_s"][b] / 3, zernike=w["zernike"][b],
                   phase_map=torch.tensor(maps[b], dtype=torch.float32, device="cuda")) for b in range(3)]
    E, I = plan.compute(stacks)
    torch.cuda.synchronize()
    assert E.shape[2] == (1 if scalar else 3)
    opt = oracle_optics(w)
    if fresnel:
        opt = _with(opt, fresnel_media=FRESNEL)
    g = OF.pupil_geometry(n_pupil, opt)
    for b in range(3):
        s = stacks[b]
        ph = OF.pupil_phase(g, opt, zernike=w["zernike"][b], phase_map=maps[b].astype(np.float32), t_s=s["t_s"])
        P = OF.base_pupil(g, opt, ph, scalar=scalar)
        ref = OF.field_separable(P, g, opt, nx, ny, 25.0, 25.0, zp + s["z_offset"], x0=s["x0"], y0=s["y0"])
        assert rel_l2(_np(E[b]), ref) < TOL, b
        assert rel_l2(_np(I[b]), OF.intensity(ref)) < TOL, b


@pytest.mark.parametrize("form", ["fourier", "chirpz"])
@pytest.mark.parametrize("n_pupil,nx,ny", [(40, 33, 29), (37, 20, 70), (130, 65, 131)])
def test_cartesian_scalar_model(lib, form, n_pupil, nx, ny):
    import torch
    rw = lib
    f = rw.FORM_FOURIER if form == "fourier" else rw.FORM_CHIRPZ
    _cart_case(rw, torch, f, n_pupil, nx, ny, scalar=True, fresnel=False)


@pytest.mark.parametrize("form", ["fourier", "chirpz"])
@pytest.mark.parametrize("n_pupil,nx,ny", [(37, 20, 70), (130, 65, 131)])
def test_cartesian_fresnel_factors(lib, form, n_pupil, nx, ny):
    # NA 1.4 > n_s = 1.33: beyond the sample's critical angle the products are complex
    import torch
    rw = lib
    f = rw.FORM_FOURIER if form == "fourier" else rw.FORM_CHIRPZ
    _cart_case(rw, torch, f, n_pupil, nx, ny, scalar=False, fresnel=True)


def test_fresnel_factors_change_the_field(lib):
    import torch
    rw = lib
    w = W.fourier_plain(n_stacks=1, seed=14)
    zp = [0.0, 400.0]
    a = _cart_plan(rw, rw.FORM_FOURIER, w, 64, 33, 33, 25.0, zp)
    b = _cart_plan(rw, rw.FORM_FOURIER, w, 64, 33, 33, 25.0, zp, fresnel=FRESNEL)
    st = [dict(t_s=500.0, zernike=w["zernike"][0])]
    _, Ia = a.compute(st, fields=False)
    _, Ib = b.compute(st, fields=False)
    torch.cuda.synchronize()
    assert rel_l2(_np(Ib), _np(Ia)) > 1e-2


# ------------------------------------------------------------------------ Bessel form
def _bessel_case(rw, torch, model, rule, n_theta, fresnel=False, extra_sz=False, apod=True):
    w = W.bessel_plain(n_stacks=2, seed=102)
    z = np.linspace(-700.0, 500.0, 5)
    o = w["optics"]
    plan = rw.Plan(form=rw.FORM_BESSEL, na=o["na"], wavelength=o["wavelength"], n_i=o["n_i"], nx=40, ny=40,
                   dx=20.0, dy=20.0, z=z, e_inc=w["e_inc"], n_theta=n_theta, n_rho=256, model=model,
                   theta_rule=rule, fresnel=FRESNEL if fresnel else None, extra_sz=extra_sz,
                   apodization=apod)
    rng = np.random.default_rng(6)
    stacks = []
    for b in range(2):
        c = np.zeros(11)
        c[3], c[10] = rng.normal(0, 0.05), rng.normal(0, 0.05)
        stacks.append(dict(z_offset=w["z_offsets"][b], x0=rng.uniform(-10, 10), y0=rng.uniform(-10, 10),
                           zernike=c))
    E, I = plan.compute(stacks)
    torch.cuda.synchronize()
    scalar = model == rw.MODEL_SCALAR
    assert E.shape[2] == (1 if scalar else 3)
    opt = O.Optics(na=o["na"], wavelength=o["wavelength"], n_i=o["n_i"], e_inc=w["e_inc"], apodization=apod,
                   fresnel_media=FRESNEL if fresnel else ())
    name = {rw.THETA_GAUSS: "gauss", rw.THETA_SIMPSON: "simpson", rw.THETA_RIEMANN: "riemann"}[rule]
    for b in range(2):
        s = stacks[b]
        ref = OB.field_bessel(opt, 40, 40, 20.0, 20.0, z + s["z_offset"], x0=s["x0"], y0=s["y0"],
                              n_theta=n_theta, zernike=s["zernike"], rule=name, scalar=scalar,
                              extra_cos=extra_sz)
        assert rel_l2(_np(E[b]), ref) < TOL, b
        assert rel_l2(_np(I[b]), OF.intensity(ref)) < TOL, b


@pytest.mark.parametrize("rule,n_theta", [(0, 200), (1, 201), (2, 200)])
@pytest.mark.parametrize("model", ["vectorial", "scalar"])
def test_bessel_models_and_theta_rules(lib, model, rule, n_theta):
    import torch
    rw = lib
    m = rw.MODEL_SCALAR if model == "scalar" else rw.MODEL_VECTORIAL
    _bessel_case(rw, torch, m, rule, n_theta)


@pytest.mark.parametrize("rule,n_theta", [(0, 200), (1, 201)])
def test_bessel_fresnel_factors(lib, rule, n_theta):
    import torch
    rw = lib
    _bessel_case(rw, torch, rw.MODEL_VECTORIAL, rule, n_theta, fresnel=True)


def test_bessel_scalar_extra_sz_no_apodization(lib):
    import torch
    rw = lib
    _bessel_case(rw, torch, rw.MODEL_SCALAR, rw.THETA_SIMPSON, 101, extra_sz=True, apod=False)


@pytest.mark.parametrize("mode", ["vectorial", "fresnel", "scalar", "simpson_envelope_gl"])
def test_bessel_few_plane_launch_matches_chunked_path(lib, mode):
    """A call of one stack takes one launch (phase, contraction and epilogue per radial
    band of a plane); a call of more stacks takes the phase kernel, the matrix-core
    contraction and the epilogue kernel.  The same six stacks (shifts, axisymmetric
    Zernike terms; in the last case also the Simpson rule, the Gaussian envelope, the
    extra s_z factor and Gibson-Lanni depths) through both, stack by stack, and the
    many-stack call against the oracle."""
    import torch
    rw = lib
    w = W.bessel_plain(n_stacks=6, seed=103)
    z = np.linspace(-900.0, 600.0, 9)
    o = w["optics"]
    scalar = mode == "scalar"
    extra = mode == "simpson_envelope_gl"
    rule, n_theta = (rw.THETA_SIMPSON, 201) if extra else (rw.THETA_GAUSS, 200)
    plan = rw.Plan(form=rw.FORM_BESSEL, na=o["na"], wavelength=o["wavelength"], n_i=o["n_i"], nx=45, ny=45,
                   dx=20.0, dy=20.0, z=z, e_inc=W.X_LINEAR, n_theta=n_theta, n_rho=256, theta_rule=rule,
                   model=rw.MODEL_SCALAR if scalar else rw.MODEL_VECTORIAL,
                   fresnel=FRESNEL if mode == "fresnel" else None, s_env=0.5 if extra else 0.0,
                   extra_sz=extra, gibson_lanni=dict(GL) if extra else None)
    rng = np.random.default_rng(8)
    stacks = []
    for b in range(6):
        c = np.zeros(22)
        c[3], c[10], c[21] = rng.normal(0, 0.05, 3)
        stacks.append(dict(z_offset=w["z_offsets"][b], x0=rng.uniform(-15, 15), y0=rng.uniform(-15, 15),
                           zernike=c, t_s=float(rng.uniform(0.0, 3000.0)) if extra else 0.0))
    E, I = plan.compute(stacks)                 # six stacks: the chunked path
    for b in range(6):
        Eb, Ib = plan.compute([stacks[b]])      # one stack of 9 planes: the single launch
        torch.cuda.synchronize()
        assert rel_l2(_np(Eb[0]), _np(E[b])) < 1e-6, b
        assert rel_l2(_np(Ib[0]), _np(I[b])) < 1e-6, b
    gl = None
    if extra:
        gl = O.GibsonLanni(n_s=GL["n_s"], n_g=GL["n_g"], n_g_design=GL["n_g_design"], n_i_design=GL["n_i_design"],
                           t_g=GL["t_g"], t_g_design=GL["t_g_design"], t_i_design=GL["t_i_design"])
    opt = O.Optics(na=o["na"], wavelength=o["wavelength"], n_i=o["n_i"], e_inc=W.X_LINEAR,
                   fresnel_media=FRESNEL if mode == "fresnel" else (), s_env=0.5 if extra else 0.0, gl=gl)
    for b in (0, 5):
        s = stacks[b]
        ref = OB.field_bessel(opt, 45, 45, 20.0, 20.0, z + s["z_offset"], x0=s["x0"], y0=s["y0"],
                              n_theta=n_theta, zernike=s["zernike"], scalar=scalar, t_s=s["t_s"],
                              rule="simpson" if extra else "gauss", extra_cos=extra)
        assert rel_l2(_np(E[b]), ref) < TOL, b
        assert rel_l2(_np(I[b]), OF.intensity(ref)) < TOL, b


# ------------------------------------------------------- accuracy benchmark (Sec. 5.2.2)
NA, LAM, NI = 1.4, 532.0, 1.518


def _airy_line(n_px=41, dx=20.0):
    k = 2 * math.pi * NI / LAM
    v = k * (NA / NI) * np.abs(O.output_axis(n_px, dx))
    safe = np.where(v > 0, v, 1.0)
    return -1j * k * (NA / NI) ** 2 / 2 * np.where(v > 0, 2 * j1(safe) / safe, 1.0)


def _airy_plan(rw, form, **kw):
    return rw.Plan(form=form, na=NA, wavelength=LAM, n_i=NI, nx=41, ny=1, dx=20.0, dy=20.0, z=[0.0],
                   apodization=False, model=rw.MODEL_SCALAR, extra_sz=True, **kw)


def test_accuracy_benchmark_convergence_orders(lib):
    """Scalar propagators with the extra s_z factor against 2 J1(v)/v: Riemann first
    order, Simpson fourth order, the Cartesian sum between first and second order."""
    import torch
    rw = lib
    ref = _airy_line()
    tmax = math.asin(NA / NI)
    orders = {}
    for rule, ns in ((rw.THETA_RIEMANN, (16, 32, 64, 128, 256)), (rw.THETA_SIMPSON, (9, 17, 33))):
        errs, hs = [], []
        for n in ns:
            p = _airy_plan(rw, rw.FORM_BESSEL, theta_rule=rule, n_theta=n, n_rho=512)
            E, _ = p.compute([dict()], intensity=False)
            torch.cuda.synchronize()
            errs.append(rel_l2(_np(E[0, 0, 0, :, 0]), ref))
            hs.append(tmax / (n if rule == rw.THETA_RIEMANN else n - 1))
        orders[rule] = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    errs, hs = [], []
    for n in (32, 64, 128, 256, 512):
        p = _airy_plan(rw, rw.FORM_FOURIER, n_pupil=n)
        E, _ = p.compute([dict()], intensity=False)
        torch.cuda.synchronize()
        errs.append(rel_l2(_np(E[0, 0, 0, :, 0]), ref))
        hs.append(2 * (NA / NI) / n)
    orders["cartesian"] = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    assert 0.9 < orders[rw.THETA_RIEMANN] < 1.1, orders
    assert 3.6 < orders[rw.THETA_SIMPSON] < 4.4, orders
    assert 1.0 <= orders["cartesian"] <= 2.0, orders
    assert errs[-1] < 2e-4


# ----------------------------------------------------------------- batched emitters
def test_batched_with_fresnel_and_extra_sz_equals_plain_plan(lib):
    import torch
    rw = lib
    w = W.batched(n_emitters=3, seed=33)
    o = w["optics"]
    b = rw.Batch(na=o["na"], wavelength=o["wavelength"], n_i=o["n_i"], pixel=w["dx"], plane_pitch=w["dz"],
                 max_emitters=4, n_pupil=w["n_pupil"], e_inc=w["e_inc"], fresnel=FRESNEL, extra_sz=True)
    crops, planes = np.array([24, 40, 64]), np.array([3, 2, 1])
    em = rw.make_emitters(w["x0"][:3], w["y0"][:3], w["z_e"][:3], crops, planes, w["zernike"][:3])
    off = rw.batch_offsets(em)
    I = torch.zeros(off[-1], dtype=torch.float32, device="cuda")
    b.compute(em, I=I)
    for i in range(3):
        S, D = int(crops[i]), int(planes[i])
        z = (np.arange(D) - 0.5 * (D - 1)) * w["dz"]
        plan = rw.Plan(form=rw.FORM_FOURIER, na=o["na"], wavelength=o["wavelength"], n_i=o["n_i"], nx=S,
                       ny=S, dx=w["dx"], dy=w["dx"], z=z, e_inc=w["e_inc"], n_pupil=w["n_pupil"],
                       fresnel=FRESNEL, extra_sz=True)
        _, Ip = plan.compute([dict(x0=w["x0"][i], y0=w["y0"][i], z_offset=-w["z_e"][i],
                                   zernike=w["zernike"][i])], fields=False)
        torch.cuda.synchronize()
        got = I[off[i]:off[i + 1]].cpu().numpy().reshape(D, S, S)
        assert rel_l2(got, Ip[0].cpu().numpy()) < 1e-6


def test_scalar_plan_rejects_adjoint_and_small_outputs(lib):
    import torch
    rw = lib
    p = _airy_plan(rw, rw.FORM_FOURIER, n_pupil=64)
    E, I = p.compute([dict()])
    with pytest.raises(rw.RwpsfError) as ei:
        p.adjoint([dict()], E, I, 0)
    assert ei.value.status == rw.ERR_UNSUPPORTED
    with pytest.raises(ValueError):
        p.compute([dict(), dict()], E=E, I=None, intensity=False)
