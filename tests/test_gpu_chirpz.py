"""Chirp-z (Bluestein) evaluation of the Fourier form against the FP64 oracle and against the
matrix-DFT evaluation (rel-L2 <= 1e-5): both compute the same discrete Cartesian sum."""
import numpy as np
import pytest

import workloads as W
from oracle import fourier as OF
from tests.helpers import oracle_fourier_stack, oracle_optics, rel_l2

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _np(t):
    return t.detach().cpu().numpy()


def _plan(rw, form, w, n_pupil, nx, ny, dx, z, gl=True):
    o = w["optics"]
    return rw.Plan(form=form, na=o["na"], wavelength=o["wavelength"], n_i=o["n_i"], nx=nx, ny=ny, dx=dx, dy=dx,
                   z=z, e_inc=w["e_inc"], gibson_lanni=w["gl"] if gl else None, n_pupil=n_pupil)


# FFT lengths from 64 to 1024, odd and even pupils, nx != ny, both radix remainders
@pytest.mark.parametrize("n_pupil,nx,ny", [(40, 17, 23), (37, 20, 70), (130, 65, 131), (256, 128, 96),
                                           (301, 40, 200)])
def test_chirpz_small_all_corrections(lib, n_pupil, nx, ny):
    import torch
    rw = lib
    w = W.fourier_plain(n_stacks=3, seed=31)
    zp = np.linspace(-700.0, 800.0, 4)
    rng = np.random.default_rng(3)
    maps = [rng.normal(0, 0.3, (n_pupil, n_pupil)) for _ in range(3)]
    plan = _plan(rw, rw.FORM_CHIRPZ, w, n_pupil, nx, ny, 25.0, zp)
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
        assert rel_l2(_np(E[b]), ref) < TOL, (b, rel_l2(_np(E[b]), ref))
        assert rel_l2(_np(I[b]), OF.intensity(ref)) < TOL


def test_chirpz_matches_matrix_dft_full_config(lib):
    """256 x 256 pupil -> 128 x 128 x 64 (the benchmark workload): chirp-z vs the folded
    matrix DFT for 16 stacks, and one whole stack against the separable oracle."""
    import torch
    rw = lib
    w = W.fourier_plain()
    zp = np.linspace(-1000.0, 1000.0, 64)
    stacks = [dict(t_s=w["t_s"][b], z_offset=-w["t_s"][b], zernike=w["zernike"][b]) for b in range(16)]
    Ec, Ic = _plan(rw, rw.FORM_CHIRPZ, w, 256, 128, 128, 20.0, zp).compute(stacks)
    Ef, If = _plan(rw, rw.FORM_FOURIER, w, 256, 128, 128, 20.0, zp).compute(stacks)
    torch.cuda.synchronize()
    assert rel_l2(_np(Ec), _np(Ef)) < TOL
    assert rel_l2(_np(Ic), _np(If)) < TOL
    ref = oracle_fourier_stack(oracle_optics(w), 256, 128, 128, 20.0, 20.0, zp - w["t_s"][5],
                               zernike=w["zernike"][5], t_s=w["t_s"][5])
    assert rel_l2(_np(Ec[5]), ref) < TOL
    assert rel_l2(_np(Ic[5]), OF.intensity(ref)) < TOL


def test_chirpz_large_pupil(lib):
    """N = 1024 pupil (FFT length 2048): a few planes against the separable oracle."""
    import torch
    rw = lib
    w = W.fourier_plain(n_stacks=1, seed=32)
    zp = np.array([-400.0, 250.0])
    plan = _plan(rw, rw.FORM_CHIRPZ, w, 1024, 96, 64, 20.0, zp, gl=False)
    E, I = plan.compute([dict(zernike=w["zernike"][0])])
    torch.cuda.synchronize()
    ref = oracle_fourier_stack(oracle_optics(w, gl=False), 1024, 96, 64, 20.0, 20.0, zp, zernike=w["zernike"][0])
    assert rel_l2(_np(E[0]), ref) < TOL
    assert rel_l2(_np(I[0]), OF.intensity(ref)) < TOL


def test_chirpz_limits_and_no_adjoint(lib):
    import torch
    rw = lib
    w = W.fourier_plain(n_stacks=1, seed=33)
    o = w["optics"]
    optics = rw.make_optics(o["na"], o["wavelength"], o["n_i"], w["e_inc"], 1.0, True, 0.0, None)
    grid = rw.make_grid(1100, 64, 20.0, 20.0, [0.0])
    num = rw.Numerics(form=rw.FORM_CHIRPZ, n_pupil=1000, n_theta=2, n_rho=8)
    assert rw.validate(optics, grid, num) == rw.ERR_UNSUPPORTED   # N + nx - 1 > 2048
    plan = _plan(rw, rw.FORM_CHIRPZ, w, 64, 32, 32, 20.0, [0.0], gl=False)
    E, _ = plan.compute([dict()])
    g = torch.zeros((1, 1, 32, 32), dtype=torch.float32, device="cuda")
    with pytest.raises(RuntimeError):
        plan.adjoint([dict()], E, g, 1)
