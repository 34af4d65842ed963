"""The hand-written adjoint against the FP64 gradient oracle, its invariants, determinism,
linearity over stacks at the full size, and the autograd.Function wrapper."""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint as OA
from oracle import fourier as OF
from tests.helpers import oracle_optics, rel_l2

pytestmark = pytest.mark.gpu


def _case(n_pupil, nx, nz, n_stacks, seed):
    w = W.adjoint(n_stacks=n_stacks, n_pupil=n_pupil, nx=nx, nz=nz, seed_truth=seed)
    rng = np.random.default_rng(seed + 7)
    shifts = [(rng.uniform(-50, 50), rng.uniform(-50, 50), rng.uniform(-200, 200)) for _ in range(n_stacks)]
    return w, shifts


def _plan(rw, w, nz_list):
    o = w["optics"]
    return rw.Plan(form=rw.FORM_FOURIER, na=o["na"], wavelength=o["wavelength"], n_i=o["n_i"], nx=w["nx"],
                   ny=w["ny"], dx=w["dx"], dy=w["dy"], z=nz_list, e_inc=w["e_inc"], n_pupil=w["n_pupil"])


def _gpu_grad(rw, torch, w, shifts, Y, scale):
    plan = _plan(rw, w, w["z"])
    w0 = torch.tensor(w["w0_eval"], dtype=torch.float32, device="cuda")
    st = [dict(x0=x0, y0=y0, z_offset=zo, zernike=w["c_eval"], phase_map=w0) for x0, y0, zo in shifts]
    E, I = plan.compute(st)
    s = torch.tensor(scale, dtype=torch.float32, device="cuda").view(-1, 1, 1, 1)
    Yt = torch.tensor(Y, dtype=torch.float32, device="cuda")
    dLdI = (2.0 * s * (s * I - Yt) / I.numel()).contiguous()
    dc, dw = plan.adjoint(st, E, dLdI, 21)
    torch.cuda.synchronize()
    return plan, st, E, dLdI, dc.cpu().numpy().astype(np.float64), dw.cpu().numpy().astype(np.float64)


def _oracle_grad(w, shifts, Y, scale):
    opt = oracle_optics(w, gl=False)
    g = OF.pupil_geometry(w["n_pupil"], opt)
    w0 = w["w0_eval"].astype(np.float32).astype(np.float64)
    _, I = OA.forward(g, opt, w["c_eval"], w0, shifts, w["nx"], w["ny"], w["dx"], w["dy"], w["z"])
    _, dLdI = OA.mse_loss(I, Y, scale)
    return OA.gradient(g, opt, w["c_eval"], w0, shifts, w["nx"], w["ny"], w["dx"], w["dy"], w["z"], dLdI)


def _targets(w, shifts):
    opt = oracle_optics(w, gl=False)
    g = OF.pupil_geometry(w["n_pupil"], opt)
    _, Itrue = OA.forward(g, opt, w["c_true"], None, shifts, w["nx"], w["ny"], w["dx"], w["dy"], w["z"])
    e_tot = Itrue[0].sum() / len(w["z"])
    scale = w["photons"][:len(shifts)] / e_tot
    Y = W.poisson(scale.reshape(-1, 1, 1, 1) * Itrue, w["noise_seed"])
    return Y, scale


@pytest.mark.parametrize("n_pupil,nx,nz,n_stacks", [(32, 16, 3, 2), (64, 32, 4, 3), (96, 48, 2, 9), (45, 32, 3, 2)])
def test_adjoint_matches_oracle_gradient(lib, n_pupil, nx, nz, n_stacks):
    import torch
    rw = lib
    w, shifts = _case(n_pupil, nx, nz, n_stacks, seed=404)
    Y, scale = _targets(w, shifts)
    _, _, _, _, dc, dw = _gpu_grad(rw, torch, w, shifts, Y, scale)
    dc_ref, dw_ref = _oracle_grad(w, shifts, Y, scale)
    assert rel_l2(dc, dc_ref) < 1e-4, rel_l2(dc, dc_ref)
    assert rel_l2(dw, dw_ref) < 1e-4, rel_l2(dw, dw_ref)
    # global-phase invariants
    assert abs(dc[0]) < 1e-4 * np.linalg.norm(dc_ref)
    assert abs(dw.sum()) < 1e-4 * np.abs(dw_ref).sum()


def test_adjoint_is_deterministic(lib):
    import torch
    rw = lib
    w, shifts = _case(64, 32, 3, 3, seed=405)
    Y, scale = _targets(w, shifts)
    plan, st, E, dLdI, dc1, dw1 = _gpu_grad(rw, torch, w, shifts, Y, scale)
    dc2, dw2 = plan.adjoint(st, E, dLdI, 21)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(dc1, dc2.cpu().numpy().astype(np.float64))
    np.testing.assert_array_equal(dw1, dw2.cpu().numpy().astype(np.float64))


def test_adjoint_full_size_oracle_and_linearity_over_stacks(lib):
    """256 x 256 pupil, 64 x 64 x 21 stacks: 4 stacks against the oracle; 64 stacks equal the sum
    of 16 calls of 4 (the gradient is additive over stacks)."""
    import torch
    rw = lib
    w, shifts = _case(256, 64, 21, 64, seed=404)
    Y, scale = _targets(w, shifts[:4])
    _, _, _, _, dc4, dw4 = _gpu_grad(rw, torch, w, shifts[:4], Y, scale)
    dc_ref, dw_ref = _oracle_grad(w, shifts[:4], Y, scale)
    assert rel_l2(dc4, dc_ref) < 1e-4 and rel_l2(dw4, dw_ref) < 1e-4
    # linearity: one call of 64 stacks vs 16 calls of 4 (same dL/dI per stack)
    plan = _plan(rw, w, w["z"])
    w0 = torch.tensor(w["w0_eval"], dtype=torch.float32, device="cuda")
    st = [dict(x0=x0, y0=y0, z_offset=zo, zernike=w["c_eval"], phase_map=w0) for x0, y0, zo in shifts]
    E, I = plan.compute(st)
    dLdI = (I - I.mean()).contiguous() * 1e-3
    dc_all, dw_all = plan.adjoint(st, E, dLdI, 21)
    dc_sum = torch.zeros_like(dc_all)
    dw_sum = torch.zeros_like(dw_all)
    for q in range(16):
        sl = slice(4 * q, 4 * q + 4)
        a, b = plan.adjoint(st[sl], E[sl].contiguous(), dLdI[sl].contiguous(), 21)
        dc_sum += a
        dw_sum += b
    torch.cuda.synchronize()
    assert rel_l2(dc_all.cpu().numpy(), dc_sum.cpu().numpy()) < 1e-5
    assert rel_l2(dw_all.cpu().numpy(), dw_sum.cpu().numpy()) < 1e-5


def test_autograd_function_backward(lib):
    import torch
    rw = lib
    w, shifts = _case(64, 32, 3, 2, seed=406)
    Y, scale = _targets(w, shifts)
    plan = _plan(rw, w, w["z"])
    c = torch.tensor(w["c_eval"], dtype=torch.float64, requires_grad=True)
    w0 = torch.tensor(w["w0_eval"], dtype=torch.float32, device="cuda", requires_grad=True)
    PSF = rw.psf_function()
    I = PSF.apply(c, w0, plan, [dict(x0=x0, y0=y0, z_offset=zo) for x0, y0, zo in shifts])
    s = torch.tensor(scale, dtype=torch.float32, device="cuda").view(-1, 1, 1, 1)
    loss = ((s * I - torch.tensor(Y, dtype=torch.float32, device="cuda")) ** 2).mean()
    loss.backward()
    dc_ref, dw_ref = _oracle_grad(w, shifts, Y, scale)
    assert rel_l2(c.grad.numpy(), dc_ref) < 1e-4
    assert rel_l2(w0.grad.cpu().numpy().astype(np.float64), dw_ref) < 1e-4
