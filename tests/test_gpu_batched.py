"""Batched emitters against the oracle, against single-stack calls, and graph replay against eager."""
import numpy as np
import pytest

import workloads as W
from oracle import fourier as OF
from tests.helpers import oracle_fourier_stack, oracle_optics, rel_l2

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _batch(rw, w, n_max):
    o = w["optics"]
    return rw.Batch(na=o["na"], wavelength=o["wavelength"], n_i=o["n_i"], pixel=w["dx"],
                    plane_pitch=w["dz"], max_emitters=n_max, n_pupil=w["n_pupil"], e_inc=w["e_inc"])


def _emitters(rw, w, idx, crop=None, planes=None):
    S = w["S"][idx] if crop is None else crop
    D = w["D"][idx] if planes is None else planes
    return rw.make_emitters(w["x0"][idx], w["y0"][idx], w["z_e"][idx], S, D, w["zernike"][idx])


def _oracle_emitter(w, x0, y0, ze, S, D, c):
    opt = oracle_optics(w, gl=False)
    z = (np.arange(D) - 0.5 * (D - 1)) * w["dz"] - ze
    return oracle_fourier_stack(opt, w["n_pupil"], S, S, w["dx"], w["dx"], z, zernike=c, x0=x0, y0=y0)


def test_batched_small_matches_oracle_fields_and_intensity(lib):
    import torch
    rw = lib
    w = W.batched(n_emitters=24, seed=31)
    crops = np.array([24, 25, 31, 32, 33, 40, 47, 48, 63, 64, 1, 2, 17, 56, 60, 29, 36, 44, 50, 61, 32, 64, 24, 39])
    planes = np.array([1, 2, 3, 1, 4, 2, 1, 3, 2, 1, 1, 2, 3, 2, 1, 4, 1, 2, 3, 1, 2, 1, 5, 2])
    em = _emitters(rw, w, np.arange(24), crops, planes)
    off = rw.batch_offsets(em)
    b = _batch(rw, w, 64)
    I = torch.zeros(off[-1], dtype=torch.float32, device="cuda")
    E = torch.zeros(3 * off[-1], dtype=torch.complex64, device="cuda")
    b.compute(em, I=I, E=E)
    torch.cuda.synchronize()
    In, En = I.cpu().numpy(), E.cpu().numpy()
    for i in range(24):
        S, D = crops[i], planes[i]
        ref = _oracle_emitter(w, w["x0"][i], w["y0"][i], w["z_e"][i], S, D, w["zernike"][i])
        got_E = En[3 * off[i]:3 * off[i + 1]].reshape(D, 3, S, S)
        got_I = In[off[i]:off[i + 1]].reshape(D, S, S)
        assert rel_l2(got_E, ref) < TOL, (i, S, D)
        assert rel_l2(got_I, OF.intensity(ref)) < TOL, (i, S, D)


def test_batched_equals_single_stack_calls(lib):
    import torch
    rw = lib
    w = W.batched(n_emitters=6, seed=32)
    b = _batch(rw, w, 16)
    crops, planes = np.array([24, 40, 64, 33, 32, 50]), np.array([3, 2, 1, 2, 3, 1])
    em = _emitters(rw, w, np.arange(6), crops, planes)
    off = rw.batch_offsets(em)
    I = torch.zeros(off[-1], dtype=torch.float32, device="cuda")
    b.compute(em, I=I)
    o = w["optics"]
    for i in range(6):
        S, D = int(crops[i]), int(planes[i])
        z = (np.arange(D) - 0.5 * (D - 1)) * w["dz"]
        plan = rw.Plan(form=rw.FORM_FOURIER, na=o["na"], wavelength=o["wavelength"], n_i=o["n_i"], nx=S,
                       ny=S, dx=w["dx"], dy=w["dx"], z=z, e_inc=w["e_inc"], n_pupil=w["n_pupil"])
        _, Ip = plan.compute([dict(x0=w["x0"][i], y0=w["y0"][i], z_offset=-w["z_e"][i],
                                   zernike=w["zernike"][i])], fields=False)
        torch.cuda.synchronize()
        got = I[off[i]:off[i + 1]].cpu().numpy().reshape(D, S, S)
        assert rel_l2(got, Ip[0].cpu().numpy()) < 1e-6


def test_batched_integer_pixel_shift_is_a_translation(lib):
    import torch
    rw = lib
    w = W.batched(n_emitters=2, seed=33)
    px = w["dx"]
    c = w["zernike"][0]
    em = rw.make_emitters([10.0, 10.0 + px], [-5.0, -5.0 - 2 * px], [120.0, 120.0], [40, 40], [2, 2], [c, c])
    b = _batch(rw, w, 4)
    off = rw.batch_offsets(em)
    I = torch.zeros(off[-1], dtype=torch.float32, device="cuda")
    b.compute(em, I=I)
    torch.cuda.synchronize()
    a0 = I[off[0]:off[1]].cpu().numpy().reshape(2, 40, 40)
    a1 = I[off[1]:off[2]].cpu().numpy().reshape(2, 40, 40)
    # emitter 1 sits one pixel further in +x and two in -y: I1[m, n] = I0[m - 1, n + 2]
    np.testing.assert_allclose(a1[:, 1:, :-2], a0[:, :-1, 2:], rtol=0, atol=2e-6 * a0.max())


def test_batched_graph_replays_match_eager(lib):
    import torch
    rw = lib
    w = W.batched(n_emitters=300, seed=34)
    em = _emitters(rw, w, np.arange(300))
    off = rw.batch_offsets(em)
    b = _batch(rw, w, 300)
    I_eager = torch.zeros(off[-1], dtype=torch.float32, device="cuda")
    b.compute(em, I=I_eager)
    torch.cuda.synchronize()
    ref = I_eager.cpu().numpy()
    s = torch.cuda.Stream()
    b.set_graph(True)
    I = torch.zeros(off[-1], dtype=torch.float32, device="cuda")
    for rep in range(4):
        with torch.cuda.stream(s):
            I.zero_()
            b.compute(em, I=I, stream=s.cuda_stream)
        s.synchronize()
        # eager work in between replays
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(I.cpu().numpy(), ref)
    # new emitter values through the same captured graph
    w2 = W.batched(n_emitters=300, seed=35)
    em2 = rw.make_emitters(w2["x0"], w2["y0"], w2["z_e"], w["S"], w["D"], w2["zernike"])
    with torch.cuda.stream(s):
        b.compute(em2, I=I, stream=s.cuda_stream)
    s.synchronize()
    b.set_graph(False)
    I2 = torch.zeros_like(I)
    b.compute(em2, I=I2)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(I.cpu().numpy(), I2.cpu().numpy())


def test_batched_autotune_and_configs_agree(lib):
    import torch
    rw = lib
    w = W.batched(n_emitters=200, seed=36)
    em = _emitters(rw, w, np.arange(200))
    off = rw.batch_offsets(em)
    b = _batch(rw, w, 200)
    I = torch.zeros(off[-1], dtype=torch.float32, device="cuda")
    cfg, ms = b.autotune(em, I)
    assert cfg["wg_per_cu"] in (1, 2, 3) and ms > 0
    assert all(r >= 16 * (q + 1) and r in (16, 32, 48, 64) for q, r in enumerate(cfg["tile_rows"]))
    assert all(k in (8, 16) for k in cfg["k_stage"])
    outs = []
    # every tile class and k-stage: each bucket on its own class, all on 64-row tiles,
    # buckets merged upwards, shallow k-stages
    for c in [dict(wg_per_cu=1), dict(wg_per_cu=2, tile_rows=(64, 64, 64, 64)),
              dict(wg_per_cu=3, tile_rows=(32, 32, 64, 64), k_stage=(8, 8, 8, 8)),
              dict(wg_per_cu=2, tile_rows=(16, 48, 48, 64), k_stage=(8, 16, 8, 16))]:
        b.set_config(**c)
        I.zero_()
        b.compute(em, I=I)
        torch.cuda.synchronize()
        outs.append(I.cpu().numpy())
    for o in outs[1:]:
        assert rel_l2(o, outs[0]) < 1e-6
    with pytest.raises(rw.RwpsfError):
        b.set_config(tile_rows=(16, 16, 48, 64))     # a 17..32 crop does not fit 16 rows
    with pytest.raises(rw.RwpsfError):
        b.set_config(k_stage=(16, 12, 16, 16))


def test_batched_full_workload_sampled(lib):
    """4096 emitters in one launch; 32 seeded emitters checked against the oracle."""
    import torch
    rw = lib
    w = W.batched()
    em = _emitters(rw, w, np.arange(4096))
    off = rw.batch_offsets(em)
    b = _batch(rw, w, 4096)
    I = torch.zeros(off[-1], dtype=torch.float32, device="cuda")
    b.compute(em, I=I)
    torch.cuda.synchronize()
    In = I.cpu().numpy()
    rng = np.random.default_rng(303)
    for i in rng.choice(4096, 32, replace=False):
        S, D = int(w["S"][i]), int(w["D"][i])
        ref = OF.intensity(_oracle_emitter(w, w["x0"][i], w["y0"][i], w["z_e"][i], S, D, w["zernike"][i]))
        assert rel_l2(In[off[i]:off[i + 1]].reshape(D, S, S), ref) < TOL, (i, S, D)


def test_batched_gibson_lanni_per_emitter_depth(lib):
    # each emitter carries its own depth below the coverslip: against the FP64 oracle
    # (fields and intensity) and against plain Fourier-form plans with the same layer
    import torch
    rw = lib
    w = W.batched(n_emitters=8, seed=38)
    w["gl"] = dict(W.GIBSON_LANNI)
    o = w["optics"]
    b = rw.Batch(na=o["na"], wavelength=o["wavelength"], n_i=o["n_i"], pixel=w["dx"], plane_pitch=w["dz"],
                 max_emitters=8, n_pupil=w["n_pupil"], e_inc=w["e_inc"], gibson_lanni=w["gl"])
    crops, planes = np.array([24, 33, 64, 40, 1, 47, 32, 60]), np.array([3, 2, 1, 2, 4, 1, 3, 2])
    t_s = np.array([0.0, 5000.0, 1234.5, 2500.0, 800.0, 4100.0, 10.0, 3333.0])
    idx = np.arange(8)
    em = rw.make_emitters(w["x0"][idx], w["y0"][idx], w["z_e"][idx], crops, planes, w["zernike"][idx], t_s=t_s)
    off = rw.batch_offsets(em)
    I = torch.zeros(off[-1], dtype=torch.float32, device="cuda")
    E = torch.zeros(3 * off[-1], dtype=torch.complex64, device="cuda")
    b.compute(em, I=I, E=E)
    torch.cuda.synchronize()
    In, En = I.cpu().numpy(), E.cpu().numpy()
    opt = oracle_optics(w)
    for i in range(8):
        S, D = int(crops[i]), int(planes[i])
        z = (np.arange(D) - 0.5 * (D - 1)) * w["dz"] - w["z_e"][i]
        ref = oracle_fourier_stack(opt, w["n_pupil"], S, S, w["dx"], w["dx"], z, zernike=w["zernike"][i],
                                   t_s=t_s[i], x0=w["x0"][i], y0=w["y0"][i])
        got_I = In[off[i]:off[i + 1]].reshape(D, S, S)
        assert rel_l2(En[3 * off[i]:3 * off[i + 1]].reshape(D, 3, S, S), ref) < TOL, (i, S, D)
        assert rel_l2(got_I, OF.intensity(ref)) < TOL, (i, S, D)
        plan = rw.Plan(form=rw.FORM_FOURIER, na=o["na"], wavelength=o["wavelength"], n_i=o["n_i"], nx=S,
                       ny=S, dx=w["dx"], dy=w["dx"], z=z + w["z_e"][i], e_inc=w["e_inc"], n_pupil=w["n_pupil"],
                       gibson_lanni=w["gl"])
        _, Ip = plan.compute([dict(x0=w["x0"][i], y0=w["y0"][i], z_offset=-w["z_e"][i], t_s=t_s[i],
                                   zernike=w["zernike"][i])], fields=False)
        torch.cuda.synchronize()
        assert rel_l2(got_I, Ip[0].cpu().numpy()) < 2e-6, i
    em_bad = rw.make_emitters(w["x0"][:1], w["y0"][:1], w["z_e"][:1], [24], [1], w["zernike"][:1], t_s=[-1.0])
    with pytest.raises(rw.RwpsfError):
        b.compute(em_bad, I=I)


def test_batched_validation(lib):
    rw = lib
    w = W.batched(n_emitters=3, seed=37)
    b = _batch(rw, w, 2)
    import torch
    em3 = _emitters(rw, w, np.arange(3))
    I = torch.zeros(rw.batch_offsets(em3)[-1], dtype=torch.float32, device="cuda")   # output large enough
    with pytest.raises(rw.RwpsfError):
        b.compute(em3, I=I)                                       # more than max_emitters
    with pytest.raises(rw.RwpsfError):
        b.compute(_emitters(rw, w, np.arange(1), crop=[65]), I=I)  # crop too large
    with pytest.raises(rw.RwpsfError):
        b.compute(_emitters(rw, w, np.arange(1), planes=[0]), I=I)


def test_batched_autotune_cache(lib, tmp_path, monkeypatch):
    import torch
    rw = lib
    path = tmp_path / "tune.json"
    path.write_text("{ this is not json")             # corrupt cache: ignored, then rewritten
    monkeypatch.setenv("RWPSF_AUTOTUNE_CACHE", str(path))
    w = W.batched(n_emitters=64, seed=38)
    em = _emitters(rw, w, np.arange(64))
    off = rw.batch_offsets(em)
    b = _batch(rw, w, 64)
    I = torch.zeros(off[-1], dtype=torch.float32, device="cuda")
    cfg1, ms1 = b.autotune(em, I)
    text = path.read_text()
    flat = [cfg1["wg_per_cu"], *cfg1["tile_rows"], *cfg1["k_stage"]]
    assert text.strip().startswith("{") and str(flat)[1:-1].replace(" ", "") in text.replace(" ", "")
    b2 = _batch(rw, w, 64)
    cfg2, ms2 = b2.autotune(em, I)                    # served from the cache, no timing
    assert cfg2 == cfg1 and abs(ms2 - ms1) < 1e-3


def test_batched_graph_recaptures_when_tile_classes_change(lib):
    """A captured graph launches only the tile classes (and grid sizes) of its capture:
    a call with the same emitter count and outputs but a crop mix that fills another
    class must not replay it."""
    import torch
    rw = lib
    n = 40
    w = W.batched(n_emitters=n, seed=37)
    b = _batch(rw, w, n)
    b.set_config(2)
    s = torch.cuda.Stream()
    # capture: every crop in 33..48 (48-row class only); then: half the crops at most 32
    crops_a = np.full(n, 48)
    crops_b = np.where(np.arange(n) % 2 == 0, 24, 40)
    planes = np.full(n, 3)
    em_a = _emitters(rw, w, np.arange(n), crops_a, planes)
    em_b = _emitters(rw, w, np.arange(n), crops_b, planes)
    size = max(rw.batch_offsets(em_a)[-1], rw.batch_offsets(em_b)[-1])
    I = torch.zeros(size, dtype=torch.float32, device="cuda")
    b.set_graph(True)
    for em in (em_a, em_b):
        with torch.cuda.stream(s):
            I.fill_(-1.0)
            b.compute(em, I=I, stream=s.cuda_stream)
        s.synchronize()
        b.set_graph(False)
        ref = torch.full_like(I, -1.0)
        b.compute(em, I=ref)
        torch.cuda.synchronize()
        b.set_graph(True)
        np.testing.assert_array_equal(I.cpu().numpy(), ref.cpu().numpy())
    b.set_graph(False)
