"""The binding refuses tensors the library would misread before any pointer reaches it
(host logic; no GPU needed)."""
import numpy as np
import pytest
import torch

import paper_2502_03170_amd as rw


def test_optional_none_is_null_and_required_none_raises():
    assert rw.check_tensor(None, "x", torch.float32, 4, required=False).value is None
    with pytest.raises(ValueError, match="required"):
        rw.check_tensor(None, "x", torch.float32, 4)


@pytest.mark.parametrize("t, msg", [
    (torch.zeros(16, dtype=torch.float64), "must be torch.float32"),
    (torch.zeros(4, 8).t(), "contiguous"),
    (torch.zeros(15), "needs at least 16"),
    (torch.zeros(16), "CUDA"),
    ([0.0] * 16, "torch tensor"),
])
def test_bad_tensors_raise(t, msg):
    with pytest.raises(ValueError, match=msg):
        rw.check_tensor(t, "x", torch.float32, 16)


def test_phase_map_checked_when_stacks_are_marshalled():
    # a float64 map would be read as the wrong floats, a CPU map dereferenced on the GPU
    with pytest.raises(ValueError, match="phase_map must be torch.float32"):
        rw.make_stacks([dict(phase_map=torch.zeros(64, 64, dtype=torch.float64))], n_pupil=64)
    with pytest.raises(ValueError, match="needs at least 4096"):
        rw.make_stacks([dict(phase_map=torch.zeros(32, 32))], n_pupil=64)
    with pytest.raises(ValueError, match="CUDA"):
        rw.make_stacks([dict(phase_map=torch.zeros(64, 64))], n_pupil=64)


def test_make_emitters_fills_every_field():
    """The NumPy view that fills the ctypes emitter array puts each value in its C field."""
    import ctypes
    rng = np.random.default_rng(0)
    n = 37
    x0, y0, z = rng.normal(size=(3, n))
    S, D = rng.integers(1, 65, n), rng.integers(1, 41, n)
    c, ts = rng.normal(size=(n, 21)), rng.uniform(0, 5000, n)
    a = rw.make_emitters(x0, y0, z, S, D, c, ts)
    assert ctypes.sizeof(a) == n * ctypes.sizeof(rw.Emitter)
    for i in range(n):
        e = a[i]
        assert (e.x0_nm, e.y0_nm, e.z_nm, e.crop, e.planes, e.t_s_nm) == (x0[i], y0[i], z[i], S[i], D[i], ts[i])
        assert list(e.zernike_waves) == list(c[i])
    b = rw.make_emitters([1.0], [2.0], [3.0], [5], [2], [[0.1, 0.2]])
    assert (b[0].crop, b[0].planes, b[0].t_s_nm) == (5, 2, 0.0)
    assert list(b[0].zernike_waves) == [0.1, 0.2] + [0.0] * 19
