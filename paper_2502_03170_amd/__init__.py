"""Python binding of librwpsf (the MI355X vectorial Richards-Wolf PSF engine).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``librwpsf.so``; PyTorch provides device memory and the stream.
The names follow the C ABI in ``include/rwpsf.h`` without the ``rwpsf_``
prefix.  If the library is missing this module raises -- there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import math
import os
from ctypes import POINTER, byref, c_double, c_int, c_size_t, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librwpsf.so")

OK = 0
ERR_INVALID_ARG = -1
ERR_NOT_AXISYMMETRIC = -2
ERR_UNSUPPORTED = -3
ERR_OOM = -4
ERR_HIP = -5
ERR_NO_DEVICE = -6
FORM_BESSEL = 0
FORM_FOURIER = 1
FORM_CHIRPZ = 2
MODEL_VECTORIAL = 0
MODEL_SCALAR = 1
THETA_GAUSS = 0
THETA_SIMPSON = 1
THETA_RIEMANN = 2
SG_GATE_FEATURES = 24
KERNEL_PUPIL_BUILD = 0
KERNEL_GEMM_PUPIL = 1
KERNEL_GEMM_IMAGE = 2
KERNEL_BESSEL_PHI = 3
KERNEL_BESSEL_CONTRACT = 4
KERNEL_BESSEL_EPILOGUE = 5
KERNEL_ADJ_H = 6
KERNEL_ADJ_G = 7
KERNEL_ADJ_REDUCE = 8
KERNEL_CZT_ROWS = 9
KERNEL_CZT_COLS = 10
KERNEL_ADJB_RADIAL = 11
KERNEL_ADJB_CONTRACT = 12
KERNEL_ADJB_REDUCE = 13
KERNEL_BESSEL_FUSED = 14
ERR_SCRATCH_LIMIT = -7
NOALLOC_SCRATCH_BYTES = 16 << 20
MAX_ZERNIKE = 36
CIRCULAR = (1 / math.sqrt(2), 1j / math.sqrt(2))


class RwpsfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"rwpsf error {status}: {msg}")
        self.status = status


class Optics(ctypes.Structure):
    _fields_ = [("na", c_double), ("wavelength_nm", c_double), ("n_i", c_double),
                ("focal_length", c_double), ("ex_re", c_double), ("ex_im", c_double),
                ("ey_re", c_double), ("ey_im", c_double), ("apodization", c_int), ("s_env", c_double),
                ("gibson_lanni", c_int), ("n_s", c_double), ("n_g", c_double),
                ("n_g_design", c_double), ("n_i_design", c_double), ("t_g_nm", c_double),
                ("t_g_design_nm", c_double), ("t_i_design_nm", c_double), ("fresnel", c_int),
                ("extra_sz", c_int)]


class Grid(ctypes.Structure):
    _fields_ = [("nx", c_int), ("ny", c_int), ("dx_nm", c_double), ("dy_nm", c_double),
                ("nz", c_int), ("z_nm", POINTER(c_double))]


class Numerics(ctypes.Structure):
    _fields_ = [("form", c_int), ("n_pupil", c_int), ("n_theta", c_int), ("n_rho", c_int),
                ("model", c_int), ("theta_rule", c_int)]


class Stack(ctypes.Structure):
    _fields_ = [("t_s_nm", c_double), ("x0_nm", c_double), ("y0_nm", c_double),
                ("z_offset_nm", c_double), ("n_zernike", c_int), ("zernike_waves", POINTER(c_double)),
                ("phase_map", c_void_p)]


BATCH_MAX_CROP = 64
BATCH_MAX_ZERNIKE = 21


class Emitter(ctypes.Structure):
    _fields_ = [("x0_nm", c_double), ("y0_nm", c_double), ("z_nm", c_double), ("crop", c_int),
                ("planes", c_int), ("zernike_waves", c_double * BATCH_MAX_ZERNIKE), ("t_s_nm", c_double)]


class BatchConfig(ctypes.Structure):
    _fields_ = [("wg_per_cu", c_int), ("tile_rows", c_int * 4), ("k_stage", c_int * 4)]

    def as_dict(self) -> dict:
        return dict(wg_per_cu=self.wg_per_cu, tile_rows=list(self.tile_rows), k_stage=list(self.k_stage))


def batch_config(wg_per_cu: int = 2, tile_rows=(16, 32, 48, 64), k_stage=(16, 16, 16, 16)) -> BatchConfig:
    """Launch configuration of the batched form: crops of 1-16, 17-32, 33-48, 49-64 pixels on
    row tiles tile_rows[q]; the class of r-row tiles stages k_stage[r / 16 - 1] pupil rows."""
    c = BatchConfig()
    c.wg_per_cu = wg_per_cu
    for q in range(4):
        c.tile_rows[q] = int(tile_rows[q])
        c.k_stage[q] = int(k_stage[q])
    return c


_lib = None


def load(path: str | None = None) -> ctypes.CDLL:
    """Load librwpsf.so (built by ``python -m paper_2502_03170_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"librwpsf.so not found at {path}; build it with "
                           "`python -m paper_2502_03170_amd.build` (no CPU fallback exists)")
    lib = ctypes.CDLL(path)
    sig = {
        "rwpsf_abi_version": (c_int, []),
        "rwpsf_status_string": (ctypes.c_char_p, [c_int]),
        "rwpsf_last_hip_error": (c_int, []),
        "rwpsf_validate": (c_int, [POINTER(Optics), POINTER(Grid), POINTER(Numerics)]),
        "rwpsf_validate_stacks": (c_int, [POINTER(Optics), POINTER(Grid), POINTER(Numerics), c_int,
                                          POINTER(Stack)]),
        "rwpsf_plan_create": (c_int, [POINTER(Optics), POINTER(Grid), POINTER(Numerics),
                                      POINTER(c_void_p)]),
        "rwpsf_plan_destroy": (None, [c_void_p]),
        "rwpsf_plan_device_bytes": (c_size_t, [c_void_p]),
        "rwpsf_compute": (c_int, [c_void_p, c_int, POINTER(Stack), c_void_p, c_void_p, c_void_p]),
        "rwpsf_compute_noalloc": (c_int, [c_void_p, c_int, POINTER(Stack), c_void_p, c_void_p, c_void_p]),
        "rwpsf_plan_set_timing": (c_int, [c_void_p, c_int]),
        "rwpsf_plan_timing": (c_int, [c_void_p, c_int, POINTER(c_double), POINTER(ctypes.c_int64)]),
        "rwpsf_adjoint": (c_int, [c_void_p, c_int, POINTER(Stack), c_void_p, c_void_p, c_int, c_void_p,
                                  c_void_p, c_void_p]),
        "rwpsf_adjoint_bessel": (c_int, [c_void_p, c_int, POINTER(Stack), c_void_p, c_void_p, c_void_p,
                                         c_void_p, c_void_p, c_void_p]),
        "rwpsf_sg_param_count": (c_size_t, []),
        "rwpsf_sg_create": (c_int, [c_int, POINTER(c_void_p)]),
        "rwpsf_sg_destroy": (None, [c_void_p]),
        "rwpsf_sg_set_state": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, ctypes.c_int64]),
        "rwpsf_sg_get_state": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                       POINTER(ctypes.c_int64)]),
        "rwpsf_sg_forward": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_int, c_void_p]),
        "rwpsf_sg_gradient": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
        "rwpsf_sg_adam": (c_int, [c_void_p, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                  c_void_p]),
        "rwpsf_sg_error_features": (c_int, [c_int, c_void_p, c_void_p, c_void_p, c_void_p]),
        "rwpsf_sg_error_predict": (c_int, [c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
        "rwpsf_batch_create": (c_int, [POINTER(Optics), c_int, c_double, c_double, c_int, POINTER(c_void_p)]),
        "rwpsf_batch_destroy": (None, [c_void_p]),
        "rwpsf_batch_offsets": (c_int, [c_int, POINTER(Emitter), POINTER(ctypes.c_int64)]),
        "rwpsf_batch_compute": (c_int, [c_void_p, c_int, POINTER(Emitter), c_void_p, c_void_p, c_void_p]),
        "rwpsf_batch_set_graph": (c_int, [c_void_p, c_int]),
        "rwpsf_batch_set_config": (c_int, [c_void_p, POINTER(BatchConfig)]),
        "rwpsf_batch_get_config": (c_int, [c_void_p, POINTER(BatchConfig)]),
        "rwpsf_batch_autotune": (c_int, [c_void_p, c_int, POINTER(Emitter), c_void_p, c_void_p,
                                         POINTER(BatchConfig), POINTER(c_double)]),
        "rwpsf_gauss_legendre": (c_int, [c_int, c_double, c_double, POINTER(c_double), POINTER(c_double)]),
        "rwpsf_bessel_j": (c_int, [c_int, c_int, POINTER(c_double), POINTER(c_double)]),
        "rwpsf_zernike": (c_int, [c_int, c_int, POINTER(c_double), POINTER(c_double), POINTER(c_double)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def status_string(status: int) -> str:
    return load().rwpsf_status_string(status).decode()


def _check(status: int):
    if status != OK:
        raise RwpsfError(status, status_string(status))


def abi_version() -> int:
    return load().rwpsf_abi_version()


def check_tensor(t, name: str, dtype, numel: int, required: bool = True) -> c_void_p:
    """The device pointer of tensor ``t`` after checking what the library will assume of
    it: ``dtype``, contiguous, at least ``numel`` elements, on the current CUDA device.
    None gives a NULL pointer when the argument is optional.  Raises ValueError before
    anything reaches the library (an undersized or mistyped buffer would otherwise be
    read or written out of bounds on the device)."""
    import torch
    if t is None:
        if required:
            raise ValueError(f"{name} is required")
        return c_void_p(0)
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor, got {type(t).__name__}")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() < numel:
        raise ValueError(f"{name} has {t.numel()} elements, needs at least {numel}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA tensor")
    if t.device.index != torch.cuda.current_device():
        raise ValueError(f"{name} is on cuda:{t.device.index}, the current device is "
                         f"cuda:{torch.cuda.current_device()}")
    return c_void_p(t.data_ptr())


# ---------------------------------------------------------------- struct builders
def make_optics(na, wavelength, n_i, e_inc=CIRCULAR, focal_length=1.0, apodization=True, s_env=0.0,
                gibson_lanni: dict | None = None, fresnel: tuple | None = None,
                extra_sz: bool = False) -> Optics:
    """``fresnel`` = (n_s, n_g): Fresnel transmission sample -> coverslip -> immersion
    (the same indices as the Gibson-Lanni layer when both are given)."""
    ex, ey = complex(e_inc[0]), complex(e_inc[1])
    o = Optics(na=na, wavelength_nm=wavelength, n_i=n_i, focal_length=focal_length, ex_re=ex.real,
               ex_im=ex.imag, ey_re=ey.real, ey_im=ey.imag, apodization=int(bool(apodization)),
               s_env=s_env)
    if gibson_lanni:
        g = gibson_lanni
        o.gibson_lanni = 1
        o.n_s = g["n_s"]
        o.n_g = g.get("n_g", 1.5)
        o.n_g_design = g.get("n_g_design", 1.5)
        o.n_i_design = g.get("n_i_design", n_i) or n_i
        o.t_g_nm = g.get("t_g", 170e3)
        o.t_g_design_nm = g.get("t_g_design", 170e3)
        o.t_i_design_nm = g.get("t_i_design", 150e3)
    if fresnel is not None:
        n_s, n_g = float(fresnel[0]), float(fresnel[1])
        if gibson_lanni and (n_s != o.n_s or n_g != o.n_g):
            raise ValueError("the Fresnel media must be the Gibson-Lanni layer's n_s, n_g")
        o.fresnel = 1
        o.n_s, o.n_g = n_s, n_g
    o.extra_sz = int(bool(extra_sz))
    return o


def make_grid(nx, ny, dx, dy, z):
    zarr = (c_double * len(z))(*[float(v) for v in z])
    g = Grid(nx=nx, ny=ny, dx_nm=dx, dy_nm=dy, nz=len(z), z_nm=zarr)
    g._keep = zarr
    return g


def make_stacks(stacks: list[dict], n_pupil: int | None = None):
    """rwpsf_stack array; a phase map must be a float32 CUDA tensor of n_pupil^2 cells
    (checked against n_pupil when it is given, else when the stacks reach a plan)."""
    import torch
    arr = (Stack * len(stacks))()
    keep = []
    for i, s in enumerate(stacks):
        c = s.get("zernike")
        arr[i].t_s_nm = float(s.get("t_s", 0.0))
        arr[i].x0_nm = float(s.get("x0", 0.0))
        arr[i].y0_nm = float(s.get("y0", 0.0))
        arr[i].z_offset_nm = float(s.get("z_offset", 0.0))
        if c is not None and len(c):
            buf = (c_double * len(c))(*[float(v) for v in c])
            keep.append(buf)
            arr[i].n_zernike = len(c)
            arr[i].zernike_waves = ctypes.cast(buf, POINTER(c_double))
        pm = s.get("phase_map")
        if pm is not None:
            keep.append(pm)
            arr[i].phase_map = check_tensor(pm, f"stacks[{i}].phase_map", torch.float32,
                                            0 if n_pupil is None else n_pupil * n_pupil)
    return arr, keep


class Stacks:
    """A list of stack dicts marshalled once into an rwpsf_stack array, for calls that
    repeat with the same stacks (the marshalling of many stacks costs host time)."""

    def __init__(self, stacks: list[dict], n_pupil: int | None = None):
        self.arr, self.keep = make_stacks(stacks, n_pupil)
        self.maps = [s["phase_map"] for s in stacks if s.get("phase_map") is not None]
        self.n = len(stacks)

    def __len__(self):
        return self.n


def _marshal(stacks, n_pupil: int | None = None):
    if isinstance(stacks, Stacks):
        if n_pupil is not None:
            for pm in stacks.maps:
                if pm.numel() < n_pupil * n_pupil:
                    raise ValueError(f"a phase map has {pm.numel()} cells, the plan's pupil {n_pupil ** 2}")
        return stacks.arr, stacks.keep
    return make_stacks(stacks, n_pupil)


# ---------------------------------------------------------------- ABI mirrors
def validate(optics: Optics, grid: Grid, num: Numerics) -> int:
    return load().rwpsf_validate(byref(optics), byref(grid), byref(num))


def validate_stacks(optics: Optics, grid: Grid, num: Numerics, stacks: list[dict]) -> int:
    arr, _keep = make_stacks(stacks)
    return load().rwpsf_validate_stacks(byref(optics), byref(grid), byref(num), len(stacks), arr)


def gauss_legendre(n: int, a: float, b: float):
    x, w = (c_double * n)(), (c_double * n)()
    _check(load().rwpsf_gauss_legendre(n, a, b, x, w))
    return list(x), list(w)


def bessel_j(order: int, xs):
    n = len(xs)
    x, out = (c_double * n)(*[float(v) for v in xs]), (c_double * n)()
    _check(load().rwpsf_bessel_j(order, n, x, out))
    return list(out)


def zernike(j: int, r, phi):
    n = len(r)
    ra, pa, out = (c_double * n)(*map(float, r)), (c_double * n)(*map(float, phi)), (c_double * n)()
    _check(load().rwpsf_zernike(j, n, ra, pa, out))
    return list(out)


def plan_create(optics: Optics, grid: Grid, num: Numerics) -> c_void_p:
    h = c_void_p()
    _check(load().rwpsf_plan_create(byref(optics), byref(grid), byref(num), byref(h)))
    return h


def plan_destroy(handle) -> None:
    load().rwpsf_plan_destroy(handle)


def plan_set_timing(handle, enable: bool) -> None:
    _check(load().rwpsf_plan_set_timing(handle, int(bool(enable))))


def plan_timing(handle, kernel: int):
    """(total milliseconds, launches) of one kernel since timing was enabled."""
    ms, n = c_double(), ctypes.c_int64()
    _check(load().rwpsf_plan_timing(handle, kernel, byref(ms), byref(n)))
    return ms.value, n.value


def _stream(stream):
    import torch
    return c_void_p(torch.cuda.current_stream().cuda_stream if stream is None else stream)


def compute(plan, stacks, E=None, I=None, stream=None, noalloc: bool = False) -> None:
    """Enqueue rwpsf_compute for a ``Plan``: E complex64 [stacks][nz][channels][nx][ny] and
    I float32 [stacks][nz][nx][ny] CUDA tensors (either may be None, not both).
    ``stacks`` is a list of dicts or a ``Stacks``.  ``noalloc`` calls the allocation-free
    variant rwpsf_compute_noalloc instead (Bessel form)."""
    import torch
    arr, _keep = _marshal(stacks, plan.num.n_pupil if plan.num.form != FORM_BESSEL else None)
    vox = len(stacks) * plan.nz * plan.nx * plan.ny
    e = check_tensor(E, "E", torch.complex64, vox * plan.nc, required=False)
    i = check_tensor(I, "I", torch.float32, vox, required=False)
    fn = load().rwpsf_compute_noalloc if noalloc else load().rwpsf_compute
    _check(fn(plan.handle, len(stacks), arr, e, i, _stream(stream)))


def adjoint(plan, stacks, E, dL_dI, n_zernike: int, dL_dc=None, dL_dW0=None, stream=None):
    """Enqueue rwpsf_adjoint for a Fourier ``Plan``: E complex64 and dL_dI float32 as
    written by ``compute``; outputs float32 dL_dc [n_zernike] and dL_dW0 [N][N] (either may
    be None).  ``stacks`` is a list of dicts or a ``Stacks``."""
    import torch
    arr, _keep = _marshal(stacks, plan.num.n_pupil)
    vox = len(stacks) * plan.nz * plan.nx * plan.ny
    if n_zernike < 0 or n_zernike > MAX_ZERNIKE:
        raise ValueError(f"n_zernike must be in 0..{MAX_ZERNIKE}")
    args = (check_tensor(E, "E", torch.complex64, vox * plan.nc), check_tensor(dL_dI, "dL_dI", torch.float32, vox),
            n_zernike, check_tensor(dL_dc, "dL_dc", torch.float32, n_zernike, required=False),
            check_tensor(dL_dW0, "dL_dW0", torch.float32, plan.num.n_pupil ** 2, required=False))
    _check(load().rwpsf_adjoint(plan.handle, len(stacks), arr, *args, _stream(stream)))


def adjoint_bessel(plan, stacks, E, dL_dI, dL_dc=None, dL_dts=None, dL_dz=None, stream=None):
    """Enqueue rwpsf_adjoint_bessel for a Bessel ``Plan`` (E complex64, dL_dI float32; outputs
    float32 CUDA tensors: dL_dc [4] for Noll 1, 4, 11, 22, dL_dts and dL_dz [n_stacks]; any
    may be None)."""
    import torch
    arr, _keep = _marshal(stacks)
    n = len(stacks)
    vox = n * plan.nz * plan.nx * plan.ny
    args = (check_tensor(E, "E", torch.complex64, vox * plan.nc), check_tensor(dL_dI, "dL_dI", torch.float32, vox),
            check_tensor(dL_dc, "dL_dc", torch.float32, 4, required=False),
            check_tensor(dL_dts, "dL_dts", torch.float32, n, required=False),
            check_tensor(dL_dz, "dL_dz", torch.float32, n, required=False))
    _check(load().rwpsf_adjoint_bessel(plan.handle, n, arr, *args, _stream(stream)))


def _psf_function():
    import torch

    class PSFFunction(torch.autograd.Function):
        """I = PSF(c, W0): intensity stacks of a Fourier plan as a differentiable function of
        Zernike coefficients c (CPU float64, Noll 1..K, waves) and a pupil phase map W0
        (CUDA float32 [N][N], radians) shared by all stacks.  The backward is rwpsf_adjoint."""

        @staticmethod
        def forward(ctx, c, w0, plan, stacks):
            st = [dict(s, zernike=c.detach().cpu().double().numpy(), phase_map=w0.detach().contiguous())
                  for s in stacks]
            E, I = plan.compute(st)
            ctx.save_for_backward(E)
            ctx.plan, ctx.stacks, ctx.nz = plan, st, c.numel()
            ctx.c_device, ctx.c_dtype = c.device, c.dtype
            return I

        @staticmethod
        def backward(ctx, grad_I):
            (E,) = ctx.saved_tensors
            n = ctx.nz
            dc = torch.empty(max(n, 1), dtype=torch.float32, device="cuda")
            dw = torch.empty_like(ctx.stacks[0]["phase_map"])
            adjoint(ctx.plan, ctx.stacks, E, grad_I.contiguous().float(), n, dc, dw)
            return dc[:n].to(ctx.c_device, ctx.c_dtype), dw, None, None

    return PSFFunction


_PSF = None


def psf_function():
    """The torch.autograd.Function class (created on first use, torch imported lazily)."""
    global _PSF
    if _PSF is None:
        _PSF = _psf_function()
    return _PSF


def make_emitters(x0, y0, z, crop, planes, zernike, t_s=None):
    """An rwpsf_emitter array from per-emitter sequences (filled through a NumPy view of the
    ctypes array, field by field).  ``t_s``: per-emitter depth below the coverslip (nm),
    read with the Gibson-Lanni layer."""
    import numpy as np
    n = len(x0)
    arr = (Emitter * n)()
    if n == 0:
        return arr
    dt = np.dtype({"names": [f[0] for f in Emitter._fields_],
                   "formats": ["f8", "f8", "f8", "i4", "i4", ("f8", (BATCH_MAX_ZERNIKE,)), "f8"],
                   "offsets": [getattr(Emitter, f[0]).offset for f in Emitter._fields_],
                   "itemsize": ctypes.sizeof(Emitter)})
    v = np.frombuffer(arr, dtype=dt)
    v["x0_nm"], v["y0_nm"], v["z_nm"] = (np.asarray(a, dtype=np.float64).reshape(n) for a in (x0, y0, z))
    v["t_s_nm"] = 0.0 if t_s is None else np.asarray(t_s, dtype=np.float64).reshape(n)
    v["crop"], v["planes"] = (np.asarray(a).reshape(n).astype(np.int32) for a in (crop, planes))
    c = np.zeros((n, BATCH_MAX_ZERNIKE))
    zz = np.asarray(zernike, dtype=np.float64).reshape(n, -1)
    q = min(zz.shape[1], BATCH_MAX_ZERNIKE)
    c[:, :q] = zz[:, :q]
    v["zernike_waves"] = c
    return arr


def batch_offsets(emitters) -> list:
    n = len(emitters)
    off = (ctypes.c_int64 * (n + 1))()
    _check(load().rwpsf_batch_offsets(n, emitters, off))
    return list(off)


class Batch:
    """Batched emitters (rwpsf_batch_*): one persistent launch for many small stacks."""

    def __init__(self, *, na, wavelength, n_i, pixel, plane_pitch, max_emitters, n_pupil=128,
                 e_inc=CIRCULAR, focal_length=1.0, apodization=True, s_env=0.0, gibson_lanni=None,
                 fresnel=None, extra_sz=False):
        self.optics = make_optics(na, wavelength, n_i, e_inc, focal_length, apodization, s_env, gibson_lanni,
                                  fresnel, extra_sz)
        h = c_void_p()
        _check(load().rwpsf_batch_create(byref(self.optics), n_pupil, pixel, plane_pitch, max_emitters,
                                         byref(h)))
        self.handle = h

    def set_graph(self, enable: bool):
        _check(load().rwpsf_batch_set_graph(self.handle, int(bool(enable))))

    def set_config(self, wg_per_cu: int = 2, tile_rows=(16, 32, 48, 64), k_stage=(16, 16, 16, 16)):
        cfg = batch_config(wg_per_cu, tile_rows, k_stage)
        _check(load().rwpsf_batch_set_config(self.handle, byref(cfg)))

    def get_config(self):
        cfg = BatchConfig()
        _check(load().rwpsf_batch_get_config(self.handle, byref(cfg)))
        return cfg.as_dict()

    def compute(self, emitters, I=None, E=None, stream=None):
        """I float32 [total voxels] and E complex64 [3 total voxels] (CUDA; either may be None)."""
        import torch
        vox = batch_offsets(emitters)[-1]
        i = check_tensor(I, "I", torch.float32, vox, required=False)
        e = check_tensor(E, "E", torch.complex64, 3 * vox, required=False)
        _check(load().rwpsf_batch_compute(self.handle, len(emitters), emitters, i, e, _stream(stream)))

    def autotune(self, emitters, I, stream=None):
        import torch
        i = check_tensor(I, "I", torch.float32, batch_offsets(emitters)[-1])
        cfg, ms = BatchConfig(), c_double()
        _check(load().rwpsf_batch_autotune(self.handle, len(emitters), emitters, i, _stream(stream),
                                           byref(cfg), byref(ms)))
        return cfg.as_dict(), ms.value

    def close(self):
        if self.handle:
            load().rwpsf_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


SG_BF16X3 = 0
SG_BF16 = 1


class Surrogate:
    """The learned surrogate (rwpsf_sg_*): parameters and Adam state live on the device."""

    def __init__(self, max_batch: int):
        h = c_void_p()
        _check(load().rwpsf_sg_create(max_batch, byref(h)))
        self.handle = h
        self.max_batch = max_batch
        self.n_params = load().rwpsf_sg_param_count()

    def set_state(self, params, m=None, v=None, step: int = 0):
        import numpy as np
        arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float32) for a in (params, m, v)]
        ptr = [c_void_p(a.ctypes.data) if a is not None else c_void_p(0) for a in arrs]
        _check(load().rwpsf_sg_set_state(self.handle, *ptr, step))

    def get_state(self):
        import numpy as np
        w, m, v, g = (np.empty(self.n_params, dtype=np.float32) for _ in range(4))
        step = ctypes.c_int64()
        _check(load().rwpsf_sg_get_state(self.handle, c_void_p(w.ctypes.data), c_void_p(m.ctypes.data),
                                         c_void_p(v.ctypes.data), c_void_p(g.ctypes.data), byref(step)))
        return dict(params=w, adam_m=m, adam_v=v, grads=g, step=step.value)

    def _inputs(self, coef, z):
        import torch
        if coef.dim() != 2 or coef.shape[1] != 21:
            raise ValueError("coef must be [B][21]")
        B = coef.shape[0]
        if not 1 <= B <= self.max_batch:
            raise ValueError(f"batch {B} outside 1..{self.max_batch}")
        return B, check_tensor(coef, "coef", torch.float32, 21 * B), check_tensor(z, "z", torch.float32, B)

    def forward(self, coef, z, out=None, precision=SG_BF16X3, stream=None):
        """out = net(coef [B][21], z [B]) as float32 [B][64][64] (CUDA tensors)."""
        import torch
        B, c, zz = self._inputs(coef, z)
        if out is None:
            out = torch.empty((B, 64, 64), dtype=torch.float32, device="cuda")
        o = check_tensor(out, "out", torch.float32, B * 64 * 64)
        _check(load().rwpsf_sg_forward(self.handle, B, c, zz, o, precision, _stream(stream)))
        return out

    def gradient(self, coef, z, target, loss=None, stream=None):
        import torch
        B, c, zz = self._inputs(coef, z)
        t = check_tensor(target, "target", torch.float32, B * 64 * 64)
        lo = check_tensor(loss, "loss", torch.float32, 1, required=False)
        _check(load().rwpsf_sg_gradient(self.handle, B, c, zz, t, lo, _stream(stream)))

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        _check(load().rwpsf_sg_adam(self.handle, lr, beta1, beta2, eps, _stream(stream)))

    def error_features(self, coef, z, out=None, stream=None):
        """Features phi(c, z) [B][24] of the gate's error model (rwpsf_sg_error_features)."""
        import torch
        B, c, zz = self._inputs(coef, z)
        if out is None:
            out = torch.empty((B, SG_GATE_FEATURES), dtype=torch.float32, device="cuda")
        o = check_tensor(out, "out", torch.float32, B * SG_GATE_FEATURES)
        _check(load().rwpsf_sg_error_features(B, c, zz, o, _stream(stream)))
        return out

    def error_predict(self, coef, z, weights, out=None, stream=None):
        """Predicted log rel-L2 w . phi(c, z) [B] for the gate weights w [24]."""
        import torch
        B, c, zz = self._inputs(coef, z)
        w = check_tensor(weights, "weights", torch.float32, SG_GATE_FEATURES)
        if out is None:
            out = torch.empty(B, dtype=torch.float32, device="cuda")
        o = check_tensor(out, "out", torch.float32, B)
        _check(load().rwpsf_sg_error_predict(B, c, zz, w, o, _stream(stream)))
        return out

    def close(self):
        if self.handle:
            load().rwpsf_sg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """A plan of the C ABI with torch-allocated outputs."""

    def __init__(self, *, form: int, na: float, wavelength: float, n_i: float, nx: int, ny: int,
                 dx: float, dy: float, z, e_inc=CIRCULAR, focal_length: float = 1.0,
                 apodization: bool = True, s_env: float = 0.0, gibson_lanni: dict | None = None,
                 n_pupil: int = 256, n_theta: int = 200, n_rho: int = 256,
                 model: int = MODEL_VECTORIAL, theta_rule: int = THETA_GAUSS,
                 fresnel: tuple | None = None, extra_sz: bool = False):
        self.optics = make_optics(na, wavelength, n_i, e_inc, focal_length, apodization, s_env,
                                  gibson_lanni, fresnel, extra_sz)
        self.grid = make_grid(nx, ny, dx, dy, list(z))
        self.num = Numerics(form=form, n_pupil=n_pupil, n_theta=n_theta, n_rho=n_rho, model=model,
                            theta_rule=theta_rule)
        self.nx, self.ny, self.nz = nx, ny, len(z)
        self.nc = 1 if model == MODEL_SCALAR else 3   # output channels
        self.handle = plan_create(self.optics, self.grid, self.num)

    def set_timing(self, enable: bool) -> None:
        plan_set_timing(self.handle, enable)

    def timing(self, kernel: int):
        return plan_timing(self.handle, kernel)

    def device_bytes(self) -> int:
        return load().rwpsf_plan_device_bytes(self.handle)

    def compute(self, stacks: list[dict], fields: bool = True, intensity: bool = True, E=None, I=None,
                stream=None, noalloc: bool = False):
        import torch
        b = len(stacks)
        if fields and E is None:
            E = torch.empty((b, self.nz, self.nc, self.nx, self.ny), dtype=torch.complex64, device="cuda")
        if intensity and I is None:
            I = torch.empty((b, self.nz, self.nx, self.ny), dtype=torch.float32, device="cuda")
        compute(self, stacks, E if fields else None, I if intensity else None, stream, noalloc)
        return E, I

    def adjoint_bessel(self, stacks, E, dL_dI, dc=None, dts=None, dz=None, stream=None):
        """(dL/dc for Noll 1, 4, 11, 22 [4], dL/dt_s [n], dL/dz_offset [n]) of the Bessel form,
        into the given float32 tensors or new ones."""
        import torch
        n = len(stacks)
        dc = torch.empty(4, dtype=torch.float32, device="cuda") if dc is None else dc
        dts = torch.empty(n, dtype=torch.float32, device="cuda") if dts is None else dts
        dz = torch.empty(n, dtype=torch.float32, device="cuda") if dz is None else dz
        adjoint_bessel(self, stacks, E, dL_dI, dc, dts, dz, stream)
        return dc, dts, dz

    def adjoint(self, stacks, E, dL_dI, n_zernike: int, dc=None, dw=None, stream=None):
        """(dL/dc [n_zernike], dL/dW0 [N][N]) for a loss with per-voxel dL/dI, into the given
        float32 tensors or new ones."""
        import torch
        if dc is None:
            dc = torch.empty(max(n_zernike, 1), dtype=torch.float32, device="cuda")
        if dw is None:
            dw = torch.empty((self.num.n_pupil, self.num.n_pupil), dtype=torch.float32, device="cuda")
        adjoint(self, stacks, E, dL_dI, n_zernike, dc, dw, stream)
        return dc[:n_zernike], dw

    def close(self):
        if self.handle:
            plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
