#!/usr/bin/env python
"""Benchmark of the vectorial Richards-Wolf PSF engine on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

A step is one ``rwpsf_compute`` call of the Fourier (Cartesian) form on the
headline workload: 16 stacks, each 128 x 128 x 64 voxels at 20 nm from a
256 x 256 pupil, NA 1.4, 600 nm, circular polarisation, Gibson-Lanni (n_s 1.33,
emitter depth U[0, 5] um) and Noll 4..21 aberrations N(0, 0.05) waves; fields
(complex64) and intensity (float32) are both written.  Inputs are synthetic and
seeded (``workloads``), resident on the GPU before the timed region.

Prints one JSON line with the throughput (voxels/s), the roofline of the
dominant kernel (per-launch time from HIP events on the library's stream during
the timed steps), the CPU oracle timed on a bounded sample, and the other forms.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3   # MI355X dense FP32 matrix
PEAK_HBM_GBS = 8000.0      # MI355X HBM3E


def fourier_workload():
    import workloads as W
    w = W.fourier_plain()
    zp = np.linspace(-1000.0, 1000.0, 64)
    stacks = [dict(t_s=w["t_s"][b], z_offset=-w["t_s"][b], zernike=w["zernike"][b]) for b in range(16)]
    return w, zp, stacks


def bench_fourier(rw, torch, steps, warmup):
    w, zp, stacks = fourier_workload()
    o = w["optics"]
    n, nx, nz, B = 256, 128, 64, len(stacks)
    plan = rw.Plan(form=rw.FORM_FOURIER, na=o["na"], wavelength=o["wavelength"], n_i=o["n_i"], nx=nx,
                   ny=nx, dx=20.0, dy=20.0, z=zp, e_inc=w["e_inc"], gibson_lanni=w["gl"], n_pupil=n)
    E = torch.empty((B, nz, 3, nx, nx), dtype=torch.complex64, device="cuda")
    I = torch.empty((B, nz, nx, nx), dtype=torch.float32, device="cuda")
    for _ in range(warmup):
        plan.compute(stacks, E=E, I=I)
    torch.cuda.synchronize()
    plan.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.compute(stacks, E=E, I=I)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / steps
    kt = {name: plan.timing(k) for name, k in (("pupil_build", rw.KERNEL_PUPIL_BUILD),
                                               ("gemm_pupil", rw.KERNEL_GEMM_PUPIL),
                                               ("gemm_image", rw.KERNEL_GEMM_IMAGE))}
    plan.set_timing(False)
    voxels = B * nz * nx * nx
    # algorithmic work of the separable matrix DFT, per component-plane
    f1 = 8.0 * n * n * nx            # T = P~ Ay^T
    f2 = 8.0 * nx * n * nx           # E = Ax T
    comp_planes = B * nz * 3
    g1_ms, g1_n = kt["gemm_pupil"]
    g2_ms, g2_n = kt["gemm_image"]
    per_launch_g1 = f1 * comp_planes * steps / g1_n      # launches are counted over all timed steps
    per_launch_g2 = f2 * comp_planes * steps / g2_n
    ach_g1 = per_launch_g1 / (g1_ms / g1_n * 1e-3) / 1e12
    ach_g2 = per_launch_g2 / (g2_ms / g2_n * 1e-3) / 1e12
    step_flops = (f1 + f2) * comp_planes
    plan.close()
    return dict(
        ms_per_step=ms_step, voxels=voxels, value=voxels / (ms_step * 1e-3),
        kernels={k: dict(total_ms=v[0], launches=v[1], avg_us=(v[0] / v[1] * 1e3 if v[1] else None))
                 for k, v in kt.items()},
        roofline=dict(kernel="gemm_pupil_kernel", bound="mfma", achieved=round(ach_g1, 3),
                      peak=PEAK_FP32_TFLOPS, unit="TFLOP/s", frac=round(ach_g1 / PEAK_FP32_TFLOPS, 4),
                      traffic=None, flops_per_launch=per_launch_g1,
                      avg_launch_us=g1_ms / g1_n * 1e3),
        image_gemm=dict(achieved_tflops=round(ach_g2, 3), frac=round(ach_g2 / PEAK_FP32_TFLOPS, 4),
                        flops_per_launch=per_launch_g2, avg_launch_us=g2_ms / g2_n * 1e3),
        step_tflops=round(step_flops / (ms_step * 1e-3) / 1e12, 3),
        step_frac=round(step_flops / (ms_step * 1e-3) / 1e12 / PEAK_FP32_TFLOPS, 4))


def bench_bessel(rw, torch, steps, warmup, n_stacks=256):
    import workloads as W
    w = W.bessel_plain(n_stacks=n_stacks)
    o = w["optics"]
    plan = rw.Plan(form=rw.FORM_BESSEL, na=o["na"], wavelength=o["wavelength"], n_i=o["n_i"], nx=65,
                   ny=65, dx=20.0, dy=20.0, z=w["z"], e_inc=w["e_inc"], n_theta=200, n_rho=256)
    stacks = [dict(z_offset=float(v)) for v in w["z_offsets"]]
    nz = len(w["z"])
    E = torch.empty((n_stacks, nz, 3, 65, 65), dtype=torch.complex64, device="cuda")
    I = torch.empty((n_stacks, nz, 65, 65), dtype=torch.float32, device="cuda")
    one = [dict()]
    for _ in range(warmup):
        plan.compute(stacks, E=E, I=I)
        plan.compute(one, E=E[:1], I=I[:1])
    torch.cuda.synchronize()
    # single stack latency
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.compute(one, E=E[:1], I=I[:1])
    torch.cuda.synchronize()
    single_ms = (time.perf_counter() - t0) * 1e3 / steps
    plan.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.compute(stacks, E=E, I=I)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    kt = {name: plan.timing(k) for name, k in (("phi", rw.KERNEL_BESSEL_PHI),
                                               ("contract", rw.KERNEL_BESSEL_CONTRACT),
                                               ("epilogue", rw.KERNEL_BESSEL_EPILOGUE))}
    plan.close()
    voxels = n_stacks * nz * 65 * 65
    e_ms, e_n = kt["epilogue"]
    bytes_per_launch = 28.0 * voxels * steps / e_n    # E (24 B) + I (4 B) per voxel written
    ach = bytes_per_launch / (e_ms / e_n * 1e-3) / 1e9
    return dict(workload="bessel_plain: NA 1.4, 532 nm, 65x65x33 at 20 nm, GL-200, 256 radial samples, "
                         f"{n_stacks} stacks per call (focal offsets U(+-100 nm))",
                value=voxels / (ms * 1e-3), unit="voxels/s", ms_per_call=ms,
                single_stack_ms=single_ms, single_stack_voxels_per_s=65 * 65 * nz / (single_ms * 1e-3),
                kernels={k: dict(total_ms=v[0], launches=v[1], avg_us=(v[0] / v[1] * 1e3 if v[1] else None))
                         for k, v in kt.items()},
                roofline=dict(kernel="bessel_epilogue_kernel", bound="hbm", achieved=round(ach, 1),
                              peak=PEAK_HBM_GBS, unit="GB/s", frac=round(ach / PEAK_HBM_GBS, 4),
                              traffic=None, bytes_per_launch=bytes_per_launch))


def cpu_baseline(seconds: float):
    """The FP64 oracle (pupil build + separable evaluation) on whole stacks for about `seconds`."""
    from oracle import fourier as OF
    from tests.helpers import oracle_optics
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = 1
    w, zp, _ = fourier_workload()
    opt = oracle_optics(w)
    g = OF.pupil_geometry(256, opt)
    t0 = time.perf_counter()
    planes = 0
    b = 0
    while time.perf_counter() - t0 < seconds:
        s = b % 16
        P = OF.base_pupil(g, opt, OF.pupil_phase(g, opt, zernike=w["zernike"][s], t_s=w["t_s"][s]))
        for z in w["z"][s]:
            OF.field_separable(P, g, opt, 128, 128, 20.0, 20.0, [z])
            planes += 1
            if time.perf_counter() - t0 > seconds:
                break
        b += 1
    dt = time.perf_counter() - t0
    return dict(value=planes * 128 * 128 / dt, unit="voxels/s", cores=threads, kind="oracle",
                sample=f"separable FP64 oracle (pupil build included) over the headline workload's "
                       f"stacks in order: {planes} planes of 128x128 (3 field components), {dt:.1f} s, "
                       f"NumPy/BLAS threads = {threads}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="bessel", help="comma list of extra forms, or 'none'")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2502_03170_amd as rw
    rw.load()
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.synchronize()
    res = bench_fourier(rw, torch, args.steps, args.warmup)
    print(f"# fourier: {res['ms_per_step']:.3f} ms/step, {res['value']:.3e} voxels/s", file=sys.stderr,
          flush=True)
    forms = {}
    if "bessel" in args.forms.split(","):
        forms["bessel"] = bench_bessel(rw, torch, args.steps, args.warmup)
        print(f"# bessel: {forms['bessel']['value']:.3e} voxels/s", file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.cpu_seconds)
    out = {
        "metric": "PSF voxels/sec (vectorial FP32) plain vs batched/surrogate at rel-L2 <=1e-5",
        "value": res["value"], "unit": "voxels/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "fourier_plain: NA 1.4, 600 nm, n_i 1.518, 256x256 pupil, Gibson-Lanni "
                               "(n_s 1.33, t_s U[0,5] um) + Noll 4-21 N(0,0.05) waves, 128x128x64 at "
                               "20 nm, fields + intensity, 16 stacks per call",
                   "stacks_per_step": 16, "voxels_per_step": res["voxels"], "form": "fourier"},
        "roofline": res["roofline"],
        "cpu_baseline": cpu,
        "kernels": res["kernels"],
        "image_gemm": res["image_gemm"],
        "step_tflops": res["step_tflops"], "step_frac": res["step_frac"],
        "forms": forms,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
