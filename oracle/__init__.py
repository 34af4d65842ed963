"""FP64 CPU oracle for the vectorial Richards-Wolf PSF.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path (no kernels, headers, tables or helpers); the two meet only through the
seeded input generators in ``workloads/``, which hold none of the method's
arithmetic.

Everything here is plain NumPy in float64 / complex128, written to be read
against the paper (Liu et al., "Revisiting PSF Models: Unifying Framework and
High-Performance Implementation", arXiv 2502.03170):

* ``optics``   -- far field (Sec. 3.3, eq. "field Gaussian sphere"), Zernike
                  (Sec. 3.4.2), Gibson-Lanni OPD (Sec. 3.4.1), apodization and
                  Gaussian envelope (Sec. 3.4.3-3.4.4), pupil grids.
* ``fourier``  -- Cartesian parameterisation (eq. "cartesian vectorial" with
                  the correction factors of eq. "vectorial general with
                  correction"), as a brute-force double sum and as its
                  separable factorisation.
* ``bessel``   -- spherical parameterisation: the polar double integral
                  (eq. "polar vectorial") and the 1-D Bessel form
                  (eq. "polar vectorial final" / "I0").
* ``adjoint``  -- analytic gradient of a stack loss through the Cartesian form
                  and central finite differences.
* ``surrogate``-- FP64 forward/backward of the surrogate network.

Pins: each function is pinned by the ``-m "not gpu"`` tests in
``tests/test_oracle_*.py`` against closed forms, invariants and brute force.
"""
