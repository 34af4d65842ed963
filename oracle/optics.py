"""Optical building blocks of the Richards-Wolf model, FP64 (oracle; test infrastructure only).

Conventions (the paper's Fig. 1 and Sec. 3.1): direction s = (sin t cos p,
sin t sin p, cos t); p measured from +s_x toward +s_y; s_max = NA / n_i; the
wavenumber is taken in the immersion medium, k = 2 pi n_i / lambda.  Lengths
are in nanometres, Zernike coefficients in waves, phases in radians.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class GibsonLanni:
    """Layer indices and thicknesses of Sec. 3.4.1 (starred = design values)."""
    n_s: float
    n_g: float = 1.5
    n_g_design: float = 1.5
    n_i_design: float | None = None   # None -> equal to the actual immersion index
    t_g: float = 170e3
    t_g_design: float = 170e3
    t_i_design: float = 150e3


@dataclass
class Optics:
    na: float
    wavelength: float           # nm
    n_i: float                  # immersion index
    f: float = 1.0              # focal length; scales the field only
    e_inc: tuple = (1 / math.sqrt(2), 1j / math.sqrt(2))   # (e_x, e_y)
    apodization: bool = True    # sqrt(cos theta), Sec. 3.4.3
    s_env: float = 0.0          # Gaussian envelope width, Sec. 3.4.4 (0 = off)
    gl: GibsonLanni | None = None
    # Fresnel transmission (Sec. 3.3): indices of the media the light crosses before
    # the immersion medium, emitter side first, e.g. (n_s, n_g); () = q_s = q_p = 1.
    fresnel_media: tuple = ()

    @property
    def k(self) -> float:
        return 2.0 * math.pi * self.n_i / self.wavelength

    @property
    def s_max(self) -> float:
        return self.na / self.n_i

    @property
    def theta_max(self) -> float:
        return math.asin(self.s_max)


# ---------------------------------------------------------------------------
# Far field on the Gaussian reference sphere (Sec. 3.3, eq. "field Gaussian sphere")
# ---------------------------------------------------------------------------
def far_field(ex, ey, cos_t, sin_t, cos_p, sin_p, qs=1.0, qp=1.0):
    """Vectorial far field e_inf(theta, phi) for e_inc = (ex, ey, 0).

    Returns an array of shape (3, ...) (x, y, z components), broadcast over the
    angle arrays.  Written from the two 3-vectors of the equation, with
    cos 2p and sin 2p formed from cos p and sin p.
    """
    cos2p = cos_p * cos_p - sin_p * sin_p
    sin2p = 2.0 * sin_p * cos_p
    vx = np.stack([
        qs * (1 - cos2p) + qp * (1 + cos2p) * cos_t,
        (-qs + qp * cos_t) * sin2p,
        -2.0 * qp * cos_p * sin_t,
    ])
    vy = np.stack([
        (-qs + qp * cos_t) * sin2p,
        qs * (1 + cos2p) + qp * (1 - cos2p) * cos_t,
        -2.0 * qp * sin_p * sin_t,
    ])
    return vx * (ex / 2.0) + vy * (ey / 2.0)


def fresnel_q(sin_t, optics: Optics):
    """Products q_s, q_p of the Fresnel transmission coefficients (Sec. 3.3, the
    coefficients that enter eq. "field Gaussian sphere").

    The media are ``optics.fresnel_media`` followed by the immersion n_i.  Every ray
    keeps n_m sin t_m = n_i sin t, and n_m cos t_m = sqrt(n_m^2 - (n_i sin t)^2) on the
    principal branch (positive imaginary beyond a critical angle).  Interface m -> m+1
    transmits q_s^m = 2 n_m cos t_m / (n_m cos t_m + n_{m+1} cos t_{m+1}) and
    q_p^m = 2 n_m cos t_m / (n_{m+1} cos t_m + n_m cos t_{m+1}).
    """
    inv2 = (optics.n_i * np.asarray(sin_t, dtype=np.float64)) ** 2
    media = [float(n) for n in optics.fresnel_media] + [float(optics.n_i)]
    qs = np.ones(np.shape(sin_t), dtype=np.complex128)
    qp = np.ones(np.shape(sin_t), dtype=np.complex128)
    for n1, n2 in zip(media[:-1], media[1:]):
        nc1 = np.sqrt((n1 * n1 - inv2).astype(np.complex128))   # n1 cos t1
        nc2 = np.sqrt((n2 * n2 - inv2).astype(np.complex128))   # n2 cos t2
        c1, c2 = nc1 / n1, nc2 / n2
        qs = qs * (2.0 * nc1 / (nc1 + nc2))
        qp = qp * (2.0 * nc1 / (n2 * c1 + n1 * c2))
    return qs, qp


# ---------------------------------------------------------------------------
# Zernike polynomials (Sec. 3.4.2), Noll single index, orthonormal on the unit disk
# ---------------------------------------------------------------------------
def noll_to_nm(j: int) -> tuple[int, int]:
    """Noll index j >= 1 -> (n, m) with signed m (m > 0: cos, m < 0: sin).

    Radial order n is the row with n(n+1)/2 < j <= (n+1)(n+2)/2; inside a row
    |m| grows; a pair with |m| > 0 takes the cosine at even j, the sine at odd j.
    """
    if j < 1:
        raise ValueError("Noll index starts at 1")
    n = 0
    while (n + 1) * (n + 2) // 2 < j:
        n += 1
    p = j - n * (n + 1) // 2 - 1          # position inside the row, 0-based
    if n % 2 == 0:
        am = 2 * ((p + 1) // 2)
    else:
        am = 2 * (p // 2) + 1
    if am == 0:
        return n, 0
    return n, (am if j % 2 == 0 else -am)


def zernike_radial(n: int, m: int, r):
    """R_n^|m|(r) as the finite factorial sum."""
    m = abs(m)
    out = np.zeros_like(np.asarray(r, dtype=np.float64))
    for s in range((n - m) // 2 + 1):
        c = ((-1) ** s * math.factorial(n - s)
             / (math.factorial(s) * math.factorial((n + m) // 2 - s) * math.factorial((n - m) // 2 - s)))
        out = out + c * np.asarray(r, dtype=np.float64) ** (n - 2 * s)
    return out


def zernike_noll(j: int, r, p):
    """Orthonormal Zernike Z_j(r, p): mean of Z_j^2 over the unit disk is 1."""
    n, m = noll_to_nm(j)
    rad = zernike_radial(n, m, r)
    if m == 0:
        return math.sqrt(n + 1) * rad
    ang = np.cos(m * p) if m > 0 else np.sin(-m * p)
    return math.sqrt(2 * (n + 1)) * rad * ang


# ---------------------------------------------------------------------------
# Gibson-Lanni optical path difference (Sec. 3.4.1)
# ---------------------------------------------------------------------------
def gibson_lanni_ti(gl: GibsonLanni, n_i: float, t_s: float) -> float:
    """Immersion thickness from the focusing condition, taken as printed."""
    n_i_star = n_i if gl.n_i_design is None else gl.n_i_design
    return t_s + n_i * (-t_s / gl.n_s - gl.t_g / gl.n_g + gl.t_g_design / gl.n_g_design
                        + gl.t_i_design / n_i_star)


def gibson_lanni_opd(sin_t, optics: Optics, t_s: float, compensated: bool = False):
    """Phase W(theta) in radians (complex: the imaginary part is evanescent decay).

    Square roots take the principal branch, so beyond the critical angle of a
    layer sqrt(n^2 - n_i^2 sin^2) is +i*|.| and exp(iW) decays.  With
    ``compensated`` the leading t_s of the focusing condition is dropped
    (the paraxial focus reading); the default is the printed relation.
    """
    gl = optics.gl
    n_i = optics.n_i
    n_i_star = n_i if gl.n_i_design is None else gl.n_i_design
    ti = gibson_lanni_ti(gl, n_i, t_s) - (t_s if compensated else 0.0)
    s2 = (n_i * np.asarray(sin_t, dtype=np.float64)) ** 2
    root = lambda n: np.sqrt((n * n - s2).astype(np.complex128))
    k0 = 2.0 * math.pi / optics.wavelength
    return k0 * (t_s * root(gl.n_s) + ti * root(n_i) - gl.t_i_design * root(n_i_star)
                 + gl.t_g * root(gl.n_g) - gl.t_g_design * root(gl.n_g_design))


def amplitude(cos_t, sin_t, optics: Optics):
    """Amplitude correction a(s): apodization sqrt(cos t) times the Gaussian envelope."""
    a = np.ones_like(np.asarray(cos_t, dtype=np.float64))
    if optics.apodization:
        a = a * np.sqrt(cos_t)
    if optics.s_env > 0:
        a = a * np.exp(-(np.asarray(sin_t) ** 2) / optics.s_env ** 2)
    return a


# ---------------------------------------------------------------------------
# Pupil sampling
# ---------------------------------------------------------------------------
def cartesian_pupil_grid(n: int, s_max: float):
    """Cell-centred n x n grid over [-s_max, s_max]^2 and the integer disk mask.

    Returns (sx[j,l], sy[j,l], mask[j,l], ds) with j indexing s_x and l indexing
    s_y.  The mask keeps cells whose centre lies in the disk, decided in
    integers: (2j+1-n)^2 + (2l+1-n)^2 <= n^2.
    """
    idx = np.arange(n)
    u = 2 * idx + 1 - n
    ds = 2.0 * s_max / n
    sx = (u[:, None] * (s_max / n)) * np.ones((1, n))
    sy = np.ones((n, 1)) * (u[None, :] * (s_max / n))
    mask = (u[:, None] ** 2 + u[None, :] ** 2) <= n * n
    return sx, sy, mask, ds


def gauss_legendre(n: int, a: float, b: float):
    """Gauss-Legendre nodes and weights on [a, b] (NumPy's leggauss, mapped)."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (b - a) * x + 0.5 * (b + a), 0.5 * (b - a) * w


def output_axis(m: int, d: float, shift: float = 0.0):
    """Pixel coordinates (i - floor(m/2)) * d - shift: pixel floor(m/2) is on axis."""
    return (np.arange(m) - (m // 2)) * d - shift
