"""Oracle: analytic primary field of a point electric dipole in a homogeneous
whole space (Appendix A, eqs. A.1-A.3), plus the skin depth (eq. 12).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Reading of Appendix A. The printed rows are garbled: the x-row has a stray
"+3 k^2 r^2" and every row lacks the parentheses that group
``(d_i d_j / r^2)(-k^2 r^2 + 3ikr + 3)``; the appendix writes ``e^{-ikr}`` with
``+3ikr``, which is the e^{+i omega t} convention, while Section 2 fixes
e^{-i omega t}. Written for the e^{-i omega t} convention and a general unit
direction p, the field of the moment I*dS is

    E_p(x) = I dS / (4 pi sigma r^3) * e^{ikr} *
             [ d (d.p) / r^2 * (3 - 3ikr - k^2 r^2) + p * (k^2 r^2 + ikr - 1) ],

with d = x - x_s, r = |d| and k = sqrt(i omega mu0 sigma) on the principal
branch (Re k > 0, Im k > 0), i.e. k = (1 + i) / delta. The three rows of the
appendix are the cases p = x, y, z of this formula with k replaced by -k
(complex conjugate convention). It equals (1/sigma)(k^2 + grad grad) G p with
G = e^{ikr} / (4 pi r), the solution of the first-order system of Section 2
(eqs. 1-2) for a point current source.

The magnetic field follows from Faraday's law of Section 2 (eq. 1 with the
e^{-i omega t} sign), H = curl E / (i omega mu0): the gradient part of E has
no curl and k^2 = i omega mu0 sigma, so H_p = I dS grad G x p.
"""
from __future__ import annotations

import numpy as np

MU0 = 4.0e-7 * np.pi


def wavenumber(freq: float, sigma: float) -> complex:
    """k with k^2 = i omega mu0 sigma, principal branch (Section 2, eqs. 1-3)."""
    omega = 2.0 * np.pi * freq
    return complex(np.sqrt(1j * omega * MU0 * sigma))


def skin_depth(freq: float, sigma: float) -> float:
    """delta = sqrt(2 / (mu0 omega sigma)) (Section 5.3, eq. 12)."""
    return float(np.sqrt(2.0 / (MU0 * 2.0 * np.pi * freq * sigma)))


def dipole_field(x: np.ndarray, src_pos, src_dir, freq: float, sigma: float,
                 moment: float = 1.0) -> np.ndarray:
    """Primary electric field (complex128 [..., 3]) at points x [..., 3]."""
    x = np.asarray(x, dtype=np.float64)
    p = np.asarray(src_dir, dtype=np.float64)
    d = x - np.asarray(src_pos, dtype=np.float64)
    r = np.sqrt(np.sum(d * d, axis=-1))
    k = wavenumber(freq, sigma)
    kr = k * r
    amp = moment / (4.0 * np.pi * sigma * r ** 3) * np.exp(1j * kr)
    dp = np.sum(d * p, axis=-1)
    a = (3.0 - 3.0j * kr - kr * kr) * dp / (r * r)
    b = kr * kr + 1j * kr - 1.0
    return amp[..., None] * (a[..., None] * d + b[..., None] * p)


def dipole_field_appendix_rows(x: np.ndarray, src_pos, axis: int, freq: float,
                               sigma: float, moment: float = 1.0) -> np.ndarray:
    """The appendix's per-axis rows, repaired (grouping restored, stray term
    dropped), kept in the appendix's own e^{-ikr} / +3ikr form with a
    caller-chosen k. Used only to pin ``dipole_field`` against the printed
    structure: with k -> -k it must agree with the formula above."""
    x = np.asarray(x, dtype=np.float64)
    d = x - np.asarray(src_pos, dtype=np.float64)
    r = np.sqrt(np.sum(d * d, axis=-1))
    k = -wavenumber(freq, sigma)
    kr = k * r
    pref = moment / (4.0 * np.pi * sigma * r ** 3) * np.exp(-1j * kr)
    out = np.empty(d.shape, dtype=np.complex128)
    for j in range(3):
        q = d[..., axis] * d[..., j] / (r * r) * (-kr * kr + 3j * kr + 3.0)
        if j == axis:
            q = q + (kr * kr - 1j * kr - 1.0)
        out[..., j] = pref * q
    return out


def dipole_magnetic_field(x: np.ndarray, src_pos, src_dir, freq: float, sigma: float,
                          moment: float = 1.0) -> np.ndarray:
    """Primary magnetic field H_p = curl E_p / (i omega mu0) = I dS grad G x p
    (complex128 [..., 3], A/m) at points x [..., 3]:
    grad G = (ikr - 1) e^{ikr} / (4 pi r^3) d, d = x - x_s."""
    x = np.asarray(x, dtype=np.float64)
    p = np.asarray(src_dir, dtype=np.float64)
    d = x - np.asarray(src_pos, dtype=np.float64)
    r = np.sqrt(np.sum(d * d, axis=-1))
    kr = wavenumber(freq, sigma) * r
    amp = moment * (1j * kr - 1.0) * np.exp(1j * kr) / (4.0 * np.pi * r ** 3)
    return amp[..., None] * np.cross(d, np.broadcast_to(p, d.shape))
