"""Oracle: primary field of a point electric dipole over a layered earth of
two half-spaces (sea over sediments), as the paper's formulation allows
(Section 2: the primary field is that of the background model, which may be
layered; the paper evaluates the whole-space case of Appendix A).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Setting (e^{-i omega t}, no displacement currents): sigma_1 for z > z0,
sigma_2 for z < z0, the dipole (moment m along p) at height zs > z0,
k_j^2 = i omega mu0 sigma_j. In the horizontal wavenumber domain (kx, ky),
kappa^2 = kx^2 + ky^2, u_j = sqrt(kappa^2 - k_j^2) with Re u_j > 0, the field
splits into a TE part E = curl(z F) and a TM part E = curl curl(z A); at the
interface F, dF/dz, dA/dz and sigma A are continuous, so that
    r_TE = (u1 - u2) / (u1 + u2),                 t_TE = 2 u1 / (u1 + u2),
    r_TM = (s2 u1 - s1 u2) / (s2 u1 + s1 u2),     t_TM = 2 s1 u1 / (s2 u1 + s1 u2).
Decomposing the whole-space dipole field of Appendix A (the incident field)
into these parts and transforming back with the Hankel identities
(1/2pi) int kappa f(kappa) J_n(kappa rho) cos / sin (n phi) gives, with
c = m / (8 pi sigma_1), rho and phi the horizontal offset from the source:

layer 1 (z > z0): E = E_whole-space(sigma_1) + E_r, Z = (z - z0) + (zs - z0),
    A_n = int k1^2 r_TE / u1 e^{-u1 Z} J_n kappa dk    B_n = int u1 r_TM e^{-u1 Z} J_n kappa dk
    E1  = int r_TM e^{-u1 Z} J_1 kappa^2 dk            V0  = int r_TM kappa^3 / u1 e^{-u1 Z} J_0 dk
  x dipole: Ex = c (A0 + B0 + cos 2phi (A2 - B2)), Ey = c sin 2phi (A2 - B2), Ez = -2c cos phi E1
  y dipole: Ex = c sin 2phi (A2 - B2), Ey = c (A0 + B0 - cos 2phi (A2 - B2)), Ez = -2c sin phi E1
  z dipole: Ex = 2c cos phi E1, Ey = 2c sin phi E1, Ez = 2c V0
layer 2 (z < z0): E = E_t, with e = exp(u2 (z - z0) - u1 (zs - z0)),
    TA_n = int k1^2 t_TE / u1 e J_n kappa dk           TB_n = int u2 t_TM e J_n kappa dk
    TE1  = int t_TM e J_1 kappa^2 dk    VE1 = int t_TM u2 / u1 e J_1 kappa^2 dk    VV0 = int t_TM kappa^3 / u1 e J_0 dk
  x dipole: Ex = c (TA0 - TB0 + cos 2phi (TA2 + TB2)), Ey = c sin 2phi (TA2 + TB2), Ez = -2c cos phi TE1
  y dipole: Ex = c sin 2phi (TA2 + TB2), Ey = c (TA0 - TB0 - cos 2phi (TA2 + TB2)), Ez = -2c sin phi TE1
  z dipole: Ex = -2c cos phi VE1, Ey = -2c sin phi VE1, Ez = 2c VV0

The Hankel integrals are summed plainly: Gauss-Legendre panels (24 nodes)
over [0, kappa_max], kappa_max = 60 / (decay length) where the exponential
has fallen below e^-60, panels no wider than a quarter of the smaller |k_j|
below 12 max |k_j| and no wider than a quarter of the Bessel period 2 pi / rho.
"""
from __future__ import annotations

import numpy as np
from scipy.special import jv

from .primary import MU0, dipole_field


def _panels(kmax, kappa_fine, h_fine, h_coarse):
    a = np.arange(0.0, min(kappa_fine, kmax), h_fine)
    b = np.arange(min(kappa_fine, kmax), kmax, h_coarse)
    return np.concatenate([a, b, [kmax]])


_GL_X, _GL_W = np.polynomial.legendre.leggauss(24)


def _nodes(kmax, k_small, k_large, rho):
    """Quadrature nodes and weights on [0, kmax]."""
    per = np.inf if rho <= 0 else 0.25 * 2.0 * np.pi / rho
    h_fine = min(0.25 * k_small, per)
    h_coarse = min(per, kmax / 64.0)
    e = _panels(kmax, 12.0 * k_large, h_fine, h_coarse)
    e = e[np.concatenate([[True], np.diff(e) > 0])]
    lo, hi = e[:-1], e[1:]
    x = (0.5 * (hi - lo))[:, None] * _GL_X[None, :] + (0.5 * (hi + lo))[:, None]
    w = (0.5 * (hi - lo))[:, None] * _GL_W[None, :]
    return x.ravel(), w.ravel()


def layered_dipole_field(x, src_pos, src_dir, freq, sigma_top, sigma_bottom, z0=0.0, moment=1.0):
    """Total primary electric field (complex128 [..., 3]) of the dipole at
    points x [..., 3] for two half-spaces sigma_top (z > z0, holding the
    source) and sigma_bottom (z < z0). Points on z = z0 take the upper
    formula."""
    x = np.asarray(x, dtype=np.float64)
    shape = x.shape
    pts = x.reshape(-1, 3)
    src = np.asarray(src_pos, dtype=np.float64)
    p = np.asarray(src_dir, dtype=np.float64)
    zs = src[2] - z0
    if not zs > 0:
        raise ValueError("the source must lie in the upper half-space")
    s1, s2 = float(sigma_top), float(sigma_bottom)
    w = 2.0 * np.pi * freq
    k1s, k2s = 1j * w * MU0 * s1, 1j * w * MU0 * s2
    ka = np.sqrt(abs(k1s)), np.sqrt(abs(k2s))
    k_small, k_large = min(ka), max(ka)
    c = moment / (8.0 * np.pi * s1)
    out = np.zeros((len(pts), 3), dtype=np.complex128)
    for n, pt in enumerate(pts):
        dx, dy = pt[0] - src[0], pt[1] - src[1]
        rho = float(np.hypot(dx, dy))
        cph, sph = (dx / rho, dy / rho) if rho > 0 else (1.0, 0.0)
        c2, s2p = cph * cph - sph * sph, 2.0 * sph * cph
        z = pt[2] - z0
        upper = z >= 0.0
        dec = (z + zs) if upper else (zs - z)
        kmax = 60.0 / dec
        kap, wq = _nodes(kmax, k_small, k_large, rho)
        u1 = np.sqrt(kap * kap - k1s)
        u2 = np.sqrt(kap * kap - k2s)
        j0, j1, j2 = jv(0, kap * rho), jv(1, kap * rho), jv(2, kap * rho)
        if upper:
            rte = (u1 - u2) / (u1 + u2)
            rtm = (s2 * u1 - s1 * u2) / (s2 * u1 + s1 * u2)
            ex = np.exp(-u1 * (z + zs))
            fa = k1s * rte / u1 * ex * kap * wq
            fb = u1 * rtm * ex * kap * wq
            A0, A2 = np.sum(fa * j0), np.sum(fa * j2)
            B0, B2 = np.sum(fb * j0), np.sum(fb * j2)
            E1 = np.sum(rtm * ex * j1 * kap * kap * wq)
            V0 = np.sum(rtm * kap ** 3 / u1 * ex * j0 * wq)
            hx = np.array([c * (A0 + B0 + c2 * (A2 - B2)), c * s2p * (A2 - B2), -2 * c * cph * E1])
            hy = np.array([c * s2p * (A2 - B2), c * (A0 + B0 - c2 * (A2 - B2)), -2 * c * sph * E1])
            vz = np.array([2 * c * cph * E1, 2 * c * sph * E1, 2 * c * V0])
            out[n] = p[0] * hx + p[1] * hy + p[2] * vz
            out[n] += dipole_field(pt[None], src, p, freq, s1, moment)[0]
        else:
            tte = 2.0 * u1 / (u1 + u2)
            ttm = 2.0 * s1 * u1 / (s2 * u1 + s1 * u2)
            ex = np.exp(u2 * z - u1 * zs)
            fa = k1s * tte / u1 * ex * kap * wq
            fb = u2 * ttm * ex * kap * wq
            TA0, TA2 = np.sum(fa * j0), np.sum(fa * j2)
            TB0, TB2 = np.sum(fb * j0), np.sum(fb * j2)
            TE1 = np.sum(ttm * ex * j1 * kap * kap * wq)
            VE1 = np.sum(ttm * u2 / u1 * ex * j1 * kap * kap * wq)
            VV0 = np.sum(ttm * kap ** 3 / u1 * ex * j0 * wq)
            hx = np.array([c * (TA0 - TB0 + c2 * (TA2 + TB2)), c * s2p * (TA2 + TB2), -2 * c * cph * TE1])
            hy = np.array([c * s2p * (TA2 + TB2), c * (TA0 - TB0 - c2 * (TA2 + TB2)), -2 * c * sph * TE1])
            vz = np.array([-2 * c * cph * VE1, -2 * c * sph * VE1, 2 * c * VV0])
            out[n] = p[0] * hx + p[1] * hy + p[2] * vz
    return out.reshape(shape[:-1] + (3,))
