"""Bulk tier: the textbook spherical-coordinate route in numpy longdouble.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Values follow Eq. real-sh-spherical with the prefactor of Eq. Flm and the
Ferrers functions from the textbook recurrence Eq. recur-p (Condon-Shortley
phase), with t = cos(theta) = z/r.  sin(theta) is taken as r_xy/r, never as
sqrt(1-t^2), so points next to the z axis keep full relative accuracy.  The
azimuth comes from atan2 and cos/sin of m*phi from libm in longdouble.

Gradients are the exact Cartesian gradients of these functions, written in
spherical coordinates,

    grad Y = (1/r) [ theta_hat dY/dtheta + phi_hat (1/sin theta) dY/dphi ],

with two textbook identities of the Ferrers functions that remove every
division by sin(theta) (checked against mpmath in the tests):

    dP_l^m/dtheta   = ( P_l^{m+1} - (l+m)(l-m+1) P_l^{m-1} ) / 2      (m >= 1)
    dP_l^0/dtheta   = P_l^1
    m P_l^m / sin t = -( P_{l-1}^{m+1} + (l+m-1)(l+m) P_{l-1}^{m-1} ) / 2  (m >= 1)

The solid harmonics are r^l Y (Sec. II), with the product rule for their
gradient: grad(r^l Y) = r^(l-1) [ l Y r_hat + (theta/phi part above times r) ].

At r = 0: the solid harmonics are polynomials and take their exact values
(only l = 0 is non-zero, only l = 1 has a non-zero gradient); the normalised
ones have no direction, and by convention Y_0^0 keeps its constant while every
other value and every gradient is 0.
"""
from __future__ import annotations

from functools import lru_cache

import mpmath
import numpy as np

from .definition import prefactor

LD = np.longdouble


@lru_cache(maxsize=None)
def _prefactors_ld(l_max: int) -> np.ndarray:
    """F_l^m (Eq. Flm) for 0 <= m <= l <= l_max as longdouble, from exact factorials."""
    F = np.zeros((l_max + 1, l_max + 1), dtype=LD)
    with mpmath.workdps(40):
        for l in range(l_max + 1):
            for m in range(l + 1):
                F[l, m] = LD(mpmath.nstr(prefactor(l, m), 30))
    return F


def ferrers_table(t: np.ndarray, s: np.ndarray, l_max: int) -> np.ndarray:
    """P_l^m(t) for 0 <= m <= l <= l_max by Eq. recur-p; shape [l_max+2, l_max+3, N].

    ``s`` is sin(theta) = sqrt(1 - t^2) supplied by the caller.  Entries with
    m > l (and the extra row l_max+1) are zero, which is the value the
    derivative identities need there.
    """
    N = t.shape[0]
    P = np.zeros((l_max + 2, l_max + 3, N), dtype=LD)
    P[0, 0] = 1
    for l in range(1, l_max + 1):
        P[l, l] = -(2 * l - 1) * s * P[l - 1, l - 1]
        P[l, l - 1] = (2 * l - 1) * t * P[l - 1, l - 1]
        for m in range(l - 1):
            P[l, m] = ((2 * l - 1) * t * P[l - 1, m] - (l + m - 1) * P[l - 2, m]) / (l - m)
    return P


def real_sph(xyz, l_max: int, normalize: bool, gradients: bool = True):
    """Real spherical harmonics (scaled solid or normalised) and their gradients.

    Parameters
    ----------
    xyz : array [N,3] (any float type; converted exactly to longdouble)
    l_max : int >= 0
    normalize : False -> r^l Y_l^m, True -> Y_l^m
    gradients : also return the Cartesian gradient

    Returns ``Y [N,K]`` (and ``dY [N,3,K]``) in longdouble, K = (l_max+1)^2,
    column k = l^2 + l + m with m ascending from -l.
    """
    P3 = np.asarray(xyz).reshape(-1, 3).astype(LD)
    N = P3.shape[0]
    K = (l_max + 1) ** 2
    x, y, z = P3[:, 0], P3[:, 1], P3[:, 2]
    rxy = np.sqrt(x * x + y * y)
    r = np.sqrt(x * x + y * y + z * z)
    zero = r == 0
    rs = np.where(zero, LD(1), r)
    t = np.where(zero, LD(1), z / rs)      # cos(theta)
    s = np.where(zero, LD(0), rxy / rs)    # sin(theta)
    phi = np.arctan2(y, x)
    cphi, sphi = np.cos(phi), np.sin(phi)

    F = _prefactors_ld(l_max)
    P = ferrers_table(t, s, l_max)
    inv_sqrt2 = 1 / np.sqrt(LD(2))

    Y = np.zeros((N, K), dtype=LD)
    G = np.zeros((N, 3, K), dtype=LD) if gradients else None
    # unit vectors of the spherical frame
    rhat = (s * cphi, s * sphi, t)
    that = (t * cphi, t * sphi, -s)
    phat = (-sphi, cphi, np.zeros_like(s))

    for l in range(l_max + 1):
        for m in range(-l, l + 1):
            mu = abs(m)
            k = l * l + l + m
            if m > 0:
                trig, dtrig = np.cos(m * phi), -m * np.sin(m * phi)
            elif m < 0:
                trig, dtrig = np.sin(mu * phi), mu * np.cos(mu * phi)
            else:
                trig, dtrig = inv_sqrt2 * np.ones_like(phi), np.zeros_like(phi)
            Fl = F[l, mu]
            Y[:, k] = Fl * P[l, mu] * trig
            if not gradients:
                continue
            # d/dtheta of P_l^mu(cos theta)
            if mu == 0:
                dP = P[l, 1]
            else:
                dP = (P[l, mu + 1] - (l + mu) * (l - mu + 1) * P[l, mu - 1]) / 2
            # P_l^mu / sin(theta), pole-free; multiplied by dtrig/mu below
            if mu == 0:
                ang = np.zeros_like(phi)
            else:
                if l >= 1:
                    mp_over_s = -(P[l - 1, mu + 1] + (l + mu - 1) * (l + mu) * P[l - 1, mu - 1]) / 2
                else:
                    mp_over_s = np.zeros_like(phi)
                ang = Fl * mp_over_s * (dtrig / mu)
            dth = Fl * dP * trig
            for a in range(3):
                G[:, a, k] = that[a] * dth + phat[a] * ang  # r * grad(Y)

    if not normalize:
        ls = np.array([l for l in range(l_max + 1) for _ in range(2 * l + 1)], dtype=LD)
        with np.errstate(divide="ignore", invalid="ignore"):
            rl = r[:, None] ** ls[None, :]
            rl1 = np.where(ls[None, :] == 0, LD(0), r[:, None] ** (ls[None, :] - 1))
        if gradients:
            rh = np.stack(rhat, axis=1)  # [N,3]
            G = rl1[:, None, :] * (ls[None, None, :] * Y[:, None, :] * rh[:, :, None] + G)
        Y = Y * rl
        return (Y, G) if gradients else Y

    if gradients:
        G = G / rs[:, None, None]
    if zero.any():
        Y[zero, 1:] = 0
        if gradients:
            G[zero] = 0
    return (Y, G) if gradients else Y
