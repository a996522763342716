"""Backward and double-backward contractions and the error metric.

TEST INFRASTRUCTURE ONLY (see the package docstring).

For a loss L that depends on the harmonics Y(x) of each point:

* backward:        dL/dx_a = sum_k gY_k dY_{a,k}          (chain rule)
* double backward: given v = dL'/d(dL/dx), the two partials of
  L' = sum_a v_a sum_k gY_k dY_{a,k} are
      dL'/dgY_k = sum_a v_a dY_{a,k}
      dL'/dx_b  = sum_k gY_k sum_a v_a d^2Y_k/(dx_a dx_b)

The paper names derivatives of any order (Sec. II, after Eq. iter-deri) and a
custom backward that reuses the forward derivatives (Sec. III); the formulas
above are plain calculus.  Second derivatives come from the exact
polynomial derivatives of the definition tier.
"""
from __future__ import annotations

import math

import numpy as np

from .definition import definition_eval_ld
from .recurrence import real_sph

LD = np.longdouble


def backward(dY, gY):
    """gxyz[n,a] = sum_k gY[n,k] dY[n,a,k], in longdouble."""
    dY = np.asarray(dY).astype(LD)
    gY = np.asarray(gY).astype(LD)
    return np.einsum("nak,nk->na", dY, gY)


def hessian_contract(H, gY, v):
    """gxyz2[n,b] = sum_k gY[n,k] sum_a v[n,a] H[n,a,b,k]."""
    H = np.asarray(H).astype(LD)
    gY = np.asarray(gY).astype(LD)
    v = np.asarray(v).astype(LD)
    return np.einsum("nabk,nk,na->nb", H, gY, v)


def double_backward(xyz, gY, v, l_max: int, normalize: bool):
    """Return ``(ggY [N,K], gxyz2 [N,3])`` in longdouble.

    Gradients come from the bulk tier, Hessians from the definition tier
    (longdouble polynomials; use for l_max <= 12).
    """
    _, dY = real_sph(xyz, l_max, normalize, gradients=True)
    _, _, H = definition_eval_ld(xyz, l_max, normalize, hessian=True)
    v = np.asarray(v).astype(LD)
    ggY = np.einsum("nak,na->nk", dY, v)
    return ggY, hessian_contract(H, gY, v)


# ------------------------------------------------------ radial expansion
def radial_expansion(xyz, offsets, R, l_max: int, normalize: bool):
    """``c[e, n, l^2+l+m] = sum_{j in e} R[j, l, n] Y_l^m(x_j)``, longdouble.

    The expansion of a set of points in radial functions times spherical
    harmonics (Sec. I, Eq. expansion).  Environment e holds the points
    ``offsets[e] <= j < offsets[e+1]`` (CSR); ``R[j, l, n]`` is the value of
    the radial function R_nl at point j, supplied by the caller (the paper
    leaves the radial basis open).  With ``normalize`` the harmonics are those
    of the direction (the equation's Y(r_hat)); without, the solid harmonics
    r^l Y, i.e. R_nl(r) r^l in the equation's terms.  Empty environments give
    zeros.
    """
    P = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    offsets = np.asarray(offsets, dtype=np.int64)
    R = np.asarray(R).astype(LD)
    n_env = offsets.size - 1
    n_max = R.shape[2]
    K = (l_max + 1) ** 2
    Y = real_sph(P, l_max, normalize, gradients=False) if P.shape[0] else np.zeros((0, K), LD)
    Y = np.asarray(Y).astype(LD)
    lk = _ls(l_max).astype(np.int64)
    c = np.zeros((n_env, n_max, K), dtype=LD)
    for e in range(n_env):
        b, t = int(offsets[e]), int(offsets[e + 1])
        if t <= b:
            continue
        # weights of column k: R[j, l(k), n]
        W = R[b:t][:, lk, :]                     # [cnt, K, n_max]
        c[e] = np.einsum("jkn,jk->nk", W, Y[b:t])
    return c


def radial_expansion_backward(xyz, offsets, R, G, l_max: int, normalize: bool):
    """Backward of :func:`radial_expansion` for an upstream gradient
    ``G[e, n, k]`` of c, in longdouble (chain rule):

    * ``grad_R[j, l, n] = sum_m G[e, n, l^2+l+m] Y_l^m(x_j)``
    * ``grad_xyz[j, a] = sum_k gY[j, k] dY_k/dx_a(x_j)`` with
      ``gY[j, k] = sum_n G[e, n, k] R[j, l(k), n]``

    for the environment e that holds point j.
    """
    P = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    offsets = np.asarray(offsets, dtype=np.int64)
    R = np.asarray(R).astype(LD)
    G = np.asarray(G).astype(LD)
    N = P.shape[0]
    K = (l_max + 1) ** 2
    gR = np.zeros(R.shape, dtype=LD)
    gx = np.zeros((N, 3), dtype=LD)
    if N == 0:
        return gx, gR
    Y, dY = real_sph(P, l_max, normalize, gradients=True)
    lk = _ls(l_max).astype(np.int64)
    for e in range(offsets.size - 1):
        b, t = int(offsets[e]), int(offsets[e + 1])
        if t <= b:
            continue
        Ge = G[e]                                           # [n_max, K]
        gY = np.einsum("nk,jkn->jk", Ge, R[b:t][:, lk, :])  # [cnt, K]
        gx[b:t] = np.einsum("jk,jak->ja", gY, dY[b:t])
        prod = np.einsum("nk,jk->jkn", Ge, Y[b:t])           # [cnt, K, n_max]
        for l in range(l_max + 1):
            gR[b:t, l, :] = prod[:, l * l:(l + 1) ** 2, :].sum(1)
    return gx, gR


# ------------------------------------------------------ e3nn's conventions
E3NN_NORMALIZATIONS = ("integral", "component", "norm")


def e3nn_convention(xyz, l_max: int, normalize: bool, normalization: str = "integral"):
    """``(Y [N,K], dY [N,3,K])`` in e3nn's conventions, longdouble.

    Sec. III.B says the method's library provides wrappers following e3nn's
    conventions without stating them; the reading here: y is the polar
    axis, i.e. the harmonics of Eq. real-sh-cartesian evaluated at the
    cyclically permuted point (z, x, y), so that degree 1 is proportional to
    (x, y, z) in that order; "integral" keeps the unit L2 norm on the
    sphere, "component" multiplies degree l by sqrt(4 pi) (sum over m of
    Y^2 = 2l+1 on the unit sphere), "norm" by sqrt(4 pi / (2l+1)) (sum 1).
    Derivatives are along the caller's x, y, z (chain rule through the
    permutation).
    """
    if normalization not in E3NN_NORMALIZATIONS:
        raise ValueError(normalization)
    xyz = np.asarray(xyz)
    perm = np.stack([xyz[:, 2], xyz[:, 0], xyz[:, 1]], axis=1)
    Y, dYp = real_sph(perm, l_max, normalize, gradients=True)
    # d/dx = d/dy', d/dy = d/dz', d/dz = d/dx'  for (x', y', z') = (z, x, y)
    dY = np.stack([dYp[:, 1], dYp[:, 2], dYp[:, 0]], axis=1)
    ls = np.array([l for l in range(l_max + 1) for _ in range(2 * l + 1)])
    if normalization == "integral":
        c = np.ones(ls.size, dtype=LD)
    elif normalization == "component":
        c = np.full(ls.size, np.sqrt(LD(4) * np.arccos(LD(-1))), dtype=LD)
    else:
        c = np.sqrt(LD(4) * np.arccos(LD(-1)) / (2 * ls + 1).astype(LD))
    return Y * c, dY * c


# ------------------------------------------------------------ error metric
def _ls(l_max):
    return np.array([l for l in range(l_max + 1) for _ in range(2 * l + 1)], dtype=np.float64)


def component_scales(xyz, l_max: int, normalize: bool):
    """Per point and per column scales ``(s [N,K], g [N,K], h [N,K])``.

    The addition theorem gives sum_m (Y_l^m)^2 = (2l+1)/(4 pi) (times r^2l for
    the solid harmonics) and sum_m |grad Y_l^m|^2 = l(l+1)(2l+1)/(4 pi r^2)
    (normalised) or l(2l+1)^2/(4 pi) r^(2l-2) (solid), so these are the natural
    sizes of a column of degree l.  ``h`` (second derivatives) uses
    (l+1)^2 sqrt((2l+1)/4pi) times r^(l-2) or r^-2.  l = 0 borrows the l = 1
    gradient and Hessian scales (its exact derivatives are zero).
    """
    P = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    r = np.sqrt((P * P).sum(axis=1))
    ls = _ls(l_max)
    lg = np.maximum(ls, 1.0)
    base = np.sqrt((2 * ls + 1) / (4 * math.pi))
    gb = np.sqrt(lg * (lg + 1) * (2 * lg + 1) / (4 * math.pi)) if normalize else \
        np.sqrt(lg * (2 * lg + 1) ** 2 / (4 * math.pi))
    hb = (lg + 1) ** 2 * np.sqrt((2 * lg + 1) / (4 * math.pi))
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        if normalize:
            rr = np.where(r > 0, r, 1.0)[:, None]
            s = np.broadcast_to(base, (P.shape[0], ls.size)).copy()
            g = gb[None, :] / rr
            h = hb[None, :] / (rr * rr)
        else:
            s = base[None, :] * r[:, None] ** ls[None, :]
            g = gb[None, :] * r[:, None] ** (lg[None, :] - 1)
            h = hb[None, :] * r[:, None] ** (lg[None, :] - 2)
    return s, g, h


def _scaled(err, scale):
    with np.errstate(divide="ignore", invalid="ignore"):
        out = np.where(scale > 0, err / np.where(scale > 0, scale, 1.0), err)
    return out


def per_l_errors(Y, Yref, xyz, l_max: int, normalize: bool, kind: str = "Y",
                 mask=None):
    """Per-l max and RMS of the scaled error.

    ``kind`` = "Y" for values [N,K]; "dY" for gradients [N,3,K].  Errors are
    |a - ref| divided by the column scale of :func:`component_scales`, so a
    value 10^-5 means "wrong in the 5th digit of a typical entry of degree l".
    ``mask`` (bool [N]) restricts the points.  Returns ``(max[l], rms[l])``.
    """
    s, g, _ = component_scales(xyz, l_max, normalize)
    A = np.asarray(Y, dtype=LD)
    B = np.asarray(Yref, dtype=LD)
    err = np.abs(A - B).astype(np.float64)
    if kind == "Y":
        e = _scaled(err, s)
    elif kind == "dY":
        e = _scaled(err, g[:, None, :])
    else:
        raise ValueError(kind)
    # non-finite comparisons are errors unless both sides agree exactly
    same = (A == B) | (np.isnan(A.astype(np.float64)) & np.isnan(B.astype(np.float64)))
    e = np.where(same, 0.0, e)
    e = np.where(np.isfinite(e), e, np.inf)
    if mask is not None:
        e = e[np.asarray(mask)]
    mx = np.zeros(l_max + 1)
    rms = np.zeros(l_max + 1)
    for l in range(l_max + 1):
        sl = e[..., l * l:(l + 1) * (l + 1)]
        if sl.size == 0:
            continue
        mx[l] = sl.max()
        rms[l] = math.sqrt(float(np.mean(sl.astype(np.float64) ** 2)))
    return mx, rms
