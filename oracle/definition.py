"""Definition tier: every solid harmonic as an explicit polynomial.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The real harmonic is Y_l^m = F_l^{|m|} P_l^{|m|}(cos t) x {sin |m|phi, 1/sqrt2,
cos m phi} (Eq. real-sh-spherical) with F_l^m from Eq. Flm and P_l^m the
Ferrers function with the Condon-Shortley phase (as in Eq. recur-p, whose
first step carries the minus sign).  Multiplying by r^l gives the solid
harmonic (Sec. II), a homogeneous polynomial of degree l.  It is written out
here from textbook facts only:

* Legendre polynomial, explicit sum:
  P_l(t) = 2^-l sum_k (-1)^k C(l,k) C(2l-2k,l) t^(l-2k);
* Ferrers function with Condon-Shortley phase:
  P_l^m(t) = (-1)^m (1-t^2)^(m/2) d^m P_l / dt^m;
* with t = z/r and (1-t^2)^(1/2) = r_xy/r, and the polar form
  r_xy^m cos(m phi) = Re (x+iy)^m, r_xy^m sin(m phi) = Im (x+iy)^m,

  r^l P_l^m(z/r) trig(m phi) = (-1)^m [sum_j d_j z^j r^(l-m-j)] Re/Im (x+iy)^m

  where d_j are the coefficients of d^m P_l/dt^m; l-m-j is even so the
  bracket is a polynomial.

Coefficients are exact ``Fraction``s; only the irrational prefactor F is a
float (mpmath at the caller's precision, or longdouble).  Derivatives are
exact polynomial derivatives.  The normalised harmonic is the solid one
divided by r^l (its derivatives by the plain quotient rule at the point).
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache
from math import comb, factorial

import mpmath
import numpy as np

Poly = dict  # {(i, j, k): Fraction} for the monomial x^i y^j z^k


# ---------------------------------------------------------------- polynomials
def _pmul(a: Poly, b: Poly) -> Poly:
    out: Poly = {}
    for (i1, j1, k1), c1 in a.items():
        for (i2, j2, k2), c2 in b.items():
            key = (i1 + i2, j1 + j2, k1 + k2)
            out[key] = out.get(key, 0) + c1 * c2
    return {k: v for k, v in out.items() if v != 0}


def _padd(a: Poly, b: Poly, sb=1) -> Poly:
    out = dict(a)
    for k, v in b.items():
        out[k] = out.get(k, 0) + sb * v
    return {k: v for k, v in out.items() if v != 0}


def _pscale(a: Poly, s) -> Poly:
    return {k: v * s for k, v in a.items() if v * s != 0}


def pdiff(a: Poly, axis: int) -> Poly:
    """Exact partial derivative of a polynomial along axis 0 (x), 1 (y), 2 (z)."""
    out: Poly = {}
    for key, c in a.items():
        e = key[axis]
        if e == 0:
            continue
        nk = list(key)
        nk[axis] = e - 1
        nk = tuple(nk)
        out[nk] = out.get(nk, 0) + c * e
    return {k: v for k, v in out.items() if v != 0}


def _r2_power(n: int) -> Poly:
    """(x^2 + y^2 + z^2)^n expanded by the multinomial theorem."""
    out: Poly = {}
    for a in range(n + 1):
        for b in range(n - a + 1):
            c = n - a - b
            coef = factorial(n) // (factorial(a) * factorial(b) * factorial(c))
            out[(2 * a, 2 * b, 2 * c)] = Fraction(coef)
    return out


def _xiy_power(m: int) -> tuple[Poly, Poly]:
    """Real and imaginary parts of (x + i y)^m, by the binomial theorem."""
    re: Poly = {}
    im: Poly = {}
    for k in range(m + 1):
        c = comb(m, k)
        # (iy)^k = i^k y^k ; i^k cycles 1, i, -1, -i
        ph = k % 4
        key = (m - k, k, 0)
        if ph == 0:
            re[key] = Fraction(c)
        elif ph == 1:
            im[key] = Fraction(c)
        elif ph == 2:
            re[key] = Fraction(-c)
        else:
            im[key] = Fraction(-c)
    return re, im


def legendre_coeffs(l: int) -> dict[int, Fraction]:
    """Coefficients {power: c} of the Legendre polynomial P_l(t), explicit sum."""
    out = {}
    for k in range(l // 2 + 1):
        out[l - 2 * k] = Fraction((-1) ** k * comb(l, k) * comb(2 * l - 2 * k, l), 2 ** l)
    return out


def _dm_coeffs(l: int, m: int) -> dict[int, Fraction]:
    """Coefficients of d^m P_l / dt^m."""
    c = legendre_coeffs(l)
    for _ in range(m):
        c = {p - 1: v * p for p, v in c.items() if p > 0}
    return c


@lru_cache(maxsize=None)
def solid_poly(l: int, m: int) -> tuple[Poly, Fraction]:
    """Return ``(poly, extra)`` with r^l Y_l^m = F_l^{|m|} * extra * poly.

    ``extra`` is 1 except for m = 0 where it is 1/2 under the square root, i.e.
    the caller multiplies by sqrt(extra_sq); to keep everything rational the
    1/sqrt2 of m = 0 is returned as extra = Fraction(1, 2) meaning "times
    sqrt(1/2)".
    """
    mu = abs(m)
    if mu > l:
        raise ValueError("|m| > l")
    d = _dm_coeffs(l, mu)
    bracket: Poly = {}
    for j, dj in d.items():
        e = l - mu - j
        assert e % 2 == 0
        term = _pmul({(0, 0, j): Fraction(1)}, _r2_power(e // 2))
        bracket = _padd(bracket, _pscale(term, dj))
    bracket = _pscale(bracket, (-1) ** mu)  # Condon-Shortley phase of P_l^m
    re, im = _xiy_power(mu)
    if m > 0:
        return _pmul(bracket, re), Fraction(1)
    if m < 0:
        return _pmul(bracket, im), Fraction(1)
    return bracket, Fraction(1, 2)


def prefactor(l: int, m: int, ctx=mpmath.mp):
    """F_l^m = (-1)^m sqrt((2l+1)/(2 pi) (l-m)!/(l+m)!)  (Eq. Flm), m >= 0."""
    ratio = Fraction((2 * l + 1) * factorial(l - m), factorial(l + m))
    v = ctx.sqrt(ctx.mpf(ratio.numerator) / ctx.mpf(ratio.denominator) / (2 * ctx.pi))
    return -v if (m % 2) else v


def _full_prefactor_mp(l: int, m: int):
    poly, extra = solid_poly(l, m)
    F = prefactor(l, abs(m))
    if extra != 1:
        F = F * mpmath.sqrt(mpmath.mpf(extra.numerator) / extra.denominator)
    return F, poly


# --------------------------------------------------------------- evaluation
def _eval_poly_mp(poly: Poly, X, Yv, Z):
    s = mpmath.mpf(0)
    for (i, j, k), c in poly.items():
        s += (mpmath.mpf(c.numerator) / c.denominator) * X ** i * Yv ** j * Z ** k
    return s


def definition_eval_mp(point, l_max: int, normalize: bool, dps: int = 50,
                       hessian: bool = False):
    """Exact-tier values at one point, evaluated in mpmath at ``dps`` digits.

    ``point`` is any triple convertible to mpmath numbers (use exact binary
    floats).  Returns ``(Y[K], dY[3,K])`` or ``(Y, dY, H[3,3,K])`` as mpf
    nested lists, K = (l_max+1)^2, index k = l^2 + l + m.
    """
    with mpmath.workdps(dps):
        X, Yv, Z = (mpmath.mpf(float(c)) for c in point)
        r2 = X * X + Yv * Yv + Z * Z
        r = mpmath.sqrt(r2)
        K = (l_max + 1) ** 2
        Yo = [mpmath.mpf(0)] * K
        G = [[mpmath.mpf(0)] * K for _ in range(3)]
        H = [[[mpmath.mpf(0)] * K for _ in range(3)] for _ in range(3)]
        xs = (X, Yv, Z)
        for l in range(l_max + 1):
            for m in range(-l, l + 1):
                k = l * l + l + m
                F, poly = _full_prefactor_mp(l, m)
                v = F * _eval_poly_mp(poly, X, Yv, Z)
                g = [F * _eval_poly_mp(pdiff(poly, a), X, Yv, Z) for a in range(3)]
                h = None
                if hessian:
                    h = [[F * _eval_poly_mp(pdiff(pdiff(poly, a), b), X, Yv, Z)
                          for b in range(3)] for a in range(3)]
                if not normalize:
                    Yo[k] = v
                    for a in range(3):
                        G[a][k] = g[a]
                    if hessian:
                        for a in range(3):
                            for b in range(3):
                                H[a][b][k] = h[a][b]
                    continue
                if r == 0:
                    # direction undefined: Y_0^0 keeps its constant, all else 0
                    Yo[k] = v if l == 0 else mpmath.mpf(0)
                    continue
                # quotient rule for Ytilde / r^l
                rl = r ** l
                Yo[k] = v / rl
                for a in range(3):
                    G[a][k] = g[a] / rl - l * v * xs[a] / (rl * r2)
                if hessian:
                    for a in range(3):
                        for b in range(3):
                            t = h[a][b] / rl
                            t -= l * (g[a] * xs[b] + g[b] * xs[a]) / (rl * r2)
                            if a == b:
                                t -= l * v / (rl * r2)
                            t += l * (l + 2) * v * xs[a] * xs[b] / (rl * r2 * r2)
                            H[a][b][k] = t
        if hessian:
            return Yo, G, H
        return Yo, G


@lru_cache(maxsize=None)
def _ld_tables(l_max: int):
    """Per-(l,m) monomial exponent/coefficient arrays in longdouble."""
    out = []
    with mpmath.workdps(40):
        for l in range(l_max + 1):
            for m in range(-l, l + 1):
                F, poly = _full_prefactor_mp(l, m)
                derivs = {(): poly}
                for a in range(3):
                    derivs[(a,)] = pdiff(poly, a)
                for a in range(3):
                    for b in range(a, 3):
                        derivs[(a, b)] = pdiff(derivs[(a,)], b)
                conv = {}
                for key, p in derivs.items():
                    if not p:
                        conv[key] = None
                        continue
                    ex = np.array(list(p.keys()), dtype=np.int64)
                    co = np.array([np.longdouble(mpmath.nstr(F * mpmath.mpf(c.numerator) / c.denominator, 30))
                                   for c in p.values()], dtype=np.longdouble)
                    conv[key] = (ex, co)
                out.append((l, m, conv))
    return out


def _eval_poly_ld(ex_co, pw):
    if ex_co is None:
        return np.zeros(pw[0].shape[1], dtype=np.longdouble)
    ex, co = ex_co
    px, py, pz = pw
    acc = np.zeros(px.shape[1], dtype=np.longdouble)
    for (i, j, k), c in zip(ex, co):
        acc += c * px[i] * py[j] * pz[k]
    return acc


def definition_eval_ld(xyz, l_max: int, normalize: bool, hessian: bool = False):
    """Definition tier vectorised over points in numpy longdouble.

    Intended for small l (<= 12) where the explicit polynomials cancel only
    mildly; the mpmath variant is the reference at any l.  Returns
    ``(Y[N,K], dY[N,3,K])`` or ``(Y, dY, H[N,3,3,K])`` in longdouble.
    """
    P = np.asarray(xyz, dtype=np.longdouble).reshape(-1, 3)
    N = P.shape[0]
    K = (l_max + 1) ** 2
    x, y, z = P[:, 0], P[:, 1], P[:, 2]
    pw = []
    for c in (x, y, z):
        t = np.ones((l_max + 1, N), dtype=np.longdouble)
        for e in range(1, l_max + 1):
            t[e] = t[e - 1] * c
        pw.append(t)
    Yt = np.zeros((N, K), dtype=np.longdouble)
    Gt = np.zeros((N, 3, K), dtype=np.longdouble)
    Ht = np.zeros((N, 3, 3, K), dtype=np.longdouble) if hessian else None
    for l, m, conv in _ld_tables(l_max):
        k = l * l + l + m
        Yt[:, k] = _eval_poly_ld(conv[()], pw)
        for a in range(3):
            Gt[:, a, k] = _eval_poly_ld(conv[(a,)], pw)
        if hessian:
            for a in range(3):
                for b in range(a, 3):
                    v = _eval_poly_ld(conv[(a, b)], pw)
                    Ht[:, a, b, k] = v
                    Ht[:, b, a, k] = v
    if not normalize:
        return (Yt, Gt, Ht) if hessian else (Yt, Gt)
    r2 = x * x + y * y + z * z
    r = np.sqrt(r2)
    zero = r == 0
    rs = np.where(zero, np.longdouble(1), r)
    r2s = rs * rs
    ls = np.array([l for l in range(l_max + 1) for _ in range(2 * l + 1)], dtype=np.longdouble)
    rl = rs[:, None] ** ls[None, :]
    Y = Yt / rl
    G = Gt / rl[:, None, :] - ls[None, None, :] * Yt[:, None, :] * P[:, :, None] / (rl * r2s[:, None])[:, None, :]
    H = None
    if hessian:
        H = Ht / rl[:, None, None, :]
        gx = Gt[:, :, None, :] * P[:, None, :, None]
        H = H - ls * (gx + np.swapaxes(gx, 1, 2)) / (rl * r2s[:, None])[:, None, None, :]
        eye = np.eye(3, dtype=np.longdouble)
        H = H - ls * Yt[:, None, None, :] * eye[None, :, :, None] / (rl * r2s[:, None])[:, None, None, :]
        H = H + ls * (ls + 2) * Yt[:, None, None, :] * (P[:, :, None] * P[:, None, :])[:, :, :, None] \
            / (rl * r2s[:, None] * r2s[:, None])[:, None, None, :]
    if zero.any():
        Y[zero] = 0
        Y[zero, 0] = Yt[zero, 0]
        G[zero] = 0
        if hessian:
            H[zero] = 0
    return (Y, G, H) if hessian else (Y, G)
