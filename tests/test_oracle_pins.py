"""Pins of the CPU oracle to facts outside itself (closed forms, library
routines, invariants, finite differences).  CPU only.

Each test names the passage or textbook fact it checks.  The mutation tests at
the end plant plausible mistakes in the oracle and show that these pins catch
them.
"""
import math

import mpmath
import numpy as np
import pytest

import oracle
from oracle import definition, recurrence
from workloads import standard_normal_points, precision_stress_points

LD = np.longdouble
PI = math.pi


def _pts(n, seed):
    return standard_normal_points(n, seed)


def _near_pole(n, seed):
    rng = np.random.default_rng(seed)
    p = np.empty((n, 3))
    p[:, 0] = rng.choice([-1, 1], n) * 10.0 ** rng.uniform(-12, -3, n)
    p[:, 1] = rng.choice([-1, 1], n) * 10.0 ** rng.uniform(-12, -3, n)
    p[:, 2] = rng.choice([-1, 1], n) * rng.uniform(0.5, 2.0, n)
    return p


# ----------------------------------------------------------- closed forms
def closed_forms(p):
    """Textbook real spherical harmonics l <= 3 (standard table, Condon-Shortley
    convention), as functions of the Cartesian point."""
    x, y, z = p
    r = math.sqrt(x * x + y * y + z * z)
    out = [0.5 / math.sqrt(PI)]
    c1 = math.sqrt(3 / (4 * PI))
    out += [c1 * y / r, c1 * z / r, c1 * x / r]
    r2 = r * r
    out += [0.5 * math.sqrt(15 / PI) * x * y / r2,
            0.5 * math.sqrt(15 / PI) * y * z / r2,
            0.25 * math.sqrt(5 / PI) * (2 * z * z - x * x - y * y) / r2,
            0.5 * math.sqrt(15 / PI) * x * z / r2,
            0.25 * math.sqrt(15 / PI) * (x * x - y * y) / r2]
    r3 = r2 * r
    out += [0.25 * math.sqrt(35 / (2 * PI)) * y * (3 * x * x - y * y) / r3,
            0.5 * math.sqrt(105 / PI) * x * y * z / r3,
            0.25 * math.sqrt(21 / (2 * PI)) * y * (4 * z * z - x * x - y * y) / r3,
            0.25 * math.sqrt(7 / PI) * z * (2 * z * z - 3 * x * x - 3 * y * y) / r3,
            0.25 * math.sqrt(21 / (2 * PI)) * x * (4 * z * z - x * x - y * y) / r3,
            0.25 * math.sqrt(105 / PI) * (x * x - y * y) * z / r3,
            0.25 * math.sqrt(35 / (2 * PI)) * x * (x * x - 3 * y * y) / r3]
    return np.array(out)


@pytest.mark.parametrize("tier", ["bulk", "definition"])
def test_closed_forms_l_le_3(tier):
    pts = np.concatenate([_pts(40, 11), _near_pole(10, 12)])
    for p in pts:
        ref = closed_forms(p)
        if tier == "bulk":
            Y = oracle.real_sph(p[None], 3, True, gradients=False)[0]
        else:
            Y = oracle.definition_eval_ld(p[None], 3, True)[0][0]
        np.testing.assert_allclose(np.asarray(Y, dtype=float), ref, rtol=1e-13, atol=1e-15)


def test_scaled_equals_r_pow_l_times_normalised():
    pts = _pts(30, 13)
    Ys = oracle.real_sph(pts, 6, False, gradients=False)
    Yn = oracle.real_sph(pts, 6, True, gradients=False)
    r = np.sqrt((pts.astype(LD) ** 2).sum(1))
    for l in range(7):
        sl = slice(l * l, (l + 1) ** 2)
        np.testing.assert_allclose(np.asarray(Ys[:, sl], float),
                                   np.asarray(Yn[:, sl] * (r ** l)[:, None], float), rtol=1e-15, atol=0)


# --------------------------------------------------------- library routine
def _real_from_mpmath(l, m, theta, phi):
    """Real harmonic from mpmath's complex spherharm (Condon-Shortley phase)
    with the standard unitary map to real functions."""
    if m == 0:
        return mpmath.re(mpmath.spherharm(l, 0, theta, phi))
    c = mpmath.spherharm(l, abs(m), theta, phi)
    s = mpmath.sqrt(2) * (-1) ** abs(m)
    return s * (mpmath.im(c) if m < 0 else mpmath.re(c))


def test_mpmath_spherharm_cross_check():
    mpmath.mp.dps = 30
    rng = np.random.default_rng(14)
    for _ in range(6):
        th, ph = rng.uniform(0.05, 3.1), rng.uniform(-3.1, 3.1)
        p = np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
        Yb = oracle.real_sph(p[None], 6, True, gradients=False)[0]
        Ym, _ = oracle.definition_eval_mp(p, 6, True, dps=30)
        th_e = mpmath.acos(mpmath.mpf(p[2]) / mpmath.sqrt(sum(mpmath.mpf(c) ** 2 for c in p)))
        ph_e = mpmath.atan2(mpmath.mpf(p[1]), mpmath.mpf(p[0]))
        for l in range(7):
            for m in range(-l, l + 1):
                ref = float(_real_from_mpmath(l, m, th_e, ph_e))
                k = l * l + l + m
                assert abs(float(Yb[k]) - ref) < 1e-15, (l, m)
                assert abs(float(Ym[k]) - ref) < 1e-15, (l, m)


def test_ferrers_table_matches_mpmath_legenp():
    mpmath.mp.dps = 30
    t = np.array([0.3, -0.77, 0.999999], dtype=LD)
    s = np.sqrt(1 - t * t)
    P = oracle.ferrers_table(t, s, 12)
    for i, tv in enumerate(t):
        for l in range(13):
            for m in range(l + 1):
                ref = mpmath.legenp(l, m, mpmath.mpf(float(tv)), type=2)
                assert abs(float(P[l, m, i]) - float(ref)) <= 1e-14 * max(1.0, abs(float(ref))), (l, m)


def test_ferrers_derivative_identities():
    """The two identities the bulk gradient relies on, against mpmath.diff."""
    mpmath.mp.dps = 30
    P = lambda l, m, t: mpmath.mpf(0) if (m < 0 or m > l) else mpmath.legenp(l, m, t, type=2)
    for th in (mpmath.mpf("0.7"), mpmath.mpf("1e-3")):
        for l in range(0, 7):
            for m in range(0, l + 1):
                d = mpmath.diff(lambda T: P(l, m, mpmath.cos(T)), th)
                rhs = P(l, 1, mpmath.cos(th)) if m == 0 else \
                    (P(l, m + 1, mpmath.cos(th)) - (l + m) * (l - m + 1) * P(l, m - 1, mpmath.cos(th))) / 2
                assert abs(d - rhs) < 1e-20
                if m >= 1:
                    lhs = m * P(l, m, mpmath.cos(th)) / mpmath.sin(th)
                    rhs2 = -(P(l - 1, m + 1, mpmath.cos(th)) + (l + m - 1) * (l + m) * P(l - 1, m - 1, mpmath.cos(th))) / 2
                    assert abs(lhs - rhs2) < 1e-20


# ------------------------------------------------------------- prefactors
def test_prefactor_appendix_c_recursion():
    """App. C: F_l^0 = sqrt((2l+1)/2pi), F_l^m = -F_l^{m-1}/sqrt((l+m)(l+1-m))."""
    mpmath.mp.dps = 40
    for l in range(33):
        f = mpmath.sqrt(mpmath.mpf(2 * l + 1) / (2 * mpmath.pi))
        assert abs(oracle.prefactor(l, 0) - f) < mpmath.mpf(10) ** -35
        for m in range(1, l + 1):
            f = -f / mpmath.sqrt(mpmath.mpf((l + m) * (l + 1 - m)))
            assert abs(oracle.prefactor(l, m) - f) <= abs(f) * mpmath.mpf(10) ** -35
    assert abs(oracle.prefactor(1, 1) + mpmath.sqrt(3 / (4 * mpmath.pi))) < 1e-30


# -------------------------------------------------------------- invariants
@pytest.mark.parametrize("normalize", [False, True])
def test_addition_theorem(normalize):
    pts = np.concatenate([_pts(20, 15), _near_pole(10, 16)])
    Y = oracle.real_sph(pts, 32, normalize, gradients=False)
    r2 = (pts.astype(LD) ** 2).sum(1)
    for l in range(33):
        ssum = (Y[:, l * l:(l + 1) ** 2] ** 2).sum(1)
        ref = LD(2 * l + 1) / (4 * LD(np.pi)) * (1 if normalize else r2 ** l)
        np.testing.assert_allclose(np.asarray(ssum / ref, float), 1.0, rtol=1e-15)


def test_orthonormality_by_quadrature():
    """Gauss-Legendre (L+1 nodes in cos theta) x (2L+1 uniform phi) is exact for
    the products of two harmonics of degree <= L, so the Gram matrix is I."""
    L = 8
    tn, tw = np.polynomial.legendre.leggauss(L + 1)
    nphi = 2 * L + 1
    phis = 2 * np.pi * np.arange(nphi) / nphi
    T, PH = np.meshgrid(tn, phis, indexing="ij")
    W = (tw[:, None] * np.full(nphi, 2 * np.pi / nphi)[None, :]).ravel()
    st = np.sqrt(1 - T ** 2)
    pts = np.stack([st * np.cos(PH), st * np.sin(PH), T], -1).reshape(-1, 3)
    Y = np.asarray(oracle.real_sph(pts, L, True, gradients=False), float)
    gram = (Y * W[:, None]).T @ Y
    np.testing.assert_allclose(gram, np.eye((L + 1) ** 2), atol=1e-13)


def test_parity_and_homogeneity():
    pts = _pts(25, 17)
    L = 10
    Y = oracle.real_sph(pts, L, False, gradients=False)
    Ym = oracle.real_sph(-pts, L, False, gradients=False)
    lam = 1.7
    Yl = oracle.real_sph(lam * pts, L, False, gradients=False)
    for l in range(L + 1):
        sl = slice(l * l, (l + 1) ** 2)
        np.testing.assert_allclose(np.asarray(Ym[:, sl], float), (-1) ** l * np.asarray(Y[:, sl], float),
                                   rtol=1e-14, atol=1e-300)
        sc = oracle.component_scales(pts, L, False)[0][:, sl]
        err = np.abs(np.asarray(Yl[:, sl] - LD(lam) ** l * Y[:, sl], float)) / (lam ** l * sc)
        assert err.max() < 1e-15, l


@pytest.mark.parametrize("normalize", [False, True])
def test_euler_identity(normalize):
    """x . grad(r^l Y) = l r^l Y (homogeneous of degree l); x . grad Y = 0."""
    pts = np.concatenate([_pts(20, 18), _near_pole(8, 19)])
    L = 12
    Y, G = oracle.real_sph(pts, L, normalize)
    P = pts.astype(LD)
    e = np.einsum("na,nak->nk", P, G)
    s, g, _ = oracle.component_scales(pts, L, normalize)
    for l in range(L + 1):
        sl = slice(l * l, (l + 1) ** 2)
        ref = 0 if normalize else l * Y[:, sl]
        r = np.sqrt((pts ** 2).sum(1))[:, None]
        err = np.abs(np.asarray(e[:, sl] - ref, float)) / (g[:, sl] * r)
        assert err.max() < 1e-15, l


@pytest.mark.parametrize("normalize", [False, True])
def test_gradient_addition_theorem(normalize):
    pts = np.concatenate([_pts(20, 20), _near_pole(8, 21)])
    L = 16
    _, G = oracle.real_sph(pts, L, normalize)
    r2 = (pts.astype(LD) ** 2).sum(1)
    for l in range(1, L + 1):
        ssum = (G[:, :, l * l:(l + 1) ** 2] ** 2).sum((1, 2))
        if normalize:
            ref = LD(l * (l + 1) * (2 * l + 1)) / (4 * LD(np.pi) * r2)
        else:
            ref = LD(l * (2 * l + 1) ** 2) / (4 * LD(np.pi)) * r2 ** (l - 1)
        np.testing.assert_allclose(np.asarray(ssum / ref, float), 1.0, rtol=1e-14)


@pytest.mark.parametrize("normalize", [False, True])
def test_gradient_vs_central_differences(normalize):
    """Central differences of the values, step 1e-6 in longdouble."""
    pts = np.concatenate([_pts(10, 22), _near_pole(5, 23)]).astype(LD)
    L = 8
    _, G = oracle.real_sph(pts, L, normalize)
    h = LD("1e-6")
    _, g, _ = oracle.component_scales(np.asarray(pts, float), L, normalize)
    for a in range(3):
        e = np.zeros(3, dtype=LD)
        e[a] = h
        fd = (oracle.real_sph(pts + e, L, normalize, gradients=False)
              - oracle.real_sph(pts - e, L, normalize, gradients=False)) / (2 * h)
        err = np.abs(np.asarray(fd - G[:, a], float)) / g
        assert err.max() < 1e-9


@pytest.mark.parametrize("normalize", [False, True])
def test_tiers_agree(normalize):
    pts = np.concatenate([_pts(30, 24), _near_pole(10, 25),
                          np.array([[0.0, 0.0, 1.3], [0.0, 0.0, -0.4], [1e-300, 0, 2.0]])])
    L = 10
    Yb, Gb = oracle.real_sph(pts, L, normalize)
    Yd, Gd = oracle.definition_eval_ld(pts, L, normalize)
    mx, _ = oracle.per_l_errors(Yb, Yd, pts, L, normalize, "Y")
    assert mx.max() < 1e-15
    mx, _ = oracle.per_l_errors(Gb, Gd, pts, L, normalize, "dY")
    assert mx.max() < 1e-15


def test_bulk_tier_at_l32_against_high_precision_definition():
    """The bulk tier at l = 32 against the exact polynomials at 80 digits."""
    pts = np.array([[0.3, -0.8, 0.52], [1e-7, 2e-8, -1.0]])
    Yb, Gb = oracle.real_sph(pts, 32, True)
    for i, p in enumerate(pts):
        Ym, Gm = oracle.definition_eval_mp(p, 32, True, dps=80)
        Yr = np.array([float(v) for v in Ym])
        Gr = np.array([[float(v) for v in row] for row in Gm])
        mx, _ = oracle.per_l_errors(Yb[i:i + 1], Yr[None], p[None], 32, True, "Y")
        assert mx.max() < 1e-15
        mx, _ = oracle.per_l_errors(Gb[i:i + 1], Gr[None], p[None], 32, True, "dY")
        assert mx.max() < 1e-15


def test_precision_stress_mix_finite():
    xyz, _ = precision_stress_points(3000, 5)
    Y, G = oracle.real_sph(xyz, 32, True)
    assert np.isfinite(np.asarray(Y, float)).all() and np.isfinite(np.asarray(G, float)).all()


# ---------------------------------------------------------------- Hessians
@pytest.mark.parametrize("L", [8, 12])
@pytest.mark.parametrize("normalize", [False, True])
def test_hessian_invariants(normalize, L):
    """Symmetric; trace 0 for the solid harmonics (they are harmonic) and
    -l(l+1) Y / r^2 for the normalised ones; Euler: H x = (l-1) grad for solid."""
    pts = np.concatenate([_pts(12, 26), _near_pole(4, 27)])
    Y, G, H = oracle.definition_eval_ld(pts, L, normalize, hessian=True)
    np.testing.assert_array_equal(np.asarray(H, float), np.asarray(np.swapaxes(H, 1, 2), float))
    tr = H[:, 0, 0] + H[:, 1, 1] + H[:, 2, 2]
    _, _, h = oracle.component_scales(pts, L, normalize)
    r2 = (pts.astype(LD) ** 2).sum(1)[:, None]
    ls = np.array([l for l in range(L + 1) for _ in range(2 * l + 1)], dtype=LD)
    ref = -ls * (ls + 1) * Y / r2 if normalize else 0 * Y
    assert (np.abs(np.asarray(tr - ref, float)) / h).max() < 1e-14
    if not normalize:
        Hx = np.einsum("nabk,nb->nak", H, pts.astype(LD))
        err = np.abs(np.asarray(Hx - (ls - 1) * G * (ls > 0), float))
        _, g, _ = oracle.component_scales(pts, L, normalize)
        assert (err / g[:, None, :]).max() < 1e-14


@pytest.mark.parametrize("L", [6, 12])
@pytest.mark.parametrize("normalize", [False, True])
def test_hessian_vs_differences_of_gradient(normalize, L):
    """The definition tier's exact Hessians against central differences of
    the bulk tier's gradients (an independent route), up to l = 12, the
    range the GPU Hessian tests compare against."""
    pts = np.concatenate([_pts(8, 28), _near_pole(4, 29)]).astype(LD)
    _, _, H = oracle.definition_eval_ld(pts, L, normalize, hessian=True)
    _, _, hs = oracle.component_scales(np.asarray(pts, float), L, normalize)
    h = LD("1e-6")
    for b in range(3):
        e = np.zeros(3, dtype=LD)
        e[b] = h
        fd = (oracle.real_sph(pts + e, L, normalize)[1] - oracle.real_sph(pts - e, L, normalize)[1]) / (2 * h)
        err = np.abs(np.asarray(fd - H[:, :, b], float)) / hs[:, None, :]
        assert err.max() < 1e-8


def test_definition_mp_hessian_matches_ld():
    p = np.array([0.4, -1.1, 0.25])
    Ym, Gm, Hm = oracle.definition_eval_mp(p, 5, True, dps=40, hessian=True)
    Y, G, H = oracle.definition_eval_ld(p[None], 5, True, hessian=True)
    Hr = np.array([[[float(v) for v in row] for row in blk] for blk in Hm])
    np.testing.assert_allclose(np.asarray(H[0], float), Hr, rtol=1e-15, atol=1e-15)


# --------------------------------------------------------- special points
def test_origin_conventions():
    p = np.zeros((1, 3))
    Y, G = oracle.real_sph(p, 4, True)
    assert float(Y[0, 0]) == pytest.approx(0.5 / math.sqrt(PI), rel=1e-18)
    assert np.all(np.asarray(Y[0, 1:], float) == 0) and np.all(np.asarray(G, float) == 0)
    Y, G = oracle.real_sph(p, 4, False)
    c = math.sqrt(3 / (4 * PI))
    assert np.all(np.asarray(Y[0, 1:], float) == 0)
    # l = 1 solid harmonics are c*(y, z, x): constant gradients
    np.testing.assert_allclose(np.asarray(G[0, :, 1:4], float), c * np.array([[0, 0, 1], [1, 0, 0], [0, 1, 0]]),
                               rtol=1e-15)
    assert np.all(np.asarray(G[0, :, 4:], float) == 0)
    Yd, Gd = oracle.definition_eval_ld(p, 4, False)
    np.testing.assert_allclose(np.asarray(G, float), np.asarray(Gd, float), atol=1e-18)


def test_exact_pole_gradient():
    p = np.array([[0.0, 0.0, 1.5], [0.0, 0.0, -0.7]])
    for normalize in (False, True):
        _, Gb = oracle.real_sph(p, 8, normalize)
        _, Gd = oracle.definition_eval_ld(p, 8, normalize)
        mx, _ = oracle.per_l_errors(Gb, Gd, p, 8, normalize, "dY")
        assert mx.max() < 1e-16


def test_backward_contraction_definition():
    rng = np.random.default_rng(30)
    dY = rng.standard_normal((5, 3, 9))
    gY = rng.standard_normal((5, 9))
    out = oracle.backward(dY, gY)
    for n in range(5):
        for a in range(3):
            assert float(out[n, a]) == pytest.approx(sum(dY[n, a, k] * gY[n, k] for k in range(9)), rel=1e-14)


# ------------------------------------------------- mutations have teeth
def test_mutation_wrong_prefactor_sign_is_caught(monkeypatch):
    def bad(l, m, ctx=mpmath.mp):
        ratio = math.factorial(l - m) / math.factorial(l + m) * (2 * l + 1)
        return ctx.sqrt(ctx.mpf(ratio) / (2 * ctx.pi))  # (-1)^m dropped
    monkeypatch.setattr(recurrence, "prefactor", bad)
    recurrence._prefactors_ld.cache_clear()
    try:
        with pytest.raises(AssertionError):
            test_closed_forms_l_le_3("bulk")
    finally:
        recurrence._prefactors_ld.cache_clear()


def test_mutation_recurrence_term_is_caught(monkeypatch):
    def bad_table(t, s, l_max):
        P = np.zeros((l_max + 2, l_max + 3, t.shape[0]), dtype=LD)
        P[0, 0] = 1
        for l in range(1, l_max + 1):
            P[l, l] = -(2 * l - 1) * s * P[l - 1, l - 1]
            P[l, l - 1] = (2 * l - 1) * t * P[l - 1, l - 1]
            for m in range(l - 1):
                P[l, m] = ((2 * l - 1) * t * P[l - 1, m] - (l + m) * P[l - 2, m]) / (l - m)  # off by one
        return P
    monkeypatch.setattr(recurrence, "ferrers_table", bad_table)
    with pytest.raises(AssertionError):
        test_addition_theorem(True)


def test_mutation_gradient_component_is_caught(monkeypatch):
    """A gradient component off by one part in 10^7 fails the differences pin."""
    src_real_sph = recurrence.real_sph

    def bad_real_sph(xyz, l_max, normalize, gradients=True):
        out = src_real_sph(xyz, l_max, normalize, gradients)
        if gradients:
            Y, G = out
            G = G.copy()
            G[:, 0, :] *= LD(1.0000001)
            return Y, G
        return out
    monkeypatch.setattr(oracle, "real_sph", bad_real_sph)
    with pytest.raises(AssertionError):
        test_gradient_vs_central_differences(True)


def test_golden_exact_tier_values(repo_root):
    """Stored exact-tier values (tests/golden/make_golden.py, 25 digits) against
    both tiers as they stand now."""
    import json
    import os
    with open(os.path.join(repo_root, "tests", "golden", "exact_tier_l6.json")) as f:
        gold = json.load(f)
    L = gold["l_max"]
    for case in gold["cases"]:
        p = np.array([float.fromhex(c) for c in case["point"]])
        n = case["normalize"]
        Yg = np.array([LD(v) for v in case["Y"]], dtype=LD)
        Gg = np.array([[LD(v) for v in row] for row in case["dY"]], dtype=LD)
        Hg = np.array([[[LD(v) for v in row] for row in blk] for blk in case["H"]], dtype=LD)
        Yb, Gb = oracle.real_sph(p[None], L, n)
        Yd, Gd, Hd = oracle.definition_eval_ld(p[None], L, n, hessian=True)
        s, g, h = oracle.component_scales(p[None], L, n)
        assert (np.abs(np.asarray(Yb[0] - Yg, float)) / s[0]).max() < 1e-16
        assert (np.abs(np.asarray(Gb[0] - Gg, float)) / g[0]).max() < 1e-16
        assert (np.abs(np.asarray(Hd[0] - Hg, float)) / h[0]).max() < 1e-16


# -------------------------------------------------- radial expansion (Eq. expansion)
def _expansion_case(seed, counts, l_max, n_max):
    rng = np.random.default_rng(seed)
    offs = np.zeros(len(counts) + 1, np.int64)
    np.cumsum(counts, out=offs[1:])
    pts = rng.standard_normal((int(offs[-1]), 3)) * rng.uniform(0.5, 2.0, (int(offs[-1]), 1))
    R = rng.standard_normal((int(offs[-1]), l_max + 1, n_max))
    return pts, offs, R


@pytest.mark.parametrize("normalize", [False, True])
def test_radial_expansion_power_spectrum_addition_theorem(normalize):
    """sum_m c_nlm c_n'lm = (2l+1)/(4 pi) sum_{j,j'} R_jln R_j'ln' s_j s_j' P_l(cos g_jj')
    by the addition theorem (s = 1, or r^l for the solid harmonics), with P_l
    from scipy: pins the sum over the environment, the degree each weight
    goes with, and the harmonics, independently of the oracle's own route."""
    from scipy.special import eval_legendre
    L, NM = 6, 3
    counts = [5, 0, 1, 9]
    pts, offs, R = _expansion_case(41, counts, L, NM)
    c = oracle.radial_expansion(pts, offs, R, L, normalize)
    assert c.shape == (4, NM, (L + 1) ** 2)
    assert np.all(c[1] == 0)
    for e in range(4):
        b, t = offs[e], offs[e + 1]
        P = pts[b:t]
        r = np.sqrt((P * P).sum(1))
        cosg = np.clip((P / r[:, None]) @ (P / r[:, None]).T, -1.0, 1.0)
        for l in range(L + 1):
            cl = np.asarray(c[e][:, l * l:(l + 1) ** 2], float)
            lhs = cl @ cl.T
            s = np.ones_like(r) if normalize else r ** l
            W = R[b:t, l, :] * s[:, None]                       # [cnt, NM]
            rhs = (2 * l + 1) / (4 * np.pi) * W.T @ eval_legendre(l, cosg) @ W
            np.testing.assert_allclose(lhs, rhs, rtol=1e-11, atol=1e-12 * (1 + np.abs(rhs).max()))


def test_radial_expansion_rotation_invariance_and_single_point():
    """The power spectrum of an environment is unchanged by a rotation of all
    its points; a one-point environment with R = 1 is that point's harmonics."""
    L, NM = 5, 2
    pts, offs, R = _expansion_case(43, [7], L, NM)
    q, _ = np.linalg.qr(np.random.default_rng(44).standard_normal((3, 3)))
    c0 = np.asarray(oracle.radial_expansion(pts, offs, R, L, True), float)[0]
    c1 = np.asarray(oracle.radial_expansion(pts @ q.T, offs, R, L, True), float)[0]
    for l in range(L + 1):
        sl = slice(l * l, (l + 1) ** 2)
        np.testing.assert_allclose(c0[:, sl] @ c0[:, sl].T, c1[:, sl] @ c1[:, sl].T, rtol=1e-11, atol=1e-13)
    one = np.array([[0.3, -1.1, 0.7]])
    c = oracle.radial_expansion(one, np.array([0, 1]), np.ones((1, L + 1, 1)), L, False)
    Y = oracle.real_sph(one, L, False, gradients=False)
    assert np.all(c[0, 0] == Y[0])


def test_mutation_expansion_degree_of_weight_is_caught(monkeypatch):
    """Weights taken from the next degree's radial function fail the pin."""
    from oracle import derived
    good = derived._ls

    def shifted(l_max):
        return np.minimum(good(l_max) + 1, l_max)
    monkeypatch.setattr(derived, "_ls", shifted)
    with pytest.raises(AssertionError):
        test_radial_expansion_power_spectrum_addition_theorem(True)


@pytest.mark.parametrize("normalize", [False, True])
def test_radial_expansion_backward_by_differences(normalize):
    """grad_xyz against central differences of the oracle's expansion, and
    grad_R against the expansion's linearity in R: <grad_R, dR> equals
    <G, c(dR)> exactly."""
    L, NM = 4, 3
    pts, offs, R = _expansion_case(47, [4, 0, 6], L, NM)
    G = np.random.default_rng(48).standard_normal((3, NM, (L + 1) ** 2))
    gx, gR = oracle.radial_expansion_backward(pts, offs, R, G, L, normalize)
    h = 1e-5
    for j in range(pts.shape[0]):
        for a in range(3):
            d = np.zeros_like(pts)
            d[j, a] = h
            cp = oracle.radial_expansion(pts + d, offs, R, L, normalize)
            cm = oracle.radial_expansion(pts - d, offs, R, L, normalize)
            fd = float(((cp - cm) * G).sum()) / (2 * h)
            assert abs(float(gx[j, a]) - fd) <= 1e-7 * (1 + abs(fd)), (j, a, float(gx[j, a]), fd)
    dR = np.random.default_rng(49).standard_normal(R.shape)
    lhs = float((gR * dR).sum())
    rhs = float((oracle.radial_expansion(pts, offs, dR, L, normalize) * G).sum())
    assert abs(lhs - rhs) <= 1e-13 * (1 + abs(rhs))


# ------------------------------------------------------ e3nn's conventions
# The reading of Sec. III.B (e3nn's conventions, not stated in the paper):
# y as the polar axis, degree 1 proportional to (x, y, z) in that order,
# normalisations "integral" / "component" / "norm".  e3nn is not installed,
# so beyond these properties the ordering within a degree is parity
# unpinned.
@pytest.mark.parametrize("normalize", [True, False])
def test_e3nn_degree_one_is_the_point(normalize):
    """Component normalisation: Y_0 = 1 and Y_1 = sqrt(3) (x, y, z) / r (times r
    for the scaled harmonics)."""
    p = _pts(50, 801)
    Y, _ = oracle.e3nn_convention(p, 1, normalize, "component")
    r = np.linalg.norm(p, axis=1, keepdims=True)
    want1 = math.sqrt(3) * (p / r if normalize else p)
    assert np.allclose(np.asarray(Y[:, 0], float), 1.0, rtol=1e-15, atol=0)
    assert np.abs(np.asarray(Y[:, 1:4], float) - want1).max() <= 1e-14 * max(1.0, float(np.abs(want1).max()))
    # the other cyclic order, (y, z, x), does not give it
    Yalt, _ = oracle.real_sph(p[:, [1, 2, 0]], 1, normalize)
    assert np.abs(math.sqrt(4 * PI) * np.asarray(Yalt[:, 1:4], float) - want1).max() > 0.1


@pytest.mark.parametrize("normalization,target", [("integral", lambda l: (2 * l + 1) / (4 * PI)),
                                                  ("component", lambda l: 2 * l + 1),
                                                  ("norm", lambda l: 1.0)])
def test_e3nn_normalisation_sums(normalization, target):
    """Addition theorem: sum_m Y_lm(u)^2 on the unit sphere is (2l+1)/(4 pi)
    for unit L2 norm, times the square of the per-degree factor."""
    p = _pts(40, 802)
    u = p / np.linalg.norm(p, axis=1, keepdims=True)
    L = 8
    Y, _ = oracle.e3nn_convention(u, L, False, normalization)
    Y = np.asarray(Y, float)
    for l in range(L + 1):
        s = (Y[:, l * l:(l + 1) ** 2] ** 2).sum(1)
        assert np.allclose(s, target(l), rtol=1e-13, atol=0), (normalization, l)


def test_e3nn_polar_axis_is_y():
    """On the y axis only the m = 0 column of each degree survives, with
    Y_l0(0, +-1, 0) = (+-1)^l sqrt((2l+1) / (4 pi)) (Legendre P_l(+-1)) for
    unit L2 norm; elsewhere on the sphere the m != 0 columns do not vanish."""
    L = 10
    p = np.array([[0.0, 1.0, 0.0], [0.0, -1.0, 0.0]])
    Y, _ = oracle.e3nn_convention(p, L, True, "integral")
    Y = np.asarray(Y, float)
    for l in range(L + 1):
        row = Y[:, l * l:(l + 1) ** 2].copy()
        want = math.sqrt((2 * l + 1) / (4 * PI))
        assert abs(row[0, l] - want) < 1e-14 and abs(row[1, l] - (-1) ** l * want) < 1e-14
        row[:, l] = 0
        assert np.abs(row).max() < 1e-14, l
    Yz, _ = oracle.e3nn_convention(np.array([[0.0, 0.0, 1.0]]), L, True, "integral")
    assert np.abs(np.asarray(Yz, float)[0, 4:9]).max() > 0.1  # the z axis is not the pole


@pytest.mark.parametrize("normalize", [True, False])
@pytest.mark.parametrize("normalization", ["integral", "component", "norm"])
def test_e3nn_gradient_by_differences(normalize, normalization):
    """dY[:, a] is the derivative along the caller's axis a (central
    differences of Y, h = 1e-6 in longdouble)."""
    p = _pts(20, 803)
    L = 6
    _, dY = oracle.e3nn_convention(p, L, normalize, normalization)
    h = 1e-6
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        Yp, _ = oracle.e3nn_convention(p + e, L, normalize, normalization)
        Ym, _ = oracle.e3nn_convention(p - e, L, normalize, normalization)
        fd = np.asarray((Yp - Ym) / (2 * h), float)
        assert np.abs(np.asarray(dY[:, a], float) - fd).max() < 1e-7 * max(1.0, float(np.abs(fd).max())), a
