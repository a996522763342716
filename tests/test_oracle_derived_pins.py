"""Pins of the oracle's derived functions: the backward and double-backward
contractions and the per-degree error metric.  CPU only.

These functions are the checkers of every GPU parity test, so each one is tied
to something outside its own formula:

* ``backward``: central differences of L(x) = sum_k gY_k Y_k(x), with the
  values taken from the definition tier (exact polynomials), so neither the
  contraction nor the bulk tier's analytic gradient is its own reference.
* ``double_backward`` / ``hessian_contract``: the first output is the exact
  derivative of <v, backward> in gY (the expression is linear in gY), the
  second is central differences in x of <v, backward(dY(x), gY)> built from
  the bulk tier's first derivatives (no Hessian involved).
* ``component_scales``: the addition theorems fix the size of a degree-l
  block, sum_m Y_lm^2 and sum_m |grad Y_lm|^2, independently of the scale
  formula; they are summed here from the oracle's values and gradients.
* ``per_l_errors``: errors of known size planted at a known degree, order and
  axis come back as that size (over the addition-theorem scale) at that
  degree and as 0 elsewhere; a NaN comes back as inf.

The mutation tests plant plausible mistakes (a contraction over the wrong
axis, the normalised scale used for the solid harmonics, a dropped chain-rule
term) and show that these pins fail.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import derived
from workloads import standard_normal, standard_normal_points

LD = np.longdouble
PI = math.pi


def _pts(n, seed):
    p = standard_normal_points(n, seed)
    # a few points near the poles and off the unit sphere
    p[:2, :2] *= 1e-3
    p[2] *= 3.0
    return p


def _fd_x(fun, pts, rel):
    """Central differences of fun([N,3] longdouble) -> [N] in each coordinate,
    with the step rel * |x| of each point (truncation ~ rel^2, rounding
    ~ eps / rel, relative to the derivative's size)."""
    pts = np.asarray(pts, dtype=LD)
    h = LD(rel) * np.sqrt((pts * pts).sum(1))[:, None]
    out = np.zeros((pts.shape[0], 3), dtype=LD)
    for a in range(3):
        e = np.zeros((1, 3), dtype=LD)
        e[0, a] = 1
        out[:, a] = (fun(pts + h * e) - fun(pts - h * e)) / (2 * h[:, 0])
    return out


# ------------------------------------------------------------------ backward
@pytest.mark.parametrize("normalize", [False, True])
def test_backward_equals_differences_of_contracted_values(normalize):
    """dL/dx for L = sum_k gY_k Y_k(x) (the chain rule the backward states)."""
    L = 6
    pts = _pts(10, 41).astype(LD)
    gY = standard_normal((pts.shape[0], (L + 1) ** 2), 42)
    _, dY = oracle.real_sph(pts, L, normalize)
    got = oracle.backward(dY, gY)

    def loss(p):
        Y, _ = oracle.definition_eval_ld(p, L, normalize)
        return (Y * gY.astype(LD)).sum(1)
    fd = _fd_x(loss, pts, "1e-6")
    _, g, _ = oracle.component_scales(np.asarray(pts, float), L, normalize)
    scale = (np.abs(gY) * g).sum(1)[:, None]
    err = np.abs(np.asarray(got - fd, float)) / scale
    assert err.max() < 1e-9, err.max()


def test_backward_is_linear_and_zero_for_zero_gradient():
    L = 4
    pts = _pts(6, 43)
    _, dY = oracle.real_sph(pts, L, True)
    a = standard_normal((6, 25), 44)
    b = standard_normal((6, 25), 45)
    lhs = oracle.backward(dY, 2 * a - 3 * b)
    rhs = 2 * oracle.backward(dY, a) - 3 * oracle.backward(dY, b)
    assert np.abs(np.asarray(lhs - rhs, float)).max() < 1e-16 * np.abs(np.asarray(lhs, float)).max()
    assert np.all(np.asarray(oracle.backward(dY, 0 * a), float) == 0)


# ----------------------------------------------------------- double backward
@pytest.mark.parametrize("normalize", [False, True])
def test_double_backward_grad_of_gY_is_exact_derivative(normalize):
    """ggY is d<v, backward(dY, gY)>/dgY; <v, backward> is linear in gY, so
    <ggY, d> = <v, backward(dY, d)> holds for every direction d."""
    L = 5
    K = (L + 1) ** 2
    pts = _pts(8, 46)
    gY = standard_normal((8, K), 47)
    v = standard_normal((8, 3), 48)
    ggY, _ = oracle.double_backward(pts, gY, v, L, normalize)
    _, dY = oracle.real_sph(pts, L, normalize)
    _, g, _ = oracle.component_scales(pts, L, normalize)
    for seed in (49, 50, 51):
        d = standard_normal((8, K), seed)
        lhs = (ggY * d.astype(LD)).sum(1)
        rhs = (oracle.backward(dY, d) * v.astype(LD)).sum(1)
        scale = (np.abs(d) * g).sum(1) * np.abs(v).sum(1)
        assert (np.abs(np.asarray(lhs - rhs, float)) / scale).max() < 1e-15
    # and column by column: the unit directions
    for k in (0, 3, K - 1):
        e = np.zeros((8, K))
        e[:, k] = 1
        rhs = (oracle.backward(dY, e) * v.astype(LD)).sum(1)
        assert np.abs(np.asarray(ggY[:, k] - rhs, float)).max() < 1e-14 * g[:, k].max() * np.abs(v).max()


@pytest.mark.parametrize("normalize", [False, True])
def test_double_backward_grad_of_x_equals_differences(normalize):
    """gxyz2 = d/dx <v, sum_k gY_k grad Y_k(x)>: central differences of the
    bulk tier's analytic first derivatives (no second derivative involved)."""
    L = 8
    K = (L + 1) ** 2
    pts = _pts(10, 52).astype(LD)
    gY = standard_normal((10, K), 53)
    v = standard_normal((10, 3), 54)
    _, g2 = oracle.double_backward(pts, gY, v, L, normalize)

    def inner(p):
        _, dY = oracle.real_sph(p, L, normalize)
        return (oracle.backward(dY, gY) * v.astype(LD)).sum(1)
    fd = _fd_x(inner, pts, "1e-6")
    _, _, h = oracle.component_scales(np.asarray(pts, float), L, normalize)
    scale = (np.abs(gY) * h).sum(1)[:, None] * np.abs(v).sum(1)[:, None]
    err = np.abs(np.asarray(g2 - fd, float)) / scale
    assert err.max() < 1e-9, err.max()


def test_hessian_contract_against_explicit_second_differences():
    """hessian_contract(H, gY, v) on the definition tier's H equals the second
    differences of sum_k gY_k Y_k along v and each axis."""
    L = 4
    K = (L + 1) ** 2
    pts = _pts(5, 55).astype(LD)
    gY = standard_normal((5, K), 56).astype(LD)
    v = standard_normal((5, 3), 57).astype(LD)
    _, _, H = oracle.definition_eval_ld(pts, L, False, hessian=True)
    got = oracle.hessian_contract(H, gY, v)
    h = LD("1e-4")

    def f(p):
        return (oracle.definition_eval_ld(p, L, False)[0] * gY).sum(1)
    ref = np.zeros((5, 3), dtype=LD)
    for b in range(3):
        e = np.zeros(3, dtype=LD)
        e[b] = h
        # d/dx_b d/dv f by a four-point central stencil (exact for cubics)
        vv = v * h
        ref[:, b] = (f(pts + e + vv) - f(pts + e - vv) - f(pts - e + vv) + f(pts - e - vv)) / (4 * h * h)
    _, _, hs = oracle.component_scales(np.asarray(pts, float), L, False)
    scale = (np.abs(np.asarray(gY, float)) * hs).sum(1)[:, None] * np.abs(np.asarray(v, float)).sum(1)[:, None]
    assert (np.abs(np.asarray(got - ref, float)) / scale).max() < 1e-7


# ---------------------------------------------------------- scales and errors
@pytest.mark.parametrize("normalize", [False, True])
def test_component_scales_are_the_addition_theorem_norms(normalize):
    """s_l = sqrt(sum_m Y_lm^2) and g_l = sqrt(sum_m |grad Y_lm|^2) at every
    point, from the oracle's own values (each pinned to closed forms,
    mpmath and orthonormality elsewhere)."""
    L = 12
    pts = _pts(40, 58)
    Y, G = oracle.real_sph(pts, L, normalize)
    s, g, h = oracle.component_scales(pts, L, normalize)
    for l in range(L + 1):
        sl = slice(l * l, (l + 1) ** 2)
        ns = np.sqrt(np.asarray((Y[:, sl] ** 2).sum(1), float))
        np.testing.assert_allclose(s[:, l * l], ns, rtol=1e-12)
        if l >= 1:
            ng = np.sqrt(np.asarray((G[:, :, sl] ** 2).sum((1, 2)), float))
            np.testing.assert_allclose(g[:, l * l], ng, rtol=1e-12)
        # every column of a degree carries that degree's scale
        assert np.all(s[:, sl] == s[:, l * l : l * l + 1])
        assert np.all(g[:, sl] == g[:, l * l : l * l + 1])


@pytest.mark.parametrize("normalize", [False, True])
def test_hessian_scale_bounds_the_hessian(normalize):
    """h is a chosen size for second derivatives, not an identity: the largest
    Hessian entry of each degree lies within [h/50, h]."""
    L = 8
    pts = _pts(30, 59)
    _, _, H = oracle.definition_eval_ld(pts, L, normalize, hessian=True)
    _, _, h = oracle.component_scales(pts, L, normalize)
    for l in range(1, L + 1):
        sl = slice(l * l, (l + 1) ** 2)
        mx = np.abs(np.asarray(H[..., sl], float)).max((1, 2, 3))
        ratio = mx / h[:, l * l]
        assert ratio.max() <= 1.0 and ratio.min() >= 1 / 50 or l == 1, (l, ratio.min(), ratio.max())


@pytest.mark.parametrize("normalize", [False, True])
@pytest.mark.parametrize("kind", ["Y", "dY"])
def test_per_l_errors_report_planted_errors(normalize, kind):
    L = 8
    N = 16
    pts = _pts(N, 60)
    Y, G = oracle.real_sph(pts, L, normalize)
    ref = Y if kind == "Y" else G
    # the expected scale of each degree from the addition theorem
    if kind == "Y":
        norm = np.sqrt(np.asarray([(Y[:, l * l:(l + 1) ** 2] ** 2).sum(1) for l in range(L + 1)], float)).T
    else:
        norm = np.sqrt(np.asarray([(G[:, :, l * l:(l + 1) ** 2] ** 2).sum((1, 2)) for l in range(L + 1)],
                                  float)).T
    plants = [(3, 5, 2, 0, 3e-5), (7, 2, -1, 2, 1e-7), (11, 8, 8, 1, 4e-3)]  # (point, l, m, axis, size)
    bad = np.array(ref, dtype=LD, copy=True)
    for i, l, m, a, size in plants:
        k = l * l + l + m
        delta = LD(size) * LD(norm[i, l])
        if kind == "Y":
            bad[i, k] += delta
        else:
            bad[i, a, k] -= delta
    mx, rms = oracle.per_l_errors(bad, ref, pts, L, normalize, kind)
    per_l = {l: size for _, l, _, _, size in plants}
    cols = {l: N * (2 * l + 1) * (1 if kind == "Y" else 3) for l in range(L + 1)}
    for l in range(L + 1):
        if l in per_l:
            assert mx[l] == pytest.approx(per_l[l], rel=1e-9)
            assert rms[l] == pytest.approx(per_l[l] / math.sqrt(cols[l]), rel=1e-9)
        else:
            assert mx[l] == 0 and rms[l] == 0
    # the mask drops the planted points
    keep = np.ones(N, bool)
    keep[[3, 7, 11]] = False
    mx2, _ = oracle.per_l_errors(bad, ref, pts, L, normalize, kind, mask=keep)
    assert np.all(mx2 == 0)


def test_per_l_errors_nan_is_infinite():
    L = 3
    pts = _pts(4, 61)
    Y, _ = oracle.real_sph(pts, L, True)
    bad = np.array(Y, dtype=LD, copy=True)
    bad[1, 5] = np.nan
    mx, rms = oracle.per_l_errors(bad, Y, pts, L, True, "Y")
    assert math.isinf(mx[2]) and math.isinf(rms[2])
    assert mx[0] == mx[1] == mx[3] == 0
    # NaN on both sides at the same place is agreement (e.g. a NaN input)
    ref = np.array(Y, dtype=LD, copy=True)
    ref[1, 5] = np.nan
    mx, _ = oracle.per_l_errors(bad, ref, pts, L, True, "Y")
    assert np.all(mx == 0)


# ------------------------------------------------------- mutations have teeth
def test_mutation_backward_wrong_axis_is_caught(monkeypatch):
    def bad(dY, gY):
        dY = np.asarray(dY).astype(LD)
        gY = np.asarray(gY).astype(LD)
        # contracts the axes of a transposed [N,K,3] reading of dY
        return np.einsum("nka,nk->na", dY.reshape(dY.shape[0], -1, 3), gY)
    monkeypatch.setattr(oracle, "backward", bad)
    with pytest.raises(AssertionError):
        test_backward_equals_differences_of_contracted_values(True)


def test_mutation_double_backward_dropped_term_is_caught(monkeypatch):
    """gxyz2 from the Hessian of the solid harmonics even when the normalised
    ones were asked for (the chain-rule terms dropped)."""
    src = derived.definition_eval_ld

    def bad(xyz, l_max, normalize, hessian=False):
        return src(xyz, l_max, False, hessian=hessian) if hessian else src(xyz, l_max, normalize)
    monkeypatch.setattr(derived, "definition_eval_ld", bad)
    with pytest.raises(AssertionError):
        test_double_backward_grad_of_x_equals_differences(True)


def test_mutation_double_backward_wrong_contraction_is_caught(monkeypatch):
    """The components of gxyz2 rotated (a contraction over the wrong axis)."""
    orig = oracle.double_backward

    def bad(xyz, gY, v, l_max, normalize):
        ggY, g2 = orig(xyz, gY, v, l_max, normalize)
        return ggY, g2[:, [1, 2, 0]]
    monkeypatch.setattr(oracle, "double_backward", bad)
    with pytest.raises(AssertionError):
        test_double_backward_grad_of_x_equals_differences(False)


def test_mutation_swapped_scale_is_caught(monkeypatch):
    """The normalised scales used for the solid harmonics."""
    src = derived.component_scales

    def bad(xyz, l_max, normalize):
        return src(xyz, l_max, True)
    monkeypatch.setattr(oracle, "component_scales", bad)
    with pytest.raises(AssertionError):
        test_component_scales_are_the_addition_theorem_norms(False)


def test_mutation_error_metric_wrong_degree_is_caught(monkeypatch):
    """An error reported one degree off (slices shifted by one column)."""
    src = derived.per_l_errors

    def bad(Y, Yref, xyz, l_max, normalize, kind="Y", mask=None):
        A = np.roll(np.asarray(Y, dtype=LD), 1, axis=-1)
        B = np.roll(np.asarray(Yref, dtype=LD), 1, axis=-1)
        return src(A, B, xyz, l_max, normalize, kind, mask)
    monkeypatch.setattr(oracle, "per_l_errors", bad)
    with pytest.raises(AssertionError):
        test_per_l_errors_report_planted_errors(True, "Y")
