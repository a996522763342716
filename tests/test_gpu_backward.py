"""Backward (sph_backward), double backward (sph_double_backward) and the
autograd wrapper against the oracle and against finite differences."""
import numpy as np
import pytest
import torch

import oracle
from workloads import SEEDS, shell_points, standard_normal, standard_normal_points

from _gpu_common import TOL, host_points, to_dev

pytestmark = pytest.mark.gpu


def _rel_err_vec(a, ref, scale):
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return np.abs(a - ref) / scale


def _contraction_scale(gY, pts, l_max, normalize):
    """Size of sum_k gY_k dY_k: sum_k |gY_k| g_l(k) (column scales)."""
    _, g, _ = oracle.component_scales(pts, l_max, normalize)
    return (np.abs(gY) * g).sum(1)[:, None]


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("l_max", [0, 1, 3, 6, 8, 12, 20, 32])
def test_backward_matches_oracle(l_max, dtype):
    import paper_2302_08381_amd as sph
    n = 150
    pts = standard_normal_points(n, 200 + l_max)
    xyz = to_dev(pts, dtype)
    K = (l_max + 1) ** 2
    gY = to_dev(standard_normal((n, K), 300 + l_max), dtype)
    _, dY = sph.sph_compute_with_gradients(xyz, l_max, True)
    gx = sph.sph_backward(dY, gY, l_max)
    hp = host_points(xyz)
    _, Gr = oracle.real_sph(hp, l_max, True)
    gYh = gY.cpu().double().numpy()
    ref = oracle.backward(Gr, gYh)
    err = _rel_err_vec(gx.cpu().numpy(), ref, _contraction_scale(gYh, hp, l_max, True))
    assert err.max() <= TOL[dtype], err.max()


@pytest.mark.parametrize("dtype,l_max", [(torch.float64, 8), (torch.float32, 4), (torch.float32, 6)])
def test_backward_resident_grid_full_size(dtype, l_max):
    """N = 1e6 (the plain GPU-sized workload's points): far more tiles than
    the resident grid holds, so every block runs the loop that loads tile
    t + G while it reduces tile t.  Compared with the oracle on 2048 rows
    that include each of the last tiles of the run, where the loop ends."""
    import paper_2302_08381_amd as sph
    n = 1_000_000
    print(f"backward resident grid {dtype} l_max={l_max} n={n}", flush=True)
    pts = standard_normal_points(n, SEEDS["plain_gpu"])
    K = (l_max + 1) ** 2
    xyz = to_dev(pts, dtype)
    gY = to_dev(standard_normal((n, K), SEEDS["plain_gpu_grad"]), dtype)
    _, dY = sph.sph_compute_with_gradients(xyz, l_max, True)
    gx = sph.sph_backward(dY, gY, l_max)
    torch.cuda.synchronize()
    rng = np.random.default_rng(17)
    # 1536 random rows plus the last 512 rows (the final tiles and the
    # ragged end of every block's walk)
    idx = np.unique(np.concatenate([rng.choice(n - 512, 1536, replace=False), np.arange(n - 512, n)]))
    ii = torch.as_tensor(idx, device="cuda")
    hp = host_points(xyz[ii])
    _, Gr = oracle.real_sph(hp, l_max, True)
    gYh = gY[ii].cpu().double().numpy()
    err = _rel_err_vec(gx[ii].cpu().numpy(), oracle.backward(Gr, gYh), _contraction_scale(gYh, hp, l_max, True))
    assert err.max() <= TOL[dtype], err.max()
    # every row written and finite
    assert np.isfinite(gx.cpu().numpy()).all()


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("normalize", [False, True])
@pytest.mark.parametrize("l_max", [0, 1, 2, 3, 4, 6, 8, 9])
def test_double_backward_matches_oracle(l_max, normalize, dtype):
    import paper_2302_08381_amd as sph
    n = 130
    pts = shell_points(n, 0.5, 5.0 if normalize else 1.6, 400 + l_max)
    xyz = to_dev(pts, dtype)
    K = (l_max + 1) ** 2
    gY = to_dev(standard_normal((n, K), 500 + l_max), dtype)
    v = to_dev(standard_normal((n, 3), 600 + l_max), dtype)
    ggY, g2 = sph.sph_double_backward(xyz, gY, v, l_max, normalize)
    hp = host_points(xyz)
    gYh = gY.cpu().double().numpy()
    vh = v.cpu().double().numpy()
    ggr, g2r = oracle.double_backward(hp, gYh, vh, l_max, normalize)
    _, g, h = oracle.component_scales(hp, l_max, normalize)
    vn = np.sqrt((vh ** 2).sum(1))[:, None]
    e1 = _rel_err_vec(ggY.cpu().numpy(), ggr, g * vn)
    assert e1.max() <= TOL[dtype], e1.max()
    s2 = (np.abs(gYh) * h).sum(1)[:, None] * vn
    e2 = _rel_err_vec(g2.cpu().numpy(), g2r, s2)
    assert e2.max() <= TOL[dtype], e2.max()
    # each output alone
    a, b = sph.sph_double_backward(xyz, gY, v, l_max, normalize, want_grad_xyz=False)
    assert b is None and torch.equal(a, ggY)
    a, b = sph.sph_double_backward(xyz, gY, v, l_max, normalize, want_grad_grad_Y=False)
    assert a is None and torch.equal(b, g2)


@pytest.mark.parametrize("normalize", [False, True])
def test_double_backward_high_l_runtime_kernel(normalize):
    """l_max = 20 and 32 go through the widest kernels; checked against the
    oracle's exact Hessians for a few points."""
    import paper_2302_08381_amd as sph
    for l_max in (20, 32):
        n = 3
        pts = shell_points(n, 0.8, 1.2, 700 + l_max)
        xyz = to_dev(pts, torch.float64)
        K = (l_max + 1) ** 2
        gY = to_dev(standard_normal((n, K), 800 + l_max), torch.float64)
        v = to_dev(standard_normal((n, 3), 900 + l_max), torch.float64)
        ggY, g2 = sph.sph_double_backward(xyz, gY, v, l_max, normalize)
        gYh, vh = gY.cpu().numpy(), v.cpu().numpy()
        _, Gr = oracle.real_sph(pts, l_max, normalize)
        ggr = np.einsum("nak,na->nk", Gr, vh.astype(np.longdouble))
        _, g, h = oracle.component_scales(pts, l_max, normalize)
        assert (_rel_err_vec(ggY.cpu().numpy(), ggr, g * np.abs(vh).sum(1)[:, None])).max() < 1e-12
        # Hessian-vector products from the exact polynomials at 60 digits
        for i in range(n):
            _, _, H = oracle.definition_eval_mp(pts[i], l_max, normalize, dps=60, hessian=True)
            Hn = np.array([[[float(x) for x in row] for row in blk] for blk in H])
            ref = np.einsum("abk,k,a->b", Hn, gYh[i], vh[i])
            scale = (np.abs(gYh[i]) * h[i]).sum() * np.abs(vh[i]).sum()
            assert np.abs(g2[i].cpu().numpy() - ref).max() / scale < 1e-12


def test_autograd_gradcheck_and_gradgradcheck():
    from paper_2302_08381_amd import spherical_harmonics
    for normalize in (False, True):
        for l_max in (0, 2, 5):
            xyz = to_dev(standard_normal_points(7, 40 + l_max), torch.float64).requires_grad_(True)
            f = lambda x: spherical_harmonics(x, l_max, normalize)  # noqa: E731
            assert torch.autograd.gradcheck(f, (xyz,), eps=1e-6, atol=1e-7, rtol=1e-6)
            assert torch.autograd.gradgradcheck(f, (xyz,), eps=1e-6, atol=1e-6, rtol=1e-5)


def test_differentiation_workload_finite_differences():
    """Ball radius 0.5..5, l_max = 6, normalised: backward and double backward
    against central differences (h = 1e-3, float64) on 1000 sampled points of
    a 4e6-point float32 run, and against the oracle."""
    import paper_2302_08381_amd as sph
    n = 4_000_000
    L = 6
    K = 49
    pts = shell_points(n, 0.5, 5.0, SEEDS["diff"])
    rng = np.random.default_rng(SEEDS["diff"])
    idx = np.sort(rng.choice(n, 1000, replace=False))
    xyz = to_dev(pts, torch.float32)
    gY = to_dev(standard_normal((n, K), 31), torch.float32)
    v = to_dev(standard_normal((n, 3), 32), torch.float32)
    _, dY = sph.sph_compute_with_gradients(xyz, L, True)
    gx = sph.sph_backward(dY, gY, L)
    ggY, g2 = sph.sph_double_backward(xyz, gY, v, L, True)
    ii = torch.as_tensor(idx, device="cuda")
    # float64 reference runs of the same kernels on the sampled (rounded) points
    x64 = xyz[ii].double()
    gY64 = gY[ii].double()
    v64 = v[ii].double()
    h = 1e-3
    fd_b = torch.zeros_like(x64)
    fd_db = torch.zeros_like(x64)
    for a in range(3):
        e = torch.zeros_like(x64)
        e[:, a] = h
        Yp = sph.sph_compute(x64 + e, L, True)
        Ym = sph.sph_compute(x64 - e, L, True)
        fd_b[:, a] = ((Yp - Ym) * gY64).sum(1) / (2 * h)
        _, dYp = sph.sph_compute_with_gradients(x64 + e, L, True)
        _, dYm = sph.sph_compute_with_gradients(x64 - e, L, True)
        gp = sph.sph_backward(dYp, gY64, L)
        gm = sph.sph_backward(dYm, gY64, L)
        fd_db[:, a] = ((gp - gm) * v64).sum(1) / (2 * h)
    hp = x64.cpu().numpy()
    _, g, hs = oracle.component_scales(hp, L, True)
    gYh = gY64.cpu().numpy()
    sb = (np.abs(gYh) * g).sum(1)[:, None]
    # FD truncation ~ h^2 |d3| / 6: on this sample (r >= 0.64) it is 4.2e-7 of
    # the scale for the backward and 3.9e-7 for the double backward (the
    # oracle's own central differences), and the float32 kernels add < 1e-6,
    # so 1e-5 of the scale is the bound.
    assert (_rel_err_vec(gx[ii].double().cpu().numpy(), fd_b.cpu().numpy(), sb)).max() < 1e-5
    vn = np.sqrt((v64.cpu().numpy() ** 2).sum(1))[:, None]
    sdb = (np.abs(gYh) * hs).sum(1)[:, None] * vn
    assert (_rel_err_vec(g2[ii].double().cpu().numpy(), fd_db.cpu().numpy(), sdb)).max() < 1e-5
    # against the oracle (float32 tolerance)
    _, Gr = oracle.real_sph(hp, L, True)
    assert (_rel_err_vec(gx[ii].cpu().numpy(), oracle.backward(Gr, gYh), sb)).max() <= TOL[torch.float32]
    ggr, g2r = oracle.double_backward(hp, gYh, v64.cpu().numpy(), L, True)
    assert (_rel_err_vec(ggY[ii].cpu().numpy(), ggr, g * vn)).max() <= TOL[torch.float32]
    assert (_rel_err_vec(g2[ii].cpu().numpy(), g2r, sdb)).max() <= TOL[torch.float32]


def test_module_forces_training_step():
    """Energy = sum(w * Y); forces by autograd with create_graph, then a loss
    on the forces is differentiated again (double backward)."""
    from paper_2302_08381_amd import SphericalHarmonics
    m = SphericalHarmonics(4, normalize=True)
    xyz = to_dev(standard_normal_points(300, 51), torch.float64).requires_grad_(True)
    w = to_dev(standard_normal((25,), 52), torch.float64)
    E = (m(xyz) * w).sum()
    (F,) = torch.autograd.grad(E, xyz, create_graph=True)
    loss = (F ** 2).sum()
    (g,) = torch.autograd.grad(loss, xyz)
    assert torch.isfinite(g).all()
    # same through the oracle: d/dx sum F^2 = 2 H F where H = sum_k w_k Hess(Y_k)
    hp = xyz.detach().cpu().numpy()
    Fh = F.detach().cpu().numpy()
    _, _, H = oracle.definition_eval_ld(hp, 4, True, hessian=True)
    ref = 2 * np.einsum("nabk,k,na->nb", H, w.cpu().numpy().astype(np.longdouble), Fh)
    err = np.abs(g.cpu().numpy() - np.asarray(ref, float)).max() / (np.abs(np.asarray(ref, float)).max() + 1e-30)
    assert err < 1e-11
