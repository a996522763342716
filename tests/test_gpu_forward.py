"""Forward kernels (sph_compute, sph_compute_with_gradients) against the
oracle, element by element, on seeded inputs that span several 64-point
tiles and a ragged tail."""
import numpy as np
import pytest
import torch

import oracle
from workloads import SEEDS, precision_stress_points, standard_normal_points

from _gpu_common import TOL, assert_bitwise_equal, assert_close_per_l, host_points, to_dev

pytestmark = pytest.mark.gpu

LMAXES = [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 16, 17, 20, 24, 25, 32]


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("normalize", [False, True])
@pytest.mark.parametrize("l_max", LMAXES)
def test_forward_matches_oracle(l_max, normalize, dtype):
    import paper_2302_08381_amd as sph
    print(f"forward l_max={l_max} normalize={normalize} dtype={dtype}", flush=True)
    n = 200  # 3 full tiles + a ragged tail of 8
    pts = standard_normal_points(n, 100 + l_max)
    xyz = to_dev(pts, dtype)
    Y, dY = sph.sph_compute_with_gradients(xyz, l_max, normalize)
    Yo = sph.sph_compute(xyz, l_max, normalize)
    torch.cuda.synchronize()
    hp = host_points(xyz)
    Yr, Gr = oracle.real_sph(hp, l_max, normalize)
    tol = TOL[dtype]
    # the values-only kernel (one lane per point) and the derivative kernel
    # (four lanes per point) both against the oracle
    assert_close_per_l(Yo.cpu().numpy(), Yr, hp, l_max, normalize, "Y", tol)
    assert_close_per_l(Y.cpu().numpy(), Yr, hp, l_max, normalize, "Y", tol)
    assert_close_per_l(dY.cpu().numpy(), Gr, hp, l_max, normalize, "dY", tol)


@pytest.mark.parametrize("normalize", [False, True])
def test_plain_cpu_workload_float64(normalize):
    """N = 1000 standard-normal points, float64, l_max = 4 (both kinds)."""
    import paper_2302_08381_amd as sph
    pts = standard_normal_points(1000, SEEDS["plain_cpu"])
    xyz = to_dev(pts, torch.float64)
    Y, dY = sph.sph_compute_with_gradients(xyz, 4, normalize)
    Yr, Gr = oracle.real_sph(pts, 4, normalize)
    assert_close_per_l(Y.cpu().numpy(), Yr, pts, 4, normalize, "Y", 1e-12)
    assert_close_per_l(dY.cpu().numpy(), Gr, pts, 4, normalize, "dY", 1e-12)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_full_size_l8_sampled(dtype):
    """N = 1e6 standard-normal points, l_max = 8, normalised: the benchmark's
    launch; 4096 sampled rows against the oracle, plus the addition theorem
    on every row."""
    import paper_2302_08381_amd as sph
    n = 1_000_000
    pts = standard_normal_points(n, SEEDS["plain_gpu"])
    xyz = to_dev(pts, dtype)
    Y, dY = sph.sph_compute_with_gradients(xyz, 8, True)
    torch.cuda.synchronize()
    rng = np.random.default_rng(7)
    idx = np.sort(rng.choice(n, 4096, replace=False))
    idx = np.concatenate([idx, [0, 63, 64, n - 1]])
    hp = host_points(xyz[torch.as_tensor(idx, device=xyz.device)])
    Yr, Gr = oracle.real_sph(hp, 8, True)
    ii = torch.as_tensor(idx, device=xyz.device)
    assert_close_per_l(Y[ii].cpu().numpy(), Yr, hp, 8, True, "Y", TOL[dtype])
    assert_close_per_l(dY[ii].cpu().numpy(), Gr, hp, 8, True, "dY", TOL[dtype])
    # sum_m Y_lm^2 = (2l+1)/(4 pi) for every point
    Yd = Y.double()
    for l in range(9):
        s = (Yd[:, l * l:(l + 1) ** 2] ** 2).sum(1)
        ref = (2 * l + 1) / (4 * np.pi)
        assert float((s / ref - 1).abs().max()) < (1e-5 if dtype == torch.float32 else 1e-12)


def test_edge_cases():
    import paper_2302_08381_amd as sph
    for dtype in (torch.float32, torch.float64):
        # n = 0
        e = torch.empty((0, 3), dtype=dtype, device="cuda")
        assert sph.sph_compute(e, 5, True).shape == (0, 36)
        # n = 1, origin, exact poles, a point on each axis
        pts = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 1.5], [0.0, 0.0, -0.25], [2.0, 0.0, 0.0],
                        [0.0, -3.0, 0.0], [1e-30, 0.0, 1.0]])
        for normalize in (False, True):
            for L in (0, 1, 5, 8, 20):
                for n in (1, len(pts)):
                    xyz = to_dev(pts[:n], dtype)
                    Y, dY = sph.sph_compute_with_gradients(xyz, L, normalize)
                    hp = host_points(xyz)
                    Yr, Gr = oracle.real_sph(hp, L, normalize)
                    assert torch.isfinite(Y).all() and torch.isfinite(dY).all()
                    assert_close_per_l(Y.cpu().numpy(), Yr, hp, L, normalize, "Y", TOL[dtype])
                    assert_close_per_l(dY.cpu().numpy(), Gr, hp, L, normalize, "dY", TOL[dtype])


def test_nan_propagates_and_neighbours_unaffected():
    import paper_2302_08381_amd as sph
    pts = standard_normal_points(70, 9)
    pts[5] = [np.nan, 0.2, 0.3]
    xyz = to_dev(pts, torch.float32)
    Y, dY = sph.sph_compute_with_gradients(xyz, 6, True)
    assert torch.isnan(Y[5, 1:]).all()
    ok = torch.ones(70, dtype=torch.bool)
    ok[5] = False
    assert torch.isfinite(Y[ok.cuda()]).all() and torch.isfinite(dY[ok.cuda()]).all()


def test_unaligned_buffers_take_the_scalar_path():
    """Outputs that start 4 bytes past a 16-byte boundary."""
    import paper_2302_08381_amd as sph
    n, L = 150, 8
    K = (L + 1) ** 2
    pts = standard_normal_points(n, 11)
    xyz = to_dev(pts, torch.float32)
    bigY = torch.zeros(n * K + 1, dtype=torch.float32, device="cuda")
    Y = bigY[1:].view(n, K)
    sph.sph_compute(xyz, L, True, Y=Y)
    Yref = sph.sph_compute(xyz, L, True)
    assert torch.equal(Y, Yref)


def test_deterministic():
    import paper_2302_08381_amd as sph
    xyz = to_dev(standard_normal_points(5000, 12), torch.float32)
    a = sph.sph_compute_with_gradients(xyz, 12, False)
    b = sph.sph_compute_with_gradients(xyz, 12, False)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_precision_stress_l32(dtype):
    """l_max = 32, normalised: unit sphere, points within 1e-12..1e-3 of the
    z axis, and radii 1e-6..1e3; per-l error per sub-population."""
    import paper_2302_08381_amd as sph
    pts, cls = precision_stress_points(4000, SEEDS["precision"])
    xyz = to_dev(pts, dtype)
    Y, dY = sph.sph_compute_with_gradients(xyz, 32, True)
    hp = host_points(xyz)
    Yr, Gr = oracle.real_sph(hp, 32, True)
    Yc, dYc = Y.cpu().numpy(), dY.cpu().numpy()
    for c in range(3):
        m = cls == c
        mx, _ = oracle.per_l_errors(Yc[m], Yr[m], hp[m], 32, True, "Y")
        assert mx.max() <= TOL[dtype], (c, mx)
        mx, _ = oracle.per_l_errors(dYc[m], Gr[m], hp[m], 32, True, "dY")
        assert mx.max() <= TOL[dtype], (c, mx)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_every_tile_written_for_grids_of_any_size(dtype):
    """Blocks take tiles in an XCD-contiguous order (a permutation of the
    grid): grids of 9..41 tiles with every remainder mod 8, full and ragged,
    must still write every row."""
    import paper_2302_08381_amd as sph
    tile = 32 if dtype == torch.float32 else 16
    for tiles, tail in ((9, 0), (10, 5), (13, 0), (19, 7), (24, 0), (31, 1), (41, 11)):
        n = tiles * tile + tail
        print(f"grid tiles={tiles} tail={tail} n={n} dtype={dtype}", flush=True)
        pts = standard_normal_points(n, 500 + n)
        xyz = to_dev(pts, dtype)
        Y = torch.full((n, 81), float("nan"), dtype=dtype, device="cuda")
        dY = torch.full((n, 3, 81), float("nan"), dtype=dtype, device="cuda")
        sph.sph_compute_with_gradients(xyz, 8, True, Y=Y, dY=dY)
        Yv = torch.full((n, 81), float("nan"), dtype=dtype, device="cuda")
        sph.sph_compute(xyz, 8, True, Y=Yv)
        torch.cuda.synchronize()
        hp = host_points(xyz)
        Yr, Gr = oracle.real_sph(hp, 8, True)
        assert_close_per_l(Y.cpu().numpy(), Yr, hp, 8, True, "Y", TOL[dtype])
        assert_close_per_l(dY.cpu().numpy(), Gr, hp, 8, True, "dY", TOL[dtype])
        assert_close_per_l(Yv.cpu().numpy(), Yr, hp, 8, True, "Y", TOL[dtype])


@pytest.mark.parametrize("dtype,l_max", [(torch.float32, 16), (torch.float32, 32), (torch.float64, 12)])
def test_groups_of_degrees_with_misaligned_outputs(dtype, l_max):
    """l_max past one group of degrees: partial rows leave with 16-byte stores
    of their aligned middles.  Outputs 1..3 elements past a 16-byte boundary
    (every head length) must equal the aligned outputs bitwise."""
    import paper_2302_08381_amd as sph
    n = 150  # several tiles and a ragged tail
    K = (l_max + 1) ** 2
    xyz = to_dev(standard_normal_points(n, 900 + l_max), dtype)
    Y0, dY0 = sph.sph_compute_with_gradients(xyz, l_max, True)
    Yv0 = sph.sph_compute(xyz, l_max, True)
    for shift in (1, 2, 3):
        print(f"misaligned outputs l_max={l_max} dtype={dtype} shift={shift}", flush=True)
        bY = torch.full((n * K + shift,), float("nan"), dtype=dtype, device="cuda")
        bdY = torch.full((n * 3 * K + shift,), float("nan"), dtype=dtype, device="cuda")
        Y = bY[shift:].view(n, K)
        dY = bdY[shift:].view(n, 3, K)
        sph.sph_compute_with_gradients(xyz, l_max, True, Y=Y, dY=dY)
        bv = torch.full((n * K + shift,), float("nan"), dtype=dtype, device="cuda")
        Yv = bv[shift:].view(n, K)
        sph.sph_compute(xyz, l_max, True, Y=Yv)
        torch.cuda.synchronize()
        assert_bitwise_equal(Y, Y0, "Y")
        assert_bitwise_equal(dY, dY0, "dY")
        assert_bitwise_equal(Yv, Yv0, "values-only Y")
        assert torch.isnan(bY[:shift]).all() and torch.isnan(bdY[:shift]).all()  # nothing written before
    hp = host_points(xyz)
    Yr, Gr = oracle.real_sph(hp, l_max, True)
    assert_close_per_l(Y0.cpu().numpy(), Yr, hp, l_max, True, "Y", TOL[dtype])
    assert_close_per_l(dY0.cpu().numpy(), Gr, hp, l_max, True, "dY", TOL[dtype])
