"""The one-lane forward for l_max <= 3 (kernel variant "one_lane"): each lane
forms the values and the three derivative rows of its own point, and a
64-point tile leaves through LDS as 16-byte stores.  Parity with the oracle
for every l_max it serves, both kinds and both element types, every output
combination of the batched entry (Y and dY; Y, dY and the fused backward;
Y and the fused backward), on one tile per block and on a looping grid,
plus the general path (ragged tiles, unaligned outputs)."""
import numpy as np
import pytest
import torch

import oracle
from workloads import csr_environments, standard_normal

from _gpu_common import TOL, assert_bitwise_equal, assert_close_per_l, host_points, to_dev

pytestmark = pytest.mark.gpu

MODES = ((True, False), (True, True), (False, True))  # (store_dY, with_backward)


def _points(seed):
    pts, offs = csr_environments(50, 8, 128, 0.5, 5.0, seed)
    # the degenerate points first: origin, poles, axes, a short vector (r^3
    # stays a normal float32 number)
    pts, offs = pts.copy(), offs.copy()
    pts[:7] = [[0, 0, 0], [0, 0, 1], [0, 0, -2], [3, 0, 0], [0, -1, 0], [1e-6, 0, 1e-6], [1, 1, 1]]
    if offs[-1] % 64 == 0:  # keep a ragged last tile
        offs[-1] -= 1
        pts = pts[:-1]
    return pts, offs


def _check_grad(gx, Gr, gYh, hp, l_max, normalize, tol, label):
    ref = np.asarray(oracle.backward(Gr, gYh), float)
    _, g, _ = oracle.component_scales(hp, l_max, normalize)
    s = (np.abs(gYh) * g).sum(1)[:, None] + 1e-300
    err = np.abs(gx.cpu().double().numpy() - ref) / s
    assert np.isfinite(err).all() and err.max() <= tol, (label, err.max())


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("normalize", [True, False])
def test_one_lane_matches_oracle(dtype, normalize):
    import paper_2302_08381_amd as sph
    pts, offs = _points(4100 + int(normalize))
    n = int(offs[-1])
    xyz = to_dev(pts, dtype)
    o = torch.as_tensor(offs, dtype=torch.int64, device="cuda")
    hp = host_points(xyz)
    for l_max in range(4):
        K = (l_max + 1) ** 2
        Yr, Gr = oracle.real_sph(hp, l_max, normalize)
        gY = to_dev(standard_normal((n, K), 4200 + l_max), dtype)
        gYh = gY.cpu().double().numpy()
        for store, bwd in MODES:
            for bpc in (0, 4):
                label = f"one_lane l_max={l_max} {dtype} normalize={normalize} dY={store} bwd={bwd} bpc={bpc}"
                print(label, flush=True)
                sph.sph_batched_set_config(l_max, normalize, dtype, store, bwd, "one_lane", bpc)
                assert "kernel=one_lane" in sph.sph_batched_get_config(l_max, normalize, dtype, store, bwd)
                out = sph.sph_batched_compute(xyz, o, l_max, normalize, store_dY=store,
                                              grad_Y=gY if bwd else None)
                torch.cuda.synchronize()
                assert_close_per_l(out["Y"].cpu().numpy(), Yr, hp, l_max, normalize, "Y", TOL[dtype], label)
                if store:
                    assert_close_per_l(out["dY"].cpu().numpy(), Gr, hp, l_max, normalize, "dY", TOL[dtype], label)
                if bwd:
                    _check_grad(out["grad_xyz"], Gr, gYh, hp, l_max, normalize, TOL[dtype], label)
                sph.sph_batched_set_config(l_max, normalize, dtype, store, bwd, "default", 0)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_one_lane_misaligned_and_small(dtype):
    """Outputs 1..3 elements past a 16-byte boundary take the general path
    and must equal the aligned outputs bitwise; inputs of 1, 63, 64 and 65
    points cover a lone ragged tile and the first full one."""
    import paper_2302_08381_amd as sph
    for l_max in range(4):
        K = (l_max + 1) ** 2
        for n in (1, 63, 64, 65, 300):
            pts = np.asarray(standard_normal((n, 3), 4300 + n), float)
            xyz = to_dev(pts, dtype)
            o = torch.tensor([0, n], dtype=torch.int64, device="cuda")
            gY = to_dev(standard_normal((n, K), 4400 + n), dtype)
            sph.sph_batched_set_config(l_max, True, dtype, True, True, "one_lane", 0)
            ref = sph.sph_batched_compute(xyz, o, l_max, True, store_dY=True, grad_Y=gY)
            for shift in (1, 2, 3):
                print(f"one_lane misaligned l_max={l_max} n={n} {dtype} shift={shift}", flush=True)
                bY = torch.full((n * K + shift,), float("nan"), dtype=dtype, device="cuda")
                bdY = torch.full((n * 3 * K + shift,), float("nan"), dtype=dtype, device="cuda")
                bgY = torch.empty((n * K + shift,), dtype=dtype, device="cuda")
                gYm = bgY[shift:].view(n, K)
                gYm.copy_(gY)
                out = sph.sph_batched_compute(xyz, o, l_max, True, store_dY=True, grad_Y=gYm,
                                              out={"Y": bY[shift:].view(n, K), "dY": bdY[shift:].view(n, 3, K)})
                torch.cuda.synchronize()
                assert_bitwise_equal(out["Y"], ref["Y"], "Y")
                assert_bitwise_equal(out["dY"], ref["dY"], "dY")
                assert_bitwise_equal(out["grad_xyz"], ref["grad_xyz"], "grad_xyz")
                assert torch.isnan(bY[:shift]).all() and torch.isnan(bdY[:shift]).all()
            hp = host_points(xyz)
            Yr, Gr = oracle.real_sph(hp, l_max, True)
            assert_close_per_l(ref["Y"].cpu().numpy(), Yr, hp, l_max, True, "Y", TOL[dtype])
            assert_close_per_l(ref["dY"].cpu().numpy(), Gr, hp, l_max, True, "dY", TOL[dtype])
            _check_grad(ref["grad_xyz"], Gr, gY.cpu().double().numpy(), hp, l_max, True, TOL[dtype], "small")
            sph.sph_batched_set_config(l_max, True, dtype, True, True, "default", 0)


def test_one_lane_only_for_small_lmax():
    import paper_2302_08381_amd as sph
    for l_max in (4, 8):
        with pytest.raises(sph.SphError):
            sph.sph_batched_set_config(l_max, True, torch.float32, True, False, "one_lane", 0)
    with pytest.raises(sph.SphError):  # the values-only kernel is one lane per point already
        sph.sph_batched_set_config(2, True, torch.float32, False, False, "one_lane", 0)
