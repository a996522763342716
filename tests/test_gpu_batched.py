"""Batched CSR entry point (sph_batched_compute): one persistent launch over
many neighbour lists, replayed from cached hipGraphs, with the backward
fused in."""
import numpy as np
import pytest
import torch

import oracle
from workloads import SEEDS, csr_environments, standard_normal

from _gpu_common import TOL, assert_bitwise_equal, assert_close_per_l, host_points, to_dev

pytestmark = pytest.mark.gpu


def _offsets(o):
    return torch.as_tensor(o, dtype=torch.int64, device="cuda")


@pytest.mark.parametrize("l_max", [3, 6, 8, 12, 20])
def test_batched_equals_plain_and_oracle(l_max):
    import paper_2302_08381_amd as sph
    pts, offs = csr_environments(400, 8, 128, 0.5, 5.0, 60 + l_max)
    n = int(offs[-1])
    K = (l_max + 1) ** 2
    xyz = to_dev(pts, torch.float32)
    gY = to_dev(standard_normal((n, K), 70 + l_max), torch.float32)
    status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    # the plain call's kernel (the run-time-degree variant rounds differently)
    sph.sph_batched_set_config(l_max, True, torch.float32, True, True, "default", 0)
    out = sph.sph_batched_compute(xyz, _offsets(offs), l_max, True, store_dY=True, grad_Y=gY, status=status)
    Y, dY = sph.sph_compute_with_gradients(xyz, l_max, True)
    gx = sph.sph_backward(dY, gY, l_max)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    # same device function on the same point: bitwise equal values
    assert_bitwise_equal(out["Y"], Y, "batched Y")
    assert_bitwise_equal(out["dY"], dY, "batched dY")
    # fused backward sums in another order
    scale = (gY.abs().double()[:, None, :] * dY.abs().double()).sum(2) + 1e-30
    rel = ((out["grad_xyz"].double() - gx.double()).abs() / scale).max()
    assert float(rel) < 1e-5
    # and against the oracle on a sample
    idx = torch.arange(0, n, 37, device="cuda")
    hp = host_points(xyz[idx])
    Yr, Gr = oracle.real_sph(hp, l_max, True)
    gYh = gY[idx].double().cpu().numpy()
    ref = oracle.backward(Gr, gYh)
    _, g, _ = oracle.component_scales(hp, l_max, True)
    s = (np.abs(gYh) * g).sum(1)[:, None]
    err = np.abs(out["grad_xyz"][idx].cpu().numpy() - np.asarray(ref, float)) / s
    assert err.max() <= TOL[torch.float32]


def test_batched_output_variants_and_graph_replay():
    import paper_2302_08381_amd as sph
    L = 6
    K = 49
    for rep in range(4):
        pts, offs = csr_environments(100 + 7 * rep, 8, 128, 0.5, 5.0, 80 + rep)
        n = int(offs[-1])
        xyz = to_dev(pts, torch.float64)
        gY = to_dev(standard_normal((n, K), 90 + rep), torch.float64)
        Y, dY = sph.sph_compute_with_gradients(xyz, L, True)
        Yv = sph.sph_compute(xyz, L, True)
        gx = sph.sph_backward(dY, gY, L)
        a = sph.sph_batched_compute(xyz, _offsets(offs), L, True, store_dY=False)
        b = sph.sph_batched_compute(xyz, _offsets(offs), L, True, store_dY=False, grad_Y=gY)
        c = sph.sph_batched_compute(xyz, _offsets(offs), L, True, store_dY=True)
        torch.cuda.synchronize()
        # values only: the same kernel as sph_compute, bitwise
        assert a["dY"] is None and a["grad_xyz"] is None
        assert_bitwise_equal(a["Y"], Yv, "batched values")
        # the values-only and the derivative kernels agree to rounding
        assert float((Yv - Y).abs().max()) < 1e-14
        assert b["dY"] is None
        assert_bitwise_equal(b["Y"], Y, "batched+bwd Y")
        assert float(((b["grad_xyz"] - gx).abs()).max()) < 1e-12 * float(gx.abs().max() + 1)
        assert_bitwise_equal(c["Y"], Y, "batched Y (dY stored)")
        assert_bitwise_equal(c["dY"], dY, "batched dY")


def test_batched_without_graph_matches():
    import paper_2302_08381_amd as sph
    pts, offs = csr_environments(200, 8, 128, 0.5, 5.0, 99)
    xyz = to_dev(pts, torch.float32)
    a = sph.sph_batched_compute(xyz, _offsets(offs), 8, True)
    sph.sph_batched_set_options(use_graph=False, autotune=True)
    try:
        b = sph.sph_batched_compute(xyz, _offsets(offs), 8, True)
    finally:
        sph.sph_batched_set_options(use_graph=True, autotune=True)
    torch.cuda.synchronize()
    assert_bitwise_equal(a["Y"], b["Y"], "graph vs direct Y")
    assert_bitwise_equal(a["dY"], b["dY"], "graph vs direct dY")


def test_batched_empty_environments_and_status():
    import paper_2302_08381_amd as sph
    rng = np.random.default_rng(5)
    counts = rng.integers(0, 5, 300)  # many empty environments
    counts[:10] = 0
    offs = np.zeros(301, np.int64)
    np.cumsum(counts, out=offs[1:])
    n = int(offs[-1])
    pts = rng.standard_normal((n, 3))
    xyz = to_dev(pts, torch.float32)
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    out = sph.sph_batched_compute(xyz, _offsets(offs), 3, False, store_dY=False, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    assert_bitwise_equal(out["Y"], sph.sph_compute(xyz, 3, False), "batched vs plain values")
    # inconsistent offsets: decreasing, wrong start, wrong end
    for bad in (np.array([0, 5, 3, n]), np.array([1, 2, 3, n]), np.array([0, 1, 2, n + 1])):
        st.fill_(-1)
        sph.sph_batched_compute(xyz, _offsets(bad), 3, False, status=st)
        torch.cuda.synchronize()
        assert int(st.item()) == 4
    # zero points, zero environments: the status is still written
    st.fill_(-1)
    e = torch.empty((0, 3), dtype=torch.float32, device="cuda")
    sph.sph_batched_compute(e, _offsets(np.zeros(1, np.int64)), 3, False, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0


def test_batched_workload_autotuned_per_lmax():
    """20 000 environments (8..128 neighbours, shell 0.5..5), float32,
    normalised, a sequence of calls with l_max drawn from {3, 6, 8, 12}."""
    import paper_2302_08381_amd as sph
    pts, offs = csr_environments(20_000, 8, 128, 0.5, 5.0, SEEDS["batched"])
    n = int(offs[-1])
    xyz = to_dev(pts, torch.float32)
    o = _offsets(offs)
    rng = np.random.default_rng(SEEDS["batched"])
    seq = rng.choice([3, 6, 8, 12], 16)
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    for L in seq:
        L = int(L)
        K = (L + 1) ** 2
        gY = to_dev(standard_normal((n, K), 1000 + L), torch.float32)
        out = sph.sph_batched_compute(xyz, o, L, True, store_dY=True, grad_Y=gY, status=st)
        torch.cuda.synchronize()
        assert int(st.item()) == 0
        cfg = sph.sph_batched_get_config(L, True, torch.float32, True, True)
        assert cfg is not None and "blocks_per_cu=" in cfg and "kernel=" in cfg
        idx = torch.arange(0, n, 1999, device="cuda")
        hp = host_points(xyz[idx])
        Yr, Gr = oracle.real_sph(hp, L, True)
        mx, _ = oracle.per_l_errors(out["Y"][idx].cpu().numpy(), Yr, hp, L, True, "Y")
        assert mx.max() <= TOL[torch.float32]
        mx, _ = oracle.per_l_errors(out["dY"][idx].cpu().numpy(), Gr, hp, L, True, "dY")
        assert mx.max() <= TOL[torch.float32]
        # the fused backward's grad_xyz on the same rows
        gYh = gY[idx].cpu().double().numpy()
        _, g, _ = oracle.component_scales(hp, L, True)
        err = np.abs(out["grad_xyz"][idx].cpu().double().numpy() - np.asarray(oracle.backward(Gr, gYh), float))
        assert (err / (np.abs(gYh) * g).sum(1)[:, None]).max() <= TOL[torch.float32], L


def test_batched_graph_reuse_across_changing_sizes():
    """An MD-like loop: the number of neighbours changes every call.  The
    cached graph of a combination is reused with the call's grid (one tile
    per block, so the grid follows n_points up and down); every call equals
    the plain kernel bitwise, and the fused backward the plain backward."""
    import paper_2302_08381_amd as sph
    L = 6
    K = 49
    sph.sph_batched_set_config(L, True, torch.float32, True, True, "default", 0)
    sph.sph_batched_set_config(L, True, torch.float32, False, False, "default", 0)
    rng = np.random.default_rng(123)
    sizes = set()
    for call in range(44):
        n_env = int(rng.integers(1, 400))
        pts, offs = csr_environments(n_env, 0, 128, 0.5, 5.0, 5000 + call)
        n = int(offs[-1])
        sizes.add(n)
        print(f"graph reuse call {call}: n_env={n_env} n_points={n}", flush=True)
        xyz = to_dev(pts, torch.float32)
        gY = to_dev(standard_normal((n, K), 6000 + call), torch.float32)
        o = _offsets(offs)
        out = sph.sph_batched_compute(xyz, o, L, True, store_dY=True, grad_Y=gY)
        vals = sph.sph_batched_compute(xyz, o, L, True, store_dY=False)
        Y, dY = sph.sph_compute_with_gradients(xyz, L, True)
        gx = sph.sph_backward(dY, gY, L)
        torch.cuda.synchronize()
        assert_bitwise_equal(out["Y"], Y, f"call {call} Y")
        assert_bitwise_equal(out["dY"], dY, f"call {call} dY")
        assert_bitwise_equal(vals["Y"], sph.sph_compute(xyz, L, True), f"call {call} values")
        scale = (gY.abs().double()[:, None, :] * dY.abs().double()).sum(2) + 1e-30
        assert float(((out["grad_xyz"].double() - gx.double()).abs() / scale).max()) < 1e-5, call
    assert len(sizes) >= 40


def test_batched_bad_offsets_raise_by_default():
    """Without a status word of the caller's, the wrapper checks the
    kernel's verdict on the offsets and raises."""
    import paper_2302_08381_amd as sph
    pts = np.random.default_rng(3).standard_normal((10, 3))
    xyz = to_dev(pts, torch.float32)
    with pytest.raises(sph.SphError) as ei:
        sph.sph_batched_compute(xyz, _offsets(np.array([0, 6, 4, 10])), 3, True)
    assert ei.value.status == 4
    R = to_dev(standard_normal((10, 4, 2), 4), torch.float32)
    with pytest.raises(sph.SphError):
        sph.sph_radial_expansion(xyz, _offsets(np.array([0, 3, 11])), R, 3, True)
    G = to_dev(standard_normal((2, 2, 16), 5), torch.float32)
    with pytest.raises(sph.SphError):
        sph.sph_radial_expansion_backward(xyz, _offsets(np.array([1, 3, 10])), R, G, 3, True)
    # consistent offsets pass, and check=False leaves the call unchecked
    sph.sph_batched_compute(xyz, _offsets(np.array([0, 4, 10])), 3, True)
    sph.sph_batched_compute(xyz, _offsets(np.array([0, 6, 4, 10])), 3, True, check=False)
    torch.cuda.synchronize()


@pytest.mark.parametrize("l_max", [3, 8, 12])
def test_every_batched_variant_matches_oracle(l_max):
    """Each kernel variant the autotuner can pick (unrolled on its default
    tile, unrolled on a 16-point tile, run-time degree), pinned with
    sph_batched_set_config, on a one-tile-per-block and a persistent grid."""
    import paper_2302_08381_amd as sph
    pts, offs = csr_environments(300, 8, 128, 0.5, 5.0, SEEDS["batched"] + l_max)
    n = int(offs[-1])
    K = (l_max + 1) ** 2
    xyz = to_dev(pts, torch.float32)
    o = _offsets(offs)
    gY = to_dev(standard_normal((n, K), 2000 + l_max), torch.float32)
    hp = host_points(xyz)
    Yr, Gr = oracle.real_sph(hp, l_max, True)
    gYh = gY.cpu().double().numpy()
    gref = np.asarray(oracle.backward(Gr, gYh), float)
    _, gsc, _ = oracle.component_scales(hp, l_max, True)
    gscale = (np.abs(gYh) * gsc).sum(1)[:, None]
    ran = []
    for variant in ("default", "tile16", "runtime_degree", "degree_split"):
        for bpc in (0, 4):
            print(f"batched variant l_max={l_max} {variant} bpc={bpc}", flush=True)
            try:
                sph.sph_batched_set_config(l_max, True, torch.float32, True, True, variant, bpc)
            except sph.SphError:
                assert variant == "degree_split" and l_max <= 8
                continue
            cfg = sph.sph_batched_get_config(l_max, True, torch.float32, True, True)
            assert f"kernel={variant}" in cfg and f"blocks_per_cu={bpc}" in cfg
            out = sph.sph_batched_compute(xyz, o, l_max, True, store_dY=True, grad_Y=gY)
            torch.cuda.synchronize()
            assert_close_per_l(out["Y"].cpu().numpy(), Yr, hp, l_max, True, "Y", TOL[torch.float32], variant)
            assert_close_per_l(out["dY"].cpu().numpy(), Gr, hp, l_max, True, "dY", TOL[torch.float32], variant)
            err = np.abs(out["grad_xyz"].cpu().double().numpy() - gref) / gscale
            assert err.max() <= TOL[torch.float32], (variant, bpc, err.max())
            ran.append(variant)
    assert "default" in ran and "runtime_degree" in ran
    assert ("degree_split" in ran) == (l_max > 8)
    sph.sph_batched_set_config(l_max, True, torch.float32, True, True, "default", 0)
