"""Radial expansion over CSR environments (sph_radial_expansion): the sum of
R_nl(r_j) Y_l^m(x_j) over each environment's points (Eq. expansion),
against the oracle on the same seeded inputs."""
import numpy as np
import pytest
import torch

import oracle
from workloads import SEEDS, csr_environments, gaussian_radial_basis, standard_normal

from _gpu_common import TOL, host_points, to_dev

pytestmark = pytest.mark.gpu

EPS = {torch.float32: float(np.finfo(np.float32).eps), torch.float64: float(np.finfo(np.float64).eps)}

# neighbour counts around the 8..128-point chunks the kernel uses
COUNTS = [0, 1, 2, 7, 8, 9, 63, 64, 65, 127, 128, 129, 200, 257, 0, 31]


def _case(counts, l_max, n_max, seed, radial="normal"):
    counts = np.asarray(counts, np.int64)
    offs = np.zeros(counts.size + 1, np.int64)
    np.cumsum(counts, out=offs[1:])
    rng = np.random.default_rng(seed)
    n = int(offs[-1])
    pts = rng.standard_normal((n, 3)) * rng.uniform(0.5, 2.0, (n, 1))
    if radial == "normal":
        R = standard_normal((n, l_max + 1, n_max), seed + 1)
    else:
        R = gaussian_radial_basis(pts, l_max, n_max, 5.0)
    return pts, offs, R


def _check(c, pts, offs, R, l_max, normalize, dt, label=""):
    """|c - c_ref| <= (TOL + cnt eps) sum_j |R_jln| s_jk per entry: each term
    carries the harmonics' scaled error plus one rounding, and a sum of cnt
    terms adds at most cnt roundings of the sum of magnitudes."""
    ref = np.asarray(oracle.radial_expansion(pts, offs, R, l_max, normalize), float)
    got = c.cpu().double().numpy()
    assert got.shape == ref.shape
    s, _, _ = oracle.component_scales(pts, l_max, normalize)
    lk = np.array([l for l in range(l_max + 1) for _ in range(2 * l + 1)])
    for e in range(offs.size - 1):
        b, t = offs[e], offs[e + 1]
        if t == b:
            assert np.all(got[e] == 0), (label, e)
            continue
        scale = np.einsum("jkn,jk->nk", np.abs(R[b:t][:, lk, :]), s[b:t]) + 1e-300
        tol = TOL[dt] + (t - b) * EPS[dt]
        err = np.abs(got[e] - ref[e]) / scale
        assert np.isfinite(got[e]).all() and err.max() <= tol, (label, e, int(t - b), float(err.max()), tol)


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
@pytest.mark.parametrize("l_max,n_max,normalize", [
    (0, 1, True), (1, 3, False), (3, 8, True), (6, 5, True), (8, 8, True), (8, 8, False),
    (12, 4, True), (8, 13, True),
    # padded channels that fill whole 16-byte vectors (float32 12 of 16;
    # float64 6 of 8, 12 of 16)
    (8, 12, True), (6, 6, False),
    # the low-degree kernels whose items are split across otherwise idle
    # threads: into 4 parts (l_max 2, 3 channels), into 2 (l_max 4 with 8
    # channels, l_max 3 with 12)
    (2, 3, False), (4, 8, True), (3, 12, True)])
def test_expansion_matches_oracle(dt, l_max, n_max, normalize):
    import paper_2302_08381_amd as sph
    print(f"expansion {dt} l_max={l_max} n_max={n_max} normalize={normalize}", flush=True)
    pts, offs, R = _case(COUNTS, l_max, n_max, 300 + 7 * l_max + n_max)
    xyz = to_dev(pts, dt)
    Rt = to_dev(R, dt)
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    c = sph.sph_radial_expansion(xyz, torch.as_tensor(offs, device="cuda"), Rt, l_max, normalize, status=st)
    # the same radial values one element off a 16-byte boundary (element loads)
    bR = torch.empty(Rt.numel() + 1, dtype=dt, device="cuda")
    bR[1:] = Rt.flatten()
    cu = sph.sph_radial_expansion(xyz, torch.as_tensor(offs, device="cuda"), bR[1:].view(Rt.shape), l_max,
                                  normalize)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    # the oracle sees the rounded inputs the kernel saw
    for out, tag in ((c, ""), (cu, " unaligned R")):
        _check(out, host_points(xyz), offs, Rt.cpu().double().numpy(), l_max, normalize, dt,
               f"{dt} L={l_max} n={n_max}{tag}")


@pytest.mark.parametrize("dt,l_max,n_max", [(torch.float32, 5, 8), (torch.float32, 8, 8), (torch.float32, 12, 3),
                                              (torch.float64, 6, 8)])
def test_expansion_chunks_across_environments(dt, l_max, n_max):
    """20 000 environments of 0..8 points (a tenth empty) and a few of 150:
    every block walks many environments, its chunks run from the end of one
    environment into the next (not across empty ones), and a chunk that
    starts a long environment leaves partial sums for the next."""
    import paper_2302_08381_amd as sph
    print(f"expansion across environments {dt} l_max={l_max} n_max={n_max}", flush=True)
    rng = np.random.default_rng(940 + l_max)
    counts = rng.integers(1, 9, 20_000)
    counts[rng.random(counts.size) < 0.1] = 0
    counts[::997] = 150
    pts, offs, R = _case(counts, l_max, n_max, 950 + l_max)
    xyz = to_dev(pts, dt)
    Rt = to_dev(R, dt)
    c = sph.sph_radial_expansion(xyz, torch.as_tensor(offs, device="cuda"), Rt, l_max, True)
    torch.cuda.synchronize()
    hp, Rh = host_points(xyz), Rt.cpu().double().numpy()
    got = c.cpu().double().numpy()
    ref = np.asarray(oracle.radial_expansion(hp, offs, Rh, l_max, True), float)
    # the bound of _check, per environment at once
    s, _, _ = oracle.component_scales(hp, l_max, True)
    lk = np.array([l for l in range(l_max + 1) for _ in range(2 * l + 1)])
    cnts = np.diff(offs)
    nz = cnts > 0
    scale = np.zeros((cnts.size, (l_max + 1) ** 2, n_max))
    scale[nz] = np.add.reduceat(np.abs(Rh[:, lk, :]) * s[:, :, None], offs[:-1][nz], axis=0)
    scale = scale.transpose(0, 2, 1) + 1e-300
    tol = (TOL[dt] + cnts * EPS[dt])[:, None, None]
    assert np.all(got[~nz] == 0)
    err = np.abs(got - ref) / scale
    assert np.isfinite(got).all() and np.all(err <= tol), float((err / tol).max())


@pytest.mark.parametrize("l_max,n_max", [(20, 4), (32, 8)])
def test_expansion_large_degree_small_chunks(l_max, n_max):
    """Large K: 8- to 32-point chunks, so long environments add many partial
    sums."""
    import paper_2302_08381_amd as sph
    dt = torch.float64
    print(f"expansion large l_max={l_max} n_max={n_max}", flush=True)
    pts, offs, R = _case([0, 1, 9, 40, 100], l_max, n_max, 77 + l_max)
    xyz = to_dev(pts, dt)
    Rt = to_dev(R, dt)
    c = sph.sph_radial_expansion(xyz, torch.as_tensor(offs, device="cuda"), Rt, l_max, True)
    torch.cuda.synchronize()
    _check(c, host_points(xyz), offs, Rt.cpu().double().numpy(), l_max, True, dt, f"L={l_max}")


def test_expansion_workload_environments_against_unfused():
    """The batched workload's environments (8..128 neighbours in the shell
    0.5..5), float32, Gaussian radial basis, l_max 3, 6, 8, 12: the fused
    expansion against the oracle on a sample of environments, and against
    the unfused composition (harmonics stored, then contracted by torch in
    float64) on all of them."""
    import paper_2302_08381_amd as sph
    pts, offs = csr_environments(2000, 8, 128, 0.5, 5.0, SEEDS["batched"])
    dt = torch.float32
    xyz = to_dev(pts, dt)
    o = torch.as_tensor(offs, device="cuda")
    env_of = torch.repeat_interleave(torch.arange(offs.size - 1, device="cuda"), o[1:] - o[:-1])
    for L in (3, 6, 8, 12):
        print(f"expansion workload l_max={L}", flush=True)
        R = gaussian_radial_basis(host_points(xyz), L, 8, 5.0)
        Rt = to_dev(R, dt)
        c = sph.sph_radial_expansion(xyz, o, Rt, L, True)
        Y = sph.sph_compute(xyz, L, True).double()
        lk = torch.tensor([l for l in range(L + 1) for _ in range(2 * l + 1)], device="cuda")
        W = Rt.double()[:, lk, :]                                    # [N, K, n]
        ref = torch.zeros((offs.size - 1, (L + 1) ** 2, 8), dtype=torch.float64, device="cuda")
        ref.index_add_(0, env_of, W * Y[:, :, None])
        ref = ref.permute(0, 2, 1)
        # error scale of each sum: sum_j |R_jln| times the size of a degree-l
        # harmonic, sqrt((2l+1)/4pi) (the scale of the oracle comparisons)
        sl = torch.sqrt((2 * lk.double() + 1) / (4 * np.pi))
        mag = torch.zeros_like(ref.permute(0, 2, 1)).index_add_(0, env_of, W.abs() * sl[None, :, None])
        mag = mag.permute(0, 2, 1)
        torch.cuda.synchronize()
        err = ((c.double() - ref).abs() / (mag + 1e-30)).max()
        assert float(err) <= 2e-5, (L, float(err))  # 1e-5 (harmonics) + 128 roundings of 2^-24
        sel = np.arange(0, offs.size - 1, 97)
        sub = np.concatenate([[0], np.cumsum(offs[sel + 1] - offs[sel])])
        rows = np.concatenate([np.arange(offs[e], offs[e + 1]) for e in sel])
        _check(c[torch.as_tensor(sel, device="cuda")], host_points(xyz)[rows], sub,
               Rt.cpu().double().numpy()[rows], L, True, dt, f"workload L={L}")


def test_expansion_status_and_degenerate_inputs():
    import paper_2302_08381_amd as sph
    dt = torch.float32
    pts, offs, R = _case([3, 0, 5], 4, 2, 11)
    xyz = to_dev(pts, dt)
    Rt = to_dev(R, dt)
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    # inconsistent offsets: decreasing, wrong start, past the end (clamped, no fault)
    for bad in (np.array([0, 5, 3, 8]), np.array([1, 2, 3, 8]), np.array([0, 1, 2, 20])):
        st.fill_(-1)
        sph.sph_radial_expansion(xyz, torch.as_tensor(bad, device="cuda"), Rt, 4, True, status=st)
        torch.cuda.synchronize()
        assert int(st.item()) == 4
    # no environments: the status is still written
    st.fill_(-1)
    e = torch.empty((0, 3), dtype=dt, device="cuda")
    c = sph.sph_radial_expansion(e, torch.zeros(1, dtype=torch.int64, device="cuda"),
                                 torch.empty((0, 5, 2), dtype=dt, device="cuda"), 4, True, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0 and c.shape == (0, 2, 25)
    # only empty environments: zeros
    c = sph.sph_radial_expansion(e, torch.zeros(4, dtype=torch.int64, device="cuda"),
                                 torch.empty((0, 5, 2), dtype=dt, device="cuda"), 4, True)
    torch.cuda.synchronize()
    assert c.shape == (3, 2, 25) and bool((c == 0).all())
    # a point at the origin (normalised: only Y_0^0 survives)
    z = torch.zeros((1, 3), dtype=dt, device="cuda")
    c = sph.sph_radial_expansion(z, torch.tensor([0, 1], device="cuda"), torch.ones((1, 5, 1), dtype=dt,
                                 device="cuda"), 4, True)
    torch.cuda.synchronize()
    ref = np.zeros(25)
    ref[0] = 0.5 / np.sqrt(np.pi)
    assert np.allclose(c.cpu().numpy()[0, 0], ref, rtol=1e-6, atol=0)


def _check_backward(gx, gR, pts, offs, R, G, l_max, normalize, dt, label=""):
    """Scaled bounds as for the expansion: grad_R[j,l,n] sums 2l+1 terms
    G Y (scale sum_m |G| s_l); grad_xyz[j,a] sums K terms gY dY with
    gY = sum_n G R (scale sum_k (sum_n |G||R|) g_l), each with the
    harmonics' error plus roundings of the sums."""
    ref_x, ref_R = oracle.radial_expansion_backward(pts, offs, R, G, l_max, normalize)
    ref_x, ref_R = np.asarray(ref_x, float), np.asarray(ref_R, float)
    s, g, _ = oracle.component_scales(pts, l_max, normalize)
    K = (l_max + 1) ** 2
    lk = np.array([l for l in range(l_max + 1) for _ in range(2 * l + 1)])
    env = np.repeat(np.arange(offs.size - 1), np.diff(offs))
    Ga = np.abs(G)[env]                                            # [N, n, K]
    Ra = np.abs(R)[:, lk, :]                                       # [N, K, n]
    gys = np.einsum("jnk,jkn->jk", Ga, Ra)                        # bound of |gY|
    nm = R.shape[2]
    tol = TOL[dt] + (K + nm) * EPS[dt]
    if gx is not None:
        scale = (gys * g).sum(1)[:, None] + 1e-300
        err = np.abs(gx.cpu().double().numpy() - ref_x) / scale
        assert np.isfinite(err).all() and err.max() <= tol, (label, "grad_xyz", float(err.max()), tol)
    if gR is not None:
        sc = np.zeros_like(ref_R)
        for l in range(l_max + 1):
            sc[:, l, :] = (Ga[:, :, l * l:(l + 1) ** 2] * s[:, None, l * l:(l + 1) ** 2]).sum(2)
        err = np.abs(gR.cpu().double().numpy() - ref_R) / (sc + 1e-300)
        assert np.isfinite(err).all() and err.max() <= tol, (label, "grad_R", float(err.max()), tol)


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
@pytest.mark.parametrize("l_max,n_max,normalize", [
    (0, 1, True), (2, 3, False), (4, 8, True), (6, 12, False), (8, 8, True), (8, 5, False), (8, 16, True),
    (10, 5, True), (11, 4, True), (20, 9, True), (28, 12, True)])
def test_expansion_backward_matches_oracle(dt, l_max, n_max, normalize):
    import paper_2302_08381_amd as sph
    print(f"expansion backward {dt} l_max={l_max} n_max={n_max} normalize={normalize}", flush=True)
    # environments across the 32- and 64-point chunk edges of the lane groups,
    # and one far longer than the rest (the groups split the points evenly)
    counts = [0, 1, 7, 32, 33, 64, 129, 0, 200, 1500, 3] if l_max <= 12 else [0, 1, 9, 40, 70]
    pts, offs, R = _case(counts, l_max, n_max, 500 + 7 * l_max + n_max)
    xyz = to_dev(pts, dt)
    Rt = to_dev(R, dt)
    G = standard_normal((offs.size - 1, n_max, (l_max + 1) ** 2), 600 + l_max)
    Gt = to_dev(G, dt)
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    o = torch.as_tensor(offs, device="cuda")
    gx, gR = sph.sph_radial_expansion_backward(xyz, o, Rt, Gt, l_max, normalize, status=st)
    only_x, none_R = sph.sph_radial_expansion_backward(xyz, o, Rt, Gt, l_max, normalize, want_grad_R=False)
    torch.cuda.synchronize()
    assert int(st.item()) == 0 and none_R is None
    assert torch.equal(only_x, gx)
    _check_backward(gx, gR, host_points(xyz), offs, Rt.cpu().double().numpy(), Gt.cpu().double().numpy(),
                    l_max, normalize, dt, f"{dt} L={l_max} n={n_max}")


@pytest.mark.parametrize("dt,l_max", [(torch.float32, 3), (torch.float32, 9), (torch.float64, 4),
                                        (torch.float64, 6)])
def test_expansion_backward_chunks_across_environments(dt, l_max):
    """20 000 environments of 0..8 points (a tenth empty): every group of
    lanes walks several environments, and its chunks run across environment
    ends, across empty environments and stop exactly at an end.  Staged
    (float32 l_max 3, float64 l_max 4) and direct (float32 l_max 9, float64
    l_max 6) radial rows."""
    import paper_2302_08381_amd as sph
    print(f"expansion backward across environments {dt} l_max={l_max}", flush=True)
    rng = np.random.default_rng(900 + l_max)
    counts = rng.integers(1, 9, 20_000)
    counts[rng.random(counts.size) < 0.1] = 0
    n_max = 8
    pts, offs, R = _case(counts, l_max, n_max, 910 + l_max)
    xyz = to_dev(pts, dt)
    Rt = to_dev(R, dt)
    Gt = to_dev(standard_normal((offs.size - 1, n_max, (l_max + 1) ** 2), 920 + l_max), dt)
    o = torch.as_tensor(offs, device="cuda")
    gx, gR = sph.sph_radial_expansion_backward(xyz, o, Rt, Gt, l_max, True)
    only_x, _ = sph.sph_radial_expansion_backward(xyz, o, Rt, Gt, l_max, True, want_grad_R=False)
    torch.cuda.synchronize()
    assert torch.equal(only_x, gx)
    _check_backward(gx, gR, host_points(xyz), offs, Rt.cpu().double().numpy(), Gt.cpu().double().numpy(),
                    l_max, True, dt, f"{dt} L={l_max} across environments")


def test_expansion_backward_through_autograd_matches_torch():
    """The backward against torch autograd of the unfused composition in
    float64 (harmonics from sph_compute_with_gradients, contracted by torch)."""
    import paper_2302_08381_amd as sph
    dt = torch.float64
    L, NM = 6, 8
    pts, offs = csr_environments(300, 8, 128, 0.5, 5.0, SEEDS["batched"] + 3)
    xyz = to_dev(pts, dt)
    o = torch.as_tensor(offs, device="cuda")
    R = to_dev(gaussian_radial_basis(pts, L, NM, 5.0), dt)
    G = to_dev(standard_normal((offs.size - 1, NM, (L + 1) ** 2), 77), dt)
    gx, gR = sph.sph_radial_expansion_backward(xyz, o, R, G, L, True)
    Y, dY = sph.sph_compute_with_gradients(xyz, L, True)
    env = torch.repeat_interleave(torch.arange(offs.size - 1, device="cuda"), o[1:] - o[:-1])
    lk = torch.tensor([l for l in range(L + 1) for _ in range(2 * l + 1)], device="cuda")
    gY = (G[env] * R[:, lk, :].permute(0, 2, 1)).sum(1)           # [N, K]
    ref_x = (gY[:, None, :] * dY).sum(2)
    ref_R = torch.zeros_like(R)
    prod = (G[env] * Y[:, None, :])                                  # [N, n, K]
    for l in range(L + 1):
        ref_R[:, l, :] = prod[:, :, l * l:(l + 1) ** 2].sum(2)
    torch.cuda.synchronize()
    assert float((gx - ref_x).abs().max()) <= 1e-10 * (1 + float(ref_x.abs().max()))
    assert float((gR - ref_R).abs().max()) <= 1e-10 * (1 + float(ref_R.abs().max()))


@pytest.mark.parametrize("dt,l_max,n_max", [(torch.float32, 11, 4), (torch.float32, 8, 12), (torch.float64, 6, 6),
                                           (torch.float32, 6, 4), (torch.float64, 4, 6)])
def test_expansion_backward_partial_vectors(dt, l_max, n_max):
    """Channels that need padding but fill whole 16-byte vectors, rows read
    directly (float32 l_max 11 and 8, float64 l_max 6) or staged through the
    LDS tile (float32 l_max 6, float64 l_max 4) as 16-byte vectors, the
    vectors past n_max zero; and the same inputs one element off a 16-byte
    boundary (element loads): both against the oracle."""
    import paper_2302_08381_amd as sph
    print(f"expansion backward partial vectors {dt} l_max={l_max} n_max={n_max}", flush=True)
    pts, offs, R = _case([0, 1, 7, 32, 33, 64, 129, 0, 200, 3], l_max, n_max, 960 + l_max + n_max)
    E, K = offs.size - 1, (l_max + 1) ** 2
    xyz = to_dev(pts, dt)
    Rt = to_dev(R, dt)
    Gt = to_dev(standard_normal((E, n_max, K), 970 + l_max), dt)
    o = torch.as_tensor(offs, device="cuda")
    bR = torch.empty(Rt.numel() + 1, dtype=dt, device="cuda")
    bR[1:] = Rt.flatten()
    Ru = bR[1:].view(Rt.shape)
    for Rin, tag in ((Rt, "aligned"), (Ru, "unaligned")):
        gx, gR = sph.sph_radial_expansion_backward(xyz, o, Rin, Gt, l_max, True)
        torch.cuda.synchronize()
        _check_backward(gx, gR, host_points(xyz), offs, Rt.cpu().double().numpy(), Gt.cpu().double().numpy(),
                        l_max, True, dt, f"{dt} L={l_max} n={n_max} {tag}")


def test_expansion_deterministic_and_unaligned_inputs():
    """No atomics: repeated calls are bitwise equal.  Inputs and outputs that
    start at odd element offsets (not 16-byte aligned) give the same results."""
    import paper_2302_08381_amd as sph
    dt = torch.float32
    L, NM = 8, 5
    pts, offs, R = _case([3, 70, 0, 129, 33], L, NM, 909)
    n, E, K = pts.shape[0], offs.size - 1, (L + 1) ** 2
    xyz = to_dev(pts, dt)
    Rt = to_dev(R, dt)
    G = to_dev(standard_normal((E, NM, K), 910), dt)
    o = torch.as_tensor(offs, device="cuda")
    c1 = sph.sph_radial_expansion(xyz, o, Rt, L, True)
    c2 = sph.sph_radial_expansion(xyz, o, Rt, L, True)
    gx1, gR1 = sph.sph_radial_expansion_backward(xyz, o, Rt, G, L, True)
    gx2, gR2 = sph.sph_radial_expansion_backward(xyz, o, Rt, G, L, True)
    # the same values one element into larger buffers
    bx = torch.empty(n * 3 + 1, dtype=dt, device="cuda")
    bx[1:] = xyz.flatten()
    bR = torch.empty(Rt.numel() + 1, dtype=dt, device="cuda")
    bR[1:] = Rt.flatten()
    bG = torch.empty(G.numel() + 1, dtype=dt, device="cuda")
    bG[1:] = G.flatten()
    bc = torch.empty(E * NM * K + 1, dtype=dt, device="cuda")
    xu, Ru, Gu = bx[1:].view(n, 3), bR[1:].view(n, L + 1, NM), bG[1:].view(E, NM, K)
    cu = sph.sph_radial_expansion(xu, o, Ru, L, True, out=bc[1:].view(E, NM, K))
    gxu, gRu = sph.sph_radial_expansion_backward(xu, o, Ru, Gu, L, True)
    torch.cuda.synchronize()
    for a, b, name in ((c1, c2, "c"), (gx1, gx2, "grad_xyz"), (gR1, gR2, "grad_R"), (c1, cu, "c unaligned"),
                       (gx1, gxu, "grad_xyz unaligned"), (gR1, gRu, "grad_R unaligned")):
        assert torch.equal(a, b), name
