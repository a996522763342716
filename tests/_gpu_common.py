"""Shared helpers of the GPU parity tests (not collected by pytest)."""
import numpy as np
import torch

import oracle

# Tolerances on the scaled per-l error of oracle.per_l_errors (a value of
# 1e-5 is "wrong in the 5th digit of a typical entry of degree l").
TOL = {torch.float32: 1e-5, torch.float64: 1e-12}


def dev():
    return torch.device("cuda", 0)


def to_dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype=dtype, device=dev()).contiguous()


def host_points(xyz_t):
    """The device inputs as exact float64 values (the oracle sees the
    rounded inputs the kernel saw)."""
    return xyz_t.detach().cpu().double().numpy()


def assert_close_per_l(A, ref, pts, l_max, normalize, kind, tol, label=""):
    mx, rms = oracle.per_l_errors(A, ref, pts, l_max, normalize, kind)
    assert np.isfinite(mx).all() and mx.max() <= tol, \
        f"{label} {kind}: per-l max scaled error {mx} exceeds {tol}"
    return mx, rms


def assert_bitwise_equal(a, b, label=""):
    """torch.equal with a report of where the tensors differ."""
    if torch.equal(a, b):
        return
    d = (a != b)
    if d.dim() > 1:
        rows = d.reshape(d.shape[0], -1).any(1).nonzero().flatten()
    else:
        rows = d.nonzero().flatten()
    nan_a = int(torch.isnan(a).sum())
    nan_b = int(torch.isnan(b).sum())
    r0 = int(rows[0]) if len(rows) else -1
    raise AssertionError(
        f"{label}: {int(d.sum())} elements differ in {len(rows)} rows (first rows {rows[:10].tolist()}), "
        f"NaNs {nan_a}/{nan_b}; row {r0}: {a[r0].flatten()[:6].tolist()} vs {b[r0].flatten()[:6].tolist()}")
