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
