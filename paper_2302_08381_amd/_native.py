"""ctypes binding of libsph.so, entry point for entry point (include/sph.h).

Argument marshalling only: every function checks tensor placement, dtype
and layout, allocates missing outputs with torch on the input's device,
passes raw device pointers and torch's current HIP stream, and raises
:class:`SphError` with the library's message on a non-zero status.  No
arithmetic of the method happens here.

The library is loaded on first use; if libsph.so has not been built the
call raises (there is no fallback implementation).
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsph.so")
_lock = threading.Lock()
_lib = None

SPH_F32 = 0
SPH_F64 = 1
SPH_OK = 0
SPH_ERR_NULL = 1
SPH_ERR_INVALID = 2
SPH_ERR_LMAX = 3
SPH_ERR_OFFSETS = 4
SPH_ERR_DEVICE = 5

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64

_SIGNATURES = {
    "sph_num_components": (_i32, [_i32]),
    "sph_max_lmax": (_i32, []),
    "sph_status_string": (ctypes.c_char_p, [_i32]),
    "sph_last_error": (ctypes.c_char_p, []),
    "sph_version": (ctypes.c_char_p, []),
    "sph_compute": (_i32, [_vp, _i64, _i32, _i32, _i32, _vp, _vp]),
    "sph_compute_with_gradients": (_i32, [_vp, _i64, _i32, _i32, _i32, _vp, _vp, _vp]),
    "sph_compute_with_hessians": (_i32, [_vp, _i64, _i32, _i32, _i32, _vp, _vp, _vp, _vp]),
    "sph_backward": (_i32, [_vp, _vp, _i64, _i32, _i32, _vp, _vp]),
    "sph_double_backward": (_i32, [_vp, _vp, _vp, _i64, _i32, _i32, _i32, _vp, _vp, _vp]),
    "sph_batched_compute": (_i32, [_vp, _vp, _i64, _i64, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp]),
    "sph_radial_expansion": (_i32, [_vp, _vp, _i64, _i64, _vp, _i32, _i32, _i32, _i32, _vp, _vp, _vp]),
    "sph_radial_expansion_backward": (_i32, [_vp, _vp, _i64, _i64, _vp, _i32, _i32, _i32, _i32, _vp, _vp, _vp,
                                              _vp, _vp]),
    "sph_e3nn_coordinates": (_i32, [_vp, _i64, _i32, _vp, _vp]),
    "sph_e3nn_convert": (_i32, [_i64, _i32, _i32, _i32, _vp, _vp, _vp]),
    "sph_batched_set_options": (_i32, [_i32, _i32]),
    "sph_batched_get_config": (_i32, [_i32, _i32, _i32, _i32, _i32, ctypes.c_char_p, _i32]),
    "sph_batched_set_config": (_i32, [_i32, _i32, _i32, _i32, _i32, _i32, _i32]),
}


class SphError(RuntimeError):
    """A libsph call returned a non-zero status."""

    def __init__(self, status: int, message: str):
        super().__init__(f"libsph status {status}: {message}")
        self.status = status


def library_path() -> str:
    return _LIB_PATH


def lib():
    """The loaded library (ctypes.CDLL).  Raises if libsph.so is missing."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                raise RuntimeError(
                    f"libsph.so not found at {_LIB_PATH}; build it with "
                    "`python -m paper_2302_08381_amd.build` (HIP/ROCm required)")
            L = ctypes.CDLL(_LIB_PATH)
            for name, (res, args) in _SIGNATURES.items():
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
            _lib = L
    return _lib


def _check(status: int):
    if status != SPH_OK:
        msg = lib().sph_last_error().decode()
        raise SphError(status, msg or lib().sph_status_string(status).decode())


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return SPH_F32
    if t.dtype == torch.float64:
        return SPH_F64
    raise TypeError(f"unsupported dtype {t.dtype} (float32 or float64)")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _need(t: torch.Tensor, name: str, shape, dtype, device):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a tensor")
    if t.device != device or t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype} on {device}, got {t.dtype} on {t.device}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _check_xyz(xyz: torch.Tensor):
    if not isinstance(xyz, torch.Tensor) or xyz.dim() != 2 or xyz.shape[1] != 3:
        raise ValueError("xyz must be a [n,3] tensor")
    if xyz.device.type != "cuda":
        raise ValueError("xyz must be on a HIP device")
    if not xyz.is_contiguous():
        raise ValueError("xyz must be contiguous")
    _dtype_code(xyz)


def _csr_status(status, check, device):
    """(status word, whether the wrapper checks it) for a CSR call.  A
    caller's status word is the caller's to read unless ``check`` is True;
    without one the wrapper allocates a word and checks it unless ``check``
    is False."""
    if status is not None:
        _need(status, "status", (1,), torch.int32, device)
        return status, bool(check)
    if check is False:
        return None, False
    return torch.empty((1,), dtype=torch.int32, device=device), True


def _raise_on_status(status, check: bool):
    """Synchronises on the status word and raises SphError(SPH_ERR_OFFSETS)
    if the kernel found the offsets inconsistent."""
    if check:
        code = int(status.item())
        if code != SPH_OK:
            raise SphError(code, "inconsistent CSR offsets: offsets[0] must be 0, offsets non-decreasing "
                                 "and offsets[n_env] equal to the number of points")


def num_components(l_max: int) -> int:
    return int(lib().sph_num_components(int(l_max)))


def max_lmax() -> int:
    return int(lib().sph_max_lmax())


def version() -> str:
    return lib().sph_version().decode()


def sph_compute(xyz: torch.Tensor, l_max: int, normalize: bool = True, Y: torch.Tensor | None = None):
    """Y[n,K] (include/sph.h: sph_compute)."""
    _check_xyz(xyz)
    n = xyz.shape[0]
    K = (int(l_max) + 1) ** 2 if l_max >= 0 else 0
    if Y is None:
        Y = torch.empty((n, max(K, 0)), dtype=xyz.dtype, device=xyz.device)
    else:
        _need(Y, "Y", (n, K), xyz.dtype, xyz.device)
    with torch.cuda.device(xyz.device):
        _check(lib().sph_compute(_ptr(xyz), n, int(l_max), int(bool(normalize)), _dtype_code(xyz),
                                 _ptr(Y), _stream(xyz.device)))
    return Y


def sph_compute_with_gradients(xyz: torch.Tensor, l_max: int, normalize: bool = True,
                               Y: torch.Tensor | None = None, dY: torch.Tensor | None = None):
    """(Y[n,K], dY[n,3,K]) (include/sph.h: sph_compute_with_gradients)."""
    _check_xyz(xyz)
    n = xyz.shape[0]
    K = (int(l_max) + 1) ** 2 if l_max >= 0 else 0
    if Y is None:
        Y = torch.empty((n, K), dtype=xyz.dtype, device=xyz.device)
    else:
        _need(Y, "Y", (n, K), xyz.dtype, xyz.device)
    if dY is None:
        dY = torch.empty((n, 3, K), dtype=xyz.dtype, device=xyz.device)
    else:
        _need(dY, "dY", (n, 3, K), xyz.dtype, xyz.device)
    with torch.cuda.device(xyz.device):
        _check(lib().sph_compute_with_gradients(_ptr(xyz), n, int(l_max), int(bool(normalize)),
                                                _dtype_code(xyz), _ptr(Y), _ptr(dY), _stream(xyz.device)))
    return Y, dY


E3NN_NORMALIZATIONS = {"integral": 0, "component": 1, "norm": 2}


def sph_e3nn_coordinates(xyz: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """(z, x, y) of every point (include/sph.h: sph_e3nn_coordinates); ``out``
    may be ``xyz`` itself."""
    _check_xyz(xyz)
    n = xyz.shape[0]
    if out is None:
        out = torch.empty_like(xyz)
    else:
        _need(out, "out", (n, 3), xyz.dtype, xyz.device)
    with torch.cuda.device(xyz.device):
        _check(lib().sph_e3nn_coordinates(_ptr(xyz), n, _dtype_code(xyz), _ptr(out), _stream(xyz.device)))
    return out


def sph_e3nn_convert(Y: torch.Tensor, dY: torch.Tensor | None, l_max: int, normalization: str = "integral"):
    """In place: Y (and dY) computed at sph_e3nn_coordinates' points into
    e3nn's convention (include/sph.h: sph_e3nn_convert).  Returns (Y, dY)."""
    if normalization not in E3NN_NORMALIZATIONS:
        raise ValueError(f"normalization must be one of {sorted(E3NN_NORMALIZATIONS)}")
    n = Y.shape[0]
    K = (int(l_max) + 1) ** 2 if l_max >= 0 else 0
    _need(Y, "Y", (n, K), Y.dtype, Y.device)
    if dY is not None:
        _need(dY, "dY", (n, 3, K), Y.dtype, Y.device)
    with torch.cuda.device(Y.device):
        _check(lib().sph_e3nn_convert(n, int(l_max), E3NN_NORMALIZATIONS[normalization], _dtype_code(Y), _ptr(Y),
                                      _ptr(dY), _stream(Y.device)))
    return Y, dY


def sph_compute_with_hessians(xyz: torch.Tensor, l_max: int, normalize: bool = True,
                              Y: torch.Tensor | None = None, dY: torch.Tensor | None = None,
                              d2Y: torch.Tensor | None = None, store_dY: bool = True):
    """(Y[n,K], dY[n,3,K] or None, d2Y[n,3,3,K]) (include/sph.h: sph_compute_with_hessians).
    With ``store_dY=False`` (and no ``dY`` given) the first derivatives are
    not stored."""
    _check_xyz(xyz)
    n = xyz.shape[0]
    K = (int(l_max) + 1) ** 2 if l_max >= 0 else 0
    if Y is None:
        Y = torch.empty((n, K), dtype=xyz.dtype, device=xyz.device)
    else:
        _need(Y, "Y", (n, K), xyz.dtype, xyz.device)
    if dY is None:
        if store_dY:
            dY = torch.empty((n, 3, K), dtype=xyz.dtype, device=xyz.device)
    else:
        _need(dY, "dY", (n, 3, K), xyz.dtype, xyz.device)
    if d2Y is None:
        d2Y = torch.empty((n, 3, 3, K), dtype=xyz.dtype, device=xyz.device)
    else:
        _need(d2Y, "d2Y", (n, 3, 3, K), xyz.dtype, xyz.device)
    with torch.cuda.device(xyz.device):
        _check(lib().sph_compute_with_hessians(_ptr(xyz), n, int(l_max), int(bool(normalize)), _dtype_code(xyz),
                                               _ptr(Y), _ptr(dY), _ptr(d2Y), _stream(xyz.device)))
    return Y, dY, d2Y


def sph_backward(dY: torch.Tensor, grad_Y: torch.Tensor, l_max: int, grad_xyz: torch.Tensor | None = None):
    """grad_xyz[n,3] = sum_k grad_Y[n,k] dY[n,:,k] (include/sph.h: sph_backward)."""
    n = dY.shape[0]
    K = (int(l_max) + 1) ** 2
    _need(dY, "dY", (n, 3, K), dY.dtype, dY.device)
    _need(grad_Y, "grad_Y", (n, K), dY.dtype, dY.device)
    if grad_xyz is None:
        grad_xyz = torch.empty((n, 3), dtype=dY.dtype, device=dY.device)
    else:
        _need(grad_xyz, "grad_xyz", (n, 3), dY.dtype, dY.device)
    with torch.cuda.device(dY.device):
        _check(lib().sph_backward(_ptr(dY), _ptr(grad_Y), n, int(l_max), _dtype_code(dY), _ptr(grad_xyz),
                                  _stream(dY.device)))
    return grad_xyz


def sph_double_backward(xyz: torch.Tensor, grad_Y: torch.Tensor, v: torch.Tensor, l_max: int,
                        normalize: bool = True, want_grad_grad_Y: bool = True, want_grad_xyz: bool = True,
                        grad_grad_Y: torch.Tensor | None = None, grad_xyz2: torch.Tensor | None = None):
    """(grad_grad_Y[n,K] or None, grad_xyz2[n,3] or None) (include/sph.h: sph_double_backward);
    the outputs may be preallocated."""
    _check_xyz(xyz)
    n = xyz.shape[0]
    K = (int(l_max) + 1) ** 2
    _need(grad_Y, "grad_Y", (n, K), xyz.dtype, xyz.device)
    _need(v, "v", (n, 3), xyz.dtype, xyz.device)
    ggY = g2 = None
    if want_grad_grad_Y:
        ggY = torch.empty((n, K), dtype=xyz.dtype, device=xyz.device) if grad_grad_Y is None else \
            _need(grad_grad_Y, "grad_grad_Y", (n, K), xyz.dtype, xyz.device)
    if want_grad_xyz:
        g2 = torch.empty((n, 3), dtype=xyz.dtype, device=xyz.device) if grad_xyz2 is None else \
            _need(grad_xyz2, "grad_xyz2", (n, 3), xyz.dtype, xyz.device)
    with torch.cuda.device(xyz.device):
        _check(lib().sph_double_backward(_ptr(xyz), _ptr(grad_Y), _ptr(v), n, int(l_max),
                                         int(bool(normalize)), _dtype_code(xyz), _ptr(ggY), _ptr(g2),
                                         _stream(xyz.device)))
    return ggY, g2


def sph_batched_compute(xyz: torch.Tensor, offsets: torch.Tensor, l_max: int, normalize: bool = True,
                        store_dY: bool = True, grad_Y: torch.Tensor | None = None,
                        status: torch.Tensor | None = None, out: dict | None = None, check: bool | None = None):
    """Batched CSR evaluation (include/sph.h: sph_batched_compute).

    Returns a dict with "Y", "dY" (or None), "grad_xyz" (or None) and
    "status" (an int32[1] device tensor written by the kernel, or None).
    ``out`` may hold preallocated "Y", "dY", "grad_xyz" tensors.

    The kernel checks the offsets on the device and writes its verdict to a
    status word.  Without a ``status`` tensor of the caller's the wrapper
    passes one of its own, waits for the call and raises SphError on
    inconsistent offsets; ``check=False`` skips that (the call stays
    asynchronous), ``check=True`` also checks a caller's status word.
    """
    _check_xyz(xyz)
    n = xyz.shape[0]
    K = (int(l_max) + 1) ** 2
    if offsets.dtype != torch.int64 or offsets.dim() != 1 or offsets.device != xyz.device \
            or not offsets.is_contiguous():
        raise ValueError("offsets must be a contiguous int64 [n_env+1] tensor on the device of xyz")
    n_env = offsets.shape[0] - 1
    if n_env < 0:
        raise ValueError("offsets needs at least one entry")
    out = {} if out is None else dict(out)
    Y = out.get("Y")
    Y = torch.empty((n, K), dtype=xyz.dtype, device=xyz.device) if Y is None else \
        _need(Y, "Y", (n, K), xyz.dtype, xyz.device)
    dY = None
    if store_dY:
        dY = out.get("dY")
        dY = torch.empty((n, 3, K), dtype=xyz.dtype, device=xyz.device) if dY is None else \
            _need(dY, "dY", (n, 3, K), xyz.dtype, xyz.device)
    gx = None
    if grad_Y is not None:
        _need(grad_Y, "grad_Y", (n, K), xyz.dtype, xyz.device)
        gx = out.get("grad_xyz")
        gx = torch.empty((n, 3), dtype=xyz.dtype, device=xyz.device) if gx is None else \
            _need(gx, "grad_xyz", (n, 3), xyz.dtype, xyz.device)
    status, check = _csr_status(status, check, xyz.device)
    with torch.cuda.device(xyz.device):
        _check(lib().sph_batched_compute(_ptr(xyz), _ptr(offsets), n_env, n, int(l_max), int(bool(normalize)),
                                         _dtype_code(xyz), _ptr(Y), _ptr(dY), _ptr(grad_Y), _ptr(gx),
                                         _ptr(status), _stream(xyz.device)))
    _raise_on_status(status, check)
    return {"Y": Y, "dY": dY, "grad_xyz": gx, "status": status}


def sph_radial_expansion(xyz: torch.Tensor, offsets: torch.Tensor, R: torch.Tensor, l_max: int,
                         normalize: bool = True, status: torch.Tensor | None = None,
                         out: torch.Tensor | None = None, check: bool | None = None) -> torch.Tensor:
    """c[n_env, n_max, K] = sum over each environment's points of R[j,l,n] Y_l^m(x_j)
    (include/sph.h: sph_radial_expansion).  R is [n_points, l_max+1, n_max].
    ``check`` as in sph_batched_compute."""
    _check_xyz(xyz)
    n = xyz.shape[0]
    K = (int(l_max) + 1) ** 2
    if offsets.dtype != torch.int64 or offsets.dim() != 1 or offsets.device != xyz.device \
            or not offsets.is_contiguous():
        raise ValueError("offsets must be a contiguous int64 [n_env+1] tensor on the device of xyz")
    n_env = offsets.shape[0] - 1
    if n_env < 0:
        raise ValueError("offsets needs at least one entry")
    if R.dim() != 3:
        raise ValueError("R must be [n_points, l_max+1, n_max]")
    n_max = R.shape[2]
    _need(R, "R", (n, int(l_max) + 1, n_max), xyz.dtype, xyz.device)
    c = torch.empty((n_env, n_max, K), dtype=xyz.dtype, device=xyz.device) if out is None else \
        _need(out, "out", (n_env, n_max, K), xyz.dtype, xyz.device)
    status, check = _csr_status(status, check, xyz.device)
    with torch.cuda.device(xyz.device):
        _check(lib().sph_radial_expansion(_ptr(xyz), _ptr(offsets), n_env, n, _ptr(R), int(n_max), int(l_max),
                                          int(bool(normalize)), _dtype_code(xyz), _ptr(c), _ptr(status),
                                          _stream(xyz.device)))
    _raise_on_status(status, check)
    return c


def sph_radial_expansion_backward(xyz: torch.Tensor, offsets: torch.Tensor, R: torch.Tensor, grad_c: torch.Tensor,
                                  l_max: int, normalize: bool = True, want_grad_xyz: bool = True,
                                  want_grad_R: bool = True, status: torch.Tensor | None = None,
                                  check: bool | None = None):
    """(grad_xyz [n,3] or None, grad_R [n, l_max+1, n_max] or None) for an
    upstream gradient grad_c [n_env, n_max, K] of sph_radial_expansion
    (include/sph.h: sph_radial_expansion_backward).  ``check`` as in
    sph_batched_compute."""
    _check_xyz(xyz)
    n = xyz.shape[0]
    K = (int(l_max) + 1) ** 2
    if offsets.dtype != torch.int64 or offsets.dim() != 1 or offsets.device != xyz.device \
            or not offsets.is_contiguous():
        raise ValueError("offsets must be a contiguous int64 [n_env+1] tensor on the device of xyz")
    n_env = offsets.shape[0] - 1
    if n_env < 0:
        raise ValueError("offsets needs at least one entry")
    if R.dim() != 3:
        raise ValueError("R must be [n_points, l_max+1, n_max]")
    n_max = R.shape[2]
    _need(R, "R", (n, int(l_max) + 1, n_max), xyz.dtype, xyz.device)
    _need(grad_c, "grad_c", (n_env, n_max, K), xyz.dtype, xyz.device)
    gx = torch.empty((n, 3), dtype=xyz.dtype, device=xyz.device) if want_grad_xyz else None
    gR = torch.empty_like(R) if want_grad_R else None
    status, check = _csr_status(status, check, xyz.device)
    with torch.cuda.device(xyz.device):
        _check(lib().sph_radial_expansion_backward(_ptr(xyz), _ptr(offsets), n_env, n, _ptr(R), int(n_max),
                                                   int(l_max), int(bool(normalize)), _dtype_code(xyz),
                                                   _ptr(grad_c), _ptr(gx), _ptr(gR), _ptr(status),
                                                   _stream(xyz.device)))
    _raise_on_status(status, check)
    return gx, gR


def sph_batched_set_options(use_graph: bool = True, autotune: bool = True):
    _check(lib().sph_batched_set_options(int(bool(use_graph)), int(bool(autotune))))


def sph_batched_get_config(l_max: int, normalize: bool, dtype: torch.dtype, store_dY: bool,
                           with_backward: bool) -> str | None:
    buf = ctypes.create_string_buffer(128)
    code = SPH_F64 if dtype == torch.float64 else SPH_F32
    st = lib().sph_batched_get_config(int(l_max), int(bool(normalize)), code, int(bool(store_dY)),
                                      int(bool(with_backward)), buf, 128)
    return buf.value.decode() if st == SPH_OK else None


BATCHED_VARIANTS = {"default": 0, "tile16": 1, "runtime_degree": 2, "degree_split": 3, "one_lane": 4}


def sph_batched_set_config(l_max: int, normalize: bool, dtype: torch.dtype, store_dY: bool,
                           with_backward: bool, variant: str = "default", blocks_per_cu: int = 0):
    """Fix the batched launch of a combination (include/sph.h: sph_batched_set_config)."""
    if variant not in BATCHED_VARIANTS:
        raise SphError(SPH_ERR_INVALID, f"unknown variant {variant!r}")
    code = SPH_F64 if dtype == torch.float64 else SPH_F32
    _check(lib().sph_batched_set_config(int(l_max), int(bool(normalize)), code, int(bool(store_dY)),
                                        int(bool(with_backward)), BATCHED_VARIANTS[variant], int(blocks_per_cu)))
