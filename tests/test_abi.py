"""The C ABI on the CPU: the library loads, exports every symbol the header
declares, and rejects bad arguments on the host before touching a device.
No call here reaches a kernel launch."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2302_08381_amd", "libsph.so")
HEADER = os.path.join(ROOT, "include", "sph.h")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libsph.so not built")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sph_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2302_08381_amd import _native
    return _native.lib()


def test_header_declares_the_documented_entry_points():
    names = header_functions()
    for required in ("sph_compute", "sph_compute_with_gradients", "sph_backward",
                     "sph_double_backward", "sph_batched_compute", "sph_radial_expansion",
                     "sph_compute_with_hessians"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    raw = ctypes.CDLL(LIB)
    for name in header_functions():
        assert hasattr(raw, name), name


def test_binding_covers_every_declared_symbol():
    from paper_2302_08381_amd import _native
    assert set(header_functions()) <= set(_native._SIGNATURES)


def test_metadata(lib):
    assert lib.sph_max_lmax() == 32
    assert lib.sph_num_components(8) == 81
    assert lib.sph_num_components(0) == 1
    assert lib.sph_num_components(-1) == -1
    assert lib.sph_status_string(0) == b"success"
    assert lib.sph_status_string(4) == b"inconsistent CSR offsets"
    assert lib.sph_status_string(99) == b"unknown status"
    assert b"gfx950" in lib.sph_version()


FAKE = ctypes.c_void_p(0x10000)  # never dereferenced: every case fails validation first


@pytest.mark.parametrize("args,code", [
    ((FAKE, -1, 4, 0, 0, FAKE, None), 2),      # n < 0
    ((FAKE, 10, -1, 0, 0, FAKE, None), 3),     # l_max < 0
    ((FAKE, 10, 33, 0, 0, FAKE, None), 3),     # l_max too large
    ((FAKE, 10, 4, 2, 0, FAKE, None), 2),      # normalize not 0/1
    ((FAKE, 10, 4, 0, 7, FAKE, None), 2),      # bad dtype
    ((None, 10, 4, 0, 0, FAKE, None), 1),      # xyz NULL
    ((FAKE, 10, 4, 0, 0, None, None), 1),      # Y NULL
    ((None, 0, 4, 0, 0, None, None), 0),       # n = 0: nothing to do
])
def test_compute_validation(lib, args, code):
    assert lib.sph_compute(*args) == code
    if code:
        assert len(lib.sph_last_error()) > 0


@pytest.mark.parametrize("args,code", [
    ((FAKE, -1, 4, 0, 0, FAKE, None, FAKE, None), 2),      # n < 0
    ((FAKE, 10, 33, 0, 0, FAKE, None, FAKE, None), 3),     # l_max too large
    ((FAKE, 10, 4, 3, 0, FAKE, None, FAKE, None), 2),      # normalize not 0/1
    ((FAKE, 10, 4, 0, 2, FAKE, None, FAKE, None), 2),      # bad dtype
    ((None, 10, 4, 0, 0, FAKE, None, FAKE, None), 1),      # xyz NULL
    ((FAKE, 10, 4, 0, 0, None, None, FAKE, None), 1),      # Y NULL
    ((FAKE, 10, 4, 0, 0, FAKE, None, None, None), 1),      # d2Y NULL
    ((None, 0, 4, 0, 0, None, None, None, None), 0),       # n = 0: nothing to do
])
def test_hessian_validation(lib, args, code):
    assert lib.sph_compute_with_hessians(*args) == code
    if code:
        assert len(lib.sph_last_error()) > 0


def test_hessian_overlap_is_rejected(lib):
    base = 0x200000
    # d2Y [10,3,3,25] float starting inside Y [10,25]
    st = lib.sph_compute_with_hessians(ctypes.c_void_p(0x100000), 10, 4, 1, 0, ctypes.c_void_p(base), None,
                                       ctypes.c_void_p(base + 400), None)
    assert st == 2 and b"overlaps" in lib.sph_last_error()


def test_overlap_is_rejected(lib):
    base = 0x100000
    # Y starts inside xyz
    st = lib.sph_compute(ctypes.c_void_p(base), 100, 2, 0, 0, ctypes.c_void_p(base + 64), None)
    assert st == 2 and b"overlaps" in lib.sph_last_error()


def test_backward_validation(lib):
    assert lib.sph_backward(FAKE, None, 5, 3, 0, FAKE, None) == 1
    assert lib.sph_backward(FAKE, FAKE, 5, 40, 0, FAKE, None) == 3
    assert lib.sph_backward(None, None, 0, 3, 0, None, None) == 0


def test_double_backward_validation(lib):
    assert lib.sph_double_backward(FAKE, None, FAKE, 5, 3, 0, 0, FAKE, None, None) == 1
    assert lib.sph_double_backward(FAKE, FAKE, FAKE, 5, 3, 3, 0, FAKE, None, None) == 2
    # nothing requested: a no-op
    assert lib.sph_double_backward(FAKE, FAKE, FAKE, 5, 3, 0, 0, None, None, None) == 0


def test_batched_validation(lib):
    b = lib.sph_batched_compute
    assert b(FAKE, None, 3, 10, 3, 1, 0, FAKE, None, None, None, None, None) == 1      # offsets NULL
    assert b(FAKE, FAKE, -1, 10, 3, 1, 0, FAKE, None, None, None, None, None) == 2     # n_env < 0
    assert b(FAKE, FAKE, 3, 10, 3, 1, 0, FAKE, None, FAKE, None, None, None) == 1      # grad_Y w/o grad_xyz
    assert b(FAKE, FAKE, 3, 10, 3, 1, 0, FAKE, None, None, FAKE, None, None) == 2      # grad_xyz w/o grad_Y
    assert b(FAKE, FAKE, 3, 0, 3, 1, 0, FAKE, None, None, None, None, None) == 0       # nothing to do


def test_set_options_validation(lib):
    assert lib.sph_batched_set_options(2, 0) == 2


def test_set_config_validation(lib):
    """Every case fails validation before any device call."""
    c = lib.sph_batched_set_config
    assert c(33, 1, 0, 1, 1, 0, 0) == 3        # l_max out of range
    assert c(8, 2, 0, 1, 1, 0, 0) == 2         # normalize
    assert c(8, 1, 7, 1, 1, 0, 0) == 2         # dtype
    assert c(8, 1, 0, 2, 1, 0, 0) == 2         # store_dY flag
    assert c(8, 1, 0, 1, 1, 4, 0) == 2         # unknown variant
    assert c(8, 1, 0, 1, 1, 3, 0) == 2         # degree_split does not exist for float l_max = 8
    assert c(3, 1, 1, 1, 1, 3, 0) == 2         # ... nor for double l_max = 3
    assert c(8, 1, 0, 1, 1, 0, 65) == 2        # blocks_per_cu
    assert c(13, 1, 0, 1, 1, 1, 0) == 2        # tile16 does not exist past the unrolled kernels
    assert c(9, 1, 1, 1, 1, 1, 0) == 2         # ... (double: l_max <= 8)
    assert c(8, 1, 0, 0, 0, 1, 0) == 2         # ... nor for the values-only kernel
    assert c(20, 1, 0, 0, 0, 2, 0) == 2        # values only: runtime_degree is the default at l_max = 20
    assert c(20, 1, 0, 1, 1, 3, 0) == 2        # no degree split with the fused backward past l_max = 12


def test_radial_expansion_validation(lib):
    """Every case fails (or finishes) on the host before any device call."""
    x = lib.sph_radial_expansion
    #        xyz   offs  n_env n   R     n_max L  norm dt  c     status stream
    assert x(FAKE, None, 3, 10, FAKE, 8, 4, 1, 0, FAKE, None, None) == 1    # offsets NULL
    assert x(FAKE, FAKE, -1, 10, FAKE, 8, 4, 1, 0, FAKE, None, None) == 2   # n_env < 0
    assert x(FAKE, FAKE, 3, 10, FAKE, 0, 4, 1, 0, FAKE, None, None) == 2    # n_max < 1
    assert x(FAKE, FAKE, 3, 10, FAKE, 65, 4, 1, 0, FAKE, None, None) == 2   # n_max > 64
    assert x(FAKE, FAKE, 3, 10, FAKE, 8, 33, 1, 0, FAKE, None, None) == 3   # l_max
    assert x(FAKE, FAKE, 3, 10, FAKE, 8, 4, 2, 0, FAKE, None, None) == 2    # normalize
    assert x(FAKE, FAKE, 3, 10, FAKE, 8, 4, 1, 5, FAKE, None, None) == 2    # dtype
    assert x(FAKE, FAKE, 3, 10, FAKE, 8, 4, 1, 0, None, None, None) == 1    # c NULL
    assert x(FAKE, FAKE, 3, 10, None, 8, 4, 1, 0, FAKE, None, None) == 1    # R NULL
    assert x(FAKE, FAKE, 0, 10, FAKE, 8, 4, 1, 0, None, None, None) == 0    # no environments, no status
    # l_max = 32 with 64 double channels: the 8-point chunk needs > 160 KiB of LDS
    assert x(FAKE, FAKE, 3, 10, FAKE, 64, 32, 1, 1, FAKE, None, None) == 2
    assert b"LDS" in lib.sph_last_error()


def test_radial_expansion_backward_validation(lib):
    x = lib.sph_radial_expansion_backward
    #        xyz   offs  n_env n   R     n_max L  norm dt gc    gx    gR    status stream
    assert x(FAKE, None, 3, 10, FAKE, 8, 4, 1, 0, FAKE, FAKE, None, None, None) == 1    # offsets NULL
    assert x(FAKE, FAKE, 3, 10, FAKE, 17, 4, 1, 0, FAKE, FAKE, None, None, None) == 2   # n_max > 16
    assert x(FAKE, FAKE, 3, 10, FAKE, 8, 4, 1, 0, None, FAKE, None, None, None) == 1    # grad_c NULL
    assert x(FAKE, FAKE, 3, 10, FAKE, 8, 40, 1, 0, FAKE, FAKE, None, None, None) == 3   # l_max
    assert x(FAKE, FAKE, 3, 10, FAKE, 8, 4, 1, 0, FAKE, None, None, None, None) == 0    # nothing requested


def test_e3nn_entry_points_validation(lib):
    """Every case fails validation before any device call."""
    assert lib.sph_e3nn_coordinates(FAKE, -1, 0, FAKE, None) == 2          # n < 0
    assert lib.sph_e3nn_coordinates(FAKE, 5, 3, FAKE, None) == 2           # dtype
    assert lib.sph_e3nn_coordinates(None, 5, 0, FAKE, None) == 1           # NULL input
    assert lib.sph_e3nn_coordinates(None, 0, 0, None, None) == 0           # nothing to do
    base = 0x100000
    assert lib.sph_e3nn_coordinates(ctypes.c_void_p(base), 10, 0, ctypes.c_void_p(base + 8), None) == 2  # overlap
    assert lib.sph_e3nn_convert(5, 4, 3, 0, FAKE, None, None) == 2         # normalization
    assert lib.sph_e3nn_convert(5, 33, 0, 0, FAKE, None, None) == 3        # l_max
    assert lib.sph_e3nn_convert(5, 4, 0, 0, None, None, None) == 1         # Y required
    assert lib.sph_e3nn_convert(10, 2, 1, 0, ctypes.c_void_p(base), ctypes.c_void_p(base + 64), None) == 2
    assert lib.sph_e3nn_convert(0, 2, 1, 0, None, None, None) == 0
