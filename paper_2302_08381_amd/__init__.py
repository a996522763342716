"""Real spherical harmonics on MI355X (gfx950) after arXiv:2302.08381.

The arithmetic lives in libsph.so (HIP kernels behind the C ABI of
include/sph.h).  This package is its thin Python face:

* :mod:`._native` -- one function per C entry point, same names
  (``sph_compute``, ``sph_compute_with_gradients``, ``sph_backward``,
  ``sph_double_backward``, ``sph_batched_compute``, ``sph_radial_expansion``
  ...), torch tensors in,
  raw device pointers and the current HIP stream out;
* :mod:`.autograd` -- ``spherical_harmonics`` / ``SphericalHarmonics`` with
  first and second derivatives, and ``e3nn_spherical_harmonics`` in e3nn's
  conventions (first derivatives).

Building: ``python -m paper_2302_08381_amd.build`` (hipcc, in-tree).
"""
from ._native import (  # noqa: F401
    SphError,
    library_path,
    max_lmax,
    num_components,
    sph_backward,
    sph_batched_compute,
    sph_batched_get_config,
    sph_batched_set_config,
    sph_batched_set_options,
    sph_compute,
    sph_compute_with_gradients,
    sph_compute_with_hessians,
    sph_double_backward,
    sph_e3nn_convert,
    sph_e3nn_coordinates,
    sph_radial_expansion,
    sph_radial_expansion_backward,
    version,
)
from .autograd import (  # noqa: F401
    SphericalHarmonics,
    e3nn_spherical_harmonics,
    e3nn_spherical_harmonics_with_gradients,
    spherical_harmonics,
    spherical_harmonics_with_gradients,
)
