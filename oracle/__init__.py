"""Plain, slow CPU oracle for the real spherical harmonics of arXiv:2302.08381.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute anything in this package: only the tests, the smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code, tables or
constants with the HIP library.

Two tiers compute the same closed-form functions (the method reaches them
exactly, up to rounding; Sec. II):

* :mod:`oracle.definition` -- the definition written out.  Each solid harmonic
  r^l Y_l^m is expanded into an explicit polynomial in x, y, z with exact
  rational coefficients (Eqs. real-sh-spherical and Flm with the textbook
  Ferrers function), so values, gradients and Hessians are exact polynomial
  arithmetic.  Evaluated either in mpmath at any precision, or vectorised in
  numpy ``longdouble`` where cancellation is mild (small l).
* :mod:`oracle.recurrence` -- the bulk tier: the textbook spherical-coordinate
  route (Eq. recur-p, Condon-Shortley phase) in numpy ``longdouble``, with the
  gradient from textbook pole-free Ferrers identities.  Stable at any l <= 32.
* :mod:`oracle.derived` -- backward and double-backward contractions, the
  radial expansion over environments (Eq. expansion), e3nn's conventions
  (Sec. III.B, a reading: pinned by the degree-1 identity, normalisation
  sums, the polar axis and finite differences; beyond those pins parity
  unpinned, e3nn not being installed) and the per-l error metric, built on
  the two tiers.

Pins (tests marked ``not gpu``) tie both tiers to closed forms, library
routines (mpmath), invariants (addition theorems, orthonormality, harmonicity,
Euler homogeneity) and finite differences.
"""
from .definition import (  # noqa: F401
    prefactor,
    solid_poly,
    definition_eval_mp,
    definition_eval_ld,
)
from .recurrence import real_sph, ferrers_table  # noqa: F401
from .derived import (  # noqa: F401
    backward,
    double_backward,
    hessian_contract,
    radial_expansion,
    radial_expansion_backward,
    e3nn_convention,
    per_l_errors,
    component_scales,
)
