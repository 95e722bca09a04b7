"""Seeded synthetic inputs for the multi-messenger Wiener filter.

This package only draws test and benchmark inputs (spectra, noise maps, masks
and a data realisation).  It holds none of the filter's arithmetic, so both the
CPU oracle and the GPU library can be fed from it without sharing any solver
code.
"""

from .maps import (  # noqa: F401
    ARCMIN,
    Problem,
    l_of_modes,
    make_problem,
    make_problems,
    make_stationary_problem,
    named_config,
    pixel_size_rad,
    uneven_batch,
)
