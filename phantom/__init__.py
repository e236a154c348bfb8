"""Seeded synthetic inputs shared by the tests, the oracle checks and the benchmark.

This package only *generates input volumes* (and their known fibre geometry);
it holds none of the structure-tensor arithmetic, so both the HIP path and the
CPU oracle can consume its output without sharing any of the method's code.
"""

from .helix import (  # noqa: F401
    Annulus,
    PhantomSpec,
    generate,
    helix_angle,
    spec_small_f32,
    spec_headline_u16,
    spec_two_annuli_u16,
)
