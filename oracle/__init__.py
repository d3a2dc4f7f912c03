"""FP64 CPU oracle of the spectral path tracer (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the HIP library; the two meet
only through the seeded input generators in ``paper_1912_05494_amd.synth``.

Parity status of each function (see the pin tests under ``tests/``):
  philox        pinned: bit-exact against rocRAND's host-callable Philox.
  fresnel/slab  pinned: closed forms (normal incidence, Brewster angle,
                lossless slab, absorbed-fraction identity, index-matched
                Beer-Lambert) and mpmath at 30 digits.
  intersect     pinned: BVH equals brute force; analytic hits.
  render        pinned: white-furnace and sun-only closed forms, band/tile
                invariance, gray-channel invariance, independent Python path
                for tiny images.
"""
from .binding import *  # noqa: F401,F403
