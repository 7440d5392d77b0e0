"""Plain FP64 CPU oracle for the RPA correlation energy path (chi0 and E_c).

TEST INFRASTRUCTURE ONLY. Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import or run anything in this package. The
product path (the HIP library and its Python binding) never calls it and
shares no code, tables or helpers with it.

Every function follows one passage of Yan, Li and O'Grady, "Graphics
Processing Unit Acceleration of the Random Phase Approximation in the
Projector Augmented Wave Method" (arXiv 1307.8052), cited by section and
equation label. Readings of passages that are silent or ambiguous are listed
in the module docstring of :mod:`oracle.rpa`.

Parity status: every function is pinned by a test in ``tests/test_oracle_pins.py``
except the PAW nabla table D of the optical limit beyond its two-level and
self-consistency checks, which is synthetic (parity unpinned against any
printed number: the paper prints no chi0 or E_c values).
"""
from .rpa import *  # noqa: F401,F403
