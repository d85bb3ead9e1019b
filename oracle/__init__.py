"""FP64 CPU oracle for the EPLL restoration path.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the restoration library.  It shares
no code with the GPU path; both only consume the seeded inputs drawn by
``fepll_synth``.
"""
from . import epll64  # noqa: F401
