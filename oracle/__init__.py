"""FP64 CPU oracle for the EE2 / LIM Cahn-Hilliard time steps.

Test infrastructure only: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.
"""
from .ch_oracle import *  # noqa: F401,F403
