"""Plain FP64 CPU oracle for GLS map-making.

Test infrastructure only: the tests, the smoke check and the benchmark's
CPU-baseline leg use it; the product path never does.
"""
from .mapmaking import *  # noqa: F401,F403
