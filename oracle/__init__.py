"""FP64 CPU oracle for FRAM -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct numpy implementation of what the GPU path
computes.  Only the test suite, the smoke check and the benchmark's CPU
baseline may import it; the library and its Python binding never do.  It
shares no code with the HIP path.
"""
from .fram64 import (  # noqa: F401
    prescale, p1, p2, p3, sdsn, fram, discretize, objective, accuracy, solve,
    SdsnInfo, FramInfo,
)
