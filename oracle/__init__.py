"""CPU FP64 oracle for the online CP hot path (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The product path (the HIP library and its binding) never calls
it and shares no code with it.
"""
from .octen_oracle import *  # noqa: F401,F403
