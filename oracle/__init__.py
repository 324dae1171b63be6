"""CPU oracle for batched link-SDF clearance -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library never does, and shares no code
with it.  See ``lsdf_oracle.c`` for what is computed and which passage of the
paper each function follows.
"""
from .oracle import *  # noqa: F401,F403
from .oracle import build_oracle, load  # noqa: F401
