"""CPU FP64 oracle for UoI_LASSO / UoI_VAR -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (``paper_1808_06992_amd``) never
imports it and shares no code with it.
"""
from .oracle import *  # noqa: F401,F403
from .oracle import build  # noqa: F401
