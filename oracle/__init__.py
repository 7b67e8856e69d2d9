"""FP64 CPU oracle for VQ-NNF template matching.

Test infrastructure only: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.
"""
from . import vqnnf_oracle  # noqa: F401
