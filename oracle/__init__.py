"""FP64 CPU oracle of the Batch-FPM hot path.

Test infrastructure only: imported by the tests, the smoke check and the CPU
baseline leg of the benchmark, never by the product package.
"""
from . import fpm_oracle  # noqa: F401
