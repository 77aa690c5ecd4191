"""CPU FP64 reference (the oracle) for the PDHG + corner-push path.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU leg of the benchmark, never by the product library.  It shares no code
with the HIP path.
"""
from .oracle import (  # noqa: F401
    OracleSolver,
    OrKKT,
    OrParams,
    OrPushResult,
    OrResult,
    build_oracle,
    num_threads,
    push_uniform,
    restart_decision,
    set_threads,
    kkt_weighted,
    weight_update,
    splitmix64,
    STATUS,
)
