"""FP64 CPU oracle for the reduced Navier-Stokes online stage.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the CPU-baseline
leg of ``bench.py``; never by the product path. It shares no code with the HIP library.
"""

from .oracle import (  # noqa: F401
    build_oracle, load_oracle, OracleSet, theta, gepp_solve, newton, picard, pressure,
    solve_batch, STATUS,
)
