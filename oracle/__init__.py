"""CPU oracle of the reacting-flow right-hand side.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.
"""
from .oracle import Oracle, build_oracle, OracleError  # noqa: F401
