"""FP64 CPU oracle of the axisymmetric D2Q9 + D2Q4 LBGK-LES step.

TEST INFRASTRUCTURE ONLY: the checker of the HIP path.  Only the tests, the
smoke check and the CPU-baseline leg of the benchmark may import it.
"""
from .oracle import RefSolver, OracleError, build, load, feq, geq, table_lookup  # noqa: F401
