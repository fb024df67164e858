"""FP64 CPU oracle for the Ohta-Kawasaki Newton-Krylov timestep.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg import this package; the product library never does.
"""
from .okref import Oracle, OracleParams, OracleInfo, local_residual, local_jacobian  # noqa: F401
