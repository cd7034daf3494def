"""CPU oracle for BDD min-marginal averaging (test infrastructure only).

A plain, slow, single-threaded fp64 reference written from the paper (Lange &
Swoboda, ICML 2021), with an fp32 mirror of the same steps. Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may use it; the
product library never does. It takes problem arrays duck-typed (``n``,
``cost``, ``row_ptr``, ``col``, ``coef``, ``sense``, ``rhs``, ``order``) and
imports nothing from the product package.
"""
from .core import Oracle, OracleError, build_row, ORC_CHECK_ALL  # noqa: F401
