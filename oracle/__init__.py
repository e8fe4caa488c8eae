"""Plain CPU FP64 oracle for the partitioned network expansion.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, calls or
links anything in this package; only the tests, the smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code with the GPU path:
its own message passing, its own explicit oblique P/Q projectors (no gauge or
slice trick), its own cluster enumerator and an explicit enumeration of every
retained configuration.

Parity status of each function is stated in its docstring; every function is
pinned by at least one test in ``tests/test_oracle_*.py`` against values the
mathematics fixes (brute-force spin sums, high-temperature closed forms, the
complete-expansion identity, ring and tree special cases, count formulas).
"""

from .pne_oracle import (  # noqa: F401
    bp_messages,
    projectors,
    vacuum,
    dangling_max,
    enumerate_clusters,
    cluster_weight,
    enumerate_collections,
    cumulant_sum,
    pne_contract,
    literal_term,
    OracleResult,
)
from .exact import (  # noqa: F401
    exact_contract,
    exact_log_contract,
    ising_bruteforce_logz,
    full_expansion_sum,
)
