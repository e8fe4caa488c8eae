"""MI355X (gfx950) partitioned network expansion: C-ABI library + thin binding.

The hot path (BP sweeps, bond gauge, excited slices, cluster contractions and
the FP64 cross-term sum) runs in hand-written HIP kernels inside libpne.so;
this package only marshals arguments.  Importing it does not load the
library; the first Context (or enumerate_clusters) call does, and fails
loudly if libpne.so has not been built.
"""

from .pne import (  # noqa: F401
    Batch,
    Context,
    Network,
    PNEError,
    Result,
    Prepared,
    Server,
    enumerate_clusters,
    count_configurations,
    load_library,
    LIB_PATH,
    PATH_BLOCK_GAUGE,
    PATH_BLOCK_TERMS,
    PATH_PERSISTENT,
    PRECISIONS,
    MODES,
    PNE_OK,
    PNE_WARN_BP_NOT_CONVERGED,
    PNE_WARN_PRECISION,
    PNE_ERR_NOT_READY,
    PNE_ERR_CANCELLED,
    PNE_ERR_CHECK,
)
