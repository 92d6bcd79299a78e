"""MI355X (gfx950) implementation of the static Louvain method's hot path.

The local-moving phase (synchronous rule, exact integer gains), the aggregation phase and the
modularity reduction of section 3.2 of Sahu, "Enhancing Efficiency in Parallel Louvain
Algorithm for Community Detection" (arXiv 2301.12390), as hand-written HIP kernels behind the C
ABI in ``include/louvain.h``. ``louvain`` is the Python binding.
"""

from .louvain import (  # noqa: F401
    LV_COLOR_CLASSES,
    LV_FORCE_WIDE,
    LV_GRAPH_REPLAY,
    LV_PREP_MAX,
    LV_PREP_PAPER,
    LV_PREP_SELF_LOOPS,
    LV_PREP_SYMMETRIZE,
    LV_SMALL_PARTS,
    LV_TRACE,
    LV_VALIDATE,
    Louvain,
    LouvainError,
    PreparedGraph,
    Server,
    load_library,
)
