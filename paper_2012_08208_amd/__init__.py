"""MI355X (gfx950) SIMP topology optimisation: matrix-free P1 FE solve,
compliance sensitivity, distance-weighted filter and OC update as HIP
kernels behind a C ABI (``include/topo.h``), after arXiv 2012.08208."""

from .binding import (  # noqa: F401
    Topo, Batch, EdmFilter, UMesh, TopoError, make_problem, load_library, status_string, check_exports,
    TOPO_SPLIT_ALT_ROWS, TOPO_SPLIT_UNIFORM, TOPO_FP64, TOPO_MIXED_FP32, TOPO_MIXED_IR,
    TOPO_MIXED_BF16, TOPO_MIXED_RU, TOPO_PASSIVE_FREE, TOPO_PASSIVE_VOID, TOPO_PASSIVE_SOLID,
    TOPO_FILTER_DISTANCE, TOPO_FILTER_HELMHOLTZ, TOPO_FILTER_DENSITY,
    TOPO_PC_JACOBI, TOPO_PC_GMG, TOPO_PC_LEARNED, TOPO_SYNC_POLL, TOPO_SYNC_NONE, TOPO_S_LEARNED_FALLBACK, SOLVE_INFO_LEN,
    LOG_LEN, LIB_PATH, num_params, BATCH_REC_LEN, oc_update_noalloc, OC_NOALLOC_MAX_CELLS,
)
