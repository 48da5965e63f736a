"""MI355X-native best-hit path of PanDelos-plus (k-mer dictionaries, BH with ties, BBH).

The compute path is libpdp.so (hand-written HIP for gfx950 behind a C-ABI,
declared in include/pdp.h); this package only binds it.
"""
from .binding import (  # noqa: F401
    PDP_E_ALPHABET, PDP_E_BUDGET, PDP_E_CAPACITY, PDP_E_HIP, PDP_E_INVAL, PDP_E_KRANGE, PDP_E_LIMIT,
    PDP_E_UNIMPL, PDP_E_WORKSPACE, PDP_K_MAX, PDP_MAX_WINDOWS, PDP_NOALLOC_SCRATCH_BYTES, PDP_OK, PDP_STATUS_TWO_PASS,
    PDP_DICT_LONG_GENES, PDP_MAX_WINDOWS_LONG, PDP_TASK_AB,
    PDP_TASK_BA, PDP_TASK_BBH, LIB_PATH, PdpError, lib,
)
from .api import (  # noqa: F401
    BBHOut, BHOut, DeviceGenome, Dictionary, DictionaryBatch, PairResults, PairRunner, Plan, Workspace, abi_version,
    Graph, RequestResult, Server, all_pairs_tasks, autotune, bbh, bh, bh_noalloc, dict_size, k_rule, new_status, params,
    read_status, status_flags,
)
