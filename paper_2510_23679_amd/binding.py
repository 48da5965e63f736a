"""ctypes binding of libpdp.so with the C-ABI's names.

Only argument marshalling lives here: every step of the path runs in the HIP
kernels behind the C-ABI.  PyTorch provides device memory (``torch.empty`` on
the ROCm device) and streams (``torch.cuda.current_stream().cuda_stream``).
If the library is missing this module raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpdp.so")

u32, u64, i32, vp = C.c_uint32, C.c_uint64, C.c_int32, C.c_void_p

PDP_OK = 0
PDP_E_INVAL = -1
PDP_E_KRANGE = -2
PDP_E_WORKSPACE = -3
PDP_E_CAPACITY = -4
PDP_E_ALPHABET = -5
PDP_E_HIP = -6
PDP_E_BUDGET = -7
PDP_E_LIMIT = -8
PDP_E_UNIMPL = -9

PDP_TASK_AB = 1
PDP_TASK_BA = 2
PDP_TASK_BBH = 4
PDP_PARAM_PERSISTENT = 1
PDP_PARAM_COLMAX = 2
PDP_PARAM_TWO_PASS = 4
PDP_STATUS_TWO_PASS = 1
PDP_K_MAX = 12
PDP_K_MAX_NT = 31
PDP_ALPHA_AMINO = 0
PDP_ALPHA_NUCLEOTIDE = 1
# alphabet names used by the Python side
ALPHABET_IDS = {"aa": PDP_ALPHA_AMINO, "nt": PDP_ALPHA_NUCLEOTIDE}


def alphabet_id(alphabet) -> int:
    """pdp_alphabet value of "aa" (amino acids) or "nt" (nucleotides)."""
    if alphabet not in ALPHABET_IDS:
        raise ValueError(f"unknown alphabet {alphabet!r} (expected 'aa' or 'nt')")
    return ALPHABET_IDS[alphabet]
PDP_MAX_WINDOWS = 65535
PDP_MAX_WINDOWS_LONG = 2147483647
PDP_DICT_LONG_GENES = 1  # pdp_dict_bind flag: genes up to PDP_MAX_WINDOWS_LONG windows (the long-gene path)

# kernels that pdp_plan_timer_start can time
PDP_NOALLOC_SCRATCH_BYTES = 64 << 20  # include/pdp.h: the fixed scratch of pdp_bh_noalloc

KERNELS = {"join": 0, "bucket": 1, "tile_count": 2, "tile_write": 3, "bbh": 4, "all": 5, "join_backup": 6}


class pdp_status(C.Structure):
    _fields_ = [("code", i32), ("flags", u32), ("needed", u64), ("where", u64)]


class pdp_genome(C.Structure):
    _fields_ = [("residues", vp), ("gene_off", vp), ("n_genes", u32), ("reserved", u32), ("n_residues", u64)]


class pdp_dict(C.Structure):
    _fields_ = [("n_genes", u32), ("k", u32), ("capacity", u64), ("n_buckets", u32), ("key_shift", u32),
                ("alphabet", u32), ("lead", u32), ("flags", u32), ("reserved", u32), ("nwin", vp), ("mv_ptr", vp), ("mv_code", vp), ("mv_cnt", vp), ("ix_dir", vp),
                ("ix_code", vp), ("ix_gene", vp), ("ix_cnt", vp), ("ix_key", vp), ("status", vp)]


class pdp_bh_out(C.Structure):
    _fields_ = [("n_rows", u32), ("reserved", u32), ("capacity", u64), ("ptr", vp), ("col", vp), ("num", vp),
                ("den", vp)]


class pdp_bbh_out(C.Structure):
    _fields_ = [("n_rows", u32), ("reserved", u32), ("capacity", u64), ("ptr", vp), ("a", vp), ("b", vp),
                ("num", vp), ("den", vp)]


class pdp_params(C.Structure):
    _fields_ = [("inc_capacity", u64), ("tile_rows", u32), ("join_entries", u32), ("lds_budget", u32),
                ("flags", u32), ("theta_num", u32), ("theta_den", u32), ("tau_num", u32), ("tau_den", u32)]


class pdp_task(C.Structure):
    _fields_ = [("a", C.POINTER(pdp_dict)), ("b", C.POINTER(pdp_dict)), ("flags", u32), ("reserved", u32)]


class pdp_plan_info(C.Structure):
    _fields_ = [("ws_bytes", u64), ("inc_capacity", u64), ("bh_rows", u32), ("bbh_rows", u32), ("n_tasks", u32),
                ("join_groups", u32), ("tiles", u32), ("tile_lds", u32), ("long_rows", u32), ("reserved", u32)]


class pdp_tune_result(C.Structure):
    _fields_ = [("best", pdp_params), ("best_ms", C.c_double), ("first_ms", C.c_double), ("tried", u32),
                ("reserved", u32)]


class pdp_server_config(C.Structure):
    _fields_ = [("budget_bytes", u64), ("slots", u32), ("k", u32), ("alphabet", u32), ("reserved", u32),
                ("params", pdp_params)]


class pdp_request_done(C.Structure):
    _fields_ = [("tag", u64), ("code", i32), ("n_genes", u32), ("attempts", u32), ("flags", u32),
                ("submit_us", C.c_double), ("admit_us", C.c_double), ("done_us", C.c_double),
                ("bh_entries", u64), ("bbh_pairs", u64), ("h2d_ms", C.c_float), ("build_ms", C.c_float),
                ("pairs_ms", C.c_float), ("d2h_ms", C.c_float)]


_P32 = C.POINTER(u32)


class pdp_request_result(C.Structure):
    _fields_ = [("code", i32), ("n_residents", u32), ("status", pdp_status), ("bh_rows", u32), ("bbh_rows", u32),
                ("ab_row", _P32), ("ba_row", _P32), ("bbh_row", _P32),
                ("bh_ptr", _P32), ("bh_col", _P32), ("bh_num", _P32), ("bh_den", _P32),
                ("bbh_ptr", _P32), ("bbh_a", _P32), ("bbh_b", _P32), ("bbh_num", _P32), ("bbh_den", _P32)]


class pdp_server_stats(C.Structure):
    _fields_ = [("admitted", u64), ("completed", u64), ("retries", u64), ("pending", u64), ("budget_bytes", u64),
                ("used_bytes", u64), ("peak_used_bytes", u64), ("inflight", u32), ("peak_inflight", u32)]


# name -> (restype, argtypes); the same names as include/pdp.h
SIGNATURES = {
    "pdp_abi_version": (u32, []),
    "pdp_strerror": (C.c_char_p, [i32]),
    "pdp_last_error": (C.c_char_p, []),
    "pdp_k_rule": (i32, [u64, u32, i32, C.POINTER(u32)]),
    "pdp_dict_size": (i32, [u32, u64, u32, u32, C.POINTER(u64), C.POINTER(u64)]),
    "pdp_dict_bind": (i32, [vp, u64, u32, u64, u32, u32, u32, C.POINTER(pdp_dict)]),
    "pdp_dict_build": (i32, [C.POINTER(pdp_genome), C.POINTER(pdp_dict), vp, u64, vp]),
    "pdp_dict_build_many_ws_size": (i32, [C.POINTER(pdp_genome), C.POINTER(C.POINTER(pdp_dict)), u32, C.POINTER(u64)]),
    "pdp_dict_build_many": (i32, [C.POINTER(pdp_genome), C.POINTER(C.POINTER(pdp_dict)), u32, vp, u64, vp]),
    "pdp_plan_create": (i32, [C.POINTER(pdp_task), u32, C.POINTER(pdp_params), C.POINTER(vp)]),
    "pdp_plan_info_get": (i32, [vp, C.POINTER(pdp_plan_info)]),
    "pdp_plan_rows": (i32, [vp, u32, C.POINTER(u32), C.POINTER(u32), C.POINTER(u32)]),
    "pdp_plan_destroy": (None, [vp]),
    "pdp_plan_upload": (i32, [vp, vp, u64, vp]),
    "pdp_plan_launch": (i32, [vp, C.POINTER(pdp_bh_out), C.POINTER(pdp_bbh_out), vp, vp, u64, vp]),
    "pdp_plan_run": (i32, [vp, C.POINTER(pdp_bh_out), C.POINTER(pdp_bbh_out), vp, vp, u64, vp]),
    "pdp_plan_families": (i32, [vp, C.POINTER(pdp_bbh_out), vp, vp, u32, vp, vp, vp, u64, vp]),
    "pdp_plan_timer_start": (i32, [vp, i32, u32]),
    "pdp_plan_timer_read": (i32, [vp, C.POINTER(C.c_double), C.POINTER(u32)]),
    "pdp_plan_timer_stop": (i32, [vp]),
    "pdp_capture_begin": (i32, [vp]),
    "pdp_capture_end": (i32, [vp, C.POINTER(vp)]),
    "pdp_graph_launch": (i32, [vp, vp]),
    "pdp_graph_destroy": (None, [vp]),
    "pdp_autotune_ws_size": (i32, [C.POINTER(pdp_task), u32, C.POINTER(pdp_params), u32, C.POINTER(u64)]),
    "pdp_autotune": (i32, [C.POINTER(pdp_task), u32, C.POINTER(pdp_params), u32, u32, C.POINTER(pdp_bh_out),
                           C.POINTER(pdp_bbh_out), vp, vp, u64, vp, C.POINTER(pdp_tune_result)]),
    "pdp_server_create": (i32, [C.POINTER(pdp_server_config), C.POINTER(C.POINTER(pdp_dict)), u32, vp, u64,
                                C.POINTER(vp)]),
    "pdp_server_submit": (i32, [vp, vp, vp, u32, u64]),
    "pdp_server_poll": (i32, [vp, C.POINTER(pdp_request_done), u32, C.POINTER(u32), u32]),
    "pdp_server_fetch": (i32, [vp, u64, C.POINTER(pdp_request_result)]),
    "pdp_server_release": (i32, [vp, u64]),
    "pdp_server_stats_get": (i32, [vp, C.POINTER(pdp_server_stats)]),
    "pdp_server_destroy": (None, [vp]),
    "pdp_bh_ws_size": (i32,[C.POINTER(pdp_dict), C.POINTER(pdp_dict), C.POINTER(pdp_params), C.POINTER(u64)]),
    "pdp_bh": (i32, [C.POINTER(pdp_dict), C.POINTER(pdp_dict), C.POINTER(pdp_params), C.POINTER(pdp_bh_out), vp, vp,
                     u64, vp]),
    "pdp_bh_noalloc": (i32, [C.POINTER(pdp_dict), C.POINTER(pdp_dict), C.POINTER(pdp_params), C.POINTER(pdp_bh_out),
                             vp, vp]),
    "pdp_bbh_ws_size": (i32, [u32, C.POINTER(u64)]),
    "pdp_bbh": (i32, [C.POINTER(pdp_bh_out), C.POINTER(pdp_bh_out), C.POINTER(pdp_bbh_out), vp, vp, u64, vp]),
}

_lib = None


class PdpError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{message} (code {code})")
        self.code = code


ABI_VERSION = 6  # the layout of the structures above; include/pdp.h defines the same number


def lib():
    """The loaded libpdp.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(the best-hit path has no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        if L.pdp_abi_version() != ABI_VERSION:
            raise RuntimeError(f"{LIB_PATH} has ABI {L.pdp_abi_version()}, this binding expects {ABI_VERSION}: "
                               "rebuild it with __graft_entry__.build()")
        _lib = L
    return _lib


def check(rc: int, what: str = "") -> None:
    if rc != PDP_OK:
        L = lib()
        msg = L.pdp_strerror(rc).decode()
        detail = L.pdp_last_error().decode()
        raise PdpError(rc, f"{what}: {msg}" + (f" ({detail})" if detail else ""))
