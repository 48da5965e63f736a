"""Python side of the best-hit library: device buffers from PyTorch, calls through the C-ABI.

Nothing here computes any part of the path; it allocates, marshals and reads
back.  All device memory is ``torch.empty`` on the current ROCm device and
every call is enqueued on a torch stream.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import binding as B
from .binding import check, lib

_U32_MASK = 0xFFFFFFFF


def _stream_handle(stream: Optional[torch.cuda.Stream]) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _device() -> torch.device:
    if not torch.cuda.is_available():
        raise RuntimeError("the best-hit path runs on a ROCm GPU and none is visible")
    return torch.device("cuda", torch.cuda.current_device())


def abi_version() -> int:
    return int(lib().pdp_abi_version())


def k_rule(total: int, alphabet: int = 20, mode: int = 0) -> int:
    """Eq. k_length through the C-ABI (host computation, no GPU needed)."""
    k = B.u32(0)
    check(lib().pdp_k_rule(int(total), int(alphabet), int(mode), C.byref(k)), "pdp_k_rule")
    return int(k.value)


def dict_size(n_genes: int, n_residues: int, k: int, alphabet: str = "aa") -> Tuple[int, int]:
    arena, ws = B.u64(0), B.u64(0)
    check(lib().pdp_dict_size(int(n_genes), int(n_residues), int(k), B.alphabet_id(alphabet), C.byref(arena),
                              C.byref(ws)), "pdp_dict_size")
    return int(arena.value), int(ws.value)


class Workspace:
    """A growable device scratch buffer shared by calls on one stream."""

    def __init__(self, nbytes: int = 0):
        self.buf = None
        self.ensure(nbytes)

    def ensure(self, nbytes: int) -> "Workspace":
        nbytes = max(int(nbytes), 256)
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = torch.empty(nbytes, dtype=torch.uint8, device=_device())
        return self

    @property
    def ptr(self) -> int:
        return self.buf.data_ptr()

    @property
    def nbytes(self) -> int:
        return self.buf.numel()


def _view(arena: torch.Tensor, ptr: int, count: int, dtype: torch.dtype) -> torch.Tensor:
    itemsize = torch.empty(0, dtype=dtype).element_size()
    off = ptr - arena.data_ptr()
    return arena[off:off + count * itemsize].view(dtype)


class DeviceGenome:
    """A genome's letters (ASCII) and gene offsets in device memory; alphabet "aa" (amino
    acids) or "nt" (nucleotides)."""

    def __init__(self, residues: np.ndarray, offsets: np.ndarray, alphabet: str = "aa"):
        B.alphabet_id(alphabet)
        self.alphabet = alphabet
        dev = _device()
        res = np.ascontiguousarray(residues, dtype=np.uint8)
        off = np.ascontiguousarray(offsets, dtype=np.uint64)
        self.residues = torch.from_numpy(res if res.size else np.zeros(1, np.uint8)).to(dev)
        self.offsets = torch.from_numpy(off.view(np.int64)).to(dev)
        self.n_genes = int(off.shape[0] - 1)
        self.n_residues = int(off[-1]) if off.size else 0
        self.longest = int(np.diff(off).max()) if self.n_genes else 0  # letters of the longest gene

    def long_genes(self, k: int) -> bool:
        """True when a gene has more than PDP_MAX_WINDOWS k-mer windows (the long-gene path)."""
        return self.longest >= k and self.longest - k + 1 > B.PDP_MAX_WINDOWS

    @classmethod
    def of(cls, genome) -> "DeviceGenome":
        return cls(genome.residues, genome.offsets, getattr(genome, "alphabet", "aa"))

    def struct(self) -> B.pdp_genome:
        return B.pdp_genome(self.residues.data_ptr(), self.offsets.data_ptr(), self.n_genes, 0, self.n_residues)


def read_status(t: torch.Tensor) -> Tuple[int, int, int]:
    """(code, needed, where) of a pdp_status held in a 24-byte device tensor (synchronises)."""
    raw = t.detach().cpu().numpy().view(np.uint8)[:24].tobytes()
    st = B.pdp_status.from_buffer_copy(raw)
    return int(st.code), int(st.needed), int(st.where)


def status_flags(t: torch.Tensor) -> int:
    """pdp_status.flags of a status tensor (PDP_STATUS_*; synchronises)."""
    raw = t.detach().cpu().numpy().view(np.uint8)[:24].tobytes()
    return int(B.pdp_status.from_buffer_copy(raw).flags)


def new_status() -> torch.Tensor:
    return torch.zeros(32, dtype=torch.uint8, device=_device())


class Dictionary:
    """The k-mer dictionary of one genome (multiplicity vectors + inverted index), on device."""

    def __init__(self, n_genes: int, n_residues: int, k: int, alphabet: str = "aa", long_genes: bool = False):
        arena_bytes, ws_bytes = dict_size(n_genes, n_residues, k, alphabet)
        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device=_device())
        self.d = B.pdp_dict()
        flags = B.PDP_DICT_LONG_GENES if long_genes else 0
        check(lib().pdp_dict_bind(self.arena.data_ptr(), arena_bytes, int(n_genes), int(n_residues), int(k),
                                  B.alphabet_id(alphabet), flags, C.byref(self.d)), "pdp_dict_bind")
        self.long_genes = bool(long_genes)
        self.ws_bytes = ws_bytes
        self.k = int(k)
        self.alphabet = alphabet
        self.n_genes = int(n_genes)
        self.n_residues = int(n_residues)
        self.genome: Optional[DeviceGenome] = None

    @classmethod
    def build_from(cls, genome, k: int, ws: Optional[Workspace] = None,
                   stream: Optional[torch.cuda.Stream] = None) -> "Dictionary":
        dg = genome if isinstance(genome, DeviceGenome) else DeviceGenome.of(genome)
        d = cls(dg.n_genes, dg.n_residues, k, dg.alphabet, long_genes=dg.long_genes(k))
        d.build(dg, ws, stream)
        return d

    def build(self, genome: DeviceGenome, ws: Optional[Workspace] = None,
              stream: Optional[torch.cuda.Stream] = None) -> None:
        ws = (ws or Workspace()).ensure(self.ws_bytes)
        self.genome = genome  # the kernels read it asynchronously
        self._ws = ws
        g = genome.struct()
        check(lib().pdp_dict_build(C.byref(g), C.byref(self.d), ws.ptr, ws.nbytes, _stream_handle(stream)),
              "pdp_dict_build")

    def status(self) -> Tuple[int, int, int]:
        return read_status(_view(self.arena, self.d.status, 24, torch.uint8))

    def check_status(self) -> None:
        code, needed, where = self.status()
        if code != 0:
            raise B.PdpError(code, f"dictionary build: {lib().pdp_strerror(code).decode()} (needed {needed}, where {where})")

    def host(self) -> dict:
        """Copies every array to host numpy (synchronises)."""
        n = self.n_genes
        out = {}
        out["nwin"] = _view(self.arena, self.d.nwin, n, torch.int32).cpu().numpy().view(np.uint32)
        out["mv_ptr"] = _view(self.arena, self.d.mv_ptr, n + 1, torch.int32).cpu().numpy().view(np.uint32)
        e = int(out["mv_ptr"][-1])
        out["mv_code"] = _view(self.arena, self.d.mv_code, e, torch.int64).cpu().numpy().view(np.uint64)
        out["mv_cnt"] = _view(self.arena, self.d.mv_cnt, e, torch.int32).cpu().numpy().view(np.uint32)
        out["ix_dir"] = _view(self.arena, self.d.ix_dir, self.d.n_buckets + 1, torch.int32).cpu().numpy().view(np.uint32)
        out["ix_code"] = _view(self.arena, self.d.ix_code, e, torch.int64).cpu().numpy().view(np.uint64)
        out["ix_gene"] = _view(self.arena, self.d.ix_gene, e, torch.int32).cpu().numpy().view(np.uint32)
        out["ix_cnt"] = _view(self.arena, self.d.ix_cnt, e, torch.int32).cpu().numpy().view(np.uint32)
        if self.d.key_shift:
            out["ix_key"] = _view(self.arena, self.d.ix_key, e, torch.int32).cpu().numpy().view(np.uint32)
        return out


class DictionaryBatch:
    """Many dictionaries built by one pdp_dict_build_many call per build()."""

    def __init__(self, genomes: Sequence[DeviceGenome], k, ws: Optional[Workspace] = None,
                 long_genes: Optional[bool] = None):
        """long_genes: bind every dictionary for long genes (True), none (False), or each one that
        holds a gene past PDP_MAX_WINDOWS windows (None)."""
        ks = list(k) if isinstance(k, (list, tuple)) else [int(k)] * len(genomes)
        self.genomes = list(genomes)
        self.dicts = [Dictionary(g.n_genes, g.n_residues, kk, g.alphabet,
                                 long_genes=g.long_genes(kk) if long_genes is None else long_genes)
                      for g, kk in zip(self.genomes, ks)]
        n = len(self.genomes)
        self._g = (B.pdp_genome * n)(*[g.struct() for g in self.genomes])
        self._d = (C.POINTER(B.pdp_dict) * n)(*[C.pointer(d.d) for d in self.dicts])
        need = B.u64(0)
        check(lib().pdp_dict_build_many_ws_size(self._g, self._d, n, C.byref(need)), "pdp_dict_build_many_ws_size")
        self.ws = (ws or Workspace()).ensure(need.value)

    def build(self, stream=None) -> None:
        check(lib().pdp_dict_build_many(self._g, self._d, len(self.dicts), self.ws.ptr, self.ws.nbytes,
                                        _stream_handle(stream)), "pdp_dict_build_many")
        for d, g in zip(self.dicts, self.genomes):
            d.genome = g

    def check_status(self) -> None:
        for d in self.dicts:
            d.check_status()


class BHOut:
    """Combined best-hit CSR output (device)."""

    def __init__(self, n_rows: int, capacity: int):
        dev = _device()
        self.n_rows = int(n_rows)
        self.capacity = int(capacity)
        self.ptr = torch.empty(self.n_rows + 1, dtype=torch.int32, device=dev)
        c = max(self.capacity, 1)
        self.col = torch.empty(c, dtype=torch.int32, device=dev)
        self.num = torch.empty(c, dtype=torch.int32, device=dev)
        self.den = torch.empty(c, dtype=torch.int32, device=dev)

    def struct(self) -> B.pdp_bh_out:
        return B.pdp_bh_out(self.n_rows, 0, self.capacity, self.ptr.data_ptr(), self.col.data_ptr(),
                            self.num.data_ptr(), self.den.data_ptr())

    def host(self):
        ptr = self.ptr.cpu().numpy().view(np.uint32)
        n = int(ptr[-1])
        return (ptr, self.col[:n].cpu().numpy().view(np.uint32), self.num[:n].cpu().numpy().view(np.uint32),
                self.den[:n].cpu().numpy().view(np.uint32))


class BBHOut:
    """Combined BBH output (device): CSR over the first genome's genes plus (a, b, num, den)."""

    def __init__(self, n_rows: int, capacity: int):
        dev = _device()
        self.n_rows = int(n_rows)
        self.capacity = int(capacity)
        self.ptr = torch.empty(self.n_rows + 1, dtype=torch.int32, device=dev)
        c = max(self.capacity, 1)
        self.a = torch.empty(c, dtype=torch.int32, device=dev)
        self.b = torch.empty(c, dtype=torch.int32, device=dev)
        self.num = torch.empty(c, dtype=torch.int32, device=dev)
        self.den = torch.empty(c, dtype=torch.int32, device=dev)

    def struct(self) -> B.pdp_bbh_out:
        return B.pdp_bbh_out(self.n_rows, 0, self.capacity, self.ptr.data_ptr(), self.a.data_ptr(), self.b.data_ptr(),
                             self.num.data_ptr(), self.den.data_ptr())

    def host(self):
        ptr = self.ptr.cpu().numpy().view(np.uint32)
        n = int(ptr[-1])
        return (ptr, self.a[:n].cpu().numpy().view(np.uint32), self.b[:n].cpu().numpy().view(np.uint32),
                self.num[:n].cpu().numpy().view(np.uint32), self.den[:n].cpu().numpy().view(np.uint32))


def params(inc_capacity: int = 0, tile_rows: int = 0, join_entries: int = 0, lds_budget: int = 0,
           persistent: bool = False, theta=None, tau=None, colmax: bool = False,
           two_pass: bool = False) -> B.pdp_params:
    """Tuning knobs and the candidate filters: theta / tau as (numerator, denominator) or None (off).
    colmax: the second genome's best hits from the column maxima of the first genome's rows.
    two_pass: the join counts its records in a pass of its own before writing them."""
    tn, td = theta if theta is not None else (0, 0)
    un, ud = tau if tau is not None else (0, 0)
    flags = (B.PDP_PARAM_PERSISTENT if persistent else 0) | (B.PDP_PARAM_COLMAX if colmax else 0) \
        | (B.PDP_PARAM_TWO_PASS if two_pass else 0)
    return B.pdp_params(int(inc_capacity), int(tile_rows), int(join_entries), int(lds_budget), flags,
                        int(tn), int(td), int(un), int(ud))


def _with_capacity(prm: B.pdp_params, capacity: int) -> B.pdp_params:
    """The same parameters with another record capacity."""
    return B.pdp_params(int(capacity), prm.tile_rows, prm.join_entries, prm.lds_budget, prm.flags, prm.theta_num,
                        prm.theta_den, prm.tau_num, prm.tau_den)


class Plan:
    """pdp_plan for a list of tasks (dictionary a, dictionary b, flags)."""

    def __init__(self, tasks: Sequence[Tuple[Dictionary, Dictionary, int]], prm: Optional[B.pdp_params] = None):
        self.dicts = [(a, b) for a, b, _ in tasks]  # keep the dictionaries alive
        arr = (B.pdp_task * len(tasks))()
        for i, (a, b, f) in enumerate(tasks):
            arr[i].a = C.pointer(a.d)
            arr[i].b = C.pointer(b.d)
            arr[i].flags = int(f)
        self.prm = prm or params()
        h = B.vp()
        check(lib().pdp_plan_create(arr, len(tasks), C.byref(self.prm), C.byref(h)), "pdp_plan_create")
        self.h = h
        info = B.pdp_plan_info()
        check(lib().pdp_plan_info_get(self.h, C.byref(info)), "pdp_plan_info_get")
        self.info = info
        self.n_tasks = len(tasks)
        self._rows = []
        for t in range(self.n_tasks):
            ab, ba, bb = B.u32(0), B.u32(0), B.u32(0)
            check(lib().pdp_plan_rows(self.h, t, C.byref(ab), C.byref(ba), C.byref(bb)), "pdp_plan_rows")
            self._rows.append((int(ab.value), int(ba.value), int(bb.value)))

    def __del__(self):
        h = getattr(self, "h", None)
        if h and h.value:
            try:
                lib().pdp_plan_destroy(h)
            except Exception:  # pragma: no cover - interpreter shutdown
                pass
            self.h = None

    def rows(self, t: int) -> Tuple[int, int, int]:
        """First row of task t in the best-hit output (AB, BA) and in the BBH output; 2^32-1 = none."""
        return self._rows[t]

    def upload(self, ws: Workspace, stream=None) -> None:
        check(lib().pdp_plan_upload(self.h, ws.ptr, ws.nbytes, _stream_handle(stream)), "pdp_plan_upload")

    def launch(self, bh: BHOut, bbh: Optional[BBHOut], status: torch.Tensor, ws: Workspace, stream=None) -> None:
        bs = bh.struct()
        bb = bbh.struct() if bbh is not None else None
        check(lib().pdp_plan_launch(self.h, C.byref(bs), C.byref(bb) if bb is not None else None,
                                    status.data_ptr(), ws.ptr, ws.nbytes, _stream_handle(stream)), "pdp_plan_launch")

    def run(self, bh: BHOut, bbh: Optional[BBHOut], status: torch.Tensor, ws: Workspace, stream=None) -> None:
        self.upload(ws, stream)
        self.launch(bh, bbh, status, ws, stream)

    def timer_start(self, kernel: int, max_launches: int) -> None:
        """HIP events around one kernel of each later launch, on the launch's own stream."""
        check(lib().pdp_plan_timer_start(self.h, int(kernel), int(max_launches)), "pdp_plan_timer_start")

    def timer_read(self) -> Tuple[float, int]:
        ms, n = C.c_double(0), B.u32(0)
        check(lib().pdp_plan_timer_read(self.h, C.byref(ms), C.byref(n)), "pdp_plan_timer_read")
        return float(ms.value), int(n.value)

    def timer_stop(self) -> None:
        check(lib().pdp_plan_timer_stop(self.h), "pdp_plan_timer_stop")


@dataclass
class PairResults:
    """Host copy of one plan run, sliced per task."""

    plan: Plan
    bh: tuple
    bbh: Optional[tuple]

    def best_hits(self, t: int, direction: int = 0):
        """(ptr, col, num, den) of task t; direction 0 = genes of a in b, 1 = genes of b in a."""
        base = self.plan.rows(t)[direction]
        if base == _U32_MASK:
            raise KeyError("task has no such direction")
        a, b = self.plan.dicts[t]
        n = (a if direction == 0 else b).n_genes
        ptr, col, num, den = self.bh
        p = ptr[base:base + n + 1].astype(np.int64)
        lo, hi = int(p[0]), int(p[-1])
        return (p - lo).astype(np.uint32), col[lo:hi], num[lo:hi], den[lo:hi]

    def bbh_pairs(self, t: int):
        """(a, b, num, den) of task t in (a, b) order."""
        base = self.plan.rows(t)[2]
        if base == _U32_MASK or self.bbh is None:
            raise KeyError("task has no BBH output")
        n = self.plan.dicts[t][0].n_genes
        ptr, a, b, num, den = self.bbh
        lo, hi = int(ptr[base]), int(ptr[base + n])
        return a[lo:hi], b[lo:hi], num[lo:hi], den[lo:hi]


class PairRunner:
    """Owns a plan with its workspace, outputs and status; grows buffers when the device reports
    PDP_E_CAPACITY and runs again."""

    def __init__(self, tasks, prm: Optional[B.pdp_params] = None, bh_capacity: Optional[int] = None,
                 bbh_capacity: Optional[int] = None):
        self.tasks = list(tasks)
        self.prm = prm or params()
        self.plan = Plan(self.tasks, self.prm)
        info = self.plan.info
        self.ws = Workspace(info.ws_bytes)
        self.bh = BHOut(info.bh_rows, bh_capacity if bh_capacity is not None else 2 * info.bh_rows + 1024)
        self.bbh = BBHOut(info.bbh_rows, bbh_capacity if bbh_capacity is not None else info.bbh_rows + 1024) \
            if info.bbh_rows else None
        self.status = new_status()
        self.fam_status = new_status()
        self.uploaded = False

    def _grow(self, where: int, needed: int) -> None:
        if where == 0:
            self.prm = _with_capacity(self.prm, int(needed * 1.25) + 1024)
            self.plan = Plan(self.tasks, self.prm)
            self.ws = Workspace(self.plan.info.ws_bytes)
            self.uploaded = False
        elif where == 1:
            self.bh = BHOut(self.plan.info.bh_rows, int(needed * 1.25) + 1024)
        elif where == 2:
            self.bbh = BBHOut(self.plan.info.bbh_rows, int(needed * 1.25) + 1024)
        else:
            raise B.PdpError(B.PDP_E_CAPACITY, f"capacity error at unknown array {where}")

    def launch(self, stream=None) -> None:
        """Enqueues one run (uploading the plan tables the first time)."""
        if not self.uploaded:
            self.plan.upload(self.ws, stream)
            self.uploaded = True
        self.plan.launch(self.bh, self.bbh, self.status, self.ws, stream)

    def run(self, stream=None, max_tries: int = 4) -> Tuple[int, int, int]:
        """Runs until no capacity error remains; returns the final status (synchronises)."""
        for _ in range(max_tries):
            self.launch(stream)
            code, needed, where = read_status(self.status)
            if code == B.PDP_E_CAPACITY:
                self._grow(where, needed)
                continue
            if code != 0:
                raise B.PdpError(code, f"best-hit run: {lib().pdp_strerror(code).decode()} "
                                       f"(needed {needed}, where {where})")
            return code, needed, where
        raise B.PdpError(B.PDP_E_CAPACITY, "capacity still too small after retries")

    def results(self) -> PairResults:
        return PairResults(self.plan, self.bh.host(), self.bbh.host() if self.bbh is not None else None)

    def families(self, node_a: Sequence[int], node_b: Sequence[int], n_nodes: int, stream=None) -> torch.Tensor:
        """pdp_plan_families on the last launch's BBH: node_a[t] / node_b[t] are the global ids of gene 0 of
        task t's genomes; returns the device labels (smallest node id of each node's family)."""
        if self.bbh is None:
            raise ValueError("no task of this plan asks for BBH")
        dev = _device()
        na = torch.tensor(np.asarray(node_a, dtype=np.int64), dtype=torch.int32, device=dev)
        nb = torch.tensor(np.asarray(node_b, dtype=np.int64), dtype=torch.int32, device=dev)
        labels = torch.empty(max(int(n_nodes), 1), dtype=torch.int32, device=dev)
        self._fam_keep = (na, nb)  # read asynchronously by the kernels
        bb = self.bbh.struct()
        check(lib().pdp_plan_families(self.plan.h, C.byref(bb), na.data_ptr(), nb.data_ptr(), int(n_nodes),
                                      labels.data_ptr(), self.fam_status.data_ptr(), self.ws.ptr, self.ws.nbytes,
                                      _stream_handle(stream)), "pdp_plan_families")
        return labels[: int(n_nodes)]


def all_pairs_tasks(dicts: Sequence[Dictionary], pairs: Optional[Sequence[Tuple[int, int]]] = None,
                    flags: int = B.PDP_TASK_AB | B.PDP_TASK_BA | B.PDP_TASK_BBH):
    if pairs is None:
        pairs = [(i, j) for i in range(len(dicts)) for j in range(i + 1, len(dicts))]
    return [(dicts[i], dicts[j], flags) for i, j in pairs]


def bh(q: Dictionary, t: Dictionary, prm: Optional[B.pdp_params] = None, capacity: Optional[int] = None,
       stream=None) -> BHOut:
    """pdp_bh: best hits of q's genes in t (synchronises to read the status)."""
    prm = prm or params()
    ws_bytes = B.u64(0)
    check(lib().pdp_bh_ws_size(C.byref(q.d), C.byref(t.d), C.byref(prm), C.byref(ws_bytes)), "pdp_bh_ws_size")
    ws = Workspace(ws_bytes.value)
    out = BHOut(q.n_genes, capacity if capacity is not None else 2 * q.n_genes + 1024)
    st = new_status()
    for _ in range(4):
        o = out.struct()
        check(lib().pdp_bh(C.byref(q.d), C.byref(t.d), C.byref(prm), C.byref(o), st.data_ptr(), ws.ptr, ws.nbytes,
                           _stream_handle(stream)), "pdp_bh")
        code, needed, where = read_status(st)
        if code == B.PDP_E_CAPACITY and where == 0:
            prm = _with_capacity(prm, int(needed * 1.25) + 1024)
            check(lib().pdp_bh_ws_size(C.byref(q.d), C.byref(t.d), C.byref(prm), C.byref(ws_bytes)), "pdp_bh_ws_size")
            ws = Workspace(ws_bytes.value)
            continue
        if code == B.PDP_E_CAPACITY and where == 1:
            out = BHOut(q.n_genes, int(needed * 1.25) + 1024)
            continue
        if code != 0:
            raise B.PdpError(code, f"pdp_bh: {lib().pdp_strerror(code).decode()}")
        return out
    raise B.PdpError(B.PDP_E_CAPACITY, "pdp_bh: capacity still too small")


def bh_noalloc(q: Dictionary, t: Dictionary, prm: Optional[B.pdp_params] = None, capacity: Optional[int] = None,
               stream=None) -> BHOut:
    """pdp_bh_noalloc: best hits of q's genes in t with the library's fixed device scratch (no
    workspace).  Grows the output and retries on a best-hit capacity error; a record capacity
    error retries with more records while the fixed scratch holds them (synchronises)."""
    prm = prm or params()
    out = BHOut(q.n_genes, capacity if capacity is not None else 2 * q.n_genes + 1024)
    st = new_status()
    for _ in range(4):
        o = out.struct()
        check(lib().pdp_bh_noalloc(C.byref(q.d), C.byref(t.d), C.byref(prm), C.byref(o), st.data_ptr(),
                                   _stream_handle(stream)), "pdp_bh_noalloc")
        code, needed, where = read_status(st)
        if code == B.PDP_E_CAPACITY and where == 0:
            prm = _with_capacity(prm, int(needed * 1.25) + 1024)
            continue
        if code == B.PDP_E_CAPACITY and where == 1:
            out = BHOut(q.n_genes, int(needed * 1.25) + 1024)
            continue
        if code != 0:
            raise B.PdpError(code, f"pdp_bh_noalloc: {lib().pdp_strerror(code).decode()}")
        return out
    raise B.PdpError(B.PDP_E_CAPACITY, "pdp_bh_noalloc: capacity still too small")


def bbh(ab: BHOut, ba: BHOut, capacity: Optional[int] = None, stream=None) -> BBHOut:
    """pdp_bbh: BBH from two best-hit outputs (synchronises to read the status)."""
    ws_bytes = B.u64(0)
    check(lib().pdp_bbh_ws_size(ab.n_rows, C.byref(ws_bytes)), "pdp_bbh_ws_size")
    ws = Workspace(ws_bytes.value)
    out = BBHOut(ab.n_rows, capacity if capacity is not None else ab.n_rows + 1024)
    st = new_status()
    for _ in range(3):
        a, b, o = ab.struct(), ba.struct(), out.struct()
        check(lib().pdp_bbh(C.byref(a), C.byref(b), C.byref(o), st.data_ptr(), ws.ptr, ws.nbytes,
                            _stream_handle(stream)), "pdp_bbh")
        code, needed, where = read_status(st)
        if code == B.PDP_E_CAPACITY:
            out = BBHOut(ab.n_rows, int(needed * 1.25) + 1024)
            continue
        if code != 0:
            raise B.PdpError(code, f"pdp_bbh: {lib().pdp_strerror(code).decode()}")
        return out
    raise B.PdpError(B.PDP_E_CAPACITY, "pdp_bbh: capacity still too small")


class Graph:
    """A HIP graph of library launches: ``with Graph.capture(stream) as g: ...`` then ``g.launch()``."""

    def __init__(self, stream: torch.cuda.Stream):
        self.stream = stream
        self.h = B.vp()
        self._destroy = lib().pdp_graph_destroy  # bound now: module globals may be gone at interpreter exit

    @classmethod
    def capture(cls, stream: torch.cuda.Stream) -> "Graph":
        return cls(stream)

    def __enter__(self) -> "Graph":
        check(lib().pdp_capture_begin(_stream_handle(self.stream)), "pdp_capture_begin")
        return self

    def __exit__(self, exc_type, exc, tb):
        rc = lib().pdp_capture_end(_stream_handle(self.stream), C.byref(self.h))
        if exc_type is None:
            check(rc, "pdp_capture_end")
        return False

    def launch(self, stream: Optional[torch.cuda.Stream] = None) -> None:
        check(lib().pdp_graph_launch(self.h, _stream_handle(stream or self.stream)), "pdp_graph_launch")

    def __del__(self):
        h = getattr(self, "h", None)
        destroy = getattr(self, "_destroy", None)
        if h is not None and h.value and destroy is not None:
            destroy(h)
            self.h = B.vp()


@dataclass
class RequestResult:
    """Host copy of one served request: per resident r, best hits both ways and BBH."""

    tag: int
    code: int
    ab_row: np.ndarray
    ba_row: np.ndarray
    bbh_row: np.ndarray
    bh: tuple  # (ptr, col, num, den)
    bbh: tuple  # (ptr, a, b, num, den)
    n_genes: int
    resident_genes: List[int]

    def best_hits(self, r: int, direction: int = 0):
        base = int((self.ab_row if direction == 0 else self.ba_row)[r])
        n = self.n_genes if direction == 0 else self.resident_genes[r]
        ptr, col, num, den = self.bh
        p = ptr[base:base + n + 1].astype(np.int64)
        lo, hi = int(p[0]), int(p[-1])
        return (p - lo).astype(np.uint32), col[lo:hi], num[lo:hi], den[lo:hi]

    def bbh_pairs(self, r: int):
        base = int(self.bbh_row[r])
        ptr, a, b, num, den = self.bbh
        lo, hi = int(ptr[base]), int(ptr[base + self.n_genes])
        return a[lo:hi], b[lo:hi], num[lo:hi], den[lo:hi]


class Server:
    """pdp_server: resident dictionaries on device, requests admitted under an HBM budget."""

    def __init__(self, residents: Sequence[Dictionary], budget_bytes: int, slots: int = 8,
                 prm: Optional[B.pdp_params] = None):
        self.residents = list(residents)
        self.k = self.residents[0].k
        self.arena = torch.empty(int(budget_bytes), dtype=torch.uint8, device=_device())
        self.alphabet = getattr(self.residents[0], "alphabet", "aa")
        cfg = B.pdp_server_config(int(budget_bytes), int(slots), self.k, B.alphabet_id(self.alphabet), 0,
                                  prm or params())
        arr = (C.POINTER(B.pdp_dict) * len(self.residents))(*[C.pointer(d.d) for d in self.residents])
        self.h = B.vp()
        torch.cuda.synchronize()  # residents built on torch streams must be complete before other streams read them
        check(lib().pdp_server_create(C.byref(cfg), arr, len(self.residents), self.arena.data_ptr(), int(budget_bytes),
                                      C.byref(self.h)), "pdp_server_create")
        self._keep = []

    def submit(self, genome, tag: int) -> None:
        al = getattr(genome, "alphabet", self.alphabet)
        if al != self.alphabet:
            raise ValueError(f"genome alphabet {al!r} differs from the residents' {self.alphabet!r}")
        res = np.ascontiguousarray(genome.residues, dtype=np.uint8)
        off = np.ascontiguousarray(genome.offsets, dtype=np.uint64)
        check(lib().pdp_server_submit(self.h, res.ctypes.data, off.ctypes.data, int(off.shape[0] - 1), int(tag)),
              "pdp_server_submit")

    def poll(self, max_n: int = 64, wait_us: int = 0) -> List[B.pdp_request_done]:
        arr = (B.pdp_request_done * max_n)()
        n = B.u32(0)
        check(lib().pdp_server_poll(self.h, arr, max_n, C.byref(n), int(wait_us)), "pdp_server_poll")
        return [arr[i] for i in range(n.value)]

    def fetch(self, tag: int) -> RequestResult:
        r = B.pdp_request_result()
        check(lib().pdp_server_fetch(self.h, int(tag), C.byref(r)), "pdp_server_fetch")
        nr = r.n_residents

        def arr(p, n):
            return np.ctypeslib.as_array(p, shape=(n,)).copy() if n else np.zeros(0, np.uint32)

        if r.code != 0:
            return RequestResult(int(tag), int(r.code), None, None, None, None, None, 0, [])
        bh_ptr = arr(r.bh_ptr, r.bh_rows + 1)
        bbh_ptr = arr(r.bbh_ptr, r.bbh_rows + 1)
        nbh, nbb = int(bh_ptr[-1]), int(bbh_ptr[-1])
        n_genes = r.bbh_rows // max(nr, 1)
        return RequestResult(int(tag), 0, arr(r.ab_row, nr), arr(r.ba_row, nr), arr(r.bbh_row, nr),
                             (bh_ptr, arr(r.bh_col, nbh), arr(r.bh_num, nbh), arr(r.bh_den, nbh)),
                             (bbh_ptr, arr(r.bbh_a, nbb), arr(r.bbh_b, nbb), arr(r.bbh_num, nbb), arr(r.bbh_den, nbb)),
                             n_genes, [d.n_genes for d in self.residents])

    def release(self, tag: int) -> None:
        check(lib().pdp_server_release(self.h, int(tag)), "pdp_server_release")

    def stats(self) -> B.pdp_server_stats:
        s = B.pdp_server_stats()
        check(lib().pdp_server_stats_get(self.h, C.byref(s)), "pdp_server_stats_get")
        return s

    def close(self) -> None:
        if getattr(self, "h", None) is not None and self.h.value:
            lib().pdp_server_destroy(self.h)
            self.h = B.vp()

    def __del__(self):
        try:
            self.close()
        except Exception:  # pragma: no cover - interpreter shutdown
            pass


def _task_array(tasks):
    arr = (B.pdp_task * len(tasks))()
    for i, (a, b, f) in enumerate(tasks):
        arr[i].a = C.pointer(a.d)
        arr[i].b = C.pointer(b.d)
        arr[i].flags = int(f)
    return arr


def autotune(tasks, candidates: Optional[Sequence[B.pdp_params]] = None, reps: int = 3, stream=None,
             base: Optional[B.pdp_params] = None):
    """pdp_autotune over a list of (dict a, dict b, flags); returns (best params, result).  The tuner
    times the launch shapes only; the candidate filters of ``base`` are carried into the result."""
    arr = _task_array(tasks)
    cand = (B.pdp_params * len(candidates))(*candidates) if candidates else None
    nc = len(candidates) if candidates else 0
    need = B.u64(0)
    check(lib().pdp_autotune_ws_size(arr, len(tasks), cand, nc, C.byref(need)), "pdp_autotune_ws_size")
    plan = Plan(tasks)
    ws = Workspace(need.value)
    bh_out = BHOut(plan.info.bh_rows, 4 * plan.info.bh_rows + 1024)
    bbh_out = BBHOut(plan.info.bbh_rows, 2 * plan.info.bbh_rows + 1024) if plan.info.bbh_rows else None
    st = new_status()
    res = B.pdp_tune_result()
    bs = bh_out.struct()
    bb = bbh_out.struct() if bbh_out is not None else None
    check(lib().pdp_autotune(arr, len(tasks), cand, nc, int(reps), C.byref(bs), C.byref(bb) if bb is not None else None,
                             st.data_ptr(), ws.ptr, ws.nbytes, _stream_handle(stream), C.byref(res)), "pdp_autotune")
    f = base or params()
    best = B.pdp_params(res.best.inc_capacity, res.best.tile_rows, res.best.join_entries, res.best.lds_budget,
                        res.best.flags, f.theta_num, f.theta_den, f.tau_num, f.tau_den)
    return best, res
