"""CPU oracle for the best-hit path -- TEST INFRASTRUCTURE ONLY.

Thin ctypes wrapper around ``pdp_oracle.c`` (a plain C rendering of the
paper's definitions over the amino-acid or the nucleotide alphabet: k rule,
Alg. 1 multiplicity vectors, Eq. jaccard_k, Eq. best_hit with ties,
Eq. bidirectional_best_hit and Alg. 3), plus ``brute`` (the same definitions
on Python strings, for tiny inputs).

Two best-hit oracles share the multiplicity vectors and the BBH set definition:
``bh`` (dense: every gene pair's two vectors merged, the sums of minima and of
maxima both computed literally) and ``bh_sparse`` (a hash map from k-mer to
postings accumulates the sums of minima of the gene pairs that share a k-mer,
and the sum of maxima follows from max + min = x + y).  The sparse one finishes
whole genome-scale workloads in seconds; the tests pin it to the dense one and
to brute force on shared inputs before it is trusted at full size.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  It shares no code with the GPU library and never loads it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pdp_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libpdp_oracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no vectorisation tricks)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    lib = C.CDLL(build())
    u32, u64, i64, vp = C.c_uint32, C.c_uint64, C.c_int64, C.c_void_p
    P = C.POINTER
    sig = {
        "orc_k_rule": (C.c_int, [u64, u32, C.c_int, P(u32)]),
        "orc_n_windows": (i64, [i64, u32]),
        "orc_k_max": (u32, [u32]),
        "orc_mv": (i64, [C.c_char_p, i64, u32, u32, P(u64), P(u32), P(i64)]),
        "orc_genome_new": (vp, [vp, vp, u32, u32, u32, P(i64)]),
        "orc_genome_free": (None, [vp]),
        "orc_genome_n": (u32, [vp]),
        "orc_genome_entries": (u64, [vp]),
        "orc_genome_ptr": (P(u64), [vp]),
        "orc_genome_ids": (P(u64), [vp]),
        "orc_genome_cnt": (P(u32), [vp]),
        "orc_genome_nwin": (P(u64), [vp]),
        "orc_jaccard_terms": (None, [P(u64), P(u32), u64, P(u64), P(u32), u64, P(u64), P(u64)]),
        "orc_compare_j": (C.c_int, [u64, u64, u64, u64]),
        "orc_pair_terms": (None, [vp, u32, vp, u32, P(u64), P(u64)]),
        "orc_bh_rows": (vp, [vp, vp, vp, u32, C.c_int]),
        "orc_bh_rows_f": (vp, [vp, vp, vp, u32, C.c_int, u64, u64, u64, u64]),
        "orc_directional_terms": (None, [P(u64), P(u32), u64, P(u64), P(u32), u64, P(u64), P(u64)]),
        "orc_bh_free": (None, [vp]),
        "orc_bh_nrows": (u32, [vp]),
        "orc_bh_ptr": (P(u64), [vp]),
        "orc_bh_col": (P(u32), [vp]),
        "orc_bh_num": (P(u64), [vp]),
        "orc_bh_den": (P(u64), [vp]),
        "orc_bbh": (vp, [vp, vp]),
        "orc_bbh_alg3": (vp, [vp, vp, vp, vp]),
        "orc_pairs_free": (None, [vp]),
        "orc_pairs_n": (u64, [vp]),
        "orc_pairs_a": (P(u32), [vp]),
        "orc_pairs_b": (P(u32), [vp]),
        "orc_pairs_num": (P(u64), [vp]),
        "orc_pairs_den": (P(u64), [vp]),
        "orc_index_new": (vp, [vp]),
        "orc_index_free": (None, [vp]),
        "orc_bh_sparse": (vp, [vp, vp, vp, vp, u32, C.c_int, u64, u64, u64, u64]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _arr(ptr, n, dtype):
    if n == 0:
        return np.zeros(0, dtype=dtype)
    return np.ctypeslib.as_array(ptr, shape=(n,)).astype(dtype, copy=True)


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except Exception:  # pragma: no cover
        return max(1, os.cpu_count() or 1)


def k_rule(total: int, alphabet: int = 20, mode: int = 0) -> int:
    """Eq. k_length in integers: mode 0 = smallest k with alphabet^k >= total, 1 = largest k with alphabet^k <= total."""
    k = C.c_uint32(0)
    if _load().orc_k_rule(int(total), int(alphabet), int(mode), C.byref(k)) != 0:
        raise ValueError("alphabet must be >= 2")
    return int(k.value)


def n_windows(length: int, k: int) -> int:
    return int(_load().orc_n_windows(int(length), int(k)))


# The two alphabets of the paper's genes: amino acids and nucleotides.
ALPHABETS = {"aa": "ACDEFGHIKLMNPQRSTVWY", "nt": "ACGT"}
_ALPHA_ID = {"aa": 0, "nt": 1}


def _alpha(alphabet) -> int:
    if alphabet not in _ALPHA_ID:
        raise ValueError(f"unknown alphabet {alphabet!r} (expected 'aa' or 'nt')")
    return _ALPHA_ID[alphabet]


def k_max(alphabet: str = "aa") -> int:
    """Largest k whose identifiers fit 64 bits for this alphabet."""
    return int(_load().orc_k_max(_alpha(alphabet)))


def mv(gene: bytes, k: int, alphabet: str = "aa"):
    """Alg. 1 for one gene: (ids ascending, multiplicities); ids are base-|alphabet| values of the windows."""
    lib = _load()
    nw = max(1, n_windows(len(gene), k))
    ids = (C.c_uint64 * nw)()
    cnt = (C.c_uint32 * nw)()
    bad = C.c_int64(-1)
    d = lib.orc_mv(gene, len(gene), int(k), _alpha(alphabet), ids, cnt, C.byref(bad))
    if d == -2:
        raise ValueError(f"k = {k} outside 1..{k_max(alphabet)} for alphabet {alphabet!r}")
    if d < 0:
        raise ValueError(f"byte outside the alphabet at offset {bad.value}")
    return np.array(ids[:d], dtype=np.uint64), np.array(cnt[:d], dtype=np.uint32)


def decode_id(i: int, k: int, alphabet: str = "aa") -> str:
    """k-mer string of a base-|alphabet| identifier (for comparing dictionaries by content)."""
    alpha = ALPHABETS[alphabet]
    s = []
    for _ in range(k):
        s.append(alpha[i % len(alpha)])
        i //= len(alpha)
    return "".join(reversed(s))


class OracleGenome:
    """Multiplicity vectors of every gene of one genome (residues + offsets).  The alphabet
    is the genome's own (``genome.alphabet``, amino acids when it has none) unless given."""

    def __init__(self, genome, k: int, alphabet: Optional[str] = None):
        lib = _load()
        self.k = int(k)
        self.alphabet = alphabet or getattr(genome, "alphabet", "aa")
        self._res = np.ascontiguousarray(genome.residues, dtype=np.uint8)
        self._off = np.ascontiguousarray(genome.offsets, dtype=np.uint64)
        n = int(self._off.shape[0] - 1)
        bad = C.c_int64(-1)
        h = lib.orc_genome_new(self._res.ctypes.data, self._off.ctypes.data, n, self.k, _alpha(self.alphabet),
                               C.byref(bad))
        if not h and bad.value == -2:
            raise ValueError(f"k = {k} outside 1..{k_max(self.alphabet)} for alphabet {self.alphabet!r}")
        if not h:
            raise ValueError(f"byte outside the alphabet at residue offset {bad.value}")
        self._h = h
        self.n = n
        e = int(lib.orc_genome_entries(h))
        self.ptr = _arr(lib.orc_genome_ptr(h), n + 1, np.uint64)
        self.ids = _arr(lib.orc_genome_ids(h), e, np.uint64)
        self.cnt = _arr(lib.orc_genome_cnt(h), e, np.uint32)
        self.nwin = _arr(lib.orc_genome_nwin(h), n, np.uint64)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_genome_free(h)
            self._h = None

    @property
    def entries(self) -> int:
        return int(self.ptr[-1])

    def mv(self, i: int):
        a, b = int(self.ptr[i]), int(self.ptr[i + 1])
        return self.ids[a:b], self.cnt[a:b]

    def terms(self, a: int, other: "OracleGenome", b: int):
        """(sum of minima over the intersection, sum of maxima over the union) for genes a, b."""
        m = C.c_uint64(0)
        d = C.c_uint64(0)
        _load().orc_pair_terms(self._h, int(a), other._h, int(b), C.byref(m), C.byref(d))
        return int(m.value), int(d.value)


def compare_j(m1: int, d1: int, m2: int, d2: int) -> int:
    return int(_load().orc_compare_j(m1, d1, m2, d2))


@dataclass
class BH:
    """Best hits in CSR form: row r's hits are col[ptr[r]:ptr[r+1]] ascending, with
    num = sum of minima, den = sum of maxima of each hit."""

    rows: np.ndarray
    ptr: np.ndarray
    col: np.ndarray
    num: np.ndarray
    den: np.ndarray
    _h: Optional[int] = None

    def row(self, r: int):
        a, b = int(self.ptr[r]), int(self.ptr[r + 1])
        return self.col[a:b], self.num[a:b], self.den[a:b]

    def __del__(self):
        if self._h and _lib is not None:
            _lib.orc_bh_free(self._h)
            self._h = None


def bh(q: OracleGenome, t: OracleGenome, rows: Optional[Sequence[int]] = None, threads: Optional[int] = None,
       theta=None, tau=None) -> BH:
    """Eq. best_hit for the given rows of q (all rows when None) against genome t.  theta / tau:
    (numerator, denominator) of the candidate filters of Eqs. length_threshold and
    directional_jaccard (None: off); a filtered pair is no best-hit candidate."""
    lib = _load()
    th = default_threads() if threads is None else int(threads)
    tn, td = theta if theta is not None else (0, 0)
    un, ud = tau if tau is not None else (0, 0)
    if rows is None:
        rws = np.arange(q.n, dtype=np.uint32)
        h = lib.orc_bh_rows_f(q._h, t._h, None, 0, th, tn, td, un, ud)
    else:
        rws = np.ascontiguousarray(rows, dtype=np.uint32)
        h = lib.orc_bh_rows_f(q._h, t._h, rws.ctypes.data, int(rws.shape[0]), th, tn, td, un, ud)
    nr = int(lib.orc_bh_nrows(h))
    ptr = _arr(lib.orc_bh_ptr(h), nr + 1, np.uint64)
    nnz = int(ptr[-1])
    return BH(rws, ptr, _arr(lib.orc_bh_col(h), nnz, np.uint32), _arr(lib.orc_bh_num(h), nnz, np.uint64),
              _arr(lib.orc_bh_den(h), nnz, np.uint64), h)


@dataclass
class Pairs:
    a: np.ndarray
    b: np.ndarray
    num: np.ndarray
    den: np.ndarray


def _pairs(h) -> Pairs:
    lib = _load()
    n = int(lib.orc_pairs_n(h))
    p = Pairs(_arr(lib.orc_pairs_a(h), n, np.uint32), _arr(lib.orc_pairs_b(h), n, np.uint32),
              _arr(lib.orc_pairs_num(h), n, np.uint64), _arr(lib.orc_pairs_den(h), n, np.uint64))
    lib.orc_pairs_free(h)
    return p


def bbh(ab: BH, ba: BH) -> Pairs:
    """Eq. bidirectional_best_hit (second condition taken in G_i); ab and ba must hold every row."""
    return _pairs(_load().orc_bbh(ab._h, ba._h))


def bbh_alg3(gi: OracleGenome, gj: OracleGenome, ab: BH, ba: BH) -> Pairs:
    """Alg. 3's column-maximum procedure; must agree with bbh()."""
    return _pairs(_load().orc_bbh_alg3(gi._h, gj._h, ab._h, ba._h))


def all_pairs(genomes, k: int, threads: Optional[int] = None, pairs=None, theta=None, tau=None,
              alphabet: Optional[str] = None):
    """BH both ways and BBH for every unordered genome pair i<j (or the given pairs)."""
    og = [OracleGenome(g, k, alphabet) for g in genomes]
    if pairs is None:
        pairs = [(i, j) for i in range(len(og)) for j in range(i + 1, len(og))]
    out = {}
    for i, j in pairs:
        ab = bh(og[i], og[j], threads=threads, theta=theta, tau=tau)
        ba = bh(og[j], og[i], threads=threads, theta=theta, tau=tau)
        out[(i, j)] = (ab, ba, bbh(ab, ba))
    return og, out


# ------------------------------------------------------------ sparse exact oracle

class SparseIndex:
    """Hash map from k-mer identifier to the postings (gene, multiplicity) of one genome."""

    def __init__(self, genome: OracleGenome):
        self.genome = genome  # the index reads its arrays; keep them alive
        self._h = _load().orc_index_new(genome._h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_index_free(h)
            self._h = None


def bh_sparse(q: OracleGenome, t: OracleGenome, index: Optional[SparseIndex] = None,
              rows: Optional[Sequence[int]] = None, threads: Optional[int] = None, theta=None, tau=None) -> BH:
    """Eq. best_hit through t's k-mer index: the same sets and (num, den) as ``bh``, visiting only
    gene pairs that share a k-mer.  ``index`` is t's SparseIndex (built here when None)."""
    lib = _load()
    ix = index if index is not None else SparseIndex(t)
    if ix.genome is not t:
        raise ValueError("the index belongs to another genome")
    th = default_threads() if threads is None else int(threads)
    tn, td = theta if theta is not None else (0, 0)
    un, ud = tau if tau is not None else (0, 0)
    if rows is None:
        rws = np.arange(q.n, dtype=np.uint32)
        h = lib.orc_bh_sparse(q._h, t._h, ix._h, None, 0, th, tn, td, un, ud)
    else:
        rws = np.ascontiguousarray(rows, dtype=np.uint32)
        h = lib.orc_bh_sparse(q._h, t._h, ix._h, rws.ctypes.data, int(rws.shape[0]), th, tn, td, un, ud)
    nr = int(lib.orc_bh_nrows(h))
    ptr = _arr(lib.orc_bh_ptr(h), nr + 1, np.uint64)
    nnz = int(ptr[-1])
    return BH(rws, ptr, _arr(lib.orc_bh_col(h), nnz, np.uint32), _arr(lib.orc_bh_num(h), nnz, np.uint64),
              _arr(lib.orc_bh_den(h), nnz, np.uint64), h)


def genomes(gens, k, threads: Optional[int] = None, alphabet: Optional[str] = None):
    """OracleGenome of every genome (k a number or one per genome), built by a pool of threads
    (each build is one C call that releases the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor

    ks = list(k) if isinstance(k, (list, tuple)) else [int(k)] * len(gens)
    th = default_threads() if threads is None else int(threads)
    with ThreadPoolExecutor(max(1, min(th, len(gens)))) as ex:
        return list(ex.map(lambda x: OracleGenome(x[0], x[1], alphabet), zip(gens, ks)))


def bh_sparse_directions(og: Sequence[OracleGenome], directions, threads: Optional[int] = None, theta=None,
                         tau=None, chunk: int = 4):
    """Sparse-oracle best hits for many (query, target) index pairs into ``og``: returns
    {(q, t): BH}.  A target's queries go in chunks of ``chunk``; each chunk is one job of a
    thread pool (largest targets first) computing its queries one thread each.  The target's
    index is built by the first of its chunks to run and freed by the last to finish, so only
    the indexes of targets in progress exist at once."""
    import threading
    from concurrent.futures import ThreadPoolExecutor

    th = default_threads() if threads is None else int(threads)
    by_target = {}
    for q, t in directions:
        by_target.setdefault(t, []).append(q)
    order = sorted(by_target, key=lambda t: -sum(og[q].entries for q in by_target[t]))
    jobs = [(t, by_target[t][c:c + chunk]) for t in order for c in range(0, len(by_target[t]), chunk)]
    lock = threading.Lock()
    left = {t: (len(by_target[t]) + chunk - 1) // chunk for t in order}
    built = {t: threading.Lock() for t in order}
    index = {}

    def job(item):
        t, qs = item
        with built[t]:
            if t not in index:
                index[t] = SparseIndex(og[t])
        ix = index[t]
        out = [((q, t), bh_sparse(og[q], og[t], ix, threads=1, theta=theta, tau=tau)) for q in qs]
        with lock:
            left[t] -= 1
            if left[t] == 0:
                del index[t]
        return out

    res = {}
    with ThreadPoolExecutor(max(1, min(th, len(jobs)))) as ex:
        for part in ex.map(job, jobs):
            res.update(part)
    return res


def all_pairs_sparse(og: Sequence[OracleGenome], pairs=None, threads: Optional[int] = None, theta=None, tau=None):
    """BH both ways (sparse oracle) and BBH for every unordered pair i<j of the given oracle
    genomes (or the given pairs), returned as {(i, j): (ab, ba, bbh)}."""
    if pairs is None:
        pairs = [(i, j) for i in range(len(og)) for j in range(i + 1, len(og))]
    dirs = [(i, j) for i, j in pairs] + [(j, i) for i, j in pairs]
    hits = bh_sparse_directions(og, dirs, threads=threads, theta=theta, tau=tau)
    return {(i, j): (hits[(i, j)], hits[(j, i)], bbh(hits[(i, j)], hits[(j, i)])) for i, j in pairs}
