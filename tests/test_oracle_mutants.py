"""The oracle's pins catch plausible mistakes: each case plants one slip into a copy
of pdp_oracle.c (on the CPU, in a temporary directory), builds it, and checks that
at least one pin (hand values, brute force, invariants) now fails."""
import ctypes as C
import os
import random
from fractions import Fraction
import shutil
import subprocess
import tempfile

import pytest

from oracle import brute

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "pdp_oracle.c")

# (name, original text, planted text)
MUTANTS = [
    ("window count |s|-k-1", "return len >= (int64_t)k ? len - (int64_t)k + 1 : 0;",
     "return len >= (int64_t)k + 2 ? len - (int64_t)k - 1 : 0;"),
    ("min and max swapped", "mn += ca[i] < cb[j] ? ca[i] : cb[j];", "mn += ca[i] > cb[j] ? ca[i] : cb[j];"),
    ("union term dropped", "mx += ca[i];               /* only in a */", "/* dropped */"),
    ("set instead of multiset", "cnt[d - 1] += 1;", "cnt[d - 1] += 0;"),
    ("first maximum only", "if (cand[b] && orc_cmp_j(m[b], d[b], m[best], d[best]) == 0) {",
     "if (cand[b] && b == best) {"),
    ("zero maximum kept", "if (have && orc_cmp_j(m[best], d[best], 0, 1) > 0) {", "if (have) {"),
    ("BBH direction typo", "if (b < ba->nrows && orc_row_has(ba, b, a)) {", "if (b < ba->nrows && orc_row_has(ab, a, b)) {"),
    ("strict comparison flipped", "if (!have || orc_cmp_j(m[b], d[b], m[best], d[best]) > 0) best = b;",
     "if (!have || orc_cmp_j(m[b], d[b], m[best], d[best]) < 0) best = b;"),
    ("length filter one-sided",
     "if (la * theta_d < (unsigned __int128)theta_n * lb || lb * theta_d < (unsigned __int128)theta_n * la) return 0;",
     "if (la * theta_d < (unsigned __int128)theta_n * lb) return 0;"),
    ("directional filter over the other gene's windows",
     "if (wa == 0 ? tau_n > 0 : (unsigned __int128)oa * tau_d < (unsigned __int128)tau_n * wa) return 0;",
     "if (wa == 0 ? tau_n > 0 : (unsigned __int128)oa * tau_d < (unsigned __int128)tau_n * wb) return 0;"),
    ("nucleotide letters out of order", '"ACDEFGHIKLMNPQRSTVWY", "ACGT"};', '"ACDEFGHIKLMNPQRSTVWY", "ACTG"};'),
    ("identifier base fixed at 20", "id = id * ORC_SIGMA[a] + (uint64_t)orc_residue(s[p + i], a);",
     "id = id * ORC_SIGMA[0] + (uint64_t)orc_residue(s[p + i], a);"),
]


def _build(text, tmp):
    src = os.path.join(tmp, "m.c")
    lib = os.path.join(tmp, "libm.so")
    with open(src, "w") as f:
        f.write(text)
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-pthread", "-o", lib, src])
    return lib


def _pins_hold(libpath, golden) -> bool:
    """Runs the oracle pins against a freshly built copy; False as soon as one fails."""
    import oracle

    saved = oracle._lib, oracle._LIB_PATH
    try:
        oracle._lib = None
        L = C.CDLL(libpath)
        oracle._LIB_PATH = libpath
        oracle._lib = None
        # reuse the wrapper's signatures on the mutant library
        orig_build = oracle.build
        oracle.build = lambda force=False: libpath
        try:
            oracle._load()
        finally:
            oracle.build = orig_build
        from synth import genome_from_strings

        def og(genes, k, alphabet="aa"):
            return oracle.OracleGenome(genome_from_strings(genes, alphabet=alphabet), k)

        for w in golden["windows"]:
            al = w.get("alphabet", "aa")
            if oracle.n_windows(len(w["gene"]), w["k"]) != w["n"]:
                return False
            ids, cnt = oracle.mv(w["gene"].encode(), w["k"], al)
            if [[oracle.decode_id(int(i), w["k"], al), int(c)] for i, c in zip(ids, cnt)] != w["mv"]:
                return False
            if "ids" in w and [int(i) for i in ids] != w["ids"]:
                return False
        for e in golden["jaccard"]:
            al = e.get("alphabet", "aa")
            if og([e["a"]], e["k"], al).terms(0, og([e["b"]], e["k"], al), 0) != (e["num"], e["den"]):
                return False
        for e in golden["best_hits"]:
            gi, gj = og(e["gi"], e["k"]), og(e["gj"], e["k"])
            ab, ba = oracle.bh(gi, gj, threads=1), oracle.bh(gj, gi, threads=1)
            rows = [[(int(c), int(n), int(d)) for c, n, d in zip(*ab.row(r))] for r in range(len(e["gi"]))]
            if rows != [[tuple(x) for x in row] for row in e["bh_ij"]]:
                return False
            p = oracle.bbh(ab, ba)
            if [[int(x), int(y)] for x, y in zip(p.a, p.b)] != e["bbh"]:
                return False
        for e in golden["filters"]:
            th = tuple(e["theta"]) if e["theta"] else None
            ta = tuple(e["tau"]) if e["tau"] else None
            gi, gj = og(e["gi"], e["k"]), og(e["gj"], e["k"])
            ab = oracle.bh(gi, gj, threads=1, theta=th, tau=ta)
            ba = oracle.bh(gj, gi, threads=1, theta=th, tau=ta)
            rows = [[(int(c), int(n), int(d)) for c, n, d in zip(*ab.row(r))] for r in range(len(e["gi"]))]
            rows_ji = [[(int(c), int(n), int(d)) for c, n, d in zip(*ba.row(r))] for r in range(len(e["gj"]))]
            if rows != [[tuple(x) for x in row] for row in e["bh_ij"]] or \
                    rows_ji != [[tuple(x) for x in row] for row in e["bh_ji"]]:
                return False
        rng = random.Random(5)
        for trial in range(15):
            th = [None, (1, 2), (3, 4)][trial % 3]
            ta = [None, (1, 2), (1, 3), (2, 5)][trial % 4]
            alpha = "ACDEFGHIKLMNPQRSTVWY"[: rng.choice([2, 3, 20])]
            k = rng.choice([1, 2, 3])
            gi = ["".join(rng.choice(alpha) for _ in range(rng.randint(0, 30))) for _ in range(rng.randint(1, 6))]
            gj = ["".join(rng.choice(alpha) for _ in range(rng.randint(0, 30))) for _ in range(rng.randint(1, 6))]
            oi, oj = og(gi, k), og(gj, k)
            ab, ba = oracle.bh(oi, oj, threads=1), oracle.bh(oj, oi, threads=1)
            want = brute.all_best_hits(gi, gj, k)
            fab = oracle.bh(oi, oj, threads=1, theta=th, tau=ta)
            fwant = brute.all_best_hits(gi, gj, k, Fraction(*th) if th else None, Fraction(*ta) if ta else None)
            if [[(int(c), int(n), int(d)) for c, n, d in zip(*fab.row(r))] for r in range(len(gi))] != \
                    [fwant[r] for r in range(len(gi))]:
                return False
            got = [[(int(c), int(n), int(d)) for c, n, d in zip(*ab.row(r))] for r in range(len(gi))]
            if got != [want[r] for r in range(len(gi))]:
                return False
            p = oracle.bbh(ab, ba)
            if list(zip(p.a.tolist(), p.b.tolist())) != brute.bbh(gi, gj, k):
                return False
        return True
    finally:
        oracle._lib, oracle._LIB_PATH = saved


def test_unmodified_copy_passes(golden):
    tmp = tempfile.mkdtemp()
    try:
        assert _pins_hold(_build(open(SRC).read(), tmp), golden)
    finally:
        shutil.rmtree(tmp)


@pytest.mark.parametrize("name,orig,planted", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(name, orig, planted, golden):
    text = open(SRC).read()
    assert orig in text, f"mutation site for '{name}' not found"
    tmp = tempfile.mkdtemp()
    try:
        assert not _pins_hold(_build(text.replace(orig, planted, 1), tmp), golden), f"'{name}' went unnoticed"
    finally:
        shutil.rmtree(tmp)
