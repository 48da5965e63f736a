"""Pins of the sparse exact oracle (a k-mer -> postings map accumulating the sums of minima of
the gene pairs that share a k-mer; Eq. jaccard_k with the sum of maxima from max + min = x + y).

Before it stands in for the dense oracle on whole genome-scale workloads it must give the same
best hits as the definitions restated independently: the hand-derived fixtures, brute force on
Python strings (with ties, both alphabets, the candidate filters of Eqs. length_threshold and
directional_jaccard), and the dense oracle, which sums minima and maxima literally, on shared
inputs including row subsets of the 10 x 3000-gene and 50-genome workloads.  Planted slips in a
copy of its code must each fail one of these pins.
"""
import os
import random
import shutil
import subprocess
import tempfile
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import brute
from synth import genome_from_strings, make_config

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "pdp_oracle.c")
ALPHA = "ACDEFGHIKLMNPQRSTVWY"


def _og(genes, k, alphabet="aa"):
    return oracle.OracleGenome(genome_from_strings(genes, alphabet=alphabet), k)


def _rows(bh, n):
    return [[(int(c), int(nu), int(d)) for c, nu, d in zip(*bh.row(r))] for r in range(n)]


def _same(x: oracle.BH, y: oracle.BH):
    assert np.array_equal(x.ptr, y.ptr), "best hits per row"
    assert np.array_equal(x.col, y.col), "columns"
    assert np.array_equal(x.num, y.num), "sums of minima"
    assert np.array_equal(x.den, y.den), "sums of maxima"


def _random_genes(rng, n, alpha, lo=0, hi=40):
    return ["".join(rng.choice(alpha) for _ in range(rng.randint(lo, hi))) for _ in range(n)]


# ------------------------------------------------------------------ hand values

def test_hand_best_hits(golden):
    for e in golden["best_hits"]:
        k = e["k"]
        gi, gj = _og(e["gi"], k), _og(e["gj"], k)
        ab, ba = oracle.bh_sparse(gi, gj), oracle.bh_sparse(gj, gi)
        assert _rows(ab, len(e["gi"])) == [[tuple(x) for x in row] for row in e["bh_ij"]], e["id"]
        assert _rows(ba, len(e["gj"])) == [[tuple(x) for x in row] for row in e["bh_ji"]], e["id"]
        p = oracle.bbh(ab, ba)
        assert [[int(x), int(y)] for x, y in zip(p.a, p.b)] == e["bbh"], e["id"]


def test_hand_filters(golden):
    for e in golden["filters"]:
        th = tuple(e["theta"]) if e["theta"] else None
        ta = tuple(e["tau"]) if e["tau"] else None
        gi, gj = _og(e["gi"], e["k"]), _og(e["gj"], e["k"])
        assert _rows(oracle.bh_sparse(gi, gj, theta=th, tau=ta), len(e["gi"])) == \
            [[tuple(x) for x in row] for row in e["bh_ij"]], e["id"]
        assert _rows(oracle.bh_sparse(gj, gi, theta=th, tau=ta), len(e["gj"])) == \
            [[tuple(x) for x in row] for row in e["bh_ji"]], e["id"]


# ------------------------------------------------------------------ brute force

@pytest.mark.parametrize("seed", range(30))
def test_brute_force_tiny_with_ties(seed):
    rng = random.Random(7000 + seed)
    alpha = ALPHA[: rng.choice([2, 3, 4, 20])]
    k = rng.choice([1, 2, 3])
    gi = _random_genes(rng, rng.randint(1, 8), alpha)
    gj = _random_genes(rng, rng.randint(1, 8), alpha)
    gj += gj[: rng.randint(0, 2)]  # duplicated genes tie exactly
    oi, oj = _og(gi, k), _og(gj, k)
    ab, ba = oracle.bh_sparse(oi, oj, threads=2), oracle.bh_sparse(oj, oi, threads=2)
    want_ab, want_ba = brute.all_best_hits(gi, gj, k), brute.all_best_hits(gj, gi, k)
    assert _rows(ab, len(gi)) == [want_ab[r] for r in range(len(gi))]
    assert _rows(ba, len(gj)) == [want_ba[r] for r in range(len(gj))]
    p = oracle.bbh(ab, ba)
    assert list(zip(p.a.tolist(), p.b.tolist())) == brute.bbh(gi, gj, k)


@pytest.mark.parametrize("seed", range(12))
def test_brute_force_nucleotide(seed):
    rng = random.Random(8000 + seed)
    k = rng.choice([1, 3, 5, 9, 15])
    gi = _random_genes(rng, rng.randint(1, 7), "ACGT", 0, 70)
    gj = _random_genes(rng, rng.randint(1, 7), "ACGT", 0, 70)
    if gi and rng.random() < 0.6:  # a mutated copy keeps shared k-mers at large k
        s = list(gi[0])
        for p in range(0, len(s), 11):
            s[p] = rng.choice("ACGT")
        gj.append("".join(s))
    oi, oj = _og(gi, k, "nt"), _og(gj, k, "nt")
    ab = oracle.bh_sparse(oi, oj, threads=1)
    want = brute.all_best_hits(gi, gj, k)
    assert _rows(ab, len(gi)) == [want[r] for r in range(len(gi))]


@pytest.mark.parametrize("seed", range(12))
def test_filters_match_brute(seed):
    rng = random.Random(9000 + seed)
    alpha = ALPHA[: rng.choice([2, 3, 4, 20])]
    k = rng.choice([1, 2, 3])
    gi = _random_genes(rng, rng.randint(1, 7), alpha, 0, 30)
    gj = _random_genes(rng, rng.randint(1, 7), alpha, 0, 30)
    gi += gi[:1]
    th = rng.choice([None, (1, 2), (3, 4), (9, 10), (0, 1)])
    ta = rng.choice([None, (1, k), (1, 2), (2, 5), (0, 1)])
    ab = oracle.bh_sparse(_og(gi, k), _og(gj, k), threads=2, theta=th, tau=ta)
    want = brute.all_best_hits(gi, gj, k, Fraction(*th) if th else None, Fraction(*ta) if ta else None)
    assert _rows(ab, len(gi)) == [want[r] for r in range(len(gi))]


# ------------------------------------------------------ the dense oracle, shared inputs

def test_planted_pair_equals_dense():
    ds = make_config(1)
    og = oracle.genomes(ds.genomes, 4)
    sparse = oracle.all_pairs_sparse(og)
    _, dense = oracle.all_pairs(ds.genomes, 4)
    for key, (ab, ba, bb) in dense.items():
        sab, sba, sbb = sparse[key]
        _same(sab, ab)
        _same(sba, ba)
        assert np.array_equal(sbb.a, bb.a) and np.array_equal(sbb.b, bb.b)
        assert np.array_equal(sbb.num, bb.num) and np.array_equal(sbb.den, bb.den)


@pytest.mark.parametrize("case", ["family", "paralogs", "nucleotide", "filters"])
def test_small_workloads_equal_dense(case):
    th = ta = None
    if case == "family":
        ds, k = make_config(2, genomes=3, genes=400), 5
    elif case == "paralogs":
        ds, k = make_config(3, genomes=3, genes_lo=300, genes_hi=500, core=150), 5
    elif case == "nucleotide":
        ds, k = make_config(2, genomes=3, genes=150, alphabet="nt"), 11
    else:
        ds, k, th, ta = make_config(2, genomes=3, genes=300), 4, (3, 4), (1, 4)
    og = oracle.genomes(ds.genomes, k)
    sparse = oracle.all_pairs_sparse(og, theta=th, tau=ta)
    _, dense = oracle.all_pairs(ds.genomes, k, theta=th, tau=ta)
    ties = 0
    for key, (ab, ba, bb) in dense.items():
        sab, sba, sbb = sparse[key]
        _same(sab, ab)
        _same(sba, ba)
        assert np.array_equal(sbb.a, bb.a) and np.array_equal(sbb.b, bb.b)
        ties += int(np.sum(np.diff(ab.ptr.astype(np.int64)) > 1))
    if case == "paralogs":
        assert ties > 0


def _evenly(n, m):
    return np.unique(np.linspace(0, n - 1, min(m, n)).astype(np.uint32))


def test_family_10x3000_rows_equal_dense():
    """Genomes 0 and 1 of the 10 x 3000-gene workload (k = 6): 400 evenly spaced rows each way."""
    ds = make_config(2)
    k = oracle.k_rule(ds.total_residues())
    assert k == 6
    og = oracle.genomes(ds.genomes[:2], k)
    for q, t in ((og[0], og[1]), (og[1], og[0])):
        rows = _evenly(q.n, 400)
        _same(oracle.bh_sparse(q, t, rows=rows), oracle.bh(q, t, rows=rows))


def test_large_workload_tie_rows_equal_dense():
    """Genomes 0 and 1 of the 50-genome workload with paralog copies (k = 7): every row the sparse
    oracle gives tied best hits plus 200 evenly spaced rows, each way, against the dense oracle."""
    ds = make_config(3)
    k = oracle.k_rule(ds.total_residues())
    assert k == 7
    og = oracle.genomes(ds.genomes[:2], k)
    tied = 0
    for q, t in ((og[0], og[1]), (og[1], og[0])):
        full = oracle.bh_sparse(q, t)
        ties = np.nonzero(np.diff(full.ptr.astype(np.int64)) > 1)[0].astype(np.uint32)
        tied += len(ties)
        rows = np.union1d(ties, _evenly(q.n, 200)).astype(np.uint32)
        _same(oracle.bh_sparse(q, t, rows=rows), oracle.bh(q, t, rows=rows))
    assert tied > 0, "paralog copies should tie"


# ------------------------------------------------------------------ planted slips

MUTANTS = [
    ("sum of maxima without the shared minima", "const uint64_t m = A->m[b], d = na + t->nwin[b] - m;",
     "const uint64_t m = A->m[b], d = na + t->nwin[b];"),
    ("maximum accumulated instead of minimum", "A->m[b] += ca < cb ? ca : cb;", "A->m[b] += ca > cb ? ca : cb;"),
    ("accumulators not cleared between rows", "A->m[b] = 0; A->oa[b] = 0; A->ob[b] = 0;", "A->oa[b] = 0; A->ob[b] = 0;"),
    ("first maximum only", "} else if (orc_cmp_j(m, d, bm, bd) == 0) {",
     "} else if (orc_cmp_j(m, d, bm, bd) == 0 && c == 0) {"),
    ("postings of one gene only", "s->len += 1;", "s->len = 1;"),
    ("directional sum over the other gene", "A->oa[b] += ca;", "A->oa[b] += cb;"),
]


def _pins_hold(libpath, golden):
    saved = oracle._lib, oracle._LIB_PATH
    orig_build = oracle.build
    try:
        oracle._lib = None
        oracle.build = lambda force=False: libpath
        oracle._load()
        for e in golden["best_hits"]:
            gi, gj = _og(e["gi"], e["k"]), _og(e["gj"], e["k"])
            if _rows(oracle.bh_sparse(gi, gj, threads=1), len(e["gi"])) != \
                    [[tuple(x) for x in row] for row in e["bh_ij"]]:
                return False
        for e in golden["filters"]:
            th = tuple(e["theta"]) if e["theta"] else None
            ta = tuple(e["tau"]) if e["tau"] else None
            gi, gj = _og(e["gi"], e["k"]), _og(e["gj"], e["k"])
            if _rows(oracle.bh_sparse(gi, gj, threads=1, theta=th, tau=ta), len(e["gi"])) != \
                    [[tuple(x) for x in row] for row in e["bh_ij"]]:
                return False
        # k = 1, tau = 1/2: "AAAAAC" shares A and C with "AC"; its occurrences of them are 6 of 6
        # windows, while the other gene's are 2 -- the directional test must use a's own
        for gi, gj, k, th, ta in ((["AAAAAC", "CD"], ["AC", "DDDDDC"], 1, None, (1, 2)),):
            got = oracle.bh_sparse(_og(gi, k), _og(gj, k), threads=1, theta=th, tau=ta)
            want = brute.all_best_hits(gi, gj, k, Fraction(*th) if th else None, Fraction(*ta) if ta else None)
            if _rows(got, len(gi)) != [want[r] for r in range(len(gi))]:
                return False
        rng = random.Random(77)
        for trial in range(20):
            alpha = ALPHA[: rng.choice([2, 3, 20])]
            k = rng.choice([1, 2, 3])
            gi = _random_genes(rng, rng.randint(1, 6), alpha, 0, 30)
            gj = _random_genes(rng, rng.randint(1, 6), alpha, 0, 30)
            gj += gj[:1]
            th = [None, (1, 2)][trial % 2]
            ta = [None, (1, 3), (1, 2)][trial % 3]
            got = oracle.bh_sparse(_og(gi, k), _og(gj, k), threads=1, theta=th, tau=ta)
            want = brute.all_best_hits(gi, gj, k, Fraction(*th) if th else None, Fraction(*ta) if ta else None)
            if _rows(got, len(gi)) != [want[r] for r in range(len(gi))]:
                return False
        return True
    finally:
        oracle.build = orig_build
        oracle._lib, oracle._LIB_PATH = saved
        oracle._lib = None


def _build(text, tmp):
    src, lib = os.path.join(tmp, "m.c"), os.path.join(tmp, "libm.so")
    with open(src, "w") as f:
        f.write(text)
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-pthread", "-o", lib, src])
    return lib


def test_unmodified_copy_passes(golden):
    tmp = tempfile.mkdtemp()
    try:
        assert _pins_hold(_build(open(SRC).read(), tmp), golden)
    finally:
        shutil.rmtree(tmp)


@pytest.mark.parametrize("name,orig,planted", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_slip_is_caught(name, orig, planted, golden):
    text = open(SRC).read()
    assert orig in text, f"mutation site for '{name}' not found"
    tmp = tempfile.mkdtemp()
    try:
        assert not _pins_hold(_build(text.replace(orig, planted, 1), tmp), golden), f"'{name}' went unnoticed"
    finally:
        shutil.rmtree(tmp)


# ------------------------------------------------------- the any-size property check

def test_property_check_rejects_missing_or_extra_bbh():
    """The check applied to every full-size GPU output rebuilds the BBH set from the two best-hit
    CSRs: a dropped mutual pair, an extra pair and a wrong num/den must each fail it."""
    import sys

    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from helpers import check_bh_properties

    ds = make_config(2, genomes=2, genes=300)
    og = oracle.genomes(ds.genomes, 5)
    ab, ba, bb = oracle.all_pairs_sparse(og)[(0, 1)]

    def g(x):
        return x.ptr.astype(np.uint32), x.col, x.num.astype(np.uint32), x.den.astype(np.uint32)

    pairs = [bb.a, bb.b, bb.num.astype(np.uint32), bb.den.astype(np.uint32)]
    check_bh_properties(g(ab), g(ba), tuple(pairs), og[0].n, og[1].n)
    assert len(bb.a) > 10
    dropped = tuple(np.delete(x, 5) for x in pairs)
    # an AB best hit whose reverse row lacks it, listed as if mutual
    lone = next((a, int(ab.col[p])) for a in range(og[0].n) for p in range(int(ab.ptr[a]), int(ab.ptr[a + 1]))
                if a not in set(ba.col[int(ba.ptr[ab.col[p]]):int(ba.ptr[ab.col[p] + 1])].tolist()))
    at = int(np.searchsorted(bb.a.astype(np.int64) * (og[1].n + 1) + bb.b, lone[0] * (og[1].n + 1) + lone[1]))
    extra = (np.insert(pairs[0], at, lone[0]), np.insert(pairs[1], at, lone[1]), np.insert(pairs[2], at, 1),
             np.insert(pairs[3], at, 2))
    wrong = (pairs[0], pairs[1], pairs[2], pairs[3] + np.uint32(1))
    for bad in (dropped, extra, wrong):
        with pytest.raises(AssertionError):
            check_bh_properties(g(ab), g(ba), bad, og[0].n, og[1].n)
