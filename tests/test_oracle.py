"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each pin is independent of the oracle's own code: hand-derived values
(tests/golden/hand_examples.json), a brute-force restatement on Python strings,
closed forms (k = 1 is the weighted Jaccard of residue counts; multiplicity-1
dictionaries give the set Jaccard), and invariants (symmetry, J(g,g) = 1,
sum of minima + sum of maxima = n_a + n_b, BBH inside both BH sets, the two
BBH procedures agreeing, relabelling equivariance).
"""
import random
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import brute
from synth import genome_from_strings, make_config

ALPHA = "ACDEFGHIKLMNPQRSTVWY"


def _og(genes, k, alphabet="aa"):
    return oracle.OracleGenome(genome_from_strings(genes, alphabet=alphabet), k)


def _bh_rows(bh):
    return [[(int(c), int(n), int(d)) for c, n, d in zip(*bh.row(r))] for r in range(len(bh.rows))]


# ----------------------------------------------------------------- hand values

def test_windows_and_mv(golden):
    for w in golden["windows"]:
        k, al = w["k"], w.get("alphabet", "aa")
        assert oracle.n_windows(len(w["gene"]), k) == w["n"], w["id"]
        ids, cnt = oracle.mv(w["gene"].encode(), k, al)
        got = [[oracle.decode_id(int(i), k, al), int(c)] for i, c in zip(ids, cnt)]
        assert got == w["mv"], w["id"]
        assert int(cnt.sum()) == w["n"]
        if "ids" in w:
            assert [int(i) for i in ids] == w["ids"], w["id"]
        og = _og([w["gene"]], k, al)
        assert [int(i) for i in og.ids] == [int(i) for i in ids], w["id"]


def test_jaccard_hand_values(golden):
    for e in golden["jaccard"]:
        al = e.get("alphabet", "aa")
        a, b = _og([e["a"]], e["k"], al), _og([e["b"]], e["k"], al)
        assert a.terms(0, b, 0) == (e["num"], e["den"]), e["id"]
        assert brute.terms(e["a"], e["b"], e["k"]) == (e["num"], e["den"]), e["id"]


def test_best_hits_hand_values(golden):
    for e in golden["best_hits"]:
        k = e["k"]
        gi, gj = _og(e["gi"], k), _og(e["gj"], k)
        ab, ba = oracle.bh(gi, gj, threads=2), oracle.bh(gj, gi, threads=2)
        want_ij = [[tuple(x) for x in row] for row in e["bh_ij"]]
        want_ji = [[tuple(x) for x in row] for row in e["bh_ji"]]
        assert _bh_rows(ab) == want_ij, e["id"]
        assert _bh_rows(ba) == want_ji, e["id"]
        p = oracle.bbh(ab, ba)
        assert [[int(x), int(y)] for x, y in zip(p.a, p.b)] == e["bbh"], e["id"]
        p3 = oracle.bbh_alg3(gi, gj, ab, ba)
        assert [[int(x), int(y)] for x, y in zip(p3.a, p3.b)] == e["bbh"], e["id"]
        assert [list(t) for t in brute.bbh(e["gi"], e["gj"], k)] == e["bbh"], e["id"]


def test_k_rule_hand_values(golden):
    for e in golden["k_rule"]:
        assert oracle.k_rule(e["total"], e["alphabet"], 0) == e["ceil"], e["id"]
        assert oracle.k_rule(e["total"], e["alphabet"], 1) == e["floor"], e["id"]


def test_k_rule_powers():
    # exact powers and their neighbours, against integer arithmetic written independently
    for a in (2, 4, 20):
        for j in range(1, 14):
            p = a ** j
            assert oracle.k_rule(p, a, 0) == j and oracle.k_rule(p, a, 1) == j
            assert oracle.k_rule(p + 1, a, 0) == j + 1 and oracle.k_rule(p + 1, a, 1) == j
            if j >= 2:
                assert oracle.k_rule(p - 1, a, 0) == j and oracle.k_rule(p - 1, a, 1) == j - 1


def test_invalid_residue_is_reported():
    with pytest.raises(ValueError):
        oracle.mv(b"MKXLA", 2)
    with pytest.raises(ValueError):
        _og(["MKVLA", "ACDBQ"], 2)
    # nucleotides: N and amino-acid letters are outside ACGT; T is valid in both alphabets
    with pytest.raises(ValueError):
        oracle.mv(b"ACGNT", 2, "nt")
    with pytest.raises(ValueError):
        _og(["ACGT", "ACDE"], 2, "nt")
    assert oracle.mv(b"ACGT", 2, "nt")[1].sum() == 3
    with pytest.raises(ValueError):
        oracle.mv(b"ACGT", 2, "rna")


def test_k_range_per_alphabet():
    # identifiers are exact 64-bit integers: |alphabet|^k <= 2^64
    assert oracle.k_max("aa") == 14 and 20 ** 14 <= 2 ** 64 < 20 ** 15
    assert oracle.k_max("nt") == 32 and 4 ** 32 == 2 ** 64
    oracle.mv(b"A" * 40, 14)
    oracle.mv(b"A" * 40, 32, "nt")
    for k, al in ((15, "aa"), (33, "nt"), (0, "aa"), (0, "nt")):
        with pytest.raises(ValueError):
            oracle.mv(b"A" * 40, k, al)
        with pytest.raises(ValueError):
            _og(["A" * 40], k, al)


# ------------------------------------------------------------- brute force

def _random_genes(rng, n, alpha, lo=0, hi=40):
    return ["".join(rng.choice(alpha) for _ in range(rng.randint(lo, hi))) for _ in range(n)]


@pytest.mark.parametrize("seed", range(40))
def test_brute_force_tiny(seed):
    rng = random.Random(1000 + seed)
    alpha = ALPHA[: rng.choice([2, 3, 4, 20])]
    k = rng.choice([1, 2, 3])
    gi = _random_genes(rng, rng.randint(1, 8), alpha)
    gj = _random_genes(rng, rng.randint(1, 8), alpha)
    # duplicates force exact ties
    if rng.random() < 0.5 and gj:
        gj.append(gj[0])
    oi, oj = _og(gi, k), _og(gj, k)
    ab, ba = oracle.bh(oi, oj, threads=3), oracle.bh(oj, oi, threads=3)
    want_ab = brute.all_best_hits(gi, gj, k)
    want_ba = brute.all_best_hits(gj, gi, k)
    assert _bh_rows(ab) == [want_ab[r] for r in range(len(gi))]
    assert _bh_rows(ba) == [want_ba[r] for r in range(len(gj))]
    p = oracle.bbh(ab, ba)
    assert list(zip(p.a.tolist(), p.b.tolist())) == brute.bbh(gi, gj, k)
    p3 = oracle.bbh_alg3(oi, oj, ab, ba)
    assert list(zip(p3.a.tolist(), p3.b.tolist())) == brute.bbh(gi, gj, k)
    for a in range(len(gi)):
        for b in range(len(gj)):
            assert oi.terms(a, oj, b) == brute.terms(gi[a], gj[b], k)


@pytest.mark.parametrize("seed", range(24))
def test_brute_force_nucleotide(seed):
    """Nucleotide genes (|alphabet| = 4) with k up to 9: windows repeat often at small k and
    rarely at large k, so both dense and sparse dictionaries are covered."""
    rng = random.Random(5000 + seed)
    k = rng.choice([1, 2, 3, 5, 7, 9])
    gi = _random_genes(rng, rng.randint(1, 7), "ACGT", 0, 70)
    gj = _random_genes(rng, rng.randint(1, 7), "ACGT", 0, 70)
    if gi and gj and rng.random() < 0.5:  # a mutated copy keeps shared k-mers at large k
        s = list(gi[0])
        for p in range(0, len(s), 9):
            s[p] = rng.choice("ACGT")
        gj.append("".join(s))
    oi, oj = _og(gi, k, "nt"), _og(gj, k, "nt")
    ab, ba = oracle.bh(oi, oj, threads=2), oracle.bh(oj, oi, threads=2)
    want_ab = brute.all_best_hits(gi, gj, k)
    want_ba = brute.all_best_hits(gj, gi, k)
    assert _bh_rows(ab) == [want_ab[r] for r in range(len(gi))]
    assert _bh_rows(ba) == [want_ba[r] for r in range(len(gj))]
    p = oracle.bbh(ab, ba)
    assert list(zip(p.a.tolist(), p.b.tolist())) == brute.bbh(gi, gj, k)
    for a, g in enumerate(gi):
        ids, cnt = oi.mv(a)
        assert {oracle.decode_id(int(i), k, "nt"): int(c) for i, c in zip(ids, cnt)} == dict(brute.multiplicities(g, k))


# --------------------------------------------------------------- invariants

def _hist(s):
    return np.bincount([ALPHA.index(c) for c in s], minlength=20) if s else np.zeros(20, int)


@pytest.mark.parametrize("seed", range(10))
def test_k1_is_weighted_jaccard_of_residue_counts(seed):
    rng = random.Random(seed)
    gi = _random_genes(rng, 5, ALPHA[:6], 1, 30)
    gj = _random_genes(rng, 5, ALPHA[:6], 1, 30)
    oi, oj = _og(gi, 1), _og(gj, 1)
    for a in range(5):
        for b in range(5):
            ha, hb = _hist(gi[a]), _hist(gj[b])
            assert oi.terms(a, oj, b) == (int(np.minimum(ha, hb).sum()), int(np.maximum(ha, hb).sum()))


def test_counts_past_16_bits_closed_form():
    # genes past 65535 windows: runs of one letter have one k-mer counted |g| - k + 1 times, and
    # (AC)^n has two k-mers counted half as often each; the sums of Eq. jaccard_k then pass 2^16
    k = 5
    oi = _og(["A" * 70000, "AC" * 35000, "MKVLA"], k)
    oj = _og(["A" * 68000, "CA" * 34000], k)
    assert oi.terms(0, oj, 0) == (68000 - k + 1, 70000 - k + 1)
    n1, n2 = 70000 - k + 1, 68000 - k + 1  # windows of (AC)^35000 and (CA)^34000, both even
    assert oi.terms(1, oj, 1) == (n2, n1)  # each k-mer min(n1/2, n2/2) twice; maxima likewise
    assert oi.terms(0, oj, 1) == (0, n1 + n2)
    ab = oracle.bh(oi, oj, threads=2)
    assert _bh_rows(ab) == [[(0, n2, n1)], [(1, n2, n1)], []]
    sparse = oracle.bh_sparse(oi, oj)
    assert _bh_rows(sparse) == _bh_rows(ab)


@pytest.mark.parametrize("seed", range(10))
def test_multiplicity_one_is_set_jaccard(seed):
    rng = random.Random(50 + seed)
    k = 4
    # random 20-letter genes of length <= 12 almost never repeat a 4-mer; skip any that do
    genes = []
    while len(genes) < 8:
        s = "".join(rng.choice(ALPHA) for _ in range(rng.randint(4, 12)))
        w = [s[p:p + k] for p in range(len(s) - k + 1)]
        if len(set(w)) == len(w):
            genes.append(s)
    genes[1] = genes[0][:2] + genes[1][2:] if len(genes[1]) > 2 else genes[1]
    og = _og(genes, k)
    for a in range(len(genes)):
        for b in range(len(genes)):
            sa = {genes[a][p:p + k] for p in range(len(genes[a]) - k + 1)}
            sb = {genes[b][p:p + k] for p in range(len(genes[b]) - k + 1)}
            if len(sa) == len(genes[a]) - k + 1 and len(sb) == len(genes[b]) - k + 1:
                assert og.terms(a, og, b) == (len(sa & sb), len(sa | sb))


@pytest.mark.parametrize("seed", range(6))
def test_invariants(seed):
    rng = random.Random(200 + seed)
    alpha = ALPHA[: rng.choice([3, 5, 20])]
    k = rng.choice([1, 2, 3])
    gi = _random_genes(rng, 12, alpha, 0, 60)
    gj = _random_genes(rng, 10, alpha, 0, 60)
    oi, oj = _og(gi, k), _og(gj, k)
    for a in range(len(gi)):
        na = int(oi.nwin[a])
        if na:
            assert oi.terms(a, oi, a) == (na, na)  # J(g, g) = 1
        for b in range(len(gj)):
            m, d = oi.terms(a, oj, b)
            assert (m, d) == oj.terms(b, oi, a)  # symmetry
            assert m + d == na + int(oj.nwin[b])  # min + max = x + y, summed
            assert 0 <= m <= d
    ab, ba = oracle.bh(oi, oj), oracle.bh(oj, oi)
    p = oracle.bbh(ab, ba)
    for a, b in zip(p.a, p.b):
        assert b in ab.row(a)[0] and a in ba.row(b)[0]
    # BBH(A, B) is the transpose of BBH(B, A)
    q = oracle.bbh(ba, ab)
    assert sorted(zip(p.a.tolist(), p.b.tolist())) == sorted(zip(q.b.tolist(), q.a.tolist()))


def test_relabelling_permutes_results():
    rng = random.Random(7)
    k = 2
    gi = _random_genes(rng, 9, ALPHA[:4], 2, 30)
    gj = _random_genes(rng, 7, ALPHA[:4], 2, 30)
    pi = list(range(len(gi)))
    pj = list(range(len(gj)))
    rng.shuffle(pi)
    rng.shuffle(pj)
    oi, oj = _og(gi, k), _og(gj, k)
    si, sj = _og([gi[x] for x in pi], k), _og([gj[x] for x in pj], k)
    p = oracle.bbh(oracle.bh(oi, oj), oracle.bh(oj, oi))
    s = oracle.bbh(oracle.bh(si, sj), oracle.bh(sj, si))
    base = set(zip(p.a.tolist(), p.b.tolist()))
    moved = {(pi[a], pj[b]) for a, b in zip(s.a.tolist(), s.b.tolist())}
    assert base == moved


def test_threads_do_not_change_results():
    ds = make_config(2, genomes=2, genes=120)
    k = 4
    a, b = (oracle.OracleGenome(g, k) for g in ds.genomes)
    r1, r8 = oracle.bh(a, b, threads=1), oracle.bh(a, b, threads=8)
    for f in ("ptr", "col", "num", "den"):
        assert np.array_equal(getattr(r1, f), getattr(r8, f))


def test_row_subset_matches_full():
    ds = make_config(2, genomes=2, genes=150)
    k = 4
    a, b = (oracle.OracleGenome(g, k) for g in ds.genomes)
    full = oracle.bh(a, b)
    rows = [5, 0, 149, 77]
    part = oracle.bh(a, b, rows=rows)
    for i, r in enumerate(rows):
        for x, y in zip(part.row(i), full.row(r)):
            assert np.array_equal(x, y)


def test_planted_homologs_are_recovered():
    """Sanity, not parity: on the tiny planted workload almost every planted pair is a BBH."""
    ds = make_config(1)
    k = oracle.k_rule(ds.total_residues(), 20, 0)
    assert k == 4
    og, res = oracle.all_pairs(ds.genomes, k)
    ab, ba, p = res[(0, 1)]
    got = set(zip(p.a.tolist(), p.b.tolist()))
    planted = {(int(a), int(b)) for a, b in ds.meta["planted"]}
    assert len(planted & got) >= 140


# ------------------------------------------------------------ families (phase (c))

def test_families_hand_cases():
    from oracle.families import components
    assert components(5, []) == [0, 1, 2, 3, 4]  # no BBH: every gene its own family
    assert components(4, [(2, 3), (1, 2)]) == [0, 1, 1, 1]  # a path: one family labelled by its smallest gene
    assert components(6, [(5, 0), (4, 3), (3, 5)]) == [0, 1, 2, 0, 0, 0]  # edge order and direction do not matter
    assert components(3, [(1, 1), (2, 1), (1, 2)]) == [0, 1, 1]  # self-loops and repeated edges change nothing


def test_families_match_library_components():
    """The union-find oracle against scipy's connected components on random graphs (labels compared as
    partitions: same component iff same label; the label is the component's smallest node)."""
    import numpy as np
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components

    from oracle.families import components
    rng = np.random.default_rng(3)
    for trial in range(20):
        n = int(rng.integers(1, 300))
        m = int(rng.integers(0, 2 * n))
        u = rng.integers(0, n, m)
        v = rng.integers(0, n, m)
        lab = np.asarray(components(n, zip(u.tolist(), v.tolist())))
        _, comp = connected_components(coo_matrix((np.ones(m), (u, v)), shape=(n, n)), directed=False)
        smallest = {}
        for x in range(n):
            smallest.setdefault(comp[x], x)
        assert np.array_equal(lab, np.array([smallest[c] for c in comp])), trial


# ------------------------------------------------ candidate filters (theta, tau)

def _rows(bh_, n):
    return [[(int(c), int(x), int(y)) for c, x, y in zip(*bh_.row(r))] for r in range(n)]


def test_filter_fixtures(golden):
    from synth import genome_from_strings
    for e in golden["filters"]:
        th = tuple(e["theta"]) if e["theta"] else None
        ta = tuple(e["tau"]) if e["tau"] else None
        gi = oracle.OracleGenome(genome_from_strings(e["gi"]), e["k"])
        gj = oracle.OracleGenome(genome_from_strings(e["gj"]), e["k"])
        ab = oracle.bh(gi, gj, threads=1, theta=th, tau=ta)
        ba = oracle.bh(gj, gi, threads=1, theta=th, tau=ta)
        assert _rows(ab, len(e["gi"])) == [[tuple(x) for x in row] for row in e["bh_ij"]], e["id"]
        assert _rows(ba, len(e["gj"])) == [[tuple(x) for x in row] for row in e["bh_ji"]], e["id"]
        p = oracle.bbh(ab, ba)
        assert [[int(x), int(y)] for x, y in zip(p.a, p.b)] == e["bbh"], e["id"]
        if "bh_ij_unfiltered" in e:
            assert _rows(oracle.bh(gi, gj, threads=1), len(e["gi"])) == \
                [[tuple(x) for x in row] for row in e["bh_ij_unfiltered"]], e["id"]


@pytest.mark.parametrize("seed", range(12))
def test_filters_match_brute(seed):
    from fractions import Fraction

    from synth import genome_from_strings
    rng = random.Random(100 + seed)
    alpha = "ACDEFGHIKLMNPQRSTVWY"[: rng.choice([2, 3, 4, 20])]
    k = rng.choice([1, 2, 3])
    gi = ["".join(rng.choice(alpha) for _ in range(rng.randint(0, 30))) for _ in range(rng.randint(1, 7))]
    gj = ["".join(rng.choice(alpha) for _ in range(rng.randint(0, 30))) for _ in range(rng.randint(1, 7))]
    gi += gi[:1]  # duplicates give ties
    th = rng.choice([None, (1, 2), (3, 4), (9, 10), (0, 1)])
    ta = rng.choice([None, (1, k), (1, 2), (2, 5), (0, 1)])
    oi = oracle.OracleGenome(genome_from_strings(gi), k)
    oj = oracle.OracleGenome(genome_from_strings(gj), k)
    ab = oracle.bh(oi, oj, threads=2, theta=th, tau=ta)
    want = brute.all_best_hits(gi, gj, k, Fraction(*th) if th else None, Fraction(*ta) if ta else None)
    assert _rows(ab, len(gi)) == [want[r] for r in range(len(gi))]


def test_zero_thresholds_filter_nothing():
    ds = make_config(2, genomes=2, genes=120)
    a, b = (oracle.OracleGenome(g, 4) for g in ds.genomes)
    plain = oracle.bh(a, b, threads=2)
    for th, ta in (((0, 1), None), (None, (0, 1)), ((0, 1), (0, 1))):
        f = oracle.bh(a, b, threads=2, theta=th, tau=ta)
        assert np.array_equal(f.ptr, plain.ptr) and np.array_equal(f.col, plain.col)


def test_filters_only_remove_candidates():
    """A row's filtered maximum never exceeds its unfiltered one, and a row whose unfiltered best hits
    all pass the filters keeps exactly them."""
    from fractions import Fraction
    ds = make_config(2, genomes=2, genes=150)
    a, b = (oracle.OracleGenome(g, 4) for g in ds.genomes)
    plain = oracle.bh(a, b, threads=2)
    filt = oracle.bh(a, b, threads=2, theta=(4, 5), tau=(1, 4))
    strs_a = [ds.genomes[0].gene(i).decode() for i in range(ds.genomes[0].n_genes)]
    strs_b = [ds.genomes[1].gene(i).decode() for i in range(ds.genomes[1].n_genes)]
    for r in range(a.n):
        pc, pn, pd = plain.row(r)
        fc, fn, fd = filt.row(r)
        if len(fc):
            assert Fraction(int(fn[0]), int(fd[0])) <= Fraction(int(pn[0]), int(pd[0]))
        if len(pc) and all(brute.candidate(strs_a[r], strs_b[int(c)], 4, Fraction(4, 5), Fraction(1, 4)) for c in pc):
            assert list(fc) == list(pc)
