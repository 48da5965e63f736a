"""GPU parity: the HIP path through the C-ABI against the CPU oracle, element by element.

Every integer output must be bit-exact: dictionaries, best-hit sets with their
(sum of minima, sum of maxima), and BBH pairs.  Each test prints its case
before touching the GPU.
"""
import random

import numpy as np
import pytest

import oracle
from helpers import check_bbh, check_bh, check_bh_properties, check_dictionary, check_pair_complete
from synth import genome_from_strings, make_config

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU collection
    pytest.skip("needs the GPU", allow_module_level=True)

import paper_2510_23679_amd as pdp  # noqa: E402

ALPHA = "ACDEFGHIKLMNPQRSTVWY"


def say(*a):
    print("[case]", *a, flush=True)


def run_all(genomes, k, prm=None, flags=pdp.PDP_TASK_BBH, pairs=None):
    dicts = [pdp.Dictionary.build_from(g, k) for g in genomes]
    runner = pdp.PairRunner(pdp.all_pairs_tasks(dicts, pairs, flags), prm)
    runner.run()
    for d in dicts:
        d.check_status()
    return dicts, runner.results()


def compare_all(genomes, k, res, pairs=None):
    og, want = oracle.all_pairs(genomes, k, pairs=pairs)
    keys = list(want.keys())
    for t, key in enumerate(keys):
        ab, ba, bb = want[key]
        check_bh(res.best_hits(t, 0), ab)
        check_bh(res.best_hits(t, 1), ba)
        check_bbh(res.bbh_pairs(t), bb)
    return og


# ------------------------------------------------------------ hand examples

def test_hand_examples(golden):
    for e in golden["best_hits"]:
        say("hand example", e["id"])
        gi, gj = genome_from_strings(e["gi"]), genome_from_strings(e["gj"])
        _, res = run_all([gi, gj], e["k"])
        for direction, key in ((0, "bh_ij"), (1, "bh_ji")):
            ptr, col, num, den = res.best_hits(0, direction)
            got = [[(int(col[p]), int(num[p]), int(den[p])) for p in range(ptr[r], ptr[r + 1])]
                   for r in range(len(ptr) - 1)]
            assert got == [[tuple(x) for x in row] for row in e[key]], e["id"]
        a, b, _, _ = res.bbh_pairs(0)
        assert [[int(x), int(y)] for x, y in zip(a, b)] == e["bbh"], e["id"]


def test_jaccard_examples(golden):
    for e in golden["jaccard"]:
        if e["num"] == 0:
            continue
        say("jaccard example", e["id"])
        al = e.get("alphabet", "aa")
        _, res = run_all([genome_from_strings([e["a"]], alphabet=al), genome_from_strings([e["b"]], alphabet=al)],
                         e["k"])
        ptr, col, num, den = res.best_hits(0, 0)
        assert (int(num[0]), int(den[0])) == (e["num"], e["den"]), e["id"]


def test_windows_examples(golden):
    for w in golden["windows"]:
        say("window example", w["id"])
        g = genome_from_strings([w["gene"]], alphabet=w.get("alphabet", "aa"))
        d = pdp.Dictionary.build_from(g, w["k"])
        d.check_status()
        check_dictionary(d.host(), oracle.OracleGenome(g, w["k"]))


# ------------------------------------------------------------- dictionaries

@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6, 7, 12])
def test_dictionary_parity(k):
    say("dictionary parity k =", k)
    ds = make_config(2, genomes=1, genes=300)
    g = ds.genomes[0]
    d = pdp.Dictionary.build_from(g, k)
    d.check_status()
    check_dictionary(d.host(), oracle.OracleGenome(g, k))


def test_dictionary_long_genes_and_big_buckets():
    # genes longer than a wave's register sort (1024 windows) and than the LDS sort (8192
    # windows), and leading-residue buckets far above the per-thread insertion sort and the
    # LDS bucket sort (low-complexity prefixes)
    rng = random.Random(3)
    genes = ["A" * 5000 + "".join(rng.choice(ALPHA) for _ in range(300))]
    genes += ["".join(rng.choice(ALPHA) for _ in range(9500))]
    genes += ["".join(rng.choice("AC") for _ in range(3000))]
    genes += ["AAAA" + "".join(rng.choice(ALPHA) for _ in range(rng.randint(4, 30))) for _ in range(3000)]
    genes += ["", "M", "MK"]
    g = genome_from_strings(genes)
    for k in (4, 6, 7):  # k = 7 sorts base-20 keys
        say("long genes / big buckets, k =", k)
        d = pdp.Dictionary.build_from(g, k)
        d.check_status()
        check_dictionary(d.host(), oracle.OracleGenome(g, k))


def test_dictionary_rejects_bad_residue():
    say("alphabet error")
    g = genome_from_strings(["MKVLA", "ACDXE", "MKB"])
    d = pdp.Dictionary.build_from(g, 2)
    code, needed, where = d.status()
    assert code == pdp.PDP_E_ALPHABET and where == 8


def test_dictionary_past_16_bit_windows():
    # a gene of 69,998 windows: bound for long genes (from the host offsets), its one k-mer is
    # counted 69,998 times; the pair path for such genomes is in test_gpu_long_genes.py
    say("dictionary past the 16-bit window limit")
    g = genome_from_strings(["A" * 70000, "MKV", "M" * 5 + "A" * 66000])
    d = pdp.Dictionary.build_from(g, 3)
    assert d.long_genes
    d.check_status()
    host = d.host()
    check_dictionary(host, oracle.OracleGenome(g, 3))
    assert int(host["mv_cnt"][0]) == 70000 - 3 + 1


# ----------------------------------------------------------- best hits, BBH

def test_planted_pair_full():
    say("planted pair, 2 x 200 genes")
    ds = make_config(1)
    k = pdp.k_rule(ds.total_residues())
    assert k == oracle.k_rule(ds.total_residues()) == 4
    dicts, res = run_all(ds.genomes, k)
    for d, g in zip(dicts, ds.genomes):
        check_dictionary(d.host(), oracle.OracleGenome(g, k))
    compare_all(ds.genomes, k, res)


@pytest.mark.parametrize("k", [4, 5, 6])
def test_family_model_small_all_pairs(k):
    say("family model, 4 genomes x 400 genes, k =", k)
    ds = make_config(2, genomes=4, genes=400)
    _, res = run_all(ds.genomes, k)
    compare_all(ds.genomes, k, res)


# The join finds a packed query entry's bucket from the low word of its code when the tail leaves
# enough leading letters there (amino acids up to k = 7, nucleotides up to 23 tail bits), and by a
# search of the item's directory otherwise: both sides of each limit, both alphabets, with and
# without column maxima.
@pytest.mark.parametrize("alphabet,k,genes", [("aa", 7, 300), ("aa", 8, 300), ("nt", 20, 250), ("nt", 21, 200)])
@pytest.mark.parametrize("colmax", [False, True])
def test_query_bucket_modes(alphabet, k, genes, colmax):
    say("query buckets:", alphabet, "k =", k, genes, "genes x 3 genomes, column maxima", colmax)
    ds = make_config(2, genomes=3, genes=genes, alphabet=alphabet)
    dicts, res = run_all(ds.genomes, k, pdp.params(colmax=colmax))
    assert all(d.d.key_shift > 0 for d in dicts)  # packed keys: the join path under test
    compare_all(ds.genomes, k, res)


# The genome with fewer entries queries the join whichever the caller names first (the plan
# swaps the task internally): both orders of a pair of unequal genomes, each with BH both ways
# and BBH, and pdp_bh with either genome as the query, against the oracle.
@pytest.mark.parametrize("colmax", [False, True])
def test_both_orders_of_unequal_genomes(colmax):
    say("both orders of an unequal pair, column maxima", colmax)
    ds = make_config(3, genomes=2, genes_lo=150, genes_hi=450, core=120)
    g0, g1 = ds.genomes
    assert abs(int(g0.offsets[-1]) - int(g1.offsets[-1])) > 1000  # unequal, so one order swaps
    pairs = [(0, 1), (1, 0)]
    dicts, res = run_all(ds.genomes, 5, pdp.params(colmax=colmax), pairs=pairs)
    compare_all(ds.genomes, 5, res, pairs=pairs)
    og = [oracle.OracleGenome(g, 5) for g in ds.genomes]
    for q, tg in ((0, 1), (1, 0)):
        check_bh(pdp.bh(dicts[q], dicts[tg]).host(), oracle.bh(og[q], og[tg]))


def test_paralog_ties():
    say("paralog copies (exact ties), 3 genomes")
    ds = make_config(3, genomes=3, genes_lo=300, genes_hi=500, core=150)
    k = 5
    _, res = run_all(ds.genomes, k)
    compare_all(ds.genomes, k, res)
    ptr = res.best_hits(0, 0)[0].astype(np.int64)
    assert np.any(np.diff(ptr) > 1), "the workload should produce tied best hits"


@pytest.mark.parametrize("seed", range(6))
def test_random_tiny_with_ties(seed):
    rng = random.Random(seed)
    alpha = ALPHA[: rng.choice([2, 3, 4, 20])]
    k = rng.choice([1, 2, 3])
    gens = []
    for _ in range(3):
        genes = ["".join(rng.choice(alpha) for _ in range(rng.randint(0, 40))) for _ in range(rng.randint(1, 30))]
        genes += genes[: rng.randint(0, 3)]  # duplicates force ties
        gens.append(genome_from_strings(genes))
    say("random tiny, seed", seed, "alphabet", len(alpha), "k", k)
    _, res = run_all(gens, k)
    compare_all(gens, k, res)


@pytest.mark.parametrize("colmax", [False, True])
def test_genome_without_genes(colmax):
    # the empty genome is the smaller one, so it takes the join's query side (the task swaps)
    say("empty genome, column maxima", colmax)
    a = genome_from_strings(["MKVLA", "MKVIA"])
    b = genome_from_strings([])
    _, res = run_all([a, b], 2, pdp.params(colmax=colmax))
    ptr, col, _, _ = res.best_hits(0, 0)
    assert list(ptr) == [0, 0, 0] and len(col) == 0
    assert len(res.best_hits(0, 1)[0]) == 1
    assert len(res.bbh_pairs(0)[0]) == 0


@pytest.mark.parametrize("prm", [dict(tile_rows=1), dict(tile_rows=7, join_entries=64),
                                 dict(lds_budget=8192, join_entries=1024), dict(inc_capacity=100),
                                 dict(persistent=True), dict(persistent=True, lds_budget=128 * 1024, join_entries=256)])
def test_tuning_knobs_do_not_change_results(prm):
    say("tuning", prm)
    ds = make_config(2, genomes=3, genes=300)
    k = 5
    _, res = run_all(ds.genomes, k, pdp.params(**prm))
    compare_all(ds.genomes, k, res)


def _mutate(rng, s, rate):
    return "".join(rng.choice(ALPHA) if rng.random() < rate else ch for ch in s)


@pytest.mark.parametrize("tile_rows", [1, 64])
def test_tiles_past_the_lds_sort(tile_rows):
    # a row whose records overflow the LDS table and sort: 13 copies of one 600-residue
    # gene (6 exact, so the row has 6 tied best hits and is rewritten by the second tile
    # launch) give its tile ~7800 records and the copies' tiles ~1200 each, so hashed,
    # grouped and dense tiles mix in one launch
    rng = random.Random(5)
    base = "".join(rng.choice(ALPHA) for _ in range(600))
    a = [base, _mutate(rng, base, 0.02)] + ["".join(rng.choice(ALPHA) for _ in range(200)) for _ in range(40)]
    b = [_mutate(rng, base, 0.03) for _ in range(7)] + [base] * 6
    b += ["".join(rng.choice(ALPHA) for _ in range(200)) for _ in range(40)]
    rng.shuffle(b)
    ga, gb = genome_from_strings(a), genome_from_strings(b)
    say("tiles past the LDS sort, tile_rows", tile_rows)
    _, res = run_all([ga, gb], 5, pdp.params(tile_rows=tile_rows))
    compare_all([ga, gb], 5, res)


def test_rows_with_many_ties():
    # rows tied with more best hits than the slab keeps: their tiles are recomputed and
    # written in column order by the second tile launch
    rng = random.Random(21)
    genes = ["".join(rng.choice(ALPHA) for _ in range(rng.randint(30, 120))) for _ in range(60)]
    a = genes[:30] + [genes[0]] * 3
    b = [genes[0]] * 7 + genes[30:] + [genes[1]] * 5 + [genes[2]] * 4
    rng.shuffle(b)
    ga, gb = genome_from_strings(a), genome_from_strings(b)
    say("rows with many ties")
    _, res = run_all([ga, gb], 4)
    compare_all([ga, gb], 4, res)
    ptr = res.best_hits(0, 0)[0].astype(np.int64)
    assert np.diff(ptr).max() >= 7


def test_dense_tile_in_several_passes():
    # 20000 target genes leave LDS room for one dense row at a time, so the overflowing
    # tile is summed in one pass per row
    rng = random.Random(9)
    base = "".join(rng.choice(ALPHA) for _ in range(500))
    a = [base] + ["".join(rng.choice(ALPHA) for _ in range(60)) for _ in range(69)]
    b = [_mutate(rng, base, 0.02) for _ in range(12)]
    b += ["".join(rng.choice(ALPHA) for _ in range(rng.randint(8, 30))) for _ in range(20000)]
    rng.shuffle(b)
    ga, gb = genome_from_strings(a), genome_from_strings(b)
    say("dense tile in several passes, 70 x 20012 genes")
    _, res = run_all([ga, gb], 4)
    compare_all([ga, gb], 4, res)


def test_capacity_overflow_reads_no_unwritten_records():
    # a record capacity far below what the join counts: the first launch must stop at the
    # count, report PDP_E_CAPACITY with the count, and touch none of the (poisoned) record
    # scratch; the retry with the reported size gives the oracle's results
    ds = make_config(1)
    k = 4
    dicts = [pdp.Dictionary.build_from(g, k) for g in ds.genomes]
    say("capacity overflow with a poisoned workspace")
    runner = pdp.PairRunner(pdp.all_pairs_tasks(dicts), pdp.params(inc_capacity=64))
    runner.ws.buf.fill_(255)  # every unwritten record would name row 255, column 2^24 - 1
    runner.launch()
    code, needed, where = pdp.read_status(runner.status)
    assert code == pdp.PDP_E_CAPACITY and where == 0 and needed > 64
    ptr = runner.bh.host()[0]
    assert int(ptr[-1]) == 0  # every row empty in the overflowed launch
    runner.run()
    compare_all(ds.genomes, k, runner.results())


def test_best_hit_capacity_overflow_with_bbh():
    # best-hit output far below the tied rows' entries, BBH on, every buffer poisoned: the launch
    # reports PDP_E_CAPACITY for the best hits (where = 1), the BBH kernels walk nothing (all BBH
    # rows empty), and the retry with the reported size gives the oracle's results
    rng = random.Random(21)
    genes = ["".join(rng.choice(ALPHA) for _ in range(rng.randint(30, 120))) for _ in range(60)]
    a = genes[:30] + [genes[0]] * 3
    b = [genes[0]] * 7 + genes[30:] + [genes[1]] * 5 + [genes[2]] * 4
    rng.shuffle(b)
    gens = [genome_from_strings(a), genome_from_strings(b)]
    k = 4
    dicts = [pdp.Dictionary.build_from(g, k) for g in gens]
    say("best-hit capacity overflow with BBH, poisoned buffers")
    runner = pdp.PairRunner(pdp.all_pairs_tasks(dicts), bh_capacity=8)
    runner.ws.buf.fill_(255)
    for t in (runner.bh.col, runner.bh.num, runner.bh.den, runner.bbh.a, runner.bbh.b):
        t.fill_(0x7F7F7F7F)  # a column read from here would index far past every array
    runner.launch()
    code, needed, where = pdp.read_status(runner.status)
    assert code == pdp.PDP_E_CAPACITY and where == 1 and needed > 8
    assert int(runner.bbh.ptr.cpu().numpy().view(np.uint32)[-1]) == 0
    runner.run()
    compare_all(gens, k, runner.results())


def test_standalone_bbh_rejects_overflowed_best_hits():
    # pdp_bbh given a best-hit output whose total exceeds its capacity (the output of an
    # overflowed call) reports PDP_E_CAPACITY (where = 1) and walks none of its entries
    from paper_2510_23679_amd import binding as B
    import ctypes as C
    ds = make_config(2, genomes=2, genes=300)
    k = 5
    da, db = (pdp.Dictionary.build_from(g, k) for g in ds.genomes)
    ab, ba = pdp.bh(da, db), pdp.bh(db, da)
    n_ab = int(ab.ptr.cpu().numpy().view(np.uint32)[-1])
    say("pdp_bbh on an overflowed best-hit output")
    short = pdp.BHOut(ab.n_rows, n_ab // 2)
    short.ptr.copy_(ab.ptr)
    short.col.fill_(0x7F7F7F7F)
    out = pdp.BBHOut(ab.n_rows, ab.n_rows + 1024)
    st = pdp.new_status()
    need = B.u64(0)
    B.check(B.lib().pdp_bbh_ws_size(ab.n_rows, C.byref(need)), "pdp_bbh_ws_size")
    ws = pdp.Workspace(need.value)
    x, y, o = short.struct(), ba.struct(), out.struct()
    B.check(B.lib().pdp_bbh(C.byref(x), C.byref(y), C.byref(o), st.data_ptr(), ws.ptr, ws.nbytes,
                            int(torch.cuda.current_stream().cuda_stream)), "pdp_bbh")
    code, needed, where = pdp.read_status(st)
    assert code == pdp.PDP_E_CAPACITY and where == 1 and needed == n_ab
    assert int(out.ptr.cpu().numpy().view(np.uint32)[-1]) == 0
    oa, ob = (oracle.OracleGenome(g, k) for g in ds.genomes)
    check_bbh(pdp.bbh(ab, ba).host()[1:], oracle.bbh(oracle.bh(oa, ob), oracle.bh(ob, oa)))


def test_join_global_search_path():
    # one leading-residue bucket holding more target entries than the join stages in LDS
    rng = random.Random(11)
    a = genome_from_strings(["WWWW" + "".join(rng.choice(ALPHA) for _ in range(8)) for _ in range(300)])
    b = genome_from_strings(["WWWW" + "".join(rng.choice(ALPHA) for _ in range(6)) for _ in range(3000)])
    say("join with a bucket past the LDS stage")
    _, res = run_all([a, b], 6, pdp.params(join_entries=16))
    compare_all([a, b], 6, res)


def test_kmer_shared_by_hundreds_of_genes():
    # a k-mer present in 300 genes of the target genome: one query entry with 300 partners in
    # the join, and a row with many tied columns
    rng = random.Random(31)
    core = "".join(rng.choice(ALPHA) for _ in range(80))
    a = [core] + ["".join(rng.choice(ALPHA) for _ in range(rng.randint(40, 120))) for _ in range(50)]
    b = [core[:40] + "".join(rng.choice(ALPHA) for _ in range(20)) for _ in range(300)]
    b += ["".join(rng.choice(ALPHA) for _ in range(rng.randint(40, 120))) for _ in range(60)]
    rng.shuffle(b)
    ga, gb = genome_from_strings(a), genome_from_strings(b)
    say("k-mer shared by 300 target genes")
    _, res = run_all([ga, gb], 5)
    compare_all([ga, gb], 5, res)


def test_single_direction_and_standalone_bbh():
    say("pdp_bh both ways + pdp_bbh")
    ds = make_config(2, genomes=2, genes=350)
    k = 5
    da, db = (pdp.Dictionary.build_from(g, k) for g in ds.genomes)
    ab = pdp.bh(da, db)
    ba = pdp.bh(db, da)
    out = pdp.bbh(ab, ba)
    oa, ob = (oracle.OracleGenome(g, k) for g in ds.genomes)
    wab, wba = oracle.bh(oa, ob), oracle.bh(ob, oa)
    check_bh(ab.host(), wab)
    check_bh(ba.host(), wba)
    ptr, a, b, num, den = out.host()
    check_bbh((a, b, num, den), oracle.bbh(wab, wba))


def test_repeat_runs_identical():
    say("determinism across runs")
    ds = make_config(2, genomes=3, genes=300)
    dicts = [pdp.Dictionary.build_from(g, 5) for g in ds.genomes]
    runner = pdp.PairRunner(pdp.all_pairs_tasks(dicts))
    runner.run()
    first = runner.results()
    for _ in range(3):
        runner.run()
        again = runner.results()
        for x, y in zip(first.bh + first.bbh, again.bh + again.bbh):
            assert np.array_equal(x, y)


@pytest.mark.timeout(900)
def test_full_size_family_model_complete():
    """All 45 pairs of the 10 x 3000-gene workload in one launch (the benchmark's configuration):
    every best-hit row both ways and every BBH set against the sparse oracle, plus sampled rows of
    five pairs against the dense oracle."""
    ds = make_config(2)
    k = pdp.k_rule(ds.total_residues())
    assert k == 6
    og = oracle.genomes(ds.genomes, k)
    want = oracle.all_pairs_sparse(og, ds.pairs())
    dicts = [pdp.Dictionary.build_from(g, k) for g in ds.genomes]
    rng = np.random.default_rng(7)
    # the launch shapes the benchmark's autotuner chooses between
    for prm in (pdp.params(), pdp.params(colmax=True), pdp.params(colmax=True, tile_rows=128),
                pdp.params(colmax=True, join_entries=768)):
        say("full-size 10 x 3000 workload, k =", k, "column maxima", bool(prm.flags & 2), "tile rows", prm.tile_rows,
            "join entries", prm.join_entries)
        runner = pdp.PairRunner(pdp.all_pairs_tasks(dicts), prm)
        runner.run()
        res = runner.results()
        for t, (i, j) in enumerate(ds.pairs()):
            ab, ba, bb = res.best_hits(t, 0), res.best_hits(t, 1), res.bbh_pairs(t)
            check_pair_complete(ab, ba, bb, want[(i, j)], ds.genomes[i].n_genes, ds.genomes[j].n_genes)
            if t % 9 == 0:
                rows = np.sort(rng.choice(ds.genomes[i].n_genes, 24, replace=False))
                check_bh(ab, oracle.bh(og[i], og[j], rows=rows), rows=rows)


@pytest.mark.timeout(900)
def test_full_size_large_workload_complete():
    """All 1225 pairs of the 50 x U{3000..5000}-gene workload with paralog copies (exact and near
    ties) in one launch, k = 7 by the rule: every best-hit row both ways and every BBH set against
    the sparse oracle; tied best hits must be present."""
    ds = make_config(3)
    k = pdp.k_rule(ds.total_residues())
    assert k == 7
    say("full-size 50-genome workload, k =", k, "pairs", len(ds.pairs()))
    dicts = pdp.DictionaryBatch([pdp.DeviceGenome.of(g) for g in ds.genomes], k)
    dicts.build()
    dicts.check_status()
    # the default launch shape and the one the benchmark's autotuner picks on this workload
    results = []
    for prm in (pdp.params(), pdp.params(colmax=True, tile_rows=128),
                pdp.params(colmax=True, tile_rows=128, join_entries=768)):
        runner = pdp.PairRunner(pdp.all_pairs_tasks(dicts.dicts), prm)
        runner.run()
        results.append(runner.results())
        del runner
    del dicts
    og = oracle.genomes(ds.genomes, k)
    want = oracle.all_pairs_sparse(og, ds.pairs())
    say("sparse oracle done; comparing 1225 pairs in three launch shapes")
    ties = 0
    for t, (i, j) in enumerate(ds.pairs()):
        w = want.pop((i, j))
        for res in results:
            ab, ba, bb = res.best_hits(t, 0), res.best_hits(t, 1), res.bbh_pairs(t)
            check_pair_complete(ab, ba, bb, w, ds.genomes[i].n_genes, ds.genomes[j].n_genes)
        ties += int(np.sum(np.diff(ab[0].astype(np.int64)) > 1))
    assert ties > 0, "the paralog copies should give tied best hits"


def test_build_many_mixed_k_and_empty_genomes():
    say("pdp_dict_build_many: 5 genomes, mixed k, an empty genome")
    ds = make_config(2, genomes=3, genes=200)
    gens = [ds.genomes[0], genome_from_strings([]), ds.genomes[1], genome_from_strings(["", "MK", "A" * 3000]),
            ds.genomes[2]]
    ks = [5, 4, 6, 3, 1]
    batch = pdp.DictionaryBatch([pdp.DeviceGenome.of(g) for g in gens], ks)
    batch.build()
    batch.check_status()
    for d, g, k in zip(batch.dicts, gens, ks):
        check_dictionary(d.host(), oracle.OracleGenome(g, k))
    batch.build()  # the same workspace again
    batch.check_status()
    for d, g, k in zip(batch.dicts, gens, ks):
        check_dictionary(d.host(), oracle.OracleGenome(g, k))


# ------------------------------------------------------------ families (phase (c))

def _families_run(genomes, k):
    dicts = [pdp.Dictionary.build_from(g, k) for g in genomes]
    pairs = [(i, j) for i in range(len(genomes)) for j in range(i + 1, len(genomes))]
    runner = pdp.PairRunner(pdp.all_pairs_tasks(dicts, pairs))
    runner.run()
    base = np.concatenate([[0], np.cumsum([g.n_genes for g in genomes])]).astype(np.int64)
    node_a = [base[i] for i, _ in pairs]
    node_b = [base[j] for _, j in pairs]
    labels = runner.families(node_a, node_b, int(base[-1]))
    assert pdp.read_status(runner.fam_status)[0] == 0
    return runner, pairs, base, node_a, node_b, labels.cpu().numpy().view(np.uint32)


def test_families_match_oracle():
    from oracle.families import bbh_edges, components
    ds = make_config(2, genomes=4, genes=300)
    k = 5
    say("families of 4 x 300 genes")
    runner, pairs, base, node_a, node_b, got = _families_run(ds.genomes, k)
    _, want = oracle.all_pairs(ds.genomes, k, pairs=pairs)
    edges = bbh_edges([want[key][2] for key in want], node_a, node_b)
    assert len(edges) > 100
    assert np.array_equal(got, np.asarray(components(int(base[-1]), edges), dtype=np.uint32))


def test_families_full_size_properties():
    """The 10 x 3000 workload: every BBH pair joins one family, each label is its family's smallest
    gene, and the partition equals the connected components of the GPU's own BBH pairs."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    ds = make_config(2)
    k = pdp.k_rule(ds.total_residues())
    say("families of the 10 x 3000 workload")
    runner, pairs, base, node_a, node_b, got = _families_run(ds.genomes, k)
    res = runner.results()
    u, v = [], []
    for t in range(len(pairs)):
        a, b, _, _ = res.bbh_pairs(t)
        u.append(node_a[t] + a.astype(np.int64))
        v.append(node_b[t] + b.astype(np.int64))
    u, v = np.concatenate(u), np.concatenate(v)
    n = int(base[-1])
    assert np.array_equal(got[u], got[v])
    assert np.all(got <= np.arange(n)) and np.array_equal(got[got], got)
    _, comp = connected_components(coo_matrix((np.ones(len(u)), (u, v)), shape=(n, n)), directed=False)
    smallest = {}
    for x in range(n):
        smallest.setdefault(comp[x], x)
    assert np.array_equal(got, np.array([smallest[c] for c in comp], dtype=np.uint32))


# ------------------------------------------------ candidate filters (theta, tau)

def test_filter_fixtures_on_gpu(golden):
    for e in golden["filters"]:
        say("filter fixture", e["id"])
        gi, gj = genome_from_strings(e["gi"]), genome_from_strings(e["gj"])
        prm = pdp.params(theta=tuple(e["theta"]) if e["theta"] else None, tau=tuple(e["tau"]) if e["tau"] else None)
        _, res = run_all([gi, gj], e["k"], prm)
        for direction, key, n in ((0, "bh_ij", len(e["gi"])), (1, "bh_ji", len(e["gj"]))):
            ptr, col, num, den = res.best_hits(0, direction)
            got = [[[int(col[p]), int(num[p]), int(den[p])] for p in range(ptr[r], ptr[r + 1])] for r in range(n)]
            assert got == e[key], (e["id"], key)
        a, b, _, _ = res.bbh_pairs(0)
        assert [[int(x), int(y)] for x, y in zip(a, b)] == e["bbh"], e["id"]


def _compare_filtered(genomes, k, res, theta, tau):
    _, want = oracle.all_pairs(genomes, k, theta=theta, tau=tau)
    for t, key in enumerate(want):
        ab, ba, bb = want[key]
        check_bh(res.best_hits(t, 0), ab)
        check_bh(res.best_hits(t, 1), ba)
        check_bbh(res.bbh_pairs(t), bb)


@pytest.mark.parametrize("theta,tau", [((3, 4), None), (None, (1, 5)), ((1, 2), (1, 3)), ((9, 10), (2, 5))])
def test_filters_family_workload(theta, tau):
    say("filters theta", theta, "tau", tau)
    ds = make_config(2, genomes=3, genes=300)
    k = 5
    _, res = run_all(ds.genomes, k, pdp.params(theta=theta, tau=tau))
    _compare_filtered(ds.genomes, k, res, theta, tau)


@pytest.mark.parametrize("tile_rows", [1, 64])
def test_filters_on_dense_and_rewritten_tiles(tile_rows):
    # the overflowing tile of test_tiles_past_the_lds_sort (dense passes, a row with 6 ties rewritten
    # by the second tile launch), with both filters on
    rng = random.Random(5)
    base = "".join(rng.choice(ALPHA) for _ in range(600))
    a = [base, _mutate(rng, base, 0.02), base[:420]] + ["".join(rng.choice(ALPHA) for _ in range(200)) for _ in range(40)]
    b = [_mutate(rng, base, 0.03) for _ in range(7)] + [base] * 6 + [base[:300]]
    b += ["".join(rng.choice(ALPHA) for _ in range(200)) for _ in range(40)]
    rng.shuffle(b)
    ga, gb = genome_from_strings(a), genome_from_strings(b)
    say("filters on dense and rewritten tiles, tile_rows", tile_rows)
    theta, tau = (3, 4), (1, 5)
    _, res = run_all([ga, gb], 5, pdp.params(tile_rows=tile_rows, theta=theta, tau=tau))
    _compare_filtered([ga, gb], 5, res, theta, tau)
