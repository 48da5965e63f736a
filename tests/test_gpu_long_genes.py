"""GPU parity of genes past 65535 k-mer windows against the CPU oracle, in both alphabets.

Such genes need 32-bit multiplicities and sums of minima (Eq. kmer_multiplicity, Eq.
jaccard_k): a 70,000-letter low-complexity gene has one k-mer about 70,000 times, and two of
them share a sum of minima above 2^16.  Their dictionaries are bound for long genes (the
Python layer does it from the host offsets), and every task that names one takes the
long-gene path.  Each test prints its case before touching the GPU.
"""
import random

import pytest

import oracle
from helpers import check_bbh, check_bh, check_dictionary
from synth import genome_from_strings

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU collection
    pytest.skip("needs the GPU", allow_module_level=True)

import paper_2510_23679_amd as pdp  # noqa: E402

LETTERS = {"aa": "ACDEFGHIKLMNPQRSTVWY", "nt": "ACGT"}
K = {"aa": 5, "nt": 13}


def say(*a):
    print("[case]", *a, flush=True)


def _mutate(s, rng, rate, letters):
    return "".join(c if rng.random() >= rate else rng.choice(letters) for c in s)


def long_genomes(alphabet, seed=11, extra_b=0):
    """Two genomes of ~130 related genes each, plus long genes: a random 70,000-letter gene and
    its 5%-mutated copy, and runs of 70,000 and 68,000 copies of one letter (one k-mer past
    2^16 occurrences on both sides).  Genome b also holds six identical copies of one of a's
    genes (a row with more ties than the first tile pass keeps) and extra_b short genes."""
    L = LETTERS[alphabet]
    rng = random.Random(seed)
    base = ["".join(rng.choice(L) for _ in range(rng.randint(40, 500))) for _ in range(120)]
    rand_long = "".join(rng.choice(L) for _ in range(70000))
    a = [_mutate(g, rng, 0.1, L) for g in base] + [rand_long, "A" * 70000, base[0], "", "A"]
    b = [_mutate(g, rng, 0.15, L) for g in base[::-1]] + ["A" * 68000, _mutate(rand_long, rng, 0.05, L)]
    b += [base[1]] * 6
    b += ["".join(rng.choice(L) for _ in range(rng.randint(20, 60))) for _ in range(extra_b)]
    return genome_from_strings(a, alphabet=alphabet), genome_from_strings(b, alphabet=alphabet)


def run_pair(genomes, k, prm=None):
    dicts = [pdp.Dictionary.build_from(g, k) for g in genomes]
    runner = pdp.PairRunner(pdp.all_pairs_tasks(dicts, None, pdp.PDP_TASK_BBH), prm)
    runner.run()
    for d in dicts:
        d.check_status()
    return dicts, runner


def compare(genomes, k, res, theta=None, tau=None):
    _, want = oracle.all_pairs(genomes, k, theta=theta, tau=tau)
    for t, key in enumerate(want):
        ab, ba, bb = want[key]
        check_bh(res.best_hits(t, 0), ab)
        check_bh(res.best_hits(t, 1), ba)
        check_bbh(res.bbh_pairs(t), bb)


@pytest.mark.parametrize("alphabet", ["aa", "nt"])
def test_dictionary_of_long_genes(alphabet):
    k = K[alphabet]
    say("long-gene dictionary", alphabet, "k =", k)
    a, _ = long_genomes(alphabet)
    d = pdp.Dictionary.build_from(a, k)
    assert d.long_genes
    d.check_status()
    host = d.host()
    check_dictionary(host, oracle.OracleGenome(a, k))
    assert int(host["mv_cnt"].max()) == 70000 - k + 1  # the run of one letter: one k-mer, counted in 32 bits


def test_dictionary_without_long_flag_rejects_long_gene():
    say("window limit without the long-gene flag")
    g = genome_from_strings(["A" * 70000, "MKV"])
    d = pdp.Dictionary(len(g.offsets) - 1, int(g.offsets[-1]), 3)
    assert not d.long_genes
    d.build(pdp.DeviceGenome.of(g))
    code, needed, where = d.status()
    assert code == pdp.PDP_E_LIMIT and where == 0 and needed == 70000 - 3 + 1


@pytest.mark.parametrize("alphabet", ["aa", "nt"])
def test_long_gene_pair_complete(alphabet):
    k = K[alphabet]
    say("long-gene pair, complete BH both ways + BBH", alphabet, "k =", k)
    gens = long_genomes(alphabet)
    dicts, runner = run_pair(gens, k)
    assert all(d.long_genes for d in dicts)
    assert runner.plan.info.long_rows == gens[0].offsets.shape[0] - 1 + gens[1].offsets.shape[0] - 1
    res = runner.results()
    compare(gens, k, res)
    # the two runs of one letter: the sum of minima passes 16 bits
    ptr, col, num, den = res.best_hits(0, 0)
    row = 121  # "A" * 70000 in genome a
    hits = [(int(col[p]), int(num[p]), int(den[p])) for p in range(ptr[row], ptr[row + 1])]
    assert hits == [(120, 68000 - k + 1, 70000 - k + 1)]


@pytest.mark.parametrize("prm", [dict(theta=(3, 4)), dict(tau=(1, 5)), dict(theta=(1, 2), tau=(1, 3)),
                                 dict(colmax=True), dict(colmax=True, tile_rows=128)])
def test_long_gene_pair_params(prm):
    say("long-gene pair with", prm)
    gens = long_genomes("aa", seed=5)
    _, runner = run_pair(gens, 5, pdp.params(**prm))
    compare(gens, 5, runner.results(), theta=prm.get("theta"), tau=prm.get("tau"))


def test_long_gene_column_blocks():
    # a column genome of more than 4096 genes: the long-gene path sums its columns in blocks
    say("long-gene pair, 4,600 column genes")
    gens = long_genomes("aa", seed=7, extra_b=4500)
    _, runner = run_pair(gens, 5)
    compare(gens, 5, runner.results())


def test_mixed_plan_long_and_default_tasks():
    # one plan: a default task between two ordinary genomes and long-gene tasks beside it
    say("mixed plan: default and long-gene tasks")
    a, b = long_genomes("aa", seed=9)
    rng = random.Random(4)
    L = LETTERS["aa"]
    c = genome_from_strings(["".join(rng.choice(L) for _ in range(rng.randint(40, 400))) for _ in range(150)])
    d = genome_from_strings(["".join(rng.choice(L) for _ in range(rng.randint(40, 400))) for _ in range(140)])
    gens = [a, b, c, d]
    dicts, runner = run_pair(gens, 5, pdp.params(colmax=True))
    assert [x.long_genes for x in dicts] == [True, True, False, False]
    info = runner.plan.info
    assert info.long_rows > 0 and info.join_groups > 0
    compare(gens, 5, runner.results())


def test_kernel_timers_on_a_plan_without_join_items():
    # every kernel group of the timer hook reads back on a plan whose tasks all take the
    # long-gene path (no join items, no tiles)
    say("kernel timers, long-gene plan")
    gens = long_genomes("aa", seed=3)
    _, runner = run_pair(gens, 5)
    assert runner.plan.info.join_groups == 0 and runner.plan.info.tiles == 0
    for name, kid in pdp.binding.KERNELS.items():
        runner.plan.timer_start(kid, 2)
        runner.launch()
        runner.launch()
        ms, n = runner.plan.timer_read()
        runner.plan.timer_stop()
        assert n == 2 and ms >= 0.0, name
    torch.cuda.synchronize()
    compare(gens, 5, runner.results())


def test_pdp_bh_and_noalloc_on_long_genes():
    # the single-pair entry points on long-gene dictionaries: pdp_bh with a workspace and the
    # no-allocation form agree with each other and with the oracle
    say("pdp_bh and pdp_bh_noalloc on a long-gene pair")
    a, b = long_genomes("aa", seed=13)
    da, db = pdp.Dictionary.build_from(a, 5), pdp.Dictionary.build_from(b, 5)
    want = oracle.bh(oracle.OracleGenome(a, 5), oracle.OracleGenome(b, 5))
    for fn in (pdp.bh, pdp.bh_noalloc):
        check_bh(fn(da, db).host(), want)


def test_served_request_with_a_long_gene():
    # the server binds a request's dictionary for long genes when one of its genes passes the
    # 16-bit window limit; its pairs with every resident then take the long-gene path
    say("serving: a request with a 70,000-letter gene against 3 residents")
    rng = random.Random(21)
    L = LETTERS["aa"]
    res_genomes = [genome_from_strings(["".join(rng.choice(L) for _ in range(rng.randint(40, 400)))
                                        for _ in range(120)]) for _ in range(3)]
    residents = [pdp.Dictionary.build_from(g, 5) for g in res_genomes]
    a, _ = long_genomes("aa", seed=17)
    short = genome_from_strings(["".join(rng.choice(L) for _ in range(rng.randint(40, 400))) for _ in range(80)])
    arrivals = [a, short]
    srv = pdp.Server(residents, 1 << 30, slots=2)
    out = {}
    try:
        for j, g in enumerate(arrivals):
            srv.submit(g, j)
        while len(out) < len(arrivals):
            for d in srv.poll(8, wait_us=200000):
                out[d.tag] = (d, srv.fetch(d.tag))
                srv.release(d.tag)
    finally:
        srv.close()
    og_res = [oracle.OracleGenome(g, 5) for g in res_genomes]
    for j, g in enumerate(arrivals):
        d, res = out[j]
        assert d.code == 0 and res.code == 0
        q = oracle.OracleGenome(g, 5)
        for r, og in enumerate(og_res):
            ab, ba = oracle.bh(q, og), oracle.bh(og, q)
            check_bh(res.best_hits(r, 0), ab)
            check_bh(res.best_hits(r, 1), ba)
            check_bbh(res.bbh_pairs(r), oracle.bbh(ab, ba))
