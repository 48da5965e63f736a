"""GPU parity of the column-maximum mode (PDP_PARAM_COLMAX): the second genome's best hits come
from the column maxima of the first genome's rows (Alg. 3's test S[l,k] = max_r S[r,k]) instead
of a second set of join records and tiles.  Every output must equal the oracle's, exactly as in
the default mode: ties, rows with more ties than a slab keeps, rows summed densely, filters,
capacity retries, nucleotides, and the full 10 x 3000 workload element by element."""
import random

import numpy as np
import pytest

import oracle
from helpers import check_bbh, check_bh, check_bh_properties
from synth import genome_from_strings, make_config

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU collection
    pytest.skip("needs the GPU", allow_module_level=True)

import paper_2510_23679_amd as pdp  # noqa: E402

ALPHA = "ACDEFGHIKLMNPQRSTVWY"


def say(*a):
    print("[case]", *a, flush=True)


def run_all(genomes, k, prm):
    dicts = [pdp.Dictionary.build_from(g, k) for g in genomes]
    runner = pdp.PairRunner(pdp.all_pairs_tasks(dicts), prm)
    runner.run()
    for d in dicts:
        d.check_status()
    return runner


def compare_all(genomes, k, res, theta=None, tau=None):
    _, want = oracle.all_pairs(genomes, k, theta=theta, tau=tau)
    for t, key in enumerate(want):
        ab, ba, bb = want[key]
        check_bh(res.best_hits(t, 0), ab)
        check_bh(res.best_hits(t, 1), ba)
        check_bbh(res.bbh_pairs(t), bb)


def _mutate(rng, s, rate, alpha=ALPHA):
    return "".join(rng.choice(alpha) if rng.random() < rate else ch for ch in s)


@pytest.mark.parametrize("k", [4, 6])
def test_colmax_family_workload(k):
    say("colmax family model, 4 genomes x 400 genes, k =", k)
    ds = make_config(2, genomes=4, genes=400)
    compare_all(ds.genomes, k, run_all(ds.genomes, k, pdp.params(colmax=True)).results())


def test_colmax_paralog_ties():
    say("colmax paralog copies (exact ties)")
    ds = make_config(3, genomes=3, genes_lo=300, genes_hi=500, core=150)
    res = run_all(ds.genomes, 5, pdp.params(colmax=True)).results()
    compare_all(ds.genomes, 5, res)
    ptr = res.best_hits(0, 1)[0].astype(np.int64)
    assert np.any(np.diff(ptr) > 1), "the workload should produce tied column best hits"


def test_colmax_rows_with_many_ties():
    # columns tied at their maximum with more rows than a slab keeps (copies in the first
    # genome), and rows of the first genome with many tied columns
    rng = random.Random(23)
    genes = ["".join(rng.choice(ALPHA) for _ in range(rng.randint(30, 120))) for _ in range(60)]
    a = genes[:30] + [genes[0]] * 6 + [genes[40]] * 9
    b = [genes[0]] * 7 + genes[30:] + [genes[1]] * 5
    rng.shuffle(a)
    rng.shuffle(b)
    ga, gb = genome_from_strings(a), genome_from_strings(b)
    say("colmax rows with many ties")
    res = run_all([ga, gb], 4, pdp.params(colmax=True)).results()
    compare_all([ga, gb], 4, res)
    assert np.diff(res.best_hits(0, 1)[0].astype(np.int64)).max() >= 9
    assert np.diff(res.best_hits(0, 0)[0].astype(np.int64)).max() >= 7


@pytest.mark.parametrize("tile_rows", [1, 64])
def test_colmax_dense_and_grouped_tiles(tile_rows):
    # a row past the LDS table is summed densely and raises its columns' maxima from there
    rng = random.Random(5)
    base = "".join(rng.choice(ALPHA) for _ in range(600))
    a = [base, _mutate(rng, base, 0.02)] + ["".join(rng.choice(ALPHA) for _ in range(200)) for _ in range(40)]
    b = [_mutate(rng, base, 0.03) for _ in range(7)] + [base] * 6
    b += ["".join(rng.choice(ALPHA) for _ in range(200)) for _ in range(40)]
    rng.shuffle(b)
    ga, gb = genome_from_strings(a), genome_from_strings(b)
    say("colmax dense and grouped tiles, tile_rows", tile_rows)
    res = run_all([ga, gb], 5, pdp.params(tile_rows=tile_rows, colmax=True)).results()
    compare_all([ga, gb], 5, res)


@pytest.mark.parametrize("theta,tau", [((3, 4), None), ((1, 2), (1, 3))])
def test_colmax_filters(theta, tau):
    say("colmax filters", theta, tau)
    ds = make_config(2, genomes=3, genes=300)
    res = run_all(ds.genomes, 5, pdp.params(theta=theta, tau=tau, colmax=True)).results()
    compare_all(ds.genomes, 5, res, theta, tau)


def test_colmax_capacity_retry_and_persistent():
    say("colmax with a tiny record capacity (retried) and persistent kernels")
    ds = make_config(2, genomes=3, genes=300)
    runner = run_all(ds.genomes, 5, pdp.params(inc_capacity=100, persistent=True, colmax=True))
    compare_all(ds.genomes, 5, runner.results())


def test_colmax_mixed_task_flags():
    # one-direction tasks keep their own tiles next to column-maximum tasks in one plan
    ds = make_config(2, genomes=3, genes=250)
    k = 5
    dicts = [pdp.Dictionary.build_from(g, k) for g in ds.genomes]
    tasks = [(dicts[0], dicts[1], pdp.PDP_TASK_BBH), (dicts[0], dicts[2], pdp.PDP_TASK_AB),
             (dicts[2], dicts[1], pdp.PDP_TASK_BA), (dicts[1], dicts[2], pdp.PDP_TASK_AB | pdp.PDP_TASK_BA)]
    say("colmax plan mixing task flags")
    runner = pdp.PairRunner(tasks, pdp.params(colmax=True))
    runner.run()
    res = runner.results()
    og = [oracle.OracleGenome(g, k) for g in ds.genomes]
    ab01, ba01 = oracle.bh(og[0], og[1]), oracle.bh(og[1], og[0])
    check_bh(res.best_hits(0, 0), ab01)
    check_bh(res.best_hits(0, 1), ba01)
    check_bbh(res.bbh_pairs(0), oracle.bbh(ab01, ba01))
    check_bh(res.best_hits(1, 0), oracle.bh(og[0], og[2]))
    check_bh(res.best_hits(2, 1), oracle.bh(og[1], og[2]))
    check_bh(res.best_hits(3, 0), oracle.bh(og[1], og[2]))
    check_bh(res.best_hits(3, 1), oracle.bh(og[2], og[1]))


def test_colmax_nucleotide():
    say("colmax nucleotide family, 3 genomes x 250 genes, k = 13")
    ds = make_config(2, genomes=3, genes=250, alphabet="nt")
    compare_all(ds.genomes, 13, run_all(ds.genomes, 13, pdp.params(colmax=True)).results())


def test_colmax_full_size_equals_default():
    """The 10 x 3000 workload: every output array of the column-maximum mode equals the
    default mode's, element by element; sampled rows also against the oracle."""
    ds = make_config(2)
    k = 6
    say("colmax full-size 10 x 3000, against the default mode")
    dicts = [pdp.Dictionary.build_from(g, k) for g in ds.genomes]
    tasks = pdp.all_pairs_tasks(dicts)
    base = pdp.PairRunner(tasks)
    base.run()
    want = base.results()
    runner = pdp.PairRunner(tasks, pdp.params(colmax=True))
    runner.run()
    got = runner.results()
    for x, y in zip(want.bh + want.bbh, got.bh + got.bbh):
        assert np.array_equal(x, y)
    og = [oracle.OracleGenome(g, k) for g in ds.genomes]
    rng = np.random.default_rng(3)
    for t, (i, j) in enumerate(ds.pairs()):
        ba = got.best_hits(t, 1)
        check_bh_properties(got.best_hits(t, 0), ba, got.bbh_pairs(t), ds.genomes[i].n_genes, ds.genomes[j].n_genes)
        if t % 9 == 0:
            cols = np.sort(rng.choice(ds.genomes[j].n_genes, 24, replace=False))
            check_bh(ba, oracle.bh(og[j], og[i], rows=cols), rows=cols)
