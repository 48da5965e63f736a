"""GPU parity on nucleotide genomes (|alphabet| = 4, 2-bit letters, k up to 31) against the CPU
oracle.  Nucleotide genes are about three times as long as proteins and k is larger, so these
cases drive the wave, work-group and global-memory sorts of the dictionary build, the 4^9
bucket directory, packed and unpacked join keys, and denser random k-mer matches per row."""
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

NT = "ACGT"


def say(*a):
    print("[case]", *a, flush=True)


def run_all(genomes, k, prm=None, flags=pdp.PDP_TASK_BBH):
    dicts = [pdp.Dictionary.build_from(g, k) for g in genomes]
    runner = pdp.PairRunner(pdp.all_pairs_tasks(dicts, None, flags), prm)
    runner.run()
    for d in dicts:
        d.check_status()
    return dicts, runner.results()


def compare_all(genomes, k, res, theta=None, tau=None):
    _, want = oracle.all_pairs(genomes, k, theta=theta, tau=tau)
    for t, key in enumerate(want):
        ab, ba, bb = want[key]
        check_bh(res.best_hits(t, 0), ab)
        check_bh(res.best_hits(t, 1), ba)
        check_bbh(res.bbh_pairs(t), bb)


def test_k_rule_nucleotide_workload():
    ds = make_config(2, alphabet="nt")
    total = ds.total_residues()
    assert pdp.k_rule(total, 4) == oracle.k_rule(total, 4) == 13


# k below, at and above the 9 bucket letters; packed keys up to k = 20 for 300 genes
# (2 (k - 9) + 9 <= 32), unpacked above
@pytest.mark.parametrize("k", [1, 3, 8, 9, 10, 13, 16, 20, 21, 31])
def test_dictionary_parity_nucleotide(k):
    say("nucleotide dictionary parity k =", k)
    ds = make_config(2, genomes=1, genes=300, alphabet="nt")
    g = ds.genomes[0]
    d = pdp.Dictionary.build_from(g, k)
    d.check_status()
    assert d.d.alphabet == pdp.binding.PDP_ALPHA_NUCLEOTIDE and d.d.lead == min(k, 9)
    check_dictionary(d.host(), oracle.OracleGenome(g, k))


def test_dictionary_nucleotide_sort_paths_and_big_buckets():
    """Window counts at the edges of the wave sort (256, 512, 1024 windows), the LDS sort
    (8192) and past it, genes shorter than k, and low-complexity genes whose k-mers crowd a
    few buckets."""
    rng = random.Random(11)
    k = 13
    lens = [0, 1, k - 1, k, 256 + k - 1, 257 + k - 1, 1024 + k - 1, 1025 + k - 1, 8192 + k - 1,
            8193 + k - 1, 12000]
    genes = ["".join(rng.choice(NT) for _ in range(n)) for n in lens]
    genes += ["A" * 3000, "AC" * 2500, "ACGT" * 1000 + "".join(rng.choice(NT) for _ in range(500))]
    genes += ["AAAAAAAAA" + "".join(rng.choice(NT) for _ in range(rng.randint(4, 40))) for _ in range(2000)]
    g = genome_from_strings(genes, alphabet="nt")
    for kk in (9, 13, 24):
        say("nucleotide sort paths / big buckets, k =", kk)
        d = pdp.Dictionary.build_from(g, kk)
        d.check_status()
        check_dictionary(d.host(), oracle.OracleGenome(g, kk))


def test_dictionary_rejects_letters_outside_acgt():
    for genes, where in ((["ACGT", "ACGNA"], 7), (["ACGU"], 3), (["ACDE", "ACGT"], 2)):
        say("nucleotide alphabet error", genes)
        d = pdp.Dictionary.build_from(genome_from_strings(genes, alphabet="nt"), 2)
        code, _, at = d.status()
        assert code == pdp.PDP_E_ALPHABET and at == where
    # the same letters are valid amino acids
    d = pdp.Dictionary.build_from(genome_from_strings(["ACDE", "ACGT"]), 2)
    d.check_status()


def test_pair_needs_one_alphabet():
    a = pdp.Dictionary.build_from(genome_from_strings(["ACGTACGT"], alphabet="nt"), 4)
    b = pdp.Dictionary.build_from(genome_from_strings(["ACGTACGT"]), 4)
    with pytest.raises(pdp.PdpError) as e:
        pdp.PairRunner(pdp.all_pairs_tasks([a, b]))
    assert e.value.code == pdp.PDP_E_INVAL


def test_planted_pair_nucleotide():
    ds = make_config(1, alphabet="nt")
    k = pdp.k_rule(ds.total_residues(), 4)
    assert k == oracle.k_rule(ds.total_residues(), 4)
    say("nucleotide planted pair, 2 x 200 genes, k =", k)
    dicts, res = run_all(ds.genomes, k)
    for d, g in zip(dicts, ds.genomes):
        check_dictionary(d.host(), oracle.OracleGenome(g, k))
    compare_all(ds.genomes, k, res)
    # the planted homologs are best hits of each other
    ptr, col, _, _ = res.best_hits(0, 0)
    planted = ds.meta["planted"]
    found = sum(int(b) in col[ptr[a]:ptr[a + 1]] for a, b in planted)
    assert found >= 0.9 * len(planted)


@pytest.mark.parametrize("k", [11, 13, 15, 22])
def test_family_model_nucleotide_all_pairs(k):
    say("nucleotide family model, 4 genomes x 300 genes, k =", k)
    ds = make_config(2, genomes=4, genes=300, alphabet="nt")
    _, res = run_all(ds.genomes, k)
    compare_all(ds.genomes, k, res)


@pytest.mark.parametrize("prm", [dict(tile_rows=8), dict(tile_rows=128, join_entries=128),
                                 dict(lds_budget=96 * 1024, persistent=True)])
def test_nucleotide_tuning_knobs(prm):
    say("nucleotide knobs", prm)
    ds = make_config(2, genomes=3, genes=250, alphabet="nt")
    _, res = run_all(ds.genomes, 13, pdp.params(**prm))
    compare_all(ds.genomes, 13, res)


@pytest.mark.parametrize("theta,tau", [((3, 4), None), ((1, 2), (1, 10))])
def test_nucleotide_filters(theta, tau):
    say("nucleotide filters theta", theta, "tau", tau)
    ds = make_config(2, genomes=3, genes=250, alphabet="nt")
    _, res = run_all(ds.genomes, 13, pdp.params(theta=theta, tau=tau))
    compare_all(ds.genomes, 13, res, theta, tau)


@pytest.mark.timeout(900)
def test_full_size_nucleotide_complete():
    """All 45 pairs of 10 nucleotide genomes x 3000 genes (k = 13) in one launch: every best-hit row
    both ways and every BBH set against the sparse oracle, one dictionary against the oracle's."""
    ds = make_config(2, alphabet="nt")
    k = pdp.k_rule(ds.total_residues(), 4)
    say("full-size nucleotide 10 x 3000 workload, k =", k)
    dicts = [pdp.Dictionary.build_from(g, k) for g in ds.genomes]
    runner = pdp.PairRunner(pdp.all_pairs_tasks(dicts))
    runner.run()
    for d in dicts:
        d.check_status()
    res = runner.results()
    og = oracle.genomes(ds.genomes, k)
    check_dictionary(dicts[3].host(), og[3])
    want = oracle.all_pairs_sparse(og, ds.pairs())
    for t, (i, j) in enumerate(ds.pairs()):
        ab, ba, bb = res.best_hits(t, 0), res.best_hits(t, 1), res.bbh_pairs(t)
        check_pair_complete(ab, ba, bb, want[(i, j)], ds.genomes[i].n_genes, ds.genomes[j].n_genes)
