"""GPU parity of the join's two layouts of the shared-k-mer records.

By default one pass searches each query entry once and writes its records into
per-tile regions that the plan sizes from the record capacity.  When a region
overflows, the count pass, the scan and the write pass run after it and lay the
records out exactly (pdp_status.flags reports PDP_STATUS_TWO_PASS), and the
regions are refitted to that launch's counts for the next launch.  PDP_PARAM_TWO_PASS
asks for the two passes from the start.  Each layout must give the oracle's best
hits and BBH, element by element.
"""
import random

import numpy as np
import pytest

import oracle
from helpers import check_bbh, check_bh
from synth import genome_from_strings, make_config

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU collection
    pytest.skip("needs the GPU", allow_module_level=True)

import paper_2510_23679_amd as pdp  # noqa: E402

ALPHA = "ACDEFGHIKLMNPQRSTVWY"


def say(*a):
    print("[case]", *a, flush=True)


def _runner(genomes, k, prm):
    dicts = [pdp.Dictionary.build_from(g, k) for g in genomes]
    runner = pdp.PairRunner(pdp.all_pairs_tasks(dicts), prm)
    return dicts, runner


def _compare(genomes, k, res):
    _, want = oracle.all_pairs(genomes, k)
    for t, key in enumerate(want.keys()):
        ab, ba, bb = want[key]
        check_bh(res.best_hits(t, 0), ab)
        check_bh(res.best_hits(t, 1), ba)
        check_bbh(res.bbh_pairs(t), bb)


def _needed_records(genomes, k, persistent):
    """The exact record count of a workload: the capacity error of a launch with room for 64."""
    _, r = _runner(genomes, k, pdp.params(inc_capacity=64, persistent=persistent))
    r.launch()
    code, needed, where = pdp.read_status(r.status)
    assert code == pdp.PDP_E_CAPACITY and where == 0
    return needed


@pytest.mark.parametrize("persistent", [False, True])
def test_one_pass_default_fits_its_regions(persistent):
    say("one-pass join, family model 4 x 400, k 5, persistent", persistent)
    ds = make_config(2, genomes=4, genes=400)
    _, r = _runner(ds.genomes, 5, pdp.params(persistent=persistent))
    code, _, _ = r.run()
    assert code == 0
    assert pdp.status_flags(r.status) == 0, "the default regions should hold this workload"
    _compare(ds.genomes, 5, r.results())


@pytest.mark.parametrize("persistent", [False, True])
def test_two_pass_flag(persistent):
    say("two-pass join by request, family model 4 x 400, k 5, persistent", persistent)
    ds = make_config(2, genomes=4, genes=400)
    _, r = _runner(ds.genomes, 5, pdp.params(two_pass=True, persistent=persistent))
    r.run()
    assert pdp.status_flags(r.status) == 0
    _compare(ds.genomes, 5, r.results())


@pytest.mark.parametrize("persistent", [False, True])
def test_region_overflow_falls_back_to_two_passes(persistent):
    # a capacity equal to the exact record count: split over the tiles by rows, some tile's
    # region is too small, so the two passes redo the layout within the same capacity
    ds = make_config(2, genomes=3, genes=300)
    k = 5
    needed = _needed_records(ds.genomes, k, persistent)
    say("region overflow, capacity", needed, "persistent", persistent)
    _, r = _runner(ds.genomes, k, pdp.params(inc_capacity=needed, persistent=persistent))
    r.ws.buf.fill_(255)  # records the fallback fails to rewrite would name row 255, column 2^24 - 1
    code, _, _ = r.run(max_tries=1)
    assert code == 0
    assert pdp.status_flags(r.status) & pdp.PDP_STATUS_TWO_PASS
    _compare(ds.genomes, k, r.results())
    # the fallback refitted the regions to the exact counts (no slack is left here): the next
    # launch of the same plan on the same dictionaries fits in one pass
    r.launch()
    assert pdp.read_status(r.status)[0] == 0 and pdp.status_flags(r.status) == 0
    _compare(ds.genomes, k, r.results())
    # a fresh upload of the plan tables restores the estimated regions, and the fallback again
    r.plan.upload(r.ws)
    r.launch()
    assert pdp.read_status(r.status)[0] == 0 and pdp.status_flags(r.status) & pdp.PDP_STATUS_TWO_PASS
    _compare(ds.genomes, k, r.results())


def test_one_pass_equals_two_pass_on_skewed_join():
    # a k-mer shared by 300 target genes and a bucket past the LDS stage: the one-pass join's
    # global-memory search and its skewed tiles, against the two-pass layout and the oracle
    rng = random.Random(5)
    core = "".join(rng.choice(ALPHA) for _ in range(80))
    a = [core] + ["WWWW" + "".join(rng.choice(ALPHA) for _ in range(rng.randint(8, 60))) for _ in range(200)]
    b = [core[:40] + "".join(rng.choice(ALPHA) for _ in range(20)) for _ in range(300)]
    b += ["WWWW" + "".join(rng.choice(ALPHA) for _ in range(rng.randint(6, 40))) for _ in range(1500)]
    rng.shuffle(b)
    gens = [genome_from_strings(a), genome_from_strings(b)]
    k = 5
    outs = []
    for two in (False, True):
        say("skewed join, two_pass", two)
        _, r = _runner(gens, k, pdp.params(two_pass=two, join_entries=16))
        r.run()
        res = r.results()
        _compare(gens, k, res)
        outs.append([np.concatenate([x.astype(np.int64) for x in res.best_hits(0, d)]) for d in (0, 1)])
    for x, y in zip(*outs):
        assert np.array_equal(x, y)


def test_one_pass_unpacked_codes():
    # k = 12 amino acids: no packed keys, the one-pass join stages 64-bit codes
    rng = random.Random(9)
    anc = ["".join(rng.choice(ALPHA) for _ in range(rng.randint(30, 200))) for _ in range(120)]
    gens = []
    for _ in range(3):
        genes = []
        for s in anc:
            t = list(s)
            for i in range(len(t)):
                if rng.random() < 0.03:
                    t[i] = rng.choice(ALPHA)
            genes.append("".join(t))
        rng.shuffle(genes)
        gens.append(genome_from_strings(genes))
    k = 12
    say("unpacked codes, k 12, 3 genomes x 120 genes")
    _, r = _runner(gens, k, pdp.params())
    r.run()
    assert pdp.status_flags(r.status) == 0
    _compare(gens, k, r.results())


def test_graph_replays_refit_after_fallback():
    # a plan whose regions overflow, captured in a HIP graph after a fresh upload of its tables:
    # the first replay falls back to two passes and refits the regions, the later replays fit in
    # one pass; eager work between the replays, every replay equal to the eager result
    ds = make_config(2, genomes=3, genes=300)
    k = 5
    needed = _needed_records(ds.genomes, k, False)
    say("graph replays around a region refit, capacity", needed)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        dicts, r = _runner(ds.genomes, k, pdp.params(inc_capacity=needed))
        r.run(stream)
        eager = r.results()
        r.plan.upload(r.ws, stream)  # back to the estimated regions
        graph = pdp.Graph.capture(stream)
        with graph:
            r.launch(stream)
        for rep in range(4):
            r.bh.col.fill_(-1)
            r.bbh.a.fill_(-1)
            scratch = torch.randn(1 << 20, device="cuda", dtype=torch.float32).sum()
            stream.synchronize()
            graph.launch(stream)
            stream.synchronize()
            assert pdp.read_status(r.status)[0] == 0
            flags = pdp.status_flags(r.status)
            assert bool(flags & pdp.PDP_STATUS_TWO_PASS) == (rep == 0), f"replay {rep}: flags {flags}"
            again = r.results()
            for x, y in zip(eager.bh + eager.bbh, again.bh + again.bbh):
                assert np.array_equal(x, y), f"replay {rep}"
            del scratch
    _compare(ds.genomes, k, eager)
