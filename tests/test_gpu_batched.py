"""GPU tests of the batched forms: many genome pairs of several independent instances in
one plan, persistent kernels, HIP-graph replay and the autotuner.  Results must equal
the oracle and the plain per-pair launches bit for bit."""
import numpy as np
import pytest

import oracle
from helpers import check_bbh, check_bh
from synth import batched_instances, make_config

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU collection
    pytest.skip("needs the GPU", allow_module_level=True)

import paper_2510_23679_amd as pdp  # noqa: E402


def say(*a):
    print("[case]", *a, flush=True)


def small_instances(n=3):
    """Independent pangenome instances with uneven genome counts and sizes (scaled down)."""
    return list(batched_instances(0, n, genomes_lo=2, genomes_hi=4, genes_lo=60, genes_hi=220))


def instance_tasks(insts, stream=None):
    """Dictionaries of every genome of every instance (one build call) and all their pairs."""
    dev, ks, owner = [], [], []
    for ii, ds in enumerate(insts):
        k = pdp.k_rule(ds.total_residues())
        for g in ds.genomes:
            dev.append(pdp.DeviceGenome.of(g))
            ks.append(k)
            owner.append(ii)
    batch = pdp.DictionaryBatch(dev, ks)
    batch.build(stream)
    tasks, keys, base = [], [], 0
    for ii, ds in enumerate(insts):
        n = ds.n_genomes
        for i, j in ds.pairs():
            tasks.append((batch.dicts[base + i], batch.dicts[base + j], pdp.PDP_TASK_BBH))
            keys.append((ii, i, j))
        base += n
    return batch, tasks, keys


def check_against_oracle(insts, res, keys):
    want = {}
    for ii, ds in enumerate(insts):
        k = pdp.k_rule(ds.total_residues())
        _, w = oracle.all_pairs(ds.genomes, k)
        for (i, j), v in w.items():
            want[(ii, i, j)] = v
    for t, key in enumerate(keys):
        ab, ba, bb = want[key]
        check_bh(res.best_hits(t, 0), ab)
        check_bh(res.best_hits(t, 1), ba)
        check_bbh(res.bbh_pairs(t), bb)


@pytest.mark.parametrize("persistent", [False, True])
def test_instances_in_one_plan(persistent):
    say("3 instances in one plan, persistent =", persistent)
    insts = small_instances()
    batch, tasks, keys = instance_tasks(insts)
    batch.check_status()
    runner = pdp.PairRunner(tasks, pdp.params(persistent=persistent))
    runner.run()
    check_against_oracle(insts, runner.results(), keys)


def test_batched_equals_per_pair_launches():
    say("batched plan vs one plan per pair")
    insts = small_instances()
    batch, tasks, keys = instance_tasks(insts)
    runner = pdp.PairRunner(tasks, pdp.params(persistent=True))
    runner.run()
    res = runner.results()
    for t, task in enumerate(tasks):
        single = pdp.PairRunner([task])
        single.run()
        one = single.results()
        for d in (0, 1):
            for x, y in zip(res.best_hits(t, d), one.best_hits(0, d)):
                assert np.array_equal(x, y)
        for x, y in zip(res.bbh_pairs(t), one.bbh_pairs(0)):
            assert np.array_equal(x, y)


def test_graph_replays_match_eager():
    """Build + pair launch captured once; replayed several times with eager work and
    synchronisations between replays; every replay equals the eager result."""
    say("graph capture and replay")
    insts = small_instances()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        batch, tasks, keys = instance_tasks(insts, stream)
        runner = pdp.PairRunner(tasks, pdp.params(persistent=True))
        runner.run(stream)  # sizes the buffers, uploads the plan
        eager = runner.results()
        graph = pdp.Graph.capture(stream)
        with graph:
            batch.build(stream)
            runner.launch(stream)
        for rep in range(4):
            # eager work in between: clobber the outputs, then replay
            runner.bh.col.fill_(-1)
            if runner.bbh is not None:
                runner.bbh.a.fill_(-1)
            scratch = torch.randn(1 << 20, device="cuda", dtype=torch.float32).sum()
            stream.synchronize()
            graph.launch(stream)
            stream.synchronize()
            assert pdp.read_status(runner.status)[0] == 0
            again = runner.results()
            for x, y in zip(eager.bh + eager.bbh, again.bh + again.bbh):
                assert np.array_equal(x, y), f"replay {rep}"
            del scratch
    check_against_oracle(insts, eager, keys)


def test_autotune_picks_a_clean_candidate():
    say("autotune on a small workload")
    ds = make_config(2, genomes=3, genes=300)
    k = 5
    dicts = [pdp.Dictionary.build_from(g, k) for g in ds.genomes]
    tasks = pdp.all_pairs_tasks(dicts)
    best, res = pdp.autotune(tasks, reps=2)
    assert res.tried >= 12 and res.best_ms > 0 and res.best_ms <= res.first_ms
    runner = pdp.PairRunner(tasks, best)
    runner.run()
    og, want = oracle.all_pairs(ds.genomes, k)
    out = runner.results()
    for t, key in enumerate(want):
        ab, ba, bb = want[key]
        check_bh(out.best_hits(t, 0), ab)
        check_bh(out.best_hits(t, 1), ba)
        check_bbh(out.bbh_pairs(t), bb)
