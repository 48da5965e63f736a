"""Full-size GPU parity for the batched and served forms, in the launch configurations the
benchmark times: the first wave of the 400-instance batched workload (independent instances of
U{4..30} genomes x U{500..5000} genes, k per instance by the rule, 128-row tiles and 512-entry
join sub-ranges, not persistent) and full-size arrivals served against all 200 resident genomes
of 4000 genes (k = 7 fixed from the residents).  Sampled rows are checked against the oracle one
by one (first and last rows included), and the outputs (every third pair of the wave, every
resident of a request) against the properties that hold at any size."""
import numpy as np
import pytest

import oracle
from helpers import check_bbh, check_bh, check_bh_properties
from synth import batched_instances, serving_workload

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU collection
    pytest.skip("needs the GPU", allow_module_level=True)

import paper_2510_23679_amd as pdp  # noqa: E402

WAVE_GENOMES = 256  # genomes per batched wave, as the benchmark packs them


def say(*a):
    print("[case]", *a, flush=True)


def sampled_rows(rng, n, m=16):
    rows = rng.choice(n, min(m, n), replace=False)
    return np.unique(np.concatenate([[0, n - 1], rows]))


def test_full_size_batched_first_wave_sampled():
    wave, genomes = [], 0
    for ds in batched_instances(0, 400):
        if wave and genomes + len(ds.genomes) > WAVE_GENOMES:
            break
        wave.append(ds)
        genomes += len(ds.genomes)
    devs, ks, spans = [], [], []
    for ds in wave:
        k = pdp.k_rule(ds.total_residues())
        spans.append((len(devs), len(ds.genomes), k))
        for g in ds.genomes:
            devs.append(pdp.DeviceGenome.of(g))
            ks.append(k)
    say("batched first wave:", len(wave), "instances,", len(devs), "genomes, k per instance", [s[2] for s in spans])
    batch = pdp.DictionaryBatch(devs, ks)
    batch.build()
    batch.check_status()
    tasks, where = [], []
    for x, (first, n, k) in enumerate(spans):
        for i in range(n):
            for j in range(i + 1, n):
                tasks.append((batch.dicts[first + i], batch.dicts[first + j],
                              pdp.PDP_TASK_AB | pdp.PDP_TASK_BA | pdp.PDP_TASK_BBH))
                where.append((x, i, j))
    runner = pdp.PairRunner(tasks, pdp.params(tile_rows=128, join_entries=512))
    runner.run()
    res = runner.results()
    rng = np.random.default_rng(41)
    picked = list(range(0, len(tasks), 97)) + [len(tasks) - 1]
    cache = {}

    def og(x, i):
        if (x, i) not in cache:
            cache[(x, i)] = oracle.OracleGenome(wave[x].genomes[i], spans[x][2])
        return cache[(x, i)]

    for t in range(0, len(where), 3):  # every third pair: the property checks loop in Python
        x, i, j = where[t]
        ab, ba, bb = res.best_hits(t, 0), res.best_hits(t, 1), res.bbh_pairs(t)
        check_bh_properties(ab, ba, bb, wave[x].genomes[i].n_genes, wave[x].genomes[j].n_genes)
    say("sampled pairs:", len(picked), "of", len(tasks))
    for t in picked:
        x, i, j = where[t]
        a, b = og(x, i), og(x, j)
        rows = sampled_rows(rng, wave[x].genomes[i].n_genes)
        check_bh(res.best_hits(t, 0), oracle.bh(a, b, rows=rows), rows=rows)
        cols = sampled_rows(rng, wave[x].genomes[j].n_genes)
        check_bh(res.best_hits(t, 1), oracle.bh(b, a, rows=cols), rows=cols)


def test_full_size_serving_sampled():
    wl = serving_workload()
    k = pdp.k_rule(wl.residents.total_residues())
    assert k == 7
    say("serving: 200 residents x 4000 genes, k =", k)
    batch = pdp.DictionaryBatch([pdp.DeviceGenome.of(g) for g in wl.residents.genomes], k)
    batch.build()
    torch.cuda.synchronize()
    batch.check_status()
    arrivals = [wl.arrival(j) for j in range(3)]
    srv = pdp.Server(batch.dicts, 32 << 30, slots=8, prm=pdp.params())
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
    rng = np.random.default_rng(43)
    residents = [0, 71, 142, 199]
    og_res = {r: oracle.OracleGenome(wl.residents.genomes[r], k) for r in residents}
    for j, g in enumerate(arrivals):
        d, res = out[j]
        assert d.code == 0 and res.code == 0
        say("arrival", j, "genes", g.n_genes)
        for r in range(len(wl.residents.genomes)):
            check_bh_properties(res.best_hits(r, 0), res.best_hits(r, 1), res.bbh_pairs(r), g.n_genes,
                                wl.residents.genomes[r].n_genes)
        q = oracle.OracleGenome(g, k)
        for r in residents:
            rows = sampled_rows(rng, g.n_genes)
            check_bh(res.best_hits(r, 0), oracle.bh(q, og_res[r], rows=rows), rows=rows)
            cols = sampled_rows(rng, wl.residents.genomes[r].n_genes)
            check_bh(res.best_hits(r, 1), oracle.bh(og_res[r], q, rows=cols), rows=cols)
        # a request's BBH against one resident, in full: both directions computed by the oracle
        ab, ba = oracle.bh(q, og_res[0]), oracle.bh(og_res[0], q)
        check_bbh(res.bbh_pairs(0), oracle.bbh(ab, ba))
