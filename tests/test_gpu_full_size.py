"""Full-size GPU parity for the batched and served forms, in the launch configurations the
benchmark times: the first wave of the 400-instance batched workload (independent instances of
U{4..30} genomes x U{500..5000} genes, k per instance by the rule, 128-row tiles and 512-entry
join sub-ranges, not persistent) and full-size arrivals served against all 200 resident genomes
of 4000 genes (k = 7 fixed from the residents; 4 slots, column maxima, 128-row tiles).  Every genome pair is compared in full -- every
best-hit row both ways and the whole BBH set -- against the sparse oracle, whose agreement with
the dense oracle and with brute force the CPU tests pin."""
import numpy as np
import pytest

import oracle
from helpers import check_bh, check_pair_complete
from synth import batched_instances, serving_workload

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU collection
    pytest.skip("needs the GPU", allow_module_level=True)

import paper_2510_23679_amd as pdp  # noqa: E402

WAVE_GENOMES = 256  # genomes per batched wave, as the benchmark packs them


def say(*a):
    print("[case]", *a, flush=True)


@pytest.mark.timeout(900)
def test_full_size_batched_first_wave_complete():
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
    del runner, batch, devs
    say("comparing", len(tasks), "pairs against the sparse oracle")
    t = 0
    for x, ds in enumerate(wave):
        og = oracle.genomes(ds.genomes, spans[x][2])
        want = oracle.all_pairs_sparse(og)
        for i in range(len(ds.genomes)):
            for j in range(i + 1, len(ds.genomes)):
                assert where[t] == (x, i, j)
                check_pair_complete(res.best_hits(t, 0), res.best_hits(t, 1), res.bbh_pairs(t), want[(i, j)],
                                    ds.genomes[i].n_genes, ds.genomes[j].n_genes)
                t += 1
    assert t == len(tasks)


@pytest.mark.timeout(900)
def test_full_size_serving_complete():
    wl = serving_workload()
    k = pdp.k_rule(wl.residents.total_residues())
    assert k == 7
    say("serving: 200 residents x 4000 genes, k =", k)
    batch = pdp.DictionaryBatch([pdp.DeviceGenome.of(g) for g in wl.residents.genomes], k)
    batch.build()
    torch.cuda.synchronize()
    batch.check_status()
    arrivals = [wl.arrival(j) for j in range(3)]
    # the benchmark's serving configuration: 4 slots, column maxima, 128-row tiles
    srv = pdp.Server(batch.dicts, 32 << 30, slots=4, prm=pdp.params(colmax=True, tile_rows=128))
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
    del batch
    og_res = oracle.genomes(wl.residents.genomes, k)
    n_res = len(og_res)
    for j, g in enumerate(arrivals):
        d, res = out[j]
        assert d.code == 0 and res.code == 0
        say("arrival", j, "genes", g.n_genes, "against all", n_res, "residents")
        og = og_res + [oracle.OracleGenome(g, k)]
        dirs = [(n_res, r) for r in range(n_res)] + [(r, n_res) for r in range(n_res)]
        hits = oracle.bh_sparse_directions(og, dirs)
        for r in range(n_res):
            ab, ba = hits[(n_res, r)], hits[(r, n_res)]
            check_pair_complete(res.best_hits(r, 0), res.best_hits(r, 1), res.bbh_pairs(r),
                                (ab, ba, oracle.bbh(ab, ba)), g.n_genes, wl.residents.genomes[r].n_genes)
        # one resident's rows against the dense oracle as well
        rows = np.unique(np.linspace(0, g.n_genes - 1, 40).astype(np.uint32))
        check_bh(res.best_hits(0, 0), oracle.bh(og[n_res], og_res[0], rows=rows), rows=rows)
