"""GPU tests of the serving runtime: results equal the oracle, each request's results are
identical alone and in a concurrent mix, and the HBM budget is enforced."""
import numpy as np
import pytest

import oracle
from helpers import check_bbh, check_bh
from synth import serving_workload

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU collection
    pytest.skip("needs the GPU", allow_module_level=True)

import paper_2510_23679_amd as pdp  # noqa: E402

K = 5


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def workload():
    wl = serving_workload(n_residents=4, resident_genes=200, n_arrivals=6, arrive_lo=80, arrive_hi=300)
    residents = [pdp.Dictionary.build_from(g, K) for g in wl.residents.genomes]
    for d in residents:
        d.check_status()
    arrivals = [wl.arrival(j) for j in range(6)]
    return wl, residents, arrivals


def run_server(residents, arrivals, slots, budget=1 << 30, one_at_a_time=False, prm=None):
    srv = pdp.Server(residents, budget, slots=slots, prm=prm)
    out = {}
    try:
        if one_at_a_time:
            for j, g in enumerate(arrivals):
                srv.submit(g, j)
                done = []
                while not done:
                    done = srv.poll(8, wait_us=200000)
                for d in done:
                    out[d.tag] = (d, srv.fetch(d.tag))
                    srv.release(d.tag)
        else:
            for j, g in enumerate(arrivals):
                srv.submit(g, j)
            while len(out) < len(arrivals):
                for d in srv.poll(8, wait_us=200000):
                    out[d.tag] = (d, srv.fetch(d.tag))
                    srv.release(d.tag)
        stats = srv.stats()
    finally:
        srv.close()
    return out, stats


def test_served_results_match_oracle(workload):
    wl, residents, arrivals = workload
    say("serving: 6 requests x 4 residents, 3 slots")
    out, stats = run_server(residents, arrivals, slots=3)
    assert stats.completed == 6 and stats.peak_inflight >= 2
    og_res = [oracle.OracleGenome(g, K) for g in wl.residents.genomes]
    for j, g in enumerate(arrivals):
        d, res = out[j]
        assert d.code == 0 and res.code == 0
        # the device times of the request's phases, from events on its slot's stream
        assert d.h2d_ms > 0 and d.build_ms > 0 and d.pairs_ms > 0 and d.d2h_ms > 0
        assert d.h2d_ms + d.build_ms + d.pairs_ms + d.d2h_ms <= (d.done_us - d.admit_us) / 1e3 + 0.5
        q = oracle.OracleGenome(g, K)
        for r, og in enumerate(og_res):
            ab, ba = oracle.bh(q, og), oracle.bh(og, q)
            check_bh(res.best_hits(r, 0), ab)
            check_bh(res.best_hits(r, 1), ba)
            check_bbh(res.bbh_pairs(r), oracle.bbh(ab, ba))


def test_served_with_column_maxima_and_tall_tiles(workload):
    # the benchmark's serving parameters: the residents' best hits from the column maxima of the
    # request's rows, 128-row tiles
    wl, residents, arrivals = workload
    say("serving with column maxima and 128-row tiles: 6 requests x 4 residents, 4 slots")
    out, stats = run_server(residents, arrivals, slots=4, prm=pdp.params(colmax=True, tile_rows=128))
    assert stats.completed == 6
    og_res = [oracle.OracleGenome(g, K) for g in wl.residents.genomes]
    for j, g in enumerate(arrivals):
        d, res = out[j]
        assert d.code == 0 and res.code == 0
        q = oracle.OracleGenome(g, K)
        for r, og in enumerate(og_res):
            ab, ba = oracle.bh(q, og), oracle.bh(og, q)
            check_bh(res.best_hits(r, 0), ab)
            check_bh(res.best_hits(r, 1), ba)
            check_bbh(res.bbh_pairs(r), oracle.bbh(ab, ba))


def test_alone_equals_mix(workload):
    _, residents, arrivals = workload
    say("serving: each request alone vs all in a mix")
    alone, _ = run_server(residents, arrivals, slots=1, one_at_a_time=True)
    mixed, stats = run_server(residents, arrivals, slots=4)
    assert stats.peak_inflight >= 2
    for j in range(len(arrivals)):
        a, m = alone[j][1], mixed[j][1]
        for x, y in zip(a.bh + a.bbh, m.bh + m.bbh):
            assert np.array_equal(x, y), f"request {j}"


def test_budget_rejects_oversized_request(workload):
    _, residents, arrivals = workload
    say("serving: budget too small for any request")
    srv = pdp.Server(residents, 1 << 20, slots=2)
    try:
        srv.submit(arrivals[0], 7)
        done = []
        while not done:
            done = srv.poll(4, wait_us=200000)
        assert done[0].tag == 7 and done[0].code == pdp.PDP_E_BUDGET
    finally:
        srv.close()


def test_budget_admits_one_request_at_a_time(workload):
    # a budget that fits the largest request but no two of the requests submitted: they are
    # submitted at once on four slots and wait for memory over many polls.  Waiting is no attempt: each runs
    # once, its admission is stamped when its memory is placed (after its submission and after
    # the previous request's completion), and its results are the oracle's.
    wl, residents, arrivals = workload
    foot = []
    for j, g in enumerate(arrivals):  # each request's footprint, alone
        _, st = run_server(residents, [g], slots=1)
        foot.append(int(st.peak_used_bytes))
    budget = max(foot) + 256
    # the requests of which no two fit together
    big = [j for j in range(len(arrivals)) if 2 * foot[j] > budget]
    assert len(big) >= 3
    say("serving: budget for one request at a time,", len(big), "requests on 4 slots")
    arrivals = [arrivals[j] for j in big]
    out, stats = run_server(residents, arrivals, slots=4, budget=budget)
    n = len(arrivals)
    assert stats.completed == n and stats.peak_inflight == 1 and stats.peak_used_bytes <= budget
    done = sorted((out[j][0] for j in range(n)), key=lambda d: d.admit_us)
    for prev, d in zip([None] + done[:-1], done):
        assert d.code == 0 and d.attempts == 1
        assert d.admit_us >= d.submit_us and d.done_us >= d.admit_us
        if prev is not None:
            assert d.admit_us >= prev.done_us
    og_res = [oracle.OracleGenome(g, K) for g in wl.residents.genomes]
    for j, g in enumerate(arrivals):
        res = out[j][1]
        q = oracle.OracleGenome(g, K)
        for r, og in enumerate(og_res):
            ab, ba = oracle.bh(q, og), oracle.bh(og, q)
            check_bh(res.best_hits(r, 0), ab)
            check_bh(res.best_hits(r, 1), ba)
            check_bbh(res.bbh_pairs(r), oracle.bbh(ab, ba))


def test_served_nucleotide_genomes():
    # residents and requests over ACGT: the server builds each request's dictionary with the
    # residents' alphabet and k
    from synth import make_config

    k = 11
    res_ds = make_config(2, genomes=3, genes=120, alphabet="nt")
    residents = [pdp.Dictionary.build_from(g, k) for g in res_ds.genomes]
    arrivals = make_config(1, alphabet="nt", n_genes=60, n_planted=40).genomes
    say("serving nucleotides: 2 requests x 3 residents, k =", k)
    out, stats = run_server(residents, arrivals, slots=2)
    assert stats.completed == 2
    og_res = [oracle.OracleGenome(g, k) for g in res_ds.genomes]
    for j, g in enumerate(arrivals):
        d, res = out[j]
        assert d.code == 0 and res.code == 0
        q = oracle.OracleGenome(g, k)
        for r, og in enumerate(og_res):
            ab, ba = oracle.bh(q, og), oracle.bh(og, q)
            check_bh(res.best_hits(r, 0), ab)
            check_bh(res.best_hits(r, 1), ba)
            check_bbh(res.bbh_pairs(r), oracle.bbh(ab, ba))
