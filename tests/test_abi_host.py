"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports every
function include/pdp.h declares, and its host-only logic (k rule, sizes, bind,
planning, validation) behaves as documented."""
import ctypes as C
import os
import re

import pytest

import oracle
import paper_2510_23679_amd as pdp
from paper_2510_23679_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pdp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pdp_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    L = pdp.lib()
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(B.SIGNATURES), "binding and header list different functions"


def test_abi_version_matches_header():
    m = re.search(r"#define PDP_ABI_VERSION (\d+)u", open(HEADER).read())
    assert pdp.abi_version() == int(m.group(1))


def test_strerror_covers_codes():
    L = pdp.lib()
    for code in range(0, -10, -1):
        assert L.pdp_strerror(code).decode() not in ("", "unknown error")
    assert L.pdp_strerror(-99).decode() == "unknown error"


def test_k_rule_matches_oracle():
    totals = [0, 1, 2, 19, 20, 21, 399, 400, 401, 160000, 160001, 10212983, 64 * 10 ** 6, 71 * 10 ** 6,
              20 ** 12, 20 ** 12 + 1, 2 ** 64 - 1]
    for t in totals:
        for a in (4, 20):
            for mode in (0, 1):
                assert pdp.k_rule(t, a, mode) == oracle.k_rule(t, a, mode), (t, a, mode)
    with pytest.raises(pdp.PdpError):
        pdp.k_rule(100, 1)


def test_dict_size_validation():
    arena, ws = pdp.dict_size(3000, 10 ** 6, 6)
    assert arena > 12 * 10 ** 6 * 2 and ws > 8 * 10 ** 6
    for k in (0, 13):
        with pytest.raises(pdp.PdpError) as e:
            pdp.dict_size(10, 100, k)
        assert e.value.code == pdp.PDP_E_KRANGE
    with pytest.raises(pdp.PdpError) as e:
        pdp.dict_size(10, 2 ** 32, 6)
    assert e.value.code == pdp.PDP_E_LIMIT
    # nucleotides: k up to 31 (62-bit codes)
    pdp.dict_size(10, 100, 31, "nt")
    for k in (0, 32):
        with pytest.raises(pdp.PdpError) as e:
            pdp.dict_size(10, 100, k, "nt")
        assert e.value.code == pdp.PDP_E_KRANGE
    a, w = B.u64(0), B.u64(0)
    assert pdp.lib().pdp_dict_size(10, 100, 6, 2, C.byref(a), C.byref(w)) == pdp.PDP_E_ALPHABET
    with pytest.raises(ValueError):
        pdp.dict_size(10, 100, 6, "rna")


def _fake_dict(n_genes, n_residues, k, base=1 << 20, alphabet="aa", flags=0):
    """Binds a dictionary to a fake (never dereferenced) aligned address: binding and
    planning only do host arithmetic on the pointers."""
    arena, _ = pdp.dict_size(n_genes, n_residues, k, alphabet)
    d = B.pdp_dict()
    B.check(pdp.lib().pdp_dict_bind(base, arena, n_genes, n_residues, k, B.alphabet_id(alphabet), flags, C.byref(d)),
            "bind")
    return d


def test_bind_checks_alignment_and_size():
    arena, _ = pdp.dict_size(10, 100, 3)
    d = B.pdp_dict()
    assert pdp.lib().pdp_dict_bind(4096 + 8, arena, 10, 100, 3, 0, 0, C.byref(d)) == pdp.PDP_E_INVAL
    assert pdp.lib().pdp_dict_bind(4096, arena - 1, 10, 100, 3, 0, 0, C.byref(d)) == pdp.PDP_E_WORKSPACE
    assert pdp.lib().pdp_dict_bind(4096, arena, 10, 100, 3, 0, 2, C.byref(d)) == pdp.PDP_E_INVAL  # unknown flag
    assert pdp.lib().pdp_dict_bind(4096, arena, 10, 100, 3, 0, 0, C.byref(d)) == 0
    assert d.n_buckets == 20 ** 3 and d.capacity == 101 and d.lead == 3 and d.alphabet == 0 and d.flags == 0
    assert d.nwin % 256 == 0 and d.ix_code > d.mv_code > d.nwin
    assert pdp.lib().pdp_dict_bind(4096, arena, 10, 100, 3, 0, pdp.PDP_DICT_LONG_GENES, C.byref(d)) == 0
    assert d.flags == pdp.PDP_DICT_LONG_GENES


def test_bind_layout_per_alphabet():
    # amino acids: 20^min(k,4) buckets, 5-bit letters; nucleotides: 4^min(k,9) buckets, 2-bit letters
    for k, lead in ((2, 2), (4, 4), (6, 4), (12, 4)):
        d = _fake_dict(100, 10000, k)
        assert (d.lead, d.n_buckets, d.alphabet) == (lead, 20 ** lead, 0)
        assert d.key_shift == (7 if 5 * (k - lead) + 7 <= 32 else 0)
    for k, lead in ((3, 3), (9, 9), (13, 9), (21, 9), (31, 9)):
        d = _fake_dict(100, 10000, k, alphabet="nt")
        assert (d.lead, d.n_buckets, d.alphabet) == (lead, 4 ** lead, 1)
        assert d.key_shift == (7 if 2 * (k - lead) + 7 <= 32 else 0)


def _plan(tasks, prm=None):
    arr = (B.pdp_task * len(tasks))()
    for i, (a, b, f) in enumerate(tasks):
        arr[i].a = C.pointer(a)
        arr[i].b = C.pointer(b)
        arr[i].flags = f
    h = B.vp()
    rc = pdp.lib().pdp_plan_create(arr, len(tasks), C.byref(prm or pdp.params()), C.byref(h))
    return rc, h


def test_plan_layout():
    a, b, c = _fake_dict(300, 90000, 5), _fake_dict(200, 60000, 5), _fake_dict(50, 9000, 5)
    rc, h = _plan([(a, b, pdp.PDP_TASK_BBH), (a, c, pdp.PDP_TASK_AB), (c, b, pdp.PDP_TASK_BA)],
                  pdp.params(tile_rows=16))
    assert rc == 0
    L = pdp.lib()
    info = B.pdp_plan_info()
    assert L.pdp_plan_info_get(h, C.byref(info)) == 0
    assert info.bh_rows == 300 + 200 + 300 + 200
    assert info.bbh_rows == 300
    assert info.tiles == 19 + 13 + 19 + 13
    rows = []
    for t in range(3):
        x, y, z = B.u32(), B.u32(), B.u32()
        assert L.pdp_plan_rows(h, t, C.byref(x), C.byref(y), C.byref(z)) == 0
        rows.append((x.value, y.value, z.value))
    none = 2 ** 32 - 1
    assert rows == [(0, 300, 0), (500, none, none), (none, 800, none)]
    assert L.pdp_plan_rows(h, 3, None, None, None) == pdp.PDP_E_INVAL
    L.pdp_plan_destroy(h)
    # tile heights are powers of two: 20 rows round down to 16
    rc, h = _plan([(a, b, pdp.PDP_TASK_BBH)], pdp.params(tile_rows=20))
    assert rc == 0 and L.pdp_plan_info_get(h, C.byref(info)) == 0 and info.tiles == 19 + 13
    L.pdp_plan_destroy(h)


def test_colmax_plan_has_tiles_for_one_direction():
    # column maxima: a task asking for both directions gets tiles (and records) for one genome's
    # rows only, the smaller one's (it queries the join), while the other's rows keep their place
    # in the output
    a, b = _fake_dict(300, 90000, 5), _fake_dict(200, 60000, 5)
    L = pdp.lib()
    info = B.pdp_plan_info()
    rc, h = _plan([(a, b, pdp.PDP_TASK_BBH), (b, a, pdp.PDP_TASK_BA)], pdp.params(tile_rows=16, colmax=True))
    assert rc == 0 and L.pdp_plan_info_get(h, C.byref(info)) == 0
    assert info.bh_rows == 300 + 200 + 300 and info.bbh_rows == 300
    assert info.tiles == 13 + 19  # b's rows of the BBH task, a's rows (as b) of the BA task
    L.pdp_plan_destroy(h)
    rc, h = _plan([(b, a, pdp.PDP_TASK_BBH)], pdp.params(tile_rows=16, colmax=True))
    assert rc == 0 and L.pdp_plan_info_get(h, C.byref(info)) == 0
    assert info.tiles == 13 and info.bbh_rows == 200  # the same pair in the other order: b's rows again
    L.pdp_plan_destroy(h)
    bad = pdp.params()
    bad.flags = 8
    assert _plan([(a, b, pdp.PDP_TASK_AB)], bad)[0] == pdp.PDP_E_INVAL
    # the two-pass join is a known flag
    rc, h = _plan([(a, b, pdp.PDP_TASK_BBH)], pdp.params(two_pass=True))
    assert rc == 0
    L.pdp_plan_destroy(h)


def test_smaller_genome_queries_the_join_in_the_callers_layout():
    # the genome with fewer entries takes the join's query side whichever the caller named first;
    # output rows (and the BBH rows, the caller's a) keep the caller's orientation
    a, b = _fake_dict(300, 90000, 5), _fake_dict(200, 60000, 5)
    L = pdp.lib()
    info = B.pdp_plan_info()
    none = 2 ** 32 - 1
    for tasks, tiles, rows in (([(a, b, pdp.PDP_TASK_AB)], 19, [(0, none, none)]),
                               ([(a, b, pdp.PDP_TASK_BA)], 13, [(none, 0, none)]),
                               ([(b, a, pdp.PDP_TASK_AB | pdp.PDP_TASK_BA)], 13 + 19, [(0, 200, none)]),
                               ([(a, b, pdp.PDP_TASK_BBH), (b, a, pdp.PDP_TASK_BBH)], 2 * (19 + 13),
                                [(0, 300, 0), (500, 700, 300)])):
        rc, h = _plan(tasks, pdp.params(tile_rows=16))
        assert rc == 0 and L.pdp_plan_info_get(h, C.byref(info)) == 0
        assert info.tiles == tiles
        got = []
        for t in range(len(tasks)):
            x, y, z = B.u32(), B.u32(), B.u32()
            assert L.pdp_plan_rows(h, t, C.byref(x), C.byref(y), C.byref(z)) == 0
            got.append((x.value, y.value, z.value))
        assert got == rows
        L.pdp_plan_destroy(h)


def test_long_gene_tasks_have_rows_but_no_join_or_tiles():
    # a task naming a long-gene dictionary computes its rows on the long-gene path: no join
    # items, no tiles, no column maxima; its rows keep their place in the output
    a, b = _fake_dict(300, 90000, 5), _fake_dict(200, 60000, 5)
    la = _fake_dict(300, 90000, 5, base=1 << 30, flags=pdp.PDP_DICT_LONG_GENES)
    L = pdp.lib()
    info = B.pdp_plan_info()
    rc, h = _plan([(a, b, pdp.PDP_TASK_BBH)], pdp.params(tile_rows=16))
    assert rc == 0 and L.pdp_plan_info_get(h, C.byref(info)) == 0
    groups = info.join_groups
    assert groups > 0 and info.tiles == 19 + 13 and info.long_rows == 0
    L.pdp_plan_destroy(h)
    for prm in (pdp.params(tile_rows=16), pdp.params(tile_rows=16, colmax=True)):
        rc, h = _plan([(a, b, pdp.PDP_TASK_BBH), (la, b, pdp.PDP_TASK_BBH), (b, la, pdp.PDP_TASK_AB)], prm)
        assert rc == 0 and L.pdp_plan_info_get(h, C.byref(info)) == 0
        assert info.bh_rows == 500 + 500 + 200 and info.bbh_rows == 300 + 300
        assert info.join_groups == groups  # the first task's items only
        assert info.tiles == (19 + 13 if not prm.flags else 13)  # column maxima: the smaller genome's rows
        assert info.long_rows == 300 + 200 + 200
        rows = []
        for t in range(3):
            x, y, z = B.u32(), B.u32(), B.u32()
            assert L.pdp_plan_rows(h, t, C.byref(x), C.byref(y), C.byref(z)) == 0
            rows.append((x.value, y.value, z.value))
        none = 2 ** 32 - 1
        assert rows == [(0, 300, 0), (500, 800, 300), (1000, none, none)]
        L.pdp_plan_destroy(h)
    # a long-gene task needs no LDS room for a dense tile row of the column genome
    big = _fake_dict(50000, 9 * 10 ** 6, 5, flags=pdp.PDP_DICT_LONG_GENES)
    assert _plan([(a, big, pdp.PDP_TASK_AB)])[0] == 0


def test_plan_rejects_bad_tasks():
    a5, b6 = _fake_dict(10, 900, 5), _fake_dict(10, 900, 6)
    assert _plan([(a5, b6, pdp.PDP_TASK_AB)])[0] == pdp.PDP_E_INVAL
    # same k, other alphabet
    assert _plan([(a5, _fake_dict(10, 900, 5, alphabet="nt"), pdp.PDP_TASK_AB)])[0] == pdp.PDP_E_INVAL
    n13 = _fake_dict(10, 900, 13, alphabet="nt")
    assert _plan([(n13, _fake_dict(20, 2000, 13, alphabet="nt"), pdp.PDP_TASK_BBH)])[0] == 0
    assert _plan([(a5, a5, 0)])[0] == pdp.PDP_E_INVAL
    # a column genome must leave room for one dense row (its window counts + sums + bitmap) in LDS
    big = _fake_dict(50000, 9 * 10 ** 6, 5)
    assert _plan([(a5, big, pdp.PDP_TASK_AB)])[0] == pdp.PDP_E_LIMIT
    assert _plan([(a5, big, pdp.PDP_TASK_BA)])[0] == 0  # the big genome as rows fits
    assert _plan([(a5, _fake_dict(30000, 9 * 10 ** 6, 5), pdp.PDP_TASK_AB)])[0] == 0
    # rows beyond 1024 tiles of 256 genes cannot be counted per tile in the join
    huge = _fake_dict(300000, 9 * 10 ** 7, 5)
    assert _plan([(huge, a5, pdp.PDP_TASK_AB)])[0] == pdp.PDP_E_LIMIT
    assert _plan([(a5, a5, 1)], pdp.params(inc_capacity=1 << 32))[0] == pdp.PDP_E_LIMIT
    assert _plan([(a5, a5, 1)], pdp.params(lds_budget=1 << 20))[0] == pdp.PDP_E_INVAL


def test_launch_validates_outputs():
    a = _fake_dict(10, 900, 5)
    rc, h = _plan([(a, a, pdp.PDP_TASK_BBH)])
    assert rc == 0
    out = B.pdp_bh_out(19, 0, 0, 4096, 0, 0, 0)  # wrong row count (plan has 20)
    rc = pdp.lib().pdp_plan_launch(h, C.byref(out), None, 4096, 4096, 1 << 30, None)
    assert rc == pdp.PDP_E_INVAL
    out = B.pdp_bh_out(20, 0, 0, 4096, 0, 0, 0)
    rc = pdp.lib().pdp_plan_launch(h, C.byref(out), None, 4096, 4096, 1 << 30, None)
    assert rc == pdp.PDP_E_INVAL  # BBH requested, no BBH output
    pdp.lib().pdp_plan_destroy(h)
