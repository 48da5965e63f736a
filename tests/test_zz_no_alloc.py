"""GPU tests of pdp_bh_noalloc (best hits with the library's fixed device scratch instead of a
caller workspace): called through the C-ABI, its output must equal pdp_bh's element by element,
on two calls in a row whose second has the smaller input (the scratch keeps the first call's
contents), and a pair needing more scratch than the fixed array holds is refused up front."""
import ctypes as C

import numpy as np
import pytest

import oracle
from helpers import check_bh
from synth import make_config

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU collection
    pytest.skip("needs the GPU", allow_module_level=True)

import paper_2510_23679_amd as pdp  # noqa: E402
from paper_2510_23679_amd import binding as B  # noqa: E402


def say(*a):
    print("[case]", *a, flush=True)


def noalloc(q, t, prm, capacity):
    out = pdp.BHOut(q.n_genes, capacity)
    st = pdp.new_status()
    o = out.struct()
    rc = B.lib().pdp_bh_noalloc(C.byref(q.d), C.byref(t.d), C.byref(prm), C.byref(o), st.data_ptr(),
                                int(torch.cuda.current_stream().cuda_stream))
    return rc, out, st


def with_workspace(q, t, prm, capacity):
    """The existing entry point, pdp_bh, with a fresh poisoned workspace."""
    need = B.u64(0)
    B.check(B.lib().pdp_bh_ws_size(C.byref(q.d), C.byref(t.d), C.byref(prm), C.byref(need)), "pdp_bh_ws_size")
    ws = pdp.Workspace(need.value)
    ws.buf.fill_(255)
    out = pdp.BHOut(q.n_genes, capacity)
    st = pdp.new_status()
    o = out.struct()
    rc = B.lib().pdp_bh(C.byref(q.d), C.byref(t.d), C.byref(prm), C.byref(o), st.data_ptr(), ws.ptr, ws.nbytes,
                        int(torch.cuda.current_stream().cuda_stream))
    return rc, out, st


def same(x, y):
    for a, b in zip(x, y):
        assert np.array_equal(a, b)


def test_noalloc_equals_pdp_bh_on_two_calls_in_a_row():
    # the larger input first, then the smaller one; each call as it comes (the planted pair's
    # shared k-mers pass the default record capacity, so both entry points report it alike),
    # then the retrying forms
    big = make_config(2, genomes=2, genes=2000)
    small = make_config(1)
    for name, ds, k in (("2 x 2000-gene family genomes", big, 6), ("planted pair, 2 x 200 genes", small, 4)):
        dicts = [pdp.Dictionary.build_from(g, k) for g in ds.genomes]
        for d in dicts:
            d.check_status()
        for q, t in ((dicts[0], dicts[1]), (dicts[1], dicts[0])):
            say("pdp_bh_noalloc vs pdp_bh:", name, "k =", k)
            cap = 2 * q.n_genes + 1024
            rc_w, out_w, st_w = with_workspace(q, t, pdp.params(), cap)
            rc_n, out_n, st_n = noalloc(q, t, pdp.params(), cap)
            assert rc_w == rc_n == pdp.PDP_OK, B.lib().pdp_last_error().decode()
            sw, sn = pdp.read_status(st_w), pdp.read_status(st_n)
            assert sw == sn, (sw, sn)
            if sw[0] == 0:
                same(out_n.host(), out_w.host())
            same(pdp.bh_noalloc(q, t).host(), pdp.bh(q, t).host())
    # the smaller input against the oracle as well
    og = oracle.genomes(small.genomes, 4)
    got = pdp.bh_noalloc(*[pdp.Dictionary.build_from(g, 4) for g in small.genomes]).host()
    check_bh(got, oracle.bh(og[0], og[1]))


def test_noalloc_capacity_retry_equals_pdp_bh():
    # a best-hit output too small: the device reports it, the retry through the binding fits
    ds = make_config(3, genomes=2, genes_lo=300, genes_hi=500, core=150)
    dicts = [pdp.Dictionary.build_from(g, 5) for g in ds.genomes]
    say("pdp_bh_noalloc capacity error then retry")
    rc, out, st = noalloc(dicts[0], dicts[1], pdp.params(), 4)
    assert rc == pdp.PDP_OK
    code, needed, where = pdp.read_status(st)
    assert code == pdp.PDP_E_CAPACITY and where == 1 and needed > 4
    same(pdp.bh_noalloc(dicts[0], dicts[1], capacity=4).host(), pdp.bh(dicts[0], dicts[1]).host())


def test_noalloc_refuses_a_pair_past_the_fixed_scratch():
    ds = make_config(1)
    dicts = [pdp.Dictionary.build_from(g, 4) for g in ds.genomes]
    need = B.u64(0)
    prm = pdp.params(inc_capacity=12_000_000)  # 96 MB of records: past the 64 MiB array
    B.check(B.lib().pdp_bh_ws_size(C.byref(dicts[0].d), C.byref(dicts[1].d), C.byref(prm), C.byref(need)), "ws size")
    assert need.value > pdp.PDP_NOALLOC_SCRATCH_BYTES
    say("pdp_bh_noalloc refuses", need.value, "bytes of scratch")
    rc, out, st = noalloc(dicts[0], dicts[1], prm, 1024)
    assert rc == pdp.PDP_E_WORKSPACE
    assert "fixed scratch" in B.lib().pdp_last_error().decode()
    # the next call is unaffected
    same(pdp.bh_noalloc(dicts[0], dicts[1]).host(), pdp.bh(dicts[0], dicts[1]).host())
