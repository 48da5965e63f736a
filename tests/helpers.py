"""Shared test helpers: comparing the GPU path's outputs with the CPU oracle."""
from __future__ import annotations

import numpy as np

import oracle

# Layout of a dictionary per alphabet, as the C-ABI documents it: symbol bits per letter,
# letters, and leading letters that name an index bucket.
BITS = {"aa": 5, "nt": 2}
SIGMA = {"aa": 20, "nt": 4}
LEAD = {"aa": 4, "nt": 9}


def gpu_code_to_id(codes: np.ndarray, k: int, alphabet: str = "aa") -> np.ndarray:
    """The GPU packs letters 5 (amino acids) or 2 (nucleotides) bits each; the oracle numbers
    k-mers in base 20 or 4.  Both are injective on k-mers, so translating one into the other
    lets the two dictionaries be compared by content."""
    bits, sigma = BITS[alphabet], SIGMA[alphabet]
    codes = codes.astype(np.uint64)
    assert np.all((codes >> np.uint64(bits * k)) == 0), "bits set above the k letters of a code"
    out = np.zeros(codes.shape, dtype=np.uint64)
    for i in range(k):
        sym = (codes >> np.uint64(bits * (k - 1 - i))) & np.uint64((1 << bits) - 1)
        assert np.all(sym < sigma), "a letter symbol outside the alphabet"
        out = out * np.uint64(sigma) + sym
    return out


def check_dictionary(host: dict, og: oracle.OracleGenome) -> None:
    """Every array of a GPU dictionary against the oracle's multiplicity vectors."""
    k, al = og.k, og.alphabet
    bits, sigma = BITS[al], SIGMA[al]
    assert np.array_equal(host["nwin"].astype(np.uint64), og.nwin), "windows per gene"
    assert np.array_equal(host["mv_ptr"].astype(np.uint64), og.ptr), "distinct k-mers per gene"
    assert np.array_equal(gpu_code_to_id(host["mv_code"], k, al), og.ids), "multiplicity-vector k-mers"
    assert np.array_equal(host["mv_cnt"], og.cnt), "multiplicities"
    # inverted index: every (k-mer, gene, count) ordered by k-mer then gene
    genes = np.repeat(np.arange(og.n, dtype=np.uint32), np.diff(og.ptr).astype(np.int64))
    order = np.lexsort((genes, og.ids))
    assert np.array_equal(gpu_code_to_id(host["ix_code"], k, al), og.ids[order]), "index codes"
    assert np.array_equal(host["ix_gene"], genes[order]), "index genes"
    assert np.array_equal(host["ix_cnt"], og.cnt[order]), "index counts"
    lead = min(k, LEAD[al])
    bucket = (og.ids // np.uint64(sigma ** (k - lead))).astype(np.int64)
    dir_ = np.zeros(sigma ** lead + 1, dtype=np.int64)
    np.add.at(dir_, bucket + 1, 1)
    assert np.array_equal(host["ix_dir"].astype(np.int64), np.cumsum(dir_)), "index directory"
    # packed join keys: the trailing k - lead letters, `bits` each, above the gene's bits
    shift = max(1, (og.n - 1).bit_length()) if og.n > 1 else 1
    tail_bits = bits * (k - lead)
    assert ("ix_key" in host) == (tail_bits + shift <= 32), "packed keys present exactly when they fit"
    if "ix_key" in host:
        rest = og.ids[order] % np.uint64(sigma ** (k - lead))
        tail = np.zeros(len(rest), dtype=np.uint64)
        for j in range(k - lead):  # base sigma -> `bits` per letter, most significant first
            digit = (rest // np.uint64(sigma ** (k - lead - 1 - j))) % np.uint64(sigma)
            tail = (tail << np.uint64(bits)) | digit
        want = (tail << np.uint64(shift)) | genes[order].astype(np.uint64)
        assert np.array_equal(host["ix_key"].astype(np.uint64), want), "packed index keys"


def check_bh(got, want: oracle.BH, rows=None) -> None:
    """got = (ptr, col, num, den) of every row; want = oracle BH of all rows, or of ``rows``."""
    ptr, col, num, den = got
    if rows is None:
        assert np.array_equal(ptr.astype(np.uint64), want.ptr), "best-hit counts per row"
        assert np.array_equal(col, want.col), "best-hit columns"
        assert np.array_equal(num.astype(np.uint64), want.num), "sums of minima"
        assert np.array_equal(den.astype(np.uint64), want.den), "sums of maxima"
        return
    for i, r in enumerate(rows):
        lo, hi = int(ptr[r]), int(ptr[r + 1])
        wc, wn, wd = want.row(i)
        assert np.array_equal(col[lo:hi], wc), f"row {r}: columns"
        assert np.array_equal(num[lo:hi].astype(np.uint64), wn), f"row {r}: sums of minima"
        assert np.array_equal(den[lo:hi].astype(np.uint64), wd), f"row {r}: sums of maxima"


def check_bbh(got, want: oracle.Pairs) -> None:
    a, b, num, den = got
    assert np.array_equal(a, want.a) and np.array_equal(b, want.b), "BBH pairs"
    assert np.array_equal(num.astype(np.uint64), want.num) and np.array_equal(den.astype(np.uint64), want.den)


def bbh_from_best_hits(bh_ab, bh_ba, n_a: int, n_b: int):
    """Eq. bidirectional_best_hit applied to two best-hit CSRs: every (a, b) with b in BH(a) and a
    in BH(b), in (a, b) order, with the (num, den) of the AB entry."""
    pab, cab = bh_ab[0].astype(np.int64), bh_ab[1].astype(np.int64)
    pba, cba = bh_ba[0].astype(np.int64), bh_ba[1].astype(np.int64)
    ra = np.repeat(np.arange(n_a, dtype=np.int64), np.diff(pab))
    rb = np.repeat(np.arange(n_b, dtype=np.int64), np.diff(pba))
    key_ab = ra * (n_b + 1) + cab            # (a, b) of every AB best hit
    key_ba = cba * (n_b + 1) + rb            # (a, b) of every BA best hit, transposed
    keep = np.isin(key_ab, key_ba)           # AB keys ascend: rows ascend, columns ascend in a row
    return (ra[keep].astype(np.uint32), cab[keep].astype(np.uint32), bh_ab[2][keep], bh_ab[3][keep])


def check_bh_properties(bh_ab, bh_ba, bbh, n_a: int, n_b: int) -> None:
    """Properties that hold at any size: CSR well-formed, columns ascending and in range,
    0 < num <= den, ties equal in value, and the BBH list exactly the mutual pairs of the two
    best-hit sets (none missing, none extra), in (a, b) order with the AB entry's num/den."""
    for (ptr, col, num, den), nrows, ncols in ((bh_ab, n_a, n_b), (bh_ba, n_b, n_a)):
        p = ptr.astype(np.int64)
        assert len(p) == nrows + 1 and p[0] == 0 and np.all(np.diff(p) >= 0)
        assert np.all(col < ncols)
        assert np.all(num > 0) and np.all(num <= den)
        rows = np.repeat(np.arange(nrows, dtype=np.int64), np.diff(p))
        key = rows * (ncols + 1) + col.astype(np.int64)
        assert np.all(np.diff(key) > 0), "columns ascending inside every row"
        first = p[:-1][np.diff(p) > 0]
        lead = np.repeat(first, np.diff(p)[np.diff(p) > 0])  # each entry's row's first entry
        x = num.astype(np.uint64) * den[lead].astype(np.uint64)
        y = num[lead].astype(np.uint64) * den.astype(np.uint64)
        assert np.array_equal(x, y), "ties share one value"
    a, b, num, den = bbh
    wa, wb, wn, wd = bbh_from_best_hits(bh_ab, bh_ba, n_a, n_b)
    assert np.array_equal(a, wa) and np.array_equal(b, wb), "BBH = the mutual pairs of the two best-hit sets"
    assert np.array_equal(num, wn) and np.array_equal(den, wd), "BBH num/den = the AB entries'"


def check_pair_complete(ab, ba, bb, want, n_a: int, n_b: int) -> None:
    """One genome pair in full: every best-hit row both ways and the whole BBH set against the
    oracle's (ab, ba, bbh), plus the any-size properties."""
    wab, wba, wbb = want
    check_bh(ab, wab)
    check_bh(ba, wba)
    check_bbh(bb, wbb)
    check_bh_properties(ab, ba, bb, n_a, n_b)
