"""Seeded synthetic genomes shaped like the paper's workloads.

The paper measures on RefSeq bacterial genomes and on PANPROVA-evolved
collections (Dataset construction section, Tables 1-2); neither is available
here, so these generators stand in for them.  Genes are strings over the 20
standard amino acids ("aa", the default) or over the nucleotides ACGT ("nt").
A gene family has one random ancestor; each member is the ancestor after
per-site substitutions (to one of the other letters of the alphabet, chosen
uniformly) and single-letter indels (insertion or deletion with equal
probability).  Protein lengths follow a lognormal law with median 300 aa and
sigma 0.5, clipped to [50, 2000]; nucleotide genes are three times as long
(the coding sequence of such a protein): median 900 nt, clipped to [150, 6000].

Every function is a pure function of its seed: the same arguments give the
same bytes on every machine.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Iterator, List, Optional, Sequence

import numpy as np

ALPHABET = b"ACDEFGHIKLMNPQRSTVWY"
ALPHABETS = {"aa": ALPHABET, "nt": b"ACGT"}
_ASCII = {a: np.frombuffer(v, dtype=np.uint8).copy() for a, v in ALPHABETS.items()}
# gene lengths (median, lower clip, upper clip) per alphabet
_LENGTHS = {"aa": (300.0, 50, 2000), "nt": (900.0, 150, 6000)}


def _sigma(alphabet: str) -> int:
    if alphabet not in ALPHABETS:
        raise ValueError(f"unknown alphabet {alphabet!r} (expected 'aa' or 'nt')")
    return len(ALPHABETS[alphabet])
BASE_SEED = 2510236790


def config_seed(config: int, *stream: int) -> np.random.SeedSequence:
    """Seed of workload ``config`` (1..5); ``stream`` picks an independent sub-stream."""
    return np.random.SeedSequence(BASE_SEED + int(config), spawn_key=tuple(int(s) for s in stream))


def _rng(seed) -> np.random.Generator:
    if isinstance(seed, np.random.Generator):
        return seed
    if not isinstance(seed, np.random.SeedSequence):
        seed = np.random.SeedSequence(int(seed))
    return np.random.Generator(np.random.PCG64(seed))


@dataclass
class Genome:
    """One genome: concatenated ASCII residues plus gene offsets (n+1 entries)."""

    residues: np.ndarray  # uint8, ASCII letters
    offsets: np.ndarray  # uint64, offsets[i]..offsets[i+1] is gene i
    name: str = ""
    alphabet: str = "aa"  # "aa": amino acids, "nt": nucleotides

    @property
    def n_genes(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def n_residues(self) -> int:
        return int(self.offsets[-1])

    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets.astype(np.int64))

    def gene(self, i: int) -> bytes:
        return self.residues[int(self.offsets[i]):int(self.offsets[i + 1])].tobytes()

    def strings(self) -> List[str]:
        return [self.gene(i).decode("ascii") for i in range(self.n_genes)]

    def subset(self, genes: Sequence[int], name: str = "") -> "Genome":
        return genome_from_strings([self.gene(int(i)).decode("ascii") for i in genes], name or self.name,
                                   self.alphabet)


@dataclass
class Dataset:
    """A list of genomes that are compared all-against-all (every unordered pair)."""

    genomes: List[Genome]
    description: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_genomes(self) -> int:
        return len(self.genomes)

    def total_residues(self) -> int:
        return int(sum(g.n_residues for g in self.genomes))

    def total_genes(self) -> int:
        return int(sum(g.n_genes for g in self.genomes))

    def pairs(self):
        n = len(self.genomes)
        return [(i, j) for i in range(n) for j in range(i + 1, n)]

    def gene_pairs(self) -> int:
        s = [g.n_genes for g in self.genomes]
        return int(sum(s[i] * s[j] for i, j in self.pairs()))


def genome_from_strings(genes: Sequence[str], name: str = "", alphabet: str = "aa") -> Genome:
    _sigma(alphabet)
    lens = np.array([len(s) for s in genes], dtype=np.uint64)
    off = np.zeros(len(genes) + 1, dtype=np.uint64)
    off[1:] = np.cumsum(lens)
    res = np.frombuffer("".join(genes).encode("ascii"), dtype=np.uint8).copy()
    return Genome(res, off, name, alphabet)


def _genome_from_symbols(sym: np.ndarray, off: np.ndarray, name: str = "", alphabet: str = "aa") -> Genome:
    return Genome(_ASCII[alphabet][sym], off.astype(np.uint64), name, alphabet)


def _lognormal_lengths(rng: np.random.Generator, n: int, median: float = 300.0,
                       sigma: float = 0.5, lo: int = 50, hi: int = 2000) -> np.ndarray:
    x = rng.lognormal(mean=np.log(median), sigma=sigma, size=n)
    return np.clip(np.rint(x), lo, hi).astype(np.int64)


def _random_symbols(rng: np.random.Generator, lens: np.ndarray, sigma: int = 20):
    lens = np.asarray(lens, dtype=np.int64)
    off = np.zeros(len(lens) + 1, dtype=np.int64)
    off[1:] = np.cumsum(lens)
    return rng.integers(0, sigma, int(off[-1]), dtype=np.uint8), off


def _gather_segments(sym: np.ndarray, off: np.ndarray, which: np.ndarray):
    which = np.asarray(which, dtype=np.int64)
    starts = off[which]
    lens = off[which + 1] - starts
    out_off = np.zeros(len(which) + 1, dtype=np.int64)
    out_off[1:] = np.cumsum(lens)
    idx = np.arange(int(out_off[-1]), dtype=np.int64) - np.repeat(out_off[:-1] - starts, lens)
    return sym[idx], out_off


def _mutate(rng: np.random.Generator, anc_sym: np.ndarray, anc_off: np.ndarray,
            which: np.ndarray, sub: np.ndarray, indel: np.ndarray, sigma: int = 20):
    """Members ``which`` of the ancestors, each with its own substitution and indel rate."""
    which = np.asarray(which, dtype=np.int64)
    n = len(which)
    src, src_off = _gather_segments(anc_sym, anc_off, which)
    src = src.copy()
    lens = np.diff(src_off)
    total = int(src_off[-1])
    sub_pos = np.repeat(np.asarray(sub, dtype=np.float64), lens)
    ind_pos = np.repeat(np.asarray(indel, dtype=np.float64), lens)
    m = rng.random(total) < sub_pos
    src[m] = (src[m] + rng.integers(1, sigma, int(m.sum()), dtype=np.uint8)) % sigma
    ev = rng.random(total) < ind_pos
    ins = ev & (rng.random(total) < 0.5)
    dele = ev & ~ins
    copies = np.ones(total, dtype=np.int64)
    copies[dele] = 0
    copies[ins] = 2
    out = np.repeat(src, copies)
    cum = np.cumsum(copies)
    slots = cum[ins] - 1
    out[slots] = rng.integers(0, sigma, len(slots), dtype=np.uint8)
    seg = np.repeat(np.arange(n), lens)
    new_lens = np.bincount(seg, weights=copies, minlength=n).astype(np.int64)
    off = np.zeros(n + 1, dtype=np.int64)
    off[1:] = np.cumsum(new_lens)
    return out, off


def _concat(parts):
    syms = [p[0] for p in parts]
    lens = [np.diff(p[1]) for p in parts]
    sym = np.concatenate(syms) if syms else np.zeros(0, np.uint8)
    ln = np.concatenate(lens) if lens else np.zeros(0, np.int64)
    off = np.zeros(len(ln) + 1, dtype=np.int64)
    off[1:] = np.cumsum(ln)
    return sym, off


def _permute(sym: np.ndarray, off: np.ndarray, perm: np.ndarray):
    return _gather_segments(sym, off, perm)


def random_genome(seed, n_genes: int, len_lo: int = 100, len_hi: int = 400, name: str = "",
                  alphabet: str = "aa") -> Genome:
    """Genes of uniform random letters with lengths uniform in [len_lo, len_hi]."""
    rng = _rng(seed)
    lens = rng.integers(len_lo, len_hi + 1, n_genes)
    sym, off = _random_symbols(rng, lens, _sigma(alphabet))
    return _genome_from_symbols(sym, off, name, alphabet)


def planted_pair(seed=None, n_genes: int = 200, n_planted: int = 150, len_lo: int = 100,
                 len_hi: int = 400, sub_lo: float = 0.05, sub_hi: float = 0.30,
                 indel_hi: float = 0.03, alphabet: str = "aa") -> Dataset:
    """Tiny workload: two genomes of ``n_genes`` uniform-letter genes; ``n_planted`` genes of B
    are mutated copies of genes of A, the rest are unrelated.  Gene order is shuffled."""
    rng = _rng(config_seed(1) if seed is None else seed)
    sg = _sigma(alphabet)
    lens = rng.integers(len_lo, len_hi + 1, n_genes)
    a_sym, a_off = _random_symbols(rng, lens, sg)
    src = rng.choice(n_genes, n_planted, replace=False)
    sub = rng.uniform(sub_lo, sub_hi, n_planted)
    ind = rng.uniform(0.0, indel_hi, n_planted)
    p_sym, p_off = _mutate(rng, a_sym, a_off, src, sub, ind, sg)
    r_sym, r_off = _random_symbols(rng, rng.integers(len_lo, len_hi + 1, n_genes - n_planted), sg)
    b_sym, b_off = _concat([(p_sym, p_off), (r_sym, r_off)])
    pa = rng.permutation(n_genes)
    pb = rng.permutation(n_genes)
    a_sym2, a_off2 = _permute(a_sym, a_off, pa)
    b_sym2, b_off2 = _permute(b_sym, b_off, pb)
    # planted mapping in the shuffled order: new index of A gene src[i] <-> new index of B gene i
    inv_a = np.empty(n_genes, np.int64)
    inv_a[pa] = np.arange(n_genes)
    inv_b = np.empty(n_genes, np.int64)
    inv_b[pb] = np.arange(n_genes)
    planted = np.stack([inv_a[src], inv_b[np.arange(n_planted)]], axis=1)
    return Dataset([_genome_from_symbols(a_sym2, a_off2, "A", alphabet),
                    _genome_from_symbols(b_sym2, b_off2, "B", alphabet)],
                   "planted pair", {"planted": planted})


def family_dataset(seed, genome_sizes: Sequence[int], n_core: int, acc_share: float = 0.75,
                   acc_occupancy: float = 5.5, sub_lo: float = 0.05, sub_hi: float = 0.30,
                   indel_hi: float = 0.03, paralog_frac: float = 0.0, near_tie_share: float = 0.5,
                   median_len: Optional[float] = None, sigma: float = 0.5, len_lo: Optional[int] = None,
                   len_hi: Optional[int] = None, name_prefix: str = "G", alphabet: str = "aa") -> Dataset:
    """Family model: ``n_core`` families with a member in every genome; the remaining genes of
    genome i are split ``acc_share`` : (1-acc_share) into accessory genes (members of families
    drawn without replacement from a shared pool sized so a family has ``acc_occupancy``
    members on average) and singletons.  With ``paralog_frac`` > 0, that fraction of each
    genome's genes is duplicated as exact copies, and ``near_tie_share`` of the copies then get
    one substitution.  Gene order is shuffled per genome.  Lengths default to the alphabet's
    law (median 300 aa or 900 nt)."""
    rng = _rng(seed)
    sg = _sigma(alphabet)
    d_med, d_lo, d_hi = _LENGTHS[alphabet]
    median_len = d_med if median_len is None else median_len
    len_lo = d_lo if len_lo is None else len_lo
    len_hi = d_hi if len_hi is None else len_hi
    sizes = np.asarray(genome_sizes, dtype=np.int64)
    g = len(sizes)
    if n_core > sizes.min():
        raise ValueError("n_core exceeds the smallest genome")
    rest = sizes - n_core
    acc = np.rint(rest * acc_share).astype(np.int64)
    sing = rest - acc
    pool = max(int(acc.max()), int(np.ceil(acc.sum() / max(acc_occupancy, 1e-9))))
    n_fam = n_core + pool
    anc_sym, anc_off = _random_symbols(rng, _lognormal_lengths(rng, n_fam, median_len, sigma, len_lo, len_hi), sg)
    genomes = []
    for i in range(g):
        fams = np.concatenate([np.arange(n_core), n_core + rng.choice(pool, int(acc[i]), replace=False)])
        nm = len(fams)
        m_sym, m_off = _mutate(rng, anc_sym, anc_off, fams, rng.uniform(sub_lo, sub_hi, nm),
                               rng.uniform(0.0, indel_hi, nm), sg)
        s_sym, s_off = _random_symbols(rng, _lognormal_lengths(rng, int(sing[i]), median_len, sigma, len_lo, len_hi),
                                       sg)
        sym, off = _concat([(m_sym, m_off), (s_sym, s_off)])
        if paralog_frac > 0:
            n = len(off) - 1
            nd = int(round(paralog_frac * n))
            dup = rng.choice(n, nd, replace=False)
            d_sym, d_off = _gather_segments(sym, off, dup)
            d_sym = d_sym.copy()
            n_near = int(round(near_tie_share * nd))
            for j in range(n_near):
                a, b = int(d_off[j]), int(d_off[j + 1])
                if b > a:
                    p = a + int(rng.integers(0, b - a))
                    d_sym[p] = (d_sym[p] + int(rng.integers(1, sg))) % sg
            sym, off = _concat([(sym, off), (d_sym, d_off)])
        perm = rng.permutation(len(off) - 1)
        sym, off = _permute(sym, off, perm)
        genomes.append(_genome_from_symbols(sym, off, f"{name_prefix}{i}", alphabet))
    return Dataset(genomes, "family model", {"n_core": n_core, "pool": pool, "alphabet": alphabet})


def make_config(config: int, **kw) -> Dataset:
    """Workloads 1-3 at full size, or scaled down through keyword overrides.

    1: two genomes x 200 genes with 150 planted homolog pairs.
    2: 10 genomes x ~3000 genes (1800 core, ~900 accessory, 300 singletons), 5-30% divergence.
    3: 50 genomes x U{3000..5000} genes, 1800 core, rest 3:1 accessory:singleton, plus 5%
       exact paralog copies per genome (half of them then carry one substitution).
    Keyword ``genomes`` / ``genes`` / ``core`` shrink the family workloads for tests;
    ``alphabet="nt"`` draws nucleotide genes (three times as long) instead of proteins.
    """
    if config == 1:
        if kw.get("alphabet", "aa") == "nt":
            kw.setdefault("len_lo", 300)
            kw.setdefault("len_hi", 1200)
        return planted_pair(config_seed(1), **kw)
    if config == 2:
        ng = kw.pop("genomes", 10)
        genes = kw.pop("genes", 3000)
        core = kw.pop("core", int(round(0.6 * genes)))
        single = kw.pop("singletons", int(round(0.1 * genes)))
        acc = genes - core - single
        rest = genes - core
        ds = family_dataset(config_seed(2), [genes] * ng, core, acc_share=acc / max(rest, 1),
                            acc_occupancy=kw.pop("acc_occupancy", 5.5), **kw)
        ds.description = f"family model, {ng} genomes x {genes} genes" + (
            " (nucleotide)" if kw.get("alphabet", "aa") == "nt" else "")
        return ds
    if config == 3:
        ng = kw.pop("genomes", 50)
        lo = kw.pop("genes_lo", 3000)
        hi = kw.pop("genes_hi", 5000)
        core = kw.pop("core", 1800)
        rng = _rng(config_seed(3, 1))
        sizes = rng.integers(lo, hi + 1, ng)
        ds = family_dataset(config_seed(3), sizes, core, acc_share=0.75, acc_occupancy=kw.pop("acc_occupancy", 10.0),
                            paralog_frac=kw.pop("paralog_frac", 0.05), **kw)
        ds.description = f"family model with paralogs, {ng} genomes x U{{{lo}..{hi}}} genes"
        return ds
    raise ValueError("workloads 4 and 5 are produced by batched_instances() and serving_workload()")


def batched_instances(start: int = 0, count: int = 400, genomes_lo: int = 4, genomes_hi: int = 30,
                      genes_lo: int = 500, genes_hi: int = 5000, sub_lo: float = 0.05,
                      sub_hi: float = 0.40) -> Iterator[Dataset]:
    """Independent pangenome instances (workload 4), produced lazily and reproducibly:
    instance i depends only on its index.  Each has U{genomes_lo..genomes_hi} genomes of
    U{genes_lo..genes_hi} genes; the family model is scaled to the smallest genome (60% core)."""
    for i in range(start, start + count):
        rng = _rng(config_seed(4, 0, i))
        ng = int(rng.integers(genomes_lo, genomes_hi + 1))
        sizes = rng.integers(genes_lo, genes_hi + 1, ng)
        core = int(round(0.6 * sizes.min()))
        ds = family_dataset(config_seed(4, 1, i), sizes, core, acc_share=0.75,
                            acc_occupancy=max(2.0, ng * 0.4), sub_lo=sub_lo, sub_hi=sub_hi,
                            name_prefix=f"I{i}G")
        ds.description = f"instance {i}: {ng} genomes"
        ds.meta["instance"] = i
        yield ds


@dataclass
class ServingWorkload:
    residents: Dataset
    arrival_times: np.ndarray  # seconds, ascending
    sizes: np.ndarray  # genes per arriving genome
    _anc_sym: np.ndarray = field(repr=False, default=None)
    _anc_off: np.ndarray = field(repr=False, default=None)
    sub_lo: float = 0.05
    sub_hi: float = 0.35

    def arrival(self, j: int) -> Genome:
        """Arriving genome j: genes drawn from random resident families, mutated 5-35%."""
        rng = _rng(config_seed(5, 2, j))
        n = int(self.sizes[j])
        nf = len(self._anc_off) - 1
        fams = rng.integers(0, nf, n)
        sym, off = _mutate(rng, self._anc_sym, self._anc_off, fams, rng.uniform(self.sub_lo, self.sub_hi, n),
                           rng.uniform(0.0, 0.03, n))
        return _genome_from_symbols(sym, off, f"Q{j}")


def serving_workload(n_residents: int = 200, resident_genes: int = 4000, n_arrivals: int = 2000,
                     arrive_lo: int = 1000, arrive_hi: int = 6000, rate_per_s: float = 100.0,
                     sub_lo: float = 0.05, sub_hi: float = 0.35) -> ServingWorkload:
    """Workload 5: resident genomes from the family model plus a Poisson stream of arrivals.
    Arrival j's genes are members of resident families (ancestors regenerated from the same
    seed), so it has homologs among the residents."""
    rng = _rng(config_seed(5, 0))
    core = int(round(0.6 * resident_genes))
    res = family_dataset(config_seed(5, 1), [resident_genes] * n_residents, core, acc_share=0.75,
                         acc_occupancy=max(2.0, 0.2 * n_residents), sub_lo=sub_lo, sub_hi=sub_hi,
                         name_prefix="R")
    # The family ancestors are the first draws of family_dataset's generator; redraw them here.
    frng = _rng(config_seed(5, 1))
    pool = res.meta["pool"]
    anc_sym, anc_off = _random_symbols(frng, _lognormal_lengths(frng, core + pool))
    gaps = rng.exponential(1.0 / rate_per_s, n_arrivals)
    times = np.cumsum(gaps)
    sizes = rng.integers(arrive_lo, arrive_hi + 1, n_arrivals)
    return ServingWorkload(res, times, sizes, anc_sym, anc_off, sub_lo, sub_hi)
