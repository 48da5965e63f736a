"""Brute-force oracle on Python strings -- TEST INFRASTRUCTURE ONLY, tiny inputs.

Independent of ``pdp_oracle.c``: k-mers are substrings, dictionaries are
``collections.Counter`` objects and similarities are ``fractions.Fraction``.
Each function restates one definition of the paper's Basic notions section.
"""
from __future__ import annotations

from collections import Counter
from fractions import Fraction
from typing import Dict, List, Sequence, Tuple


def windows(s: str, k: int) -> List[str]:
    """The substrings s[p..p+k-1] for every start p that leaves k characters (Alg. 1's window loop)."""
    return [s[p:p + k] for p in range(0, len(s) - k + 1)] if k >= 1 else []


def multiplicities(s: str, k: int) -> Counter:
    """mult_g(alpha) = |occ_g(alpha)| for every alpha in D_k(g) (Eqs. kmer_occurrences, kmer_multiplicity)."""
    return Counter(windows(s, k))


def terms(a: str, b: str, k: int) -> Tuple[int, int]:
    """(sum over D(a) & D(b) of min multiplicity, sum over D(a) | D(b) of max multiplicity), Eq. jaccard_k."""
    ma, mb = multiplicities(a, k), multiplicities(b, k)
    num = sum(min(ma[w], mb[w]) for w in set(ma) & set(mb))
    den = sum(max(ma[w], mb[w]) for w in set(ma) | set(mb))
    return num, den


def jaccard(a: str, b: str, k: int) -> Fraction:
    num, den = terms(a, b, k)
    return Fraction(num, den) if den else Fraction(0)


def directional(s: str, t: str, k: int) -> Fraction:
    """Eq. directional_jaccard: occurrences in s of the k-mers s shares with t, over s's windows
    (0 for a string without windows)."""
    ms, mt = multiplicities(s, k), multiplicities(t, k)
    n = max(0, len(s) - k + 1)
    return Fraction(sum(ms[w] for w in set(ms) & set(mt)), n) if n else Fraction(0)


def candidate(a: str, b: str, k: int, theta=None, tau=None) -> bool:
    """Eq. length_threshold (|a| >= theta |b| and |b| >= theta |a|) and the directional filter
    (both directional similarities >= tau); a None threshold is off."""
    if theta is not None and (len(a) < theta * len(b) or len(b) < theta * len(a)):
        return False
    if tau is not None and (directional(a, b, k) < tau or directional(b, a, k) < tau):
        return False
    return True


def best_hits(a: str, target: Sequence[str], k: int, theta=None, tau=None) -> List[int]:
    """Eq. best_hit over the candidates: indices of target genes at the maximum J among the pairs
    that pass the filters, if that maximum is above zero."""
    cand = [i for i, b in enumerate(target) if candidate(a, b, k, theta, tau)]
    if not cand:
        return []
    js = {i: jaccard(a, target[i], k) for i in cand}
    top = max(js.values())
    if top <= 0:
        return []
    return [i for i in cand if js[i] == top]


def bbh(gi: Sequence[str], gj: Sequence[str], k: int) -> List[Tuple[int, int]]:
    """Eq. bidirectional_best_hit: (l, m) with m in BH(g_il, G_j) and l in BH(g_jm, G_i), in (l, m) order."""
    bh_ij = {l: set(best_hits(a, gj, k)) for l, a in enumerate(gi)}
    bh_ji = {m: set(best_hits(b, gi, k)) for m, b in enumerate(gj)}
    return sorted((l, m) for l in bh_ij for m in bh_ij[l] if l in bh_ji[m])


def all_best_hits(gi: Sequence[str], gj: Sequence[str], k: int, theta=None,
                  tau=None) -> Dict[int, List[Tuple[int, int, int]]]:
    """Row -> [(column, num, den)] for every row of gi, columns ascending."""
    out = {}
    for l, a in enumerate(gi):
        out[l] = [(m, *terms(a, gj[m], k)) for m in best_hits(a, gj, k, theta, tau)]
    return out
