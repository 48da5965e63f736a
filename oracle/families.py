"""Gene families for the oracle -- TEST INFRASTRUCTURE ONLY.

Phase (c) of the pipeline extracts gene families from the network the
bidirectional best hits form (overview of the pipeline; the paper describes no
refinement of that network).  Reading: a family is a connected component of
the BBH network over all genes of all genomes.  Each gene is labelled with the
smallest global gene id of its family; a gene without BBH pairs is a family of
its own.  Plain union-find, written for clarity, not speed.
"""
from __future__ import annotations

from typing import Iterable, List, Tuple


def components(n_nodes: int, edges: Iterable[Tuple[int, int]]) -> List[int]:
    """Label of every node = the smallest node id in its connected component."""
    parent = list(range(n_nodes))

    def root(x: int) -> int:
        while parent[x] != x:
            x = parent[x]
        return x

    for u, v in edges:
        ru, rv = root(u), root(v)
        if ru != rv:
            # the smaller root stays a root, so a component's root is its smallest node
            if ru < rv:
                parent[rv] = ru
            else:
                parent[ru] = rv
    return [root(x) for x in range(n_nodes)]


def bbh_edges(pairs_by_task, node_a, node_b) -> List[Tuple[int, int]]:
    """Global edges from per-task BBH lists: pair (a, b) of task t joins nodes
    node_a[t] + a and node_b[t] + b."""
    edges = []
    for t, pairs in enumerate(pairs_by_task):
        for a, b in zip(pairs.a, pairs.b):
            edges.append((int(node_a[t]) + int(a), int(node_b[t]) + int(b)))
    return edges
