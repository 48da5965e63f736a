"""Seeded synthetic protein-genome generator.

This package only draws random inputs (genomes, gene orders, arrival times).
It holds none of the similarity, best-hit, k-rule or dictionary arithmetic:
both the CPU oracle and the HIP path consume what it produces, and neither is
imported from here.
"""
from .genomes import (  # noqa: F401
    ALPHABET,
    BASE_SEED,
    Genome,
    Dataset,
    config_seed,
    random_genome,
    genome_from_strings,
    planted_pair,
    family_dataset,
    make_config,
    serving_workload,
    batched_instances,
)
