"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench."""
from .workloads import (DNA, PROTEIN, PLAIN, PlainWorkload, ServedWorkload, batched_workload,
                        dna_text, pattern_set, patterns_to_csr, plain_workload, protein_probs,
                        protein_text, random_pattern_csr, served_workload)

__all__ = ["DNA", "PROTEIN", "PLAIN", "PlainWorkload", "ServedWorkload", "batched_workload", "dna_text",
           "pattern_set", "patterns_to_csr", "plain_workload", "protein_probs", "protein_text",
           "random_pattern_csr", "served_workload"]
