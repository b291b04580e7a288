"""Seeded synthetic inputs for the ISCI sigma step.

This package only draws random numbers and assembles integral arrays.  It
holds none of the method's arithmetic (no strings, signs, screening or
matrix elements), so both the CPU oracle and the HIP library can consume
its arrays without sharing any code with each other.
"""
from .recipes import (recipe_a, recipe_b, recipe_random, canonicalize_eri,
                      symmetrize_h, random_vectors)
from .workloads import WORKLOADS, Workload, workload

__all__ = ["recipe_a", "recipe_b", "recipe_random", "canonicalize_eri",
           "symmetrize_h", "random_vectors", "WORKLOADS", "Workload",
           "workload"]
