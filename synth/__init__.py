"""Seeded synthetic inputs shared by the oracle side and the HIP side.

Input generation only: nothing here computes pin counts, gains or moves.
"""
from .hypergraphs import (Instance, describe, random_power_law, sparse_matrix,  # noqa: F401
                          tiny_plain, vlsi_grid, with_k)
