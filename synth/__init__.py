"""Seeded synthetic inputs shared by the oracle side and the HIP side.

Input generation only: nothing here computes pin counts, gains or moves.
"""
from .hypergraphs import (Instance, batch_instances, describe, random_power_law,  # noqa: F401
                          sparse_matrix, tiny_plain, vlsi_grid, with_k)
