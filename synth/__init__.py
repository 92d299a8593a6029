"""Seeded synthetic inputs shared by the oracle side and the HIP side.

Input generation only: nothing here computes pin counts, gains or moves.
"""
from .hypergraphs import (Instance, Request, batch_instances, describe,  # noqa: F401
                          neighbour_clusters, random_power_law, served_pool, served_trace, sparse_matrix,
                          tiny_plain, vlsi_grid, with_k)
