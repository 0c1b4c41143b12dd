"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This package holds no arithmetic of the method itself: it only draws random
numbers (SplitMix64) and lays out the fracture tables and the workload sizes.
Both the CPU oracle and the HIP path receive what it produces as plain inputs.
"""
from .splitmix import SplitMix64
from .fractures import (disc_table, rect_table, rect_network_table, c1_crack, DISC_COLS, RECT_COLS)
from .configs import WORKLOADS, Workload, hierarchy_nodes_per_side, level_cells

__all__ = ["SplitMix64", "disc_table", "rect_table", "rect_network_table", "c1_crack", "DISC_COLS",
           "RECT_COLS", "WORKLOADS", "Workload", "hierarchy_nodes_per_side",
           "level_cells"]
