"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds no arithmetic of the RBF-FD method: it only lays out
scattered-but-staggered node sets (the stand-in for the paper's DistMesh
grids, Sec. 3), boundary tags/normals, boundary values and test fields.
Both the CPU oracle and the GPU path consume what it produces.
"""
from .nodes import (splitmix64, uniform01, cavity_nodes, hex_cavity_nodes, cylinder_nodes,
                    square_nodes,
                    build_nodes, NodeSet, TAG_INTERIOR, TAG_WALL, TAG_LID)
from .fields import (wave_field, random_vector, cavity_bc)

__all__ = ["splitmix64", "uniform01", "cavity_nodes", "hex_cavity_nodes", "cylinder_nodes",
           "square_nodes",
           "build_nodes", "NodeSet", "TAG_INTERIOR", "TAG_WALL", "TAG_LID",
           "wave_field", "random_vector", "cavity_bc"]
