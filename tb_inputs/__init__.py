"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

Holds lattice generators and the serving request trace; none of the
propagation arithmetic lives here.
"""
from .lattices import (Lattice, PrimCell, graphene, bilayer, square, honeycomb3, supercell,
                       graphene_cell, bilayer_cell, square_cell, honeycomb3_cell, cell_by_name,
                       sample_sites, rescale_for, state_from_sites, positions, hop_displacements,
                       current_operator, density_operator, area_per_orbital)

__all__ = ["Lattice", "PrimCell", "graphene", "bilayer", "square", "honeycomb3", "supercell",
           "graphene_cell", "bilayer_cell", "square_cell", "honeycomb3_cell", "cell_by_name",
           "sample_sites", "rescale_for", "state_from_sites", "positions", "hop_displacements",
           "current_operator", "density_operator", "area_per_orbital"]
