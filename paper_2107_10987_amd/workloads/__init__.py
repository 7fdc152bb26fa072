"""Seeded synthetic inputs shared by the library's tests, the benchmark and the
CPU oracle.  Geometry and initial states only: nothing here computes a step
of the hydro method."""
from .tree import (GHOST, NX, OUTFLOW, PERIODIC, LeafSet, Tree, from_tiles8, morton3,  # noqa: F401
                   split_octets, to_tiles8, uniform_tree)
from .setups import (EGAS, FIELD_NAMES, GAMMA, NF, RHO, SPC, SX, SY, SZ, TAU,  # noqa: F401
                     Workload, binary_star, blast_single_leaf, conserved_from_primitive,
                     lane_emden, polytrope_tree, rotating_polytrope, sedov_uniform,
                     uneven_batches)
