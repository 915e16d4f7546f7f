"""Seeded synthetic inputs for KCM chains.

This package only draws numbers: residue-type parameter tables, sequences,
initial dihedral angles, batch lengths and serving arrival streams.  It holds
none of the method's arithmetic (no geometry, no forces, no torques), so that
both the HIP library and the CPU oracle can consume the same inputs without
sharing any computation.
"""
from .chains import (  # noqa: F401
    ATOMS_PER_RES,
    BASE_SEED,
    N_TYPES,
    TYPE_TABLE_SEED,
    ResidueTypes,
    alanine_like_types,
    batch_lengths,
    config_seed,
    load_globule,
    mc_moves,
    polyala_starts,
    random_chi,
    random_dihedrals,
    residue_types,
    sequence,
    serving_jobs,
)
