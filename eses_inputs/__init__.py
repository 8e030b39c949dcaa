"""Seeded synthetic inputs shared by the HIP path, its tests and the oracle.

This package holds input generation only (no surface arithmetic): protein-like
atom sets, the radius table and the grid box recipe.  Both the product path and
the oracle receive the arrays it returns; neither imports the other.
"""
from .globule import (
    RADII_TABLE,
    RADII_PROB,
    globule,
    bbox_from_atoms,
    grid_dims,
    workload,
    molecule,
    Molecule,
    batch_sizes,
    batch,
    build,
    WORKLOADS,
    PROBE_RADIUS,
    MARGIN,
)

__all__ = [
    "RADII_TABLE",
    "RADII_PROB",
    "globule",
    "bbox_from_atoms",
    "grid_dims",
    "workload",
    "molecule",
    "Molecule",
    "PROBE_RADIUS",
    "MARGIN",
    "batch_sizes",
    "batch",
    "build",
    "WORKLOADS",
]
