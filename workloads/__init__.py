"""Seeded synthetic inputs for the collision-operator hot path.

This package is shared by the CPU oracle tests, the GPU parity tests and the
benchmark. It holds only the definition of the inputs (velocity nodes, the
Maxwellian of the paper's eq. (M), the BKW initial datum, random draws) and none
of the collision operator's arithmetic. `workloads.mesh` adds the seeded
polygonal meshes and initial data of the transport workload.
"""

from .synth import (  # noqa: F401
    velocity_nodes,
    maxwellian,
    bkw_initial,
    mixture_cells,
    noisy_mixture_cells,
    config_inputs,
    CONFIGS,
)
