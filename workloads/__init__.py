"""Seeded synthetic workloads shared by the oracle and the GPU path.

This package only *draws inputs*: gate matrices, Kraus sets, noise placements,
input and target states.  It holds none of the method's arithmetic (no
superoperators, no decompositions, no contractions), so the oracle and the
HIP path can both read the same circuits without sharing any code that
computes a result.
"""
from .circuits import (  # noqa: F401
    Op, Circuit, haar_su2, gate_h, gate_x, gate_y, gate_z, gate_t, gate_rx,
    gate_ry, gate_rz, gate_cz, gate_rzz, kraus_depolarizing, kraus_ad_pd,
    chain_layers, grid_layers, qaoa_3regular, place_noises, config, CONFIG_NAMES,
    random_isometry_kraus, tiny_random_circuit, trajectory_uniforms,
)
