"""Seeded synthetic optimal-transport instances.

This package only draws problem data (marginals, coordinates, cost matrices).
It holds none of the solver's arithmetic and is shared by the tests, the
benchmark and the oracle checks, so both sides of every parity test see the
same bytes.
"""
from .generators import (  # noqa: F401
    Instance,
    points_sqeuclid,
    grid_pair,
    gmm_euclid,
    batch_instances,
    serving_stream,
    config_instance,
)
