"""Seeded synthetic inputs shared by the HIP path's tests/bench and the oracle's tests.

This package only draws random scenes and query batches; it holds none of the
metric's arithmetic (no covariance, no distance, no reduction).
"""
from .generators import (  # noqa: F401
    Scene,
    Queries,
    Bodies,
    common_attrs,
    uniform_box_scene,
    room_scene,
    tabletop_scene,
    stone_circle_scene,
    uniform_queries,
    mppi_walk_queries,
    chain_queries,
    chain_ellipsoids,
    random_ellipsoids,
    grid_queries,
    serving_stream,
    config,
    CONFIG_NAMES,
)
