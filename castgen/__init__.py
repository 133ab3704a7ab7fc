"""Seeded synthetic inputs for the casting-solidification step (no method arithmetic)."""
from . import rng, meshes, configs  # noqa: F401
