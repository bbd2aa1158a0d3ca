"""Seeded synthetic Stokes problems: meshes, finite-element assembly, workloads."""
from .stokes import StokesProblem, config, make_config, make_problem  # noqa: F401
