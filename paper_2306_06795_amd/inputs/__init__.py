"""Seeded synthetic Stokes problems: meshes, finite-element assembly, workloads."""
from .stokes import (SERVE_MESHES, StokesProblem, config, make_config, make_problem,  # noqa: F401
                     make_serve_mesh, random_rhs, serve_mesh_key, serve_stream)
