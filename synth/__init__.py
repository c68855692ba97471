"""Seeded synthetic inputs (meshes, masks, materials, actuation draws).

Shared by the oracle and the GPU path; holds none of the method's arithmetic.
"""
from . import meshes, scenes  # noqa: F401
from .scenes import Workload  # noqa: F401
