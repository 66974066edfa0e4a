"""Seeded synthetic inputs shared by the CPU oracle tests and the GPU path."""
from . import matrices, workloads  # noqa: F401
