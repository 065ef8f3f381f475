"""Seeded synthetic OT instances shared by the oracle tests, the GPU tests and
the benchmark (problem data only, no solver arithmetic)."""
from .instances import *  # noqa: F401,F403
