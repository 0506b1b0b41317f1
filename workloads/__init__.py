"""Seeded synthetic workloads (matrices and right-hand sides); no method arithmetic."""
from .generators import *  # noqa: F401,F403
