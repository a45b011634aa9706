"""Seeded synthetic problem data shared by the oracle tests, the GPU tests and the bench."""
from .generators import *  # noqa: F401,F403
