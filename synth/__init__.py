"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path."""
from .generators import *  # noqa: F401,F403
