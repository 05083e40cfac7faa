"""Seeded synthetic inputs shared by the oracle tests and the GPU path (no method arithmetic)."""
from .scenes import *  # noqa: F401,F403
