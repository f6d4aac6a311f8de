"""Seeded synthetic inputs shared by tests and benchmarks (no method code)."""
from .inputs import *  # noqa: F401,F403
