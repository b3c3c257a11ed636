"""Seeded synthetic inputs shared by the oracle and the GPU path (no PCA arithmetic)."""
from . import philox, fixtures  # noqa: F401
