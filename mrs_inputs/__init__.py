"""Seeded synthetic inputs shared by the renderer and its FP64 reference."""
from . import scenes  # noqa: F401
