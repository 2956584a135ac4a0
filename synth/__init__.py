"""Seeded synthetic inputs (inputs only: none of the normalization method's arithmetic lives here)."""
from .generator import *  # noqa: F401,F403
