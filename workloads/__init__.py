"""Seeded synthetic workloads (no method arithmetic); shared by both sides."""
from .cases import *  # noqa: F401,F403
