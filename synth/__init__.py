"""Seeded synthetic quantum states shared by the parity tests, the benchmark and the oracle's tests.

This package only prepares state vectors (random amplitudes and random circuits applied to product
states).  It holds none of the arithmetic of the magic computation itself.
"""
from .states import *  # noqa: F401,F403
