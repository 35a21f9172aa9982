"""Seeded synthetic inputs shared by the oracle tests and the HIP path.

This package only draws random numbers and lays them out (cores, noise,
initial cores, smooth fields).  It holds none of the ALS arithmetic, and it
imports neither ``oracle`` nor the HIP package.
"""
from .synth import *  # noqa: F401,F403
