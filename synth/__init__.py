"""Seeded synthetic inputs for greedy column subset selection.

This package only draws random numbers and lays them out; it holds none of
the selection method's arithmetic.  Both the CPU oracle's tests and the GPU
path's tests/bench take their inputs from here.
"""
from .gen import *  # noqa: F401,F403
