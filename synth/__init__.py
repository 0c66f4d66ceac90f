"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module builds particle sets, species assignments, interaction-strength
matrices and force-factor tables. It holds none of the tree method's
arithmetic (no keys, sorting, tree, monopoles, opening test, interpolation
or force sums): everything here is an *input* to the method.
"""
from .generators import *  # noqa: F401,F403
