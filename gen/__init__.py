"""Seeded synthetic workloads shared by the tests, the benchmark and the smoke check.

This package only draws inputs (points, values, polygons, viewport queries);
it holds none of the approximation or aggregation arithmetic.
"""
from .workloads import *  # noqa: F401,F403
