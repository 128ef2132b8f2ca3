"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This package holds no arithmetic of the method: it only draws random numbers and
writes down the workloads (potential term lists, packet parameters, instance draws).
Both the oracle and the HIP path receive what it produces as plain arrays.
"""
from .workloads import *  # noqa: F401,F403
