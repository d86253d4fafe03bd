"""Seeded synthetic inputs shared by the GPU path's tests/bench and the CPU oracle.

This package holds workload parameters and random draws only: it performs none of
the method's arithmetic (no model steps, no covariance square roots, no Hessian
products). Everything the method computes is done separately by the HIP library
and by the oracle.
"""
from .workloads import *  # noqa: F401,F403
