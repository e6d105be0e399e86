"""Seeded synthetic problem descriptions.

This package only describes inputs (geometry, meshes, KL parameters, the
collocation rule, request streams).  It performs none of the method's
arithmetic, so both the CPU oracle and the GPU library binding may read it.
"""
from .configs import problem, serving_stream, PROBLEM_NAMES  # noqa: F401
