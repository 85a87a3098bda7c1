"""Hierarchical Jacobi (Islam & Wang, arXiv:2006.16465) on MI355X / gfx950.

The solver lives in the HIP library ``libhj.so`` behind the C ABI declared in
``include/hj.h``; ``hj`` is its Python binding (torch tensors in, status
codes out) and ``workloads`` draws the seeded synthetic Poisson inputs.
"""
from . import hj, workloads  # noqa: F401

__all__ = ["hj", "workloads"]
