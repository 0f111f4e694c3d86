"""Seeded synthetic workloads shaped like the paper's experiments.

This module only draws inputs (point clouds, right-hand sides, request
streams).  It holds none of the method's arithmetic, so both the CPU oracle
and the GPU path may import it.

Workload shapes:
  * ``disk``      area-uniform points in the unit disk (small Laplace case);
  * ``ellipses``  three disjoint, non-nested ellipses sampled uniformly in
                  arclength with a small tangential jitter (boundary-element
                  style point sets, Introduction and Theorem 1 assume points
                  on a curve);
  * ``square``    points uniform in the unit square (Section 7.1, where two
                  sets of N points uniform in a square are used);
  * ``star``      a closed star-shaped curve r(t) = r0 (1 + sum a_m cos(m t + p_m)),
                  sampled uniformly in arclength (Helmholtz and serving cases).
All generators use ``numpy.random.default_rng(seed)``.
"""
from .workloads import (disk_points, square_points, ellipse_points, star_points, serving_curve,
                        curve_weights, real_rhs, complex_rhs, request_stream, WORKLOADS, make_workload)

__all__ = ["disk_points", "square_points", "ellipse_points", "star_points", "serving_curve", "curve_weights",
           "real_rhs", "complex_rhs", "request_stream", "WORKLOADS", "make_workload"]
