"""Seeded joint-space waypoints: a natural cubic spline per joint through four
configurations drawn uniformly inside the joint limits, sampled at C evenly
spaced parameters and clamped to the limits.

Stands in for the paper's RRT plan with TOPP-RA gridpoints (300-500
waypoints per trajectory, Sec. IV-C), which needs a planner and a robot model
that are not available.  Input generation only.
"""
from __future__ import annotations

import numpy as np
from scipy.interpolate import CubicSpline


def make_waypoints(qmin: np.ndarray, qmax: np.ndarray, C: int, seed: int,
                   n_knots: int = 4) -> np.ndarray:
    """float64 [C][dof] joint angles (radians)."""
    rng = np.random.default_rng(seed)
    dof = qmin.shape[0]
    knots = rng.uniform(qmin, qmax, size=(n_knots, dof))
    t_knots = np.linspace(0.0, 1.0, n_knots)
    spline = CubicSpline(t_knots, knots, axis=0, bc_type="natural")
    if C == 1:
        t = np.zeros(1)
    else:
        t = np.arange(C, dtype=np.float64) / (C - 1)
    q = spline(t)
    return np.clip(q, qmin, qmax)
