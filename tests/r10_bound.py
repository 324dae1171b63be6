"""Rounding bound of the single-precision query order against the same pair
evaluated in double (test helper; numpy only, no oracle or library code).

The single-precision order (the canonical order of the clearance query) maps
a world point x to grid coordinates of link i with the pose's inverse and the
grid scaling folded into one homogeneous map (the form of the paper's Eq. 4),
then interpolates with seven two-rounding lerps.  In exact arithmetic the map
gives u_a = (R^T (x - t) - lo)_a / h_a, the definition of Sec. III-A.

Rounding count on the way to u_a (unit roundoff u = 2^-24): invh_a (1), each
map entry invh_a R_ba (1), R^T t by a product and two fma (3), the map offset
by one fma (1), cen_a (1), the point's three-fma chain (3), the final + half
(1): 11 roundings, each of a quantity no larger in magnitude than

    S_a = invh_a (sum_b |R_ba| (|x_b| + |t_b|) + |lo_a|) + |cen_a| + (n_a - 1),

so |u_twin - u_exact| <= K_MAP u S_a with K_MAP = 16 (11 plus slack for the
second-order terms).  The interpolant is Lipschitz along axis a with constant
D_a = the largest difference of neighbouring nodes along a, and each lerp
level adds at most 2u max|corner| (two roundings of convex combinations), so
a pair's value moves by at most

    sum_a D_a K_MAP u S_a + K_LERP u max|G|,   K_LERP = 8 (6 plus slack).
"""
from __future__ import annotations

import numpy as np

U32 = 2.0 ** -24
K_MAP = 16
K_LERP = 8


def coord_bound(T, lo, hi, n, points):
    """Bound [C][L][M][3], in grid units, on the single-precision order's
    grid-coordinate error for poses T [C][L][3][4] and points [M][3]."""
    T = np.asarray(T, np.float64)
    lo, hi = np.asarray(lo, np.float64), np.asarray(hi, np.float64)
    n = np.asarray(n, np.float64)
    P = np.abs(np.asarray(points, np.float64).reshape(-1, 3))
    invh = (n - 1.0) / (hi - lo)                              # [L][3]
    cen = np.abs(-lo * invh - 0.5 * (n - 1.0))                # [L][3]
    absR = np.abs(T[..., :3])                                 # [C][L][b][a]
    at = np.einsum("clba,clb->cla", absR, np.abs(T[..., 3]))  # sum_b |R_ba| |t_b|
    ax = P @ absR                                             # sum_b |x_b| |R_ba|, [C][L][M][3]
    S = invh[None, :, None, :] * (ax + at[:, :, None, :] + np.abs(lo)[None, :, None, :]) \
        + (cen + (n - 1.0))[None, :, None, :]
    return K_MAP * U32 * S


def node_slopes(grid):
    """D_a: the largest difference of neighbouring nodes along x, y, z of a
    grid stored [n_z][n_y][n_x]."""
    g = np.asarray(grid, np.float64)
    return np.array([np.abs(np.diff(g, axis=2)).max(), np.abs(np.diff(g, axis=1)).max(),
                     np.abs(np.diff(g, axis=0)).max()])


def value_bound(du, grids):
    """Bound [C][L][M] on a pair's value error from the coordinate bound du
    [C][L][M][3] and the link grids."""
    D = np.stack([node_slopes(g) for g in grids])             # [L][3]
    gmax = np.array([np.abs(np.asarray(g, np.float64)).max() for g in grids])
    return (du * D[None, :, None, :]).sum(-1) + K_LERP * U32 * gmax[None, :, None]


def face_slack(u, n):
    """Per axis, how far grid coordinates u [...][3] lie inside [0, n_a - 1]
    (negative outside), in grid units; n is [L][3] and u is [C][L][M][3]."""
    top = (np.asarray(n, np.float64) - 1.0)[None, :, None, :]
    return np.minimum(u, top - u)
