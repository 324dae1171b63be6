"""Values the paper prints, checked against the oracle's helpers."""
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def test_clearance_threshold_is_sum_of_half_cell_diagonals(orc):
    """Sec. IV-C sets the clearance threshold to the environment-voxel and
    Link-SDF discretisation bounds added together and prints about 4.3 cm;
    the oracle's half-cell-diagonal bound must give the same number."""
    g = json.load(open(GOLDEN))["clearance_threshold"]
    re, rr = g["environment_voxel_m"], g["link_sdf_resolution_m"]
    total = orc.grid_bound(np.full(3, re)) + orc.grid_bound(np.full(3, rr))
    assert round(total * 100, g["printed_digits"]) == g["printed_value_cm"]
    assert abs(total - 0.043301270189) < 1e-12
