"""Regression of the oracle against its stored fixture (tests/golden/)."""
import json
import os

import numpy as np

from tests.golden import make_golden as G


def test_oracle_matches_stored_fixture():
    with open(G.OUT) as fh:
        ref = json.load(fh)
    cur = G.summary()
    for k in ("total_mass", "mean_abs_F_minus_I", "max_abs_C"):
        assert abs(cur[k] - ref[k]) <= 1e-12 * max(1.0, abs(ref[k])), k
    for k in ("centre_of_mass", "momentum", "x_first_particles"):
        np.testing.assert_allclose(np.asarray(cur[k]), np.asarray(ref[k]), rtol=1e-12, atol=1e-15)
    # free fall before contact: the momentum is exactly sum m * n dt g
    g = -9.8 * ref["substeps"] * 1e-4 * ref["total_mass"]
    assert abs(ref["momentum"][1] - g) < 1e-9 * abs(g)
