"""The SUPAv1-v5 presets (Table 2) on the oracle: v1 is fully fixed by the
paper (128 points of E0/128 in layer 0 per event); v2-v5 need the plotted
probabilities and check their layer configurations and angle settings."""
import math

import numpy as np
import pytest

from oracle import supa_oracle as O
from paper_2202_05012_amd import presets, supa


@pytest.mark.parametrize("kin", ["3d", "literal"])
def test_v1_exact(kin):
    g = presets.supa(1, kinematics=kin)
    supa.validate_geometry(g)                      # the library accepts it (host check)
    e0, pol, az = presets.incident(5)
    r = O.simulate(g, e0, pol, az, seed=3)
    assert (r["counts"][:, 1] == 128).all() and (r["hit_layer"] == 0).all()
    assert (r["hit_plane"] == 7).all() and (r["hit_e"] == 65 * 2 ** 14).all()


def test_layer_configurations_of_table_2():
    assert presets.layer_of_plane(1) == [-1] * 5 + [0] * 6
    assert presets.layer_of_plane(2) == [-1] * 7 + [0] * 14
    assert presets.layer_of_plane(4) == [-1] * 7 + [0] * 6
    assert presets.layer_of_plane(5) == [-1] * 7 + [0] * 6 + [1] * 16


def test_v2_to_v5_need_the_plotted_probabilities():
    for v in (2, 3, 4, 5):
        with pytest.raises(ValueError):
            presets.supa(v)
    with pytest.raises(ValueError):
        presets.supa(1, p_split=[1.0] * 11, p_stop=[0.0] * 11)


def test_v3_angles_and_fractions():
    N = presets.N_PLANES[3]
    g = presets.supa(3, p_split=[1.0] * 5 + [0.0] * (N - 5), p_stop=[0.0] * 5 + [1.0] + [0.0] * (N - 6))
    assert g["angle_mode"] == "uniform" and g["angle_a"] == math.pi / 32 and g["angle_b"] == math.pi / 16
    assert (g["frac_lo"], g["frac_hi"]) == (0.25, 0.75)     # eps ~ U(-theta/4, theta/4)
    e0, pol, az = presets.incident(20)
    r = O.simulate(g, e0, pol, az, seed=8)
    assert (r["counts"][:, 1] == 32).all()                   # five certain splits, then a stop
    assert (r["hit_layer"] == -1).all()                      # sub-layer 5 is dead material
    fr = r["node_e"][r["node_parent"] == 0] / (65 * 2 ** 21)
    assert ((fr >= 0.25 - 1e-6) & (fr <= 0.75 + 1e-6)).all()
