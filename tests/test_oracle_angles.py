"""Pins for the oracle's cylindrical frame, helix angle and intrusion angle (CPU only).

Expected values are derived by hand below (right-handed frame, e_theta =
a x e_r), plus field-wide closed forms and the behaviour under rotations and
reflections of the voxel grid.
"""

import math

import numpy as np
import pytest

import oracle

S2 = 1.0 / math.sqrt(2.0)

# (center, direction, voxel (z, y, x), e3 (z, y, x), HA, IA) -- derivations:
#  axis +z through the origin, voxel (3, 0, 5): e_r = +x, e_theta = z x x = +y
#  axis +z through the origin, voxel (0, 4, 0): e_r = +y, e_theta = z x y = -x
#  axis +x through the origin, voxel (2, 0, 7): e_r = +z, e_theta = x x z = -y
HAND = [
    ((0, 0, 0), (1, 0, 0), (3, 0, 5), (0, 1, 0), 0.0, 0.0),               # circumferential
    ((0, 0, 0), (1, 0, 0), (3, 0, 5), (S2, S2, 0), math.pi / 4, 0.0),     # e_theta + axis
    ((0, 0, 0), (1, 0, 0), (3, 0, 5), (S2, -S2, 0), -math.pi / 4, 0.0),   # -e_theta + axis
    ((0, 0, 0), (1, 0, 0), (3, 0, 5), (-S2, -S2, 0), math.pi / 4, 0.0),   # sign flip of row 2
    ((0, 0, 0), (1, 0, 0), (3, 0, 5), (0, math.sqrt(3) / 2, 0.5), 0.0, math.pi / 6),  # e_theta cos30 + e_r sin30
    ((0, 0, 0), (1, 0, 0), (3, 0, 5), (1, 0, 0), math.pi / 2, 0.0),       # along the axis (f_theta = 0)
    ((0, 0, 0), (1, 0, 0), (0, 4, 0), (0, 0, 1), 0.0, 0.0),               # -e_theta: HA 0
    ((0, 0, 0), (1, 0, 0), (0, 4, 0), (S2, 0, -S2), math.pi / 4, 0.0),    # e_theta + axis
    ((0, 0, 0), (0, 0, 1), (2, 0, 7), (0, -0.5, math.sqrt(3) / 2), math.pi / 3, 0.0),
    ((0, 0, 0), (0, 0, 5), (2, 0, 7), (0, -0.5, math.sqrt(3) / 2), math.pi / 3, 0.0),  # unnormalised direction
    ((1.5, 2.0, 3.5), (1, 0, 0), (1, 2, 8), (S2, S2, 0), math.pi / 4, 0.0),  # shifted centre: e_r = +x again
]


def _single(center, direction, voxel, e3):
    shape = tuple(v + 1 for v in voxel)
    frame = oracle.cylindrical_frame(shape, center, direction)
    e = np.zeros((3,) + shape)
    e[(slice(None),) + tuple(voxel)] = e3
    ha, ia, on = oracle.helix_intrusion(e, frame)
    return ha[tuple(voxel)], ia[tuple(voxel)], on[tuple(voxel)]


@pytest.mark.parametrize("center,direction,voxel,e3,ha,ia", HAND)
def test_hand_derived_angles(center, direction, voxel, e3, ha, ia):
    got_ha, got_ia, on = _single(center, direction, voxel, e3)
    assert not on
    assert abs(got_ha - ha) < 1e-15 and abs(got_ia - ia) < 1e-15


def test_on_axis_voxels_are_flagged_and_zero():
    got_ha, got_ia, on = _single((2, 3, 3), (1, 0, 0), (0, 3, 3), (0, 1, 0))
    assert on and got_ha == 0.0 and got_ia == 0.0


def test_handedness_e_theta():
    # axis +z: at +x the circumferential direction is +y, at +y it is -x (counter-clockwise)
    e_r, e_t, a, r = oracle.cylindrical_frame((1, 9, 9), (0, 4, 4), (1, 0, 0))
    np.testing.assert_allclose(e_t[:, 0, 4, 8], [0, 1, 0], atol=1e-15)
    np.testing.assert_allclose(e_t[:, 0, 8, 4], [0, 0, -1], atol=1e-15)
    assert r[0, 4, 8] == 4.0


@pytest.mark.parametrize("direction", [(1, 0, 0), (0.3, -0.5, 0.8)])
def test_field_closed_forms(direction):
    shape = (9, 10, 11)
    center = (4.2, 4.7, 5.1)
    e_r, e_t, a, r = oracle.cylindrical_frame(shape, center, direction)
    alpha = np.linspace(-1.4, 1.4, e_r[0].size).reshape(shape)
    helix = np.cos(alpha) * e_t + np.sin(alpha) * a.reshape(3, 1, 1, 1)
    ha, ia, on = oracle.helix_intrusion(helix, (e_r, e_t, a, r))
    np.testing.assert_allclose(ha, alpha, atol=1e-14)
    np.testing.assert_allclose(ia, 0.0, atol=1e-14)
    intr = np.cos(alpha) * e_t + np.sin(alpha) * e_r
    ha, ia, on = oracle.helix_intrusion(intr, (e_r, e_t, a, r))
    np.testing.assert_allclose(ia, alpha, atol=1e-14)
    np.testing.assert_allclose(ha, 0.0, atol=1e-14)
    # sign invariance
    ha2, ia2, _ = oracle.helix_intrusion(-intr, (e_r, e_t, a, r))
    np.testing.assert_allclose(ia2, ia, atol=1e-14)


def _wrap(d):
    d = np.abs(d) % np.pi
    return np.minimum(d, np.pi - d)


def test_grid_rotation_and_reflection():
    """A cyclic axis permutation is a rotation (angles unchanged); swapping z and y is a
    reflection, which flips the handedness of e_theta and so negates HA and IA."""
    rng = np.random.default_rng(2)
    V = rng.random((14, 15, 16))
    c = (6.5, 7.2, 7.9)
    base = oracle.compute(V, sigma=1.0, rho=1.5, axis_center=c, axis_direction=(1, 0, 0))
    ok = base["gap"] >= 1e-2
    # rotation: new (z', y', x') = old (y, x, z)
    Vr = V.transpose(1, 2, 0)
    rot = oracle.compute(Vr, sigma=1.0, rho=1.5, axis_center=(c[1], c[2], c[0]), axis_direction=(0, 0, 1))
    okr = ok.transpose(1, 2, 0)
    assert _wrap(rot["ha"] - base["ha"].transpose(1, 2, 0))[okr].max() < 1e-9
    assert _wrap(rot["ia"] - base["ia"].transpose(1, 2, 0))[okr].max() < 1e-9
    np.testing.assert_allclose(rot["fa"], base["fa"].transpose(1, 2, 0), atol=1e-12)
    # reflection: swap z and y
    Vs = V.transpose(1, 0, 2)
    ref = oracle.compute(Vs, sigma=1.0, rho=1.5, axis_center=(c[1], c[0], c[2]), axis_direction=(0, 1, 0))
    oks = ok.transpose(1, 0, 2)
    assert _wrap(ref["ha"] + base["ha"].transpose(1, 0, 2))[oks].max() < 1e-9
    assert _wrap(ref["ia"] + base["ia"].transpose(1, 0, 2))[oks].max() < 1e-9
