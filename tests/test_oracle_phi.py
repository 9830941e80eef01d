"""Pins of the oracle's field law against closed-form values.

Reading: phi(d) = k*|d|_2^alpha on the square window |d|_inf <= R, with no
strength at the field's own centre (Table I: a 1x1 geometry has fan-out 0) and
the paper's example constants k = 1, alpha = -0.5 (Fig. 1 caption).
"""
import math

import numpy as np
import pytest


@pytest.mark.parametrize("k,alpha", [(1.0, -0.5), (2.5, -1.0), (0.75, -2.0), (1.0, 0.5)])
def test_closed_form_values(orc, k, alpha):
    R = 5
    # own centre carries nothing
    assert orc.phi(0, 0, R, k, alpha) == 0.0
    # unit axial neighbour: |d| = 1 so phi = k exactly
    assert orc.phi(1, 0, R, k, alpha) == k
    assert orc.phi(0, -1, R, k, alpha) == k
    # diagonal neighbour: |d| = sqrt(2)
    assert math.isclose(orc.phi(1, 1, R, k, alpha), k * 2.0 ** (alpha / 2), rel_tol=1e-15)
    # 3-4-5 triangle
    assert math.isclose(orc.phi(3, 4, R, k, alpha), k * 5.0 ** alpha, rel_tol=1e-15)
    assert math.isclose(orc.phi(-4, 3, R, k, alpha), k * 5.0 ** alpha, rel_tol=1e-15)
    # window corner is inside, one beyond is outside (square window)
    assert math.isclose(orc.phi(R, R, R, k, alpha), k * (2.0 * R * R) ** (alpha / 2),
                        rel_tol=1e-15)
    assert orc.phi(R + 1, 0, R, k, alpha) == 0.0
    assert orc.phi(0, R + 1, R, k, alpha) == 0.0
    assert orc.phi(-R - 1, R, R, k, alpha) == 0.0


def test_paper_constants_values(orc):
    # k = 1, alpha = -0.5: phi = |d|^-1/2
    assert orc.phi(2, 0, 3, 1.0, -0.5) == pytest.approx(1 / math.sqrt(2), rel=1e-15)
    assert orc.phi(3, 3, 3, 1.0, -0.5) == pytest.approx(18 ** -0.25, rel=1e-15)
    assert orc.phi(1, 2, 3, 1.0, -0.5) == pytest.approx(5 ** -0.25, rel=1e-15)


def test_table_layout_and_symmetry(orc):
    R = 4
    t = orc.phi_table(R, 1.0, -0.5)
    assert t.shape == (9, 9)
    assert t[R, R] == 0.0
    # [dy+R, dx+R] layout against single evaluations
    for dy in range(-R, R + 1):
        for dx in range(-R, R + 1):
            assert t[dy + R, dx + R] == orc.phi(dx, dy, R, 1.0, -0.5)
    # eightfold symmetry of an isotropic law
    assert np.array_equal(t, t[::-1, :])
    assert np.array_equal(t, t[:, ::-1])
    assert np.array_equal(t, t.T)


def test_radius_zero_has_no_strength(orc):
    # Table I, 1x1 geometry: fan-out 0, the field touches no other su
    t = orc.phi_table(0, 1.0, -0.5)
    assert t.shape == (1, 1) and t[0, 0] == 0.0
