"""Pins of the oracle's field law against closed-form values.

Reading: phi(d) = fl32(k*|d|_2^alpha) on the square window |d|_inf <= R, with
no strength at the field's own centre (Table I: a 1x1 geometry has fan-out 0)
and the paper's example constants k = 1, alpha = -0.5 (Fig. 1 caption).  The
strengths are FP32 numbers, the precision of the paper's float caches
(Algorithms 2 and 3): the law is evaluated exactly enough and rounded once.
"""
import math

import numpy as np
import pytest


def f32(v):
    """The FP32 number nearest to v, as a Python float."""
    return float(np.float32(v))


@pytest.mark.parametrize("k,alpha", [(1.0, -0.5), (2.5, -1.0), (0.75, -2.0), (1.0, 0.5)])
def test_closed_form_values(orc, k, alpha):
    R = 5
    # own centre carries nothing
    assert orc.phi(0, 0, R, k, alpha) == 0.0
    # unit axial neighbour: |d| = 1 so phi = k exactly
    assert orc.phi(1, 0, R, k, alpha) == k
    assert orc.phi(0, -1, R, k, alpha) == k
    # diagonal neighbour: |d| = sqrt(2)
    assert orc.phi(1, 1, R, k, alpha) == f32(k * 2.0 ** (alpha / 2))
    # 3-4-5 triangle
    assert orc.phi(3, 4, R, k, alpha) == f32(k * 5.0 ** alpha)
    assert orc.phi(-4, 3, R, k, alpha) == f32(k * 5.0 ** alpha)
    # window corner is inside, one beyond is outside (square window)
    assert orc.phi(R, R, R, k, alpha) == f32(k * (2.0 * R * R) ** (alpha / 2))
    assert orc.phi(R + 1, 0, R, k, alpha) == 0.0
    assert orc.phi(0, R + 1, R, k, alpha) == 0.0
    assert orc.phi(-R - 1, R, R, k, alpha) == 0.0


def test_paper_constants_values(orc):
    # k = 1, alpha = -0.5: phi = |d|^-1/2
    assert orc.phi(2, 0, 3, 1.0, -0.5) == f32(1 / math.sqrt(2))
    assert orc.phi(3, 3, 3, 1.0, -0.5) == f32(18 ** -0.25)
    assert orc.phi(1, 2, 3, 1.0, -0.5) == f32(5 ** -0.25)
    # the values are FP32 numbers, within half an FP32 ulp of the exact law
    for dx, dy in [(1, 1), (2, 1), (3, 2), (3, 3)]:
        exact = (dx * dx + dy * dy) ** -0.25
        v = orc.phi(dx, dy, 3, 1.0, -0.5)
        assert float(np.float32(v)) == v
        assert abs(v - exact) <= 2.0 ** -24 * exact


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


@pytest.mark.parametrize("R,k,alpha", [(4, 1.0, -0.5), (12, -0.1, -0.5), (32, 2.0, -0.5),
                                       (48, 1.0, -0.5), (16, 0.7, 1.0), (9, -1.3, -2.0)])
def test_sums_of_strengths_are_exact(orc, R, k, alpha):
    # Every field is a sum of FP32 strengths formed in FP64.  For these laws
    # the strengths span few binades, so every partial sum of a window is an
    # exact FP64 number: the oracle's superposition equals the rational sum of
    # the same FP32 values (Python fractions, no rounding at all), whatever
    # the order of the terms.
    from fractions import Fraction

    rng = np.random.default_rng(R)
    W = H = 2 * R + 7
    src = (rng.random(W * H) < 0.4).astype(np.uint8)
    got = orc.source_field(W, H, src, R, k, alpha)
    tab = [[Fraction(orc.phi(dx, dy, R, k, alpha)) for dx in range(-R, R + 1)]
           for dy in range(-R, R + 1)]
    cells = rng.choice(W * H, size=12, replace=False)
    for c in cells:
        x, y = int(c % W), int(c // W)
        exact = Fraction(0)
        for sy in range(max(0, y - R), min(H, y + R + 1)):
            for sx in range(max(0, x - R), min(W, x + R + 1)):
                if src[sy * W + sx]:
                    exact += tab[y - sy + R][x - sx + R]
        assert Fraction(got[c]) == exact, (c, float(got[c]), float(exact))
