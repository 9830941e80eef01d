"""GPU tests of the incremental field update (sf_set_field_update).

Between full superpositions, each tick adds the stamps at the su its
winners entered and subtracts those at the su they left, into an exact FP64
pedestrian field.  Bar: the same as the full path (parity.py: the field bit
for bit, no mismatched decision) at every tick of a refresh period;
bit-for-bit independence of the launch shape and of the refresh period;
batches refuse such scenes.
"""
import numpy as np
import pytest

import oracle
from paper_1803_04782_amd import scenes

pytestmark = pytest.mark.gpu

from parity import assert_parity, lockstep  # noqa: E402


@pytest.fixture(scope="module")
def sf():
    from paper_1803_04782_amd import sf as _sf

    _sf.load()
    return _sf


def _say(*a):
    print(*a, flush=True)


CASES = [
    ("room64", lambda: scenes.room64(), 16, 200, 1),
    ("dense", lambda: scenes.random_scene(150, 140, n_peds=0, radius=8, seed=41, bernoulli=0.03,
                                          exits=("E", "W"), exit_width=8, occupancy=0.4),
     32, 80, 1),
    ("wide-R", lambda: scenes.random_scene(200, 131, n_peds=1500, radius=33, seed=7,
                                           exits=("N",), exit_width=8), 8, 40, 1),
    ("hall1024", lambda: scenes.hall1024(), 32, 200, 10),
    ("max-R-torus", lambda: scenes.flow_scene(130, 100, 0.3, 8, radius=48, seed=42), 8, 30, 1),
]


@pytest.mark.parametrize("name,make,K,ticks,every", CASES, ids=[c[0] for c in CASES])
def test_incremental_lockstep(sf, name, make, K, ticks, every):
    sc = make()
    st = oracle.statics(sc)
    with sf.GpuScene(sc) as g:
        g.set_field_update(K)
        rep = lockstep(g, st, sc.start_step, ticks, every)
    _say(f"[incremental K={K}] {name}", rep)
    assert_parity(rep)


def test_incremental_tile_shape_invariance(sf, monkeypatch):
    sc = scenes.random_scene(130, 90, n_peds=1500, radius=7, seed=33, bernoulli=0.03)
    out = []
    for shape in ("16x2x2x8", "32x4x2x4", "8x2x2x4", "16x4x4x8", "8x4x4x4", "16x4x4x16"):
        monkeypatch.setenv("SF_TILE", shape)
        with sf.GpuScene(sc) as g:
            g.set_field_update(16)
            g.step(12)
            out.append((g.field(), g.positions()))
    for f, p in out[1:]:
        assert np.array_equal(f, out[0][0])
        assert np.array_equal(p, out[0][1])


def test_refresh_one_is_the_full_superposition(sf):
    sc = scenes.random_scene(90, 70, n_peds=600, radius=5, seed=3, bernoulli=0.02)
    with sf.GpuScene(sc) as a, sf.GpuScene(sc) as b:
        b.set_field_update(1)
        a.step(20)
        b.step(20)
        assert np.array_equal(a.field(), b.field())
        assert np.array_equal(a.positions(), b.positions())


def test_incremental_scene_cannot_join_a_batch(sf):
    sc = scenes.random_scene(40, 40, n_peds=50, radius=3, seed=1)
    with sf.GpuScene(sc) as g:
        g.set_field_update(8)
        with pytest.raises(sf.SfError):
            sf.Batch([g])
        g.set_field_update(0)
        with sf.Batch([g]) as b:
            b.step(2)
            with pytest.raises(sf.SfError):
                g.set_field_update(8)


@pytest.mark.parametrize("K", [2, 16, 1000])
def test_update_is_the_full_field_bit_for_bit(sf, K):
    """The pedestrian field is kept exactly, so between refreshes every
    updated field equals the full superposition of the same positions, bit
    for bit, however long the refresh period (no drift to bound)."""
    sc = scenes.random_scene(180, 120, n_peds=3000, radius=9, seed=77, bernoulli=0.04,
                             exits=("E", "W", "S"), exit_width=8, k=-0.6, k_obs=0.4)
    with sf.GpuScene(sc) as a, sf.GpuScene(sc) as b:
        b.set_field_update(K)
        for t in range(60):
            a.step(1)
            b.step(1)
            assert np.array_equal(a.positions(), b.positions()), t
            assert np.array_equal(a.field(), b.field()), t
