"""GPU parity of pedestrians larger than one su (section 2 odd footprints;
the footprint experiment of Table VI) against the FP64 oracle.

Bar (parity.py): the field bit for bit (the field radiates from the centres),
no mismatch of target, election or position, in lockstep on walled rooms
and tori with 3x3 .. 7x7 bodies, headings and walk periods; a lone walker's
closed form; bad bodies rejected; batches refuse body scenes; the incremental
update gives the full field bit for bit.
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


ROOMS = [
    ("3x3", lambda: scenes.body_room(90, 70, 3, 3, 220, 4, seed=1, exits=("E", "W"),
                                     exit_width=12, bernoulli=0.02)),
    ("5x3", lambda: scenes.body_room(100, 64, 5, 3, 150, 6, seed=2, exits=("E", "N"),
                                     exit_width=13, bernoulli=0.01)),
    ("3x5-attractive", lambda: scenes.body_room(96, 80, 3, 5, 180, 5, seed=3,
                                                exits=("S", "W"), exit_width=11, k=-0.3,
                                                k_obs=0.6)),
    ("7x7", lambda: scenes.body_room(130, 110, 7, 7, 70, 12, seed=4, exits=("E",),
                                     exit_width=21)),
]


@pytest.mark.parametrize("name,make", ROOMS, ids=[r[0] for r in ROOMS])
def test_body_room_lockstep(sf, name, make):
    sc = make()
    st = oracle.statics(sc)
    with sf.GpuScene(sc) as g:
        rep = lockstep(g, st, sc.start_step, 30)
        s = g.stats()
    _say(f"[bodies] {name}", rep, f"moved {s['moved']}, left {s['evacuated']}")
    assert_parity(rep)
    assert s["moved"] > 0


TORI = [
    ("torus-3x3-k8", lambda: scenes.body_flow_scene(128, 96, 0.45, 8, 3, radius=9, seed=5)),
    ("torus-5x5-k4-walk", lambda: scenes.body_flow_scene(150, 120, 0.5, 4, 5, radius=15, seed=6,
                                                         max_walk_period=5)),
    ("torus-1x1-k2", lambda: scenes.body_flow_scene(100, 70, 0.5, 2, 1, radius=3, seed=7)),
]


@pytest.mark.parametrize("name,make", TORI, ids=[t[0] for t in TORI])
def test_body_torus_lockstep(sf, name, make):
    sc = make()
    st = oracle.statics(sc)
    with sf.GpuScene(sc) as g:
        rep = lockstep(g, st, sc.start_step, 25)
        assert g.stats()["live"] == sc.n_peds
    _say(f"[bodies] {name}", rep)
    assert_parity(rep)


def test_lone_body_walker(sf):
    W, H = 30, 13
    ob = np.zeros((H, W), np.uint8)
    ob[0, :] = ob[-1, :] = 1
    ob[:, 0] = ob[:, -1] = 1
    ex = np.zeros((H, W), np.uint8)
    ex[1:H - 1, W - 1] = 1
    ob[1:H - 1, W - 1] = 0
    x0, y0 = 4, 6
    sc = scenes.Scene(width=W, height=H, obstacle=ob.ravel(), exit=ex.ravel(),
                      pos=np.array([y0 * W + x0], np.int32), radius=3, k_obs=0.0,
                      body_w=5, body_h=3)
    with sf.GpuScene(sc) as g:
        d0, a = W - 1 - x0, 2
        for t in range(d0 - a - 1):
            g.step(1)
            assert g.positions()[0] >= 0, t
        g.step(1)
        assert g.positions()[0] == -1
        assert g.stats()["evacuated"] == 1


def test_bad_bodies_rejected(sf):
    W, H = 40, 30
    sc = scenes.body_room(W, H, 3, 3, 10, 2, seed=9, exits=("E",), exit_width=9)
    overlap = np.array([10 * W + 10, 11 * W + 11], np.int32)  # blocks share su (11, 11)
    rc, msg = sf.create_error(sc.with_params(pos=overlap))
    assert rc == sf.SF_EINVAL and "shares" in msg, msg
    rc, msg = sf.create_error(sc.with_params(pos=np.array([1 * W + 1], np.int32)))
    assert rc == sf.SF_EINVAL and "obstacle" in msg, msg  # the block covers the walls
    rc, msg = sf.create_error(sc.with_params(body_w=4))
    assert rc == sf.SF_EINVAL and "odd" in msg, msg
    with sf.GpuScene(sc) as g:
        with pytest.raises(sf.SfError):
            sf.Batch([g])


def test_body_incremental_update_is_the_full_field(sf):
    sc = scenes.body_flow_scene(128, 100, 0.4, 8, 3, radius=6, seed=8)
    with sf.GpuScene(sc) as a, sf.GpuScene(sc) as b:
        b.set_field_update(32)
        for t in range(20):
            a.step(1)
            b.step(1)
            assert np.array_equal(a.positions(), b.positions()), t
            assert np.array_equal(a.field(), b.field()), t
