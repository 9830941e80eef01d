"""GPU tests of the destination field D (multi-source 8-neighbour BFS from the
exit su, computed at scene creation): bit-for-bit equal to the oracle's BFS
on grids built to stress the tiled search: serpentine walls whose shortest
paths cross tile borders hundreds of times, widths and heights off the
64-su word and the tile size, a grid narrower than one word, a grid of more
tiles than the device runs at once (later workgroups of a launch must still
see the launch's starting state), an unreachable pocket far from the
exit, and a room of more than 2^28 su checked against closed forms."""
import numpy as np
import pytest

import oracle
from paper_1803_04782_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sf():
    from paper_1803_04782_amd import sf as _sf

    _sf.load()
    return _sf


def _serpentine(W, H, gap_every=4, seed=0):
    """Walls on the border and on every gap_every-th row, each with one gap
    at alternating ends; the exit is on the west wall near the top."""
    ob = np.zeros((H, W), np.uint8)
    ob[0, :] = ob[-1, :] = 1
    ob[:, 0] = ob[:, -1] = 1
    for k, y in enumerate(range(gap_every, H - 1, gap_every)):
        ob[y, :] = 1
        ob[y, (W - 2) if k % 2 == 0 else 1] = 0
    ex = np.zeros((H, W), np.uint8)
    ex[1, 0] = 1
    ob[1, 0] = 0
    rng = np.random.default_rng(seed)
    free = np.flatnonzero((ob.ravel() == 0) & (ex.ravel() == 0))
    pos = np.sort(rng.choice(free, size=min(50, free.size), replace=False)).astype(np.int32)
    return scenes.Scene(width=W, height=H, obstacle=ob.ravel(), exit=ex.ravel(), pos=pos,
                        radius=1, name=f"serpentine{W}x{H}")


CASES = [
    ("serpentine-70x301", lambda: _serpentine(70, 301)),
    ("serpentine-517x600", lambda: _serpentine(517, 600, gap_every=3)),
    ("serpentine-1030x258", lambda: _serpentine(1030, 258, gap_every=5)),
    ("serpentine-5x40", lambda: _serpentine(5, 40)),
    ("random-700x300", lambda: scenes.random_scene(700, 300, n_peds=500, radius=3, seed=8,
                                                   bernoulli=0.3, exits=("S",), exit_width=4)),
    ("random-257x1100", lambda: scenes.random_scene(257, 1100, n_peds=500, radius=2, seed=9,
                                                    bernoulli=0.2, exits=("N", "E"),
                                                    exit_width=3)),
    # 17 x 17 tiles of 256 x 256 su
    ("random-4352x4200", lambda: scenes.random_scene(4352, 4200, n_peds=1000, radius=2,
                                                     seed=10, bernoulli=0.1, exits=("N",),
                                                     exit_width=16)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_destination_field_matches_oracle(sf, name, make):
    sc = make()
    st = oracle.statics(sc, with_obstacle_field=False)
    print(f"[statics] {name}: Dmax {int(st.D.max())}", flush=True)
    with sf.GpuScene(sc) as g:
        _, D = g.static_field()
    assert np.array_equal(D, st.D)


def test_unreachable_pocket_across_tiles(sf):
    W, H = 600, 400
    ob = np.zeros((H, W), np.uint8)
    ob[0, :] = ob[-1, :] = 1
    ob[:, 0] = ob[:, -1] = 1
    ob[300:340, 500] = ob[300:340, 540] = 1  # a closed box far from the exit
    ob[300, 500:541] = ob[340, 500:541] = 1
    ex = np.zeros((H, W), np.uint8)
    ex[5:9, 0] = 1
    ob[5:9, 0] = 0
    sc = scenes.Scene(width=W, height=H, obstacle=ob.ravel(), exit=ex.ravel(),
                      pos=np.array([10 * W + 10], np.int32), radius=2)
    rc, msg = sf.create_error(sc)
    assert rc == sf.SF_EUNREACHABLE, msg
    assert "1521 free su" in msg  # the 39 x 39 su inside the box


def test_room_beyond_2_28_su(sf):
    """A walled room of 16448 x 16448 su (2^28 + 2.1 M su) with one 16-su exit
    on the east wall: the set-up kernels that take one thread per su (exit
    seeds, reachability count, S) must reach the su beyond index 2^28.  In an
    empty room D is the Chebyshev distance to the exit segment (closed form);
    beyond the walls' obstacle window S = D exactly; and wherever no
    pedestrian is within R the field is S."""
    W = H = 16448
    R = 2
    y0 = H // 2 - 8
    ob = np.zeros((H, W), np.uint8)
    ob[0, :] = ob[-1, :] = 1
    ob[:, 0] = ob[:, -1] = 1
    ex = np.zeros((H, W), np.uint8)
    ex[y0:y0 + 16, W - 1] = 1
    ob[y0:y0 + 16, W - 1] = 0
    rng = np.random.default_rng(17)
    px = rng.integers(1, W - 1, 3000)
    py = np.concatenate([rng.integers(H - 400, H - 1, 2000), rng.integers(1, H - 1, 1000)])
    pos = np.unique(py * W + px).astype(np.int32)
    sc = scenes.Scene(width=W, height=H, obstacle=ob.ravel(), exit=ex.ravel(), pos=pos,
                      radius=R, name="room16448")
    del ob, ex
    print(f"[room16448] {W * H} su, {pos.size} pedestrians", flush=True)
    with sf.GpuScene(sc) as g:
        S, D = g.static_field()
        P = g.field()
        g.step(3)
        after = g.positions()
    xs = np.concatenate([rng.integers(1, W - 1, 6000), rng.integers(W - 40, W - 1, 500)])
    # rows from 16321 on hold only su beyond index 2^28
    ys = np.concatenate([rng.integers(1, H - 1, 3000), rng.integers(H - 120, H - 1, 3500)])
    idx = ys.astype(np.int64) * W + xs
    assert np.count_nonzero(idx >= (1 << 28)) >= 3500
    dy = np.where(ys < y0, y0 - ys, np.where(ys > y0 + 15, ys - (y0 + 15), 0))
    want = np.maximum(W - 1 - xs, dy)
    assert np.array_equal(D[idx], want)
    far = (xs > R) & (xs < W - 1 - R) & (ys > R) & (ys < H - 1 - R)
    assert np.array_equal(S[idx[far]], want[far].astype(np.float32))
    qx, qy = pos % W, pos // W
    alone = np.array([not np.any((np.abs(qx - x) <= R) & (np.abs(qy - y) <= R))
                      for x, y in zip(xs, ys)])
    assert alone.sum() > 5000
    # no pedestrian within R: Phi = 0 and P is S (FP64) rounded once
    assert np.array_equal(P[idx[alone]], S[idx[alone]].astype(np.float32))
    assert D[W - 1 + (y0 + 3) * W] == 0 and D[(H - 1) * W + W // 2] == -1
    live = after[after >= 0]
    assert np.all(after >= -1) and np.all(live < W * H) and np.unique(live).size == live.size
