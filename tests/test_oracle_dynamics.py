"""Pins of the oracle's tick (Algorithm 1: decide, register-and-elect, move).

* Closed forms: a lone pedestrian with no obstacle field walks the BFS
  gradient and leaves after exactly D(x0) ticks; a single-file queue in a
  one-su corridor with R = 0 drains at one pedestrian per two ticks
  (pedestrian k leaves at tick d0 + 2k - 1), which follows from targets
  having to be free at the start of the tick.
* Invariants of the discrete model: v_max = 1, one pedestrian per su, no
  pedestrian on an obstacle, at most 8 registrants per su and exactly one
  winner per claimed su, losers stay, the head-count is conserved.
* Hand-worked scenes under tests/golden (expected moves derived by hand).
* The point-evaluation route (used at full scale) agrees with the full grid.
"""
import os

import numpy as np
import pytest

from paper_1803_04782_amd import scenes

HERE = os.path.dirname(os.path.abspath(__file__))


def _room(W, H, exits, peds, obst_cells=(), **params):
    ob = np.zeros((H, W), np.uint8)
    ob[0, :] = ob[-1, :] = 1
    ob[:, 0] = ob[:, -1] = 1
    for (x, y) in obst_cells:
        ob[y, x] = 1
    ex = np.zeros((H, W), np.uint8)
    for (x, y) in exits:
        ob[y, x] = 0
        ex[y, x] = 1
    pos = np.array([y * W + x for (x, y) in peds], np.int32)
    return scenes.Scene(width=W, height=H, obstacle=ob.ravel(), exit=ex.ravel(), pos=pos,
                        **params)


@pytest.mark.parametrize("start", [(1, 1), (5, 9), (12, 3), (2, 10), (13, 10)])
def test_lone_pedestrian_leaves_after_bfs_distance(orc, start):
    W, H = 15, 12
    obst = [(6, y) for y in range(2, 10)] + [(9, y) for y in range(3, 11)]
    sc = _room(W, H, exits=[(14, 6)], peds=[start], obst_cells=obst, radius=3, k_obs=0.0)
    st = orc.statics(sc)
    d0 = int(st.D[sc.pos[0]])
    assert d0 > 0
    res = orc.run(st, sc.pos, 0, d0 + 2)
    left_at = [t for t, r in enumerate(res) if r.left]
    assert left_at == [d0 - 1]
    # every tick moves one su down the gradient
    pos = sc.pos[0]
    for t in range(d0 - 1):
        nxt = res[t].pos[0]
        assert st.D[nxt] == st.D[pos] - 1
        pos = nxt


@pytest.mark.parametrize("d0,n", [(5, 10), (1, 4), (3, 1)])
def test_corridor_queue_outflow(orc, d0, n):
    # one-su corridor: rows 0 and 2 are wall, exit at the east end of row 1
    W = d0 + n + 3
    H = 3
    ex = (W - 1, 1)
    peds = [(W - 1 - d0 - k, 1) for k in range(n)]
    sc = _room(W, H, exits=[ex], peds=peds, radius=0)
    st = orc.statics(sc)
    assert [int(st.D[p]) for p in sc.pos] == [d0 + k for k in range(n)]
    res = orc.run(st, sc.pos, 0, d0 + 2 * n + 2)
    for k in range(n):
        left = [t for t, r in enumerate(res) if r.pos[k] < 0 and (t == 0 or res[t - 1].pos[k] >= 0)]
        assert left == [d0 + 2 * k - 1], (k, left)


def _check_invariants(st, before, r, t, seed):
    W, H = st.W, st.H
    live_b = before >= 0
    # head-count conserved
    assert (r.pos >= 0).sum() + r.left == live_b.sum()
    live_a = r.pos[r.pos >= 0]
    # one pedestrian per su, never on an obstacle, never on an exit
    assert len(np.unique(live_a)) == len(live_a)
    assert not st.obstacle[live_a].any()
    assert not st.exit[live_a].any()
    occ = np.zeros(W * H, bool)
    occ[before[live_b]] = True
    claims = {}
    for i in np.flatnonzero(live_b):
        p, q = int(before[i]), int(r.target[i])
        dx = abs(q % W - p % W)
        dy = abs(q // W - p // W)
        assert max(dx, dy) <= 1  # v_max = 1
        if q != p:
            assert not occ[q] and not st.obstacle[q]  # only free su are voted on
            claims.setdefault(q, []).append(i)
        if r.moved[i]:
            assert q != p
            assert r.pos[i] == (-1 if st.exit[q] else q)
        else:
            assert r.pos[i] == p  # losers and stayers keep their su
    import oracle as _o
    for q, who in claims.items():
        assert len(who) <= 8
        winners = [i for i in who if r.moved[i]]
        assert len(winners) == 1
        keys = {i: _o.claim_key(int(i), t, seed) for i in who}
        assert winners[0] == min(keys, key=keys.get)


@pytest.mark.parametrize("W,H,n,R,seed", [(24, 18, 120, 2, 0), (31, 9, 60, 3, 1), (40, 40, 500, 4, 2)])
def test_invariants_on_random_runs(orc, W, H, n, R, seed):
    sc = scenes.random_scene(W, H, n_peds=n, radius=R, seed=seed, bernoulli=0.08,
                             exits=("E", "N"), exit_width=3)
    st = orc.statics(sc)
    pos = sc.pos.copy()
    for t in range(40):
        r = orc.step(st, pos, t)
        _check_invariants(st, pos, r, t, sc.seed)
        pos = r.pos


def test_processing_order_does_not_matter(orc):
    # relabelling pedestrians permutes ids, so use the same ids in another
    # array order: results must be the same per id
    sc = scenes.random_scene(30, 22, n_peds=150, radius=3, seed=9, bernoulli=0.05)
    st = orc.statics(sc)
    r1 = orc.step(st, sc.pos, 4)
    # the oracle processes ids in index order; reversing the whole pipeline's
    # order is equivalent to relabelling, so compare against the per-id
    # point-evaluation route instead (independent of any processing order)
    occ = orc.occupancy(st.W, st.H, sc.pos)
    owner = np.full(st.W * st.H, -1, np.int64)
    owner[sc.pos] = np.arange(len(sc.pos))
    for i in range(len(sc.pos))[::-1]:
        tgt, mv, tied = orc.outcome_at(st, occ, owner, sc.pos, i, 4)
        assert tgt == r1.target[i] and mv == bool(r1.moved[i]) and tied == bool(r1.tied[i])


def test_point_route_matches_full_grid(orc):
    sc = scenes.random_scene(27, 19, n_peds=90, radius=4, seed=11, bernoulli=0.1,
                             k_obs=0.6, radius_obs=2)
    st = orc.statics(sc)
    occ = orc.occupancy(st.W, st.H, sc.pos)
    P = orc.total_field(st, sc.pos)
    cells = np.arange(st.W * st.H)
    Pp = orc.field_at(st, occ, cells)
    np.testing.assert_allclose(Pp, P, rtol=1e-13, atol=1e-12)
    r = orc.step(st, sc.pos, 0, P=P)
    for i, p in enumerate(sc.pos):
        tgt, tied, _ = orc.decide_at(st, occ, int(p))
        assert tgt == r.target[i] and tied == bool(r.tied[i])


# ---- hand-worked scenes -------------------------------------------------------

def _load_golden(name):
    """Parse a golden scene: a character map ('#' obstacle, 'E' exit, '.' free,
    a letter a-z = pedestrian with id = letter index), parameter lines and
    expected outcomes 'id -> x,y' (or 'id -> out')."""
    path = os.path.join(HERE, "golden", name)
    grid, params, expect = [], {}, {}
    section = None
    for line in open(path):
        line = line.rstrip("\n")
        if not line or line.startswith(";"):
            continue
        if line in ("[map]", "[params]", "[expect]"):
            section = line
            continue
        if section == "[map]":
            grid.append(line)
        elif section == "[params]":
            key, val = line.split("=")
            params[key.strip()] = float(val) if "." in val or "e" in val else int(val)
        elif section == "[expect]":
            lhs, rhs = line.split("->")
            expect[lhs.strip()] = rhs.strip()
    H, W = len(grid), len(grid[0])
    ob = np.zeros(W * H, np.uint8)
    ex = np.zeros(W * H, np.uint8)
    peds = {}
    for y, row in enumerate(grid):
        for x, ch in enumerate(row):
            if ch == "#":
                ob[y * W + x] = 1
            elif ch == "E":
                ex[y * W + x] = 1
            elif ch.isalpha():
                peds[ord(ch) - ord("a")] = y * W + x
    pos = np.array([peds[i] for i in range(len(peds))], np.int32)
    t = int(params.pop("t", 0))
    sc = scenes.Scene(width=W, height=H, obstacle=ob, exit=ex, pos=pos,
                      radius=int(params.pop("R")), **params)
    return sc, t, expect


GOLDEN = sorted(f for f in os.listdir(os.path.join(HERE, "golden")) if f.endswith(".scene"))


@pytest.mark.parametrize("name", GOLDEN)
def test_golden_scene(orc, name):
    sc, t, expect = _load_golden(name)
    st = orc.statics(sc)
    r = orc.step(st, sc.pos, t)
    W = sc.width
    for key, want in expect.items():
        if key.startswith("tied "):
            i = ord(key.split()[1]) - ord("a")
            assert bool(r.tied[i]) == (want == "yes"), (name, key)
            continue
        i = ord(key) - ord("a")
        if want == "out":
            assert r.pos[i] == -1, (name, key)
        else:
            x, y = (int(v) for v in want.split(","))
            assert r.pos[i] == y * W + x, (name, key, r.pos[i] % W, r.pos[i] // W)


# ---- edges of the near-tie band ------------------------------------------------

BAND_SCENES = [("near_tie_d200_in.scene", 0.9e-5), ("near_tie_d200_out.scene", 1.1e-5),
               ("near_tie_floor_in.scene", 0.9e-5), ("near_tie_floor_out.scene", 1.1e-5)]


@pytest.mark.parametrize("name,ratio", BAND_SCENES)
def test_near_tie_band_edges(orc, name, ratio):
    """The golden scenes sit just inside (0.9e-5) and just outside (1.1e-5) the
    band, once with |u| near 200 (the scale is max(|u1|, |u2|)) and once with
    |u| below 1 (the floor of 1 applies).  Their candidate values are written
    out here independently of the oracle (Chebyshev distance to the exit in an
    empty room, obstacle strengths as FP32 numbers summed by brute force; the
    pedestrian's own field cancels), the gap ratio is checked, and the oracle's
    flag must be the band's verdict.  An absolute band, a ten times wider band
    or a band without the floor of 1 each flips one of the four verdicts."""
    sc, t, expect = _load_golden(name)
    W, H = sc.width, sc.height
    x0, y0 = int(sc.pos[0] % W), int(sc.pos[0] // W)
    exits = [(c % W, c // W) for c in np.flatnonzero(sc.exit)]
    obst = [(c % W, c // W) for c in np.flatnonzero(sc.obstacle)]
    Ro = sc.r_obs

    def dist(x, y):
        return min(max(abs(x - ex), abs(y - ey)) for ex, ey in exits)

    def obstacle_field(x, y):
        v = 0.0
        for ox, oy in obst:
            dx, dy = x - ox, y - oy
            if max(abs(dx), abs(dy)) <= Ro and (dx or dy):
                v += float(np.float32(sc.k_obs * np.hypot(dx, dy) ** sc.alpha_obs))
        return v

    vals = []
    for dx, dy in oracle_dirs():
        x, y = x0 + dx, y0 + dy
        if sc.obstacle[y * W + x]:
            continue
        vals.append(sc.w_dest * dist(x, y) + obstacle_field(x, y))
    u1, u2 = sorted(vals)[:2]
    scale = max(abs(u1), abs(u2), 1.0)
    assert abs((u2 - u1) / scale - ratio) < 0.02 * ratio
    band_says = (u2 - u1) <= 1e-5 * scale
    assert band_says == (expect["tied a"] == "yes")
    st = orc.statics(sc)
    r = orc.step(st, sc.pos, t)
    assert bool(r.tied[0]) == band_says


def oracle_dirs():
    return ((0, 0), (1, 0), (1, 1), (0, 1), (-1, 1), (-1, 0), (-1, -1), (0, -1), (1, -1))
