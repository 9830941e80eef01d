"""Pins of the oracle's multi-su pedestrians (section 2: odd width and height,
one centre su; the footprints of Table VI).

Reading (oracle header): a body is a bw x bh block centred on the pedestrian's
su; a move needs the whole shifted body inside the grid, off obstacles and off
other bodies; a mover registers for the su its body enters and wins if its key
is the smallest at all of them; a winner whose body reaches an exit leaves;
the field radiates from the centre.

* Closed form: a lone bw x bh walker with no obstacle field in a room whose
  east wall is all exit (between the corners) leaves on tick D(x0) - a - 1
  (a = (bw - 1) / 2), every tick one su closer.
* Invariants of random runs, checked by code written here (not the oracle's):
  bodies stay disjoint, inside the grid and off obstacles; centres move at most
  one su; the su a winner enters were free at the tick start and no two winners
  enter the same su; each winner holds the smallest key at every su it
  enters; losers and stayers keep their su; the head-count is conserved.
* A hand-worked collision of two 3x3 bodies whose entered columns coincide.
* One-su bodies reduce to the one-su model (the rest of the oracle's pins).
"""
import numpy as np
import pytest

from paper_1803_04782_amd import scenes


def _room(W, H, body, peds, **params):
    ob = np.zeros((H, W), np.uint8)
    ob[0, :] = ob[-1, :] = 1
    ob[:, 0] = ob[:, -1] = 1
    ex = np.zeros((H, W), np.uint8)
    ex[1:H - 1, W - 1] = 1  # the east wall between the corners is exit
    ob[1:H - 1, W - 1] = 0
    pos = np.array([y * W + x for (x, y) in peds], np.int32)
    return scenes.Scene(width=W, height=H, obstacle=ob.ravel(), exit=ex.ravel(), pos=pos,
                        body_w=body[0], body_h=body[1], **params)


@pytest.mark.parametrize("body,start", [((3, 3), (4, 5)), ((5, 3), (5, 4)), ((3, 5), (3, 6)),
                                        ((1, 1), (2, 5)), ((7, 7), (5, 5))])
def test_lone_body_walker_closed_form(orc, body, start):
    W, H = 24, 12
    sc = _room(W, H, body, [start], radius=3, k_obs=0.0)
    st = orc.statics(sc)
    a = (body[0] - 1) // 2
    d0 = int(st.D[sc.pos[0]])
    assert d0 == W - 1 - start[0]
    res = orc.run(st, sc.pos, 0, d0 + 2)
    left_at = [t for t, r in enumerate(res) if r.left]
    assert left_at == [d0 - a - 1]
    pos = int(sc.pos[0])
    for t in range(d0 - a - 1):
        nxt = int(res[t].pos[0])
        assert st.D[nxt] == st.D[pos] - 1
        pos = nxt


def _bodies_ok(W, H, obst, pos, bw, bh, periodic):
    a, b = (bw - 1) // 2, (bh - 1) // 2
    cover = np.zeros(W * H, np.int64)
    for p in pos[pos >= 0]:
        x, y = int(p % W), int(p // W)
        for j in range(-b, b + 1):
            for i in range(-a, a + 1):
                sx, sy = x + i, y + j
                if periodic:
                    sx, sy = sx % W, sy % H
                elif not (0 <= sx < W and 0 <= sy < H):
                    return False
                cover[sy * W + sx] += 1
    return cover.max(initial=0) <= 1 and not (cover[obst == 1] > 0).any()


def _entered(W, H, bw, bh, periodic, p, q):
    a, b = (bw - 1) // 2, (bh - 1) // 2
    ox, oy, tx, ty = p % W, p // W, q % W, q // W
    dx, dy = tx - ox, ty - oy
    if periodic:
        dx = (dx + 1) % W - 1
        dy = (dy + 1) % H - 1
    cx, cy = ox + dx, oy + dy
    out = []
    for j in range(-b, b + 1):
        for i in range(-a, a + 1):
            x, y = cx + i, cy + j
            if ox - a <= x <= ox + a and oy - b <= y <= oy + b:
                continue
            if periodic:
                x, y = x % W, y % H
            out.append(y * W + x)
    return out


def _check_tick(orc, st, before, r, t):
    W, H, bw, bh, per = st.W, st.H, st.body_w, st.body_h, st.periodic
    live = before >= 0
    assert (r.pos >= 0).sum() + r.left == live.sum()
    assert _bodies_ok(W, H, st.obstacle, r.pos, bw, bh, per)
    a, b = (bw - 1) // 2, (bh - 1) // 2
    covered = np.zeros(W * H, bool)
    # step-start cover
    for p in before[live]:
        x, y = int(p % W), int(p // W)
        for j in range(-b, b + 1):
            for i in range(-a, a + 1):
                sx, sy = (x + i) % W if per else x + i, (y + j) % H if per else y + j
                covered[sy * W + sx] = True
    regs = {}
    for i in np.flatnonzero(live):
        p, q = int(before[i]), int(r.target[i])
        dx = abs(q % W - p % W)
        dy = abs(q // W - p // W)
        if per:
            dx, dy = min(dx, W - dx), min(dy, H - dy)
        assert max(dx, dy) <= 1
        if q != p:
            ent = _entered(W, H, bw, bh, per, p, q)
            assert not covered[ent].any()  # entered su were free at the tick start
            for c in ent:
                regs.setdefault(c, []).append(i)
        if not r.moved[i]:
            assert r.pos[i] == p
    winners = np.flatnonzero(r.moved == 1)
    seen = set()
    for i in winners:
        ent = _entered(W, H, bw, bh, per, int(before[i]), int(r.target[i]))
        k = orc.claim_key(int(i), t, st.seed)
        for c in ent:
            assert c not in seen  # no two winners enter the same su
            seen.add(c)
            assert k == min(orc.claim_key(int(j), t, st.seed) for j in regs[c])
        left = any(st.exit[c] for c in ent)
        assert r.pos[i] == (-1 if left else r.target[i])
    # a mover holding the smallest key at every su it enters wins
    for i in np.flatnonzero(live & (r.target != before) & (r.moved == 0)):
        ent = _entered(W, H, bw, bh, per, int(before[i]), int(r.target[i]))
        k = orc.claim_key(int(i), t, st.seed)
        assert any(k != min(orc.claim_key(int(j), t, st.seed) for j in regs[c]) for c in ent)


@pytest.mark.parametrize("bw,bh,n,R,seed", [(3, 3, 40, 3, 0), (5, 3, 25, 4, 1), (3, 5, 30, 2, 2),
                                            (1, 1, 120, 3, 3)])
def test_body_invariants_bounded(orc, bw, bh, n, R, seed):
    sc = scenes.body_room(48, 36, bw, bh, n, R, seed=seed, exits=("E", "W"), exit_width=11,
                          bernoulli=0.02)
    st = orc.statics(sc)
    assert _bodies_ok(st.W, st.H, st.obstacle, sc.pos, bw, bh, False)
    pos = sc.pos.copy()
    moved = 0
    for t in range(30):
        r = orc.step(st, pos, t)
        _check_tick(orc, st, pos, r, t)
        moved += int(r.moved.sum())
        pos = r.pos
    assert moved > n  # the crowd does move


@pytest.mark.parametrize("body,seed", [(3, 4), (5, 5)])
def test_body_invariants_torus(orc, body, seed):
    sc = scenes.body_flow_scene(64, 45, 0.4, 8, body, radius=3, seed=seed)
    st = orc.statics(sc)
    assert st.periodic and _bodies_ok(st.W, st.H, st.obstacle, sc.pos, body, body, True)
    pos = sc.pos.copy()
    for t in range(20):
        r = orc.step(st, pos, t)
        _check_tick(orc, st, pos, r, t)
        pos = r.pos
    assert (pos >= 0).all()


def test_body_collision_hand_worked(orc):
    """Two 3x3 bodies face each other across one free column: A (centre
    (4,5)) heads east, B (centre (8,5)) heads west, no fields (k = k_obs =
    w_dest = 0), heading weight 1, so each one's best move is straight ahead
    (value -1).  Both register for column 6, rows 4..6; the one with the
    smaller election key at tick 0 moves, the other stays."""
    W, H = 14, 11
    ob = np.zeros((H, W), np.uint8)
    ob[0, :] = ob[-1, :] = 1
    ob[:, 0] = ob[:, -1] = 1
    ex = np.zeros((H, W), np.uint8)
    ex[5, 0] = 1
    ob[5, 0] = 0
    pos = np.array([5 * W + 4, 5 * W + 8], np.int32)
    sc = scenes.Scene(width=W, height=H, obstacle=ob.ravel(), exit=ex.ravel(), pos=pos,
                      radius=2, k=0.0, k_obs=0.0, w_dest=0.0, seed=12345,
                      heading=np.array([1, 5], np.uint8), w_heading=1.0, body_w=3, body_h=3)
    st = orc.statics(sc)
    r = orc.step(st, sc.pos, 0)
    assert r.target[0] == 5 * W + 5 and r.target[1] == 5 * W + 7
    ka, kb = orc.claim_key(0, 0, 12345), orc.claim_key(1, 0, 12345)
    win = 0 if ka < kb else 1
    assert r.moved[win] == 1 and r.moved[1 - win] == 0
    assert r.pos[win] == r.target[win] and r.pos[1 - win] == sc.pos[1 - win]
