"""GPU tests of the paper's own field path (sf_set_field_sect): the 8-sect
store with strength fan-out and Algorithm 3's K-slot FP32 sums, full and
incremental.

The kernel adds the fan-out terms in the oracle's order, so the bar is bit
for bit: P = fl32(S + Phi32) with Phi32 the oracle's Algorithm 3 sums, the 8
sect planes equal to the oracle's, and every decision, election and move
equal to the oracle's taken on that same FP32 field (tied or not).  Under the
incremental update the oracle carries its own FP32 field through the same
updates, so the FP32 drift is reproduced exactly too.
"""
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


def _say(*a):
    print(*a, flush=True)


def _occ(W, H, pos):
    m = np.zeros(W * H, np.uint8)
    m[pos[pos >= 0]] = 1
    return m


def _bits_equal(a, b):
    return np.array_equal(np.asarray(a, np.float32).view(np.uint32),
                          np.asarray(b, np.float32).view(np.uint32))


# (name, scene, K values, ticks)
CASES = [
    ("room-R0", lambda: scenes.random_scene(70, 45, n_peds=300, radius=0, seed=2,
                                            exits=("E",), exit_width=4), (8,), 4),
    ("room-R3", lambda: scenes.random_scene(150, 97, n_peds=1800, radius=3, seed=4,
                                            bernoulli=0.04, exits=("E", "W"), exit_width=6),
     (2, 4, 8, 16), 6),
    ("attractive-R7", lambda: scenes.random_scene(131, 77, n_peds=900, radius=7, seed=6,
                                                  exits=("N",), exit_width=8, k=-0.6),
     (4, 16), 6),
    ("torus-R3", lambda: scenes.flow_scene(128, 96, 0.5, 8, radius=3, seed=8), (8, 16), 6),
    ("torus-R16", lambda: scenes.flow_scene(100, 70, 0.2, 4, radius=16, seed=9), (2, 8), 3),
    ("room-R48", lambda: scenes.random_scene(140, 120, n_peds=700, radius=48, seed=12,
                                             exits=("S",), exit_width=8), (16,), 2),
]


@pytest.mark.parametrize("name,make,Ks,ticks", CASES, ids=[c[0] for c in CASES])
def test_sect_path_lockstep(sf, name, make, Ks, ticks):
    sc = make()
    st = oracle.statics(sc)
    S = st.S
    W, H = sc.width, sc.height
    for K in Ks:
        with sf.GpuScene(sc) as g:
            g.set_field_sect(K, image=True)
            pos = g.positions()
            for t in range(sc.start_step, sc.start_step + ticks):
                P = g.field()
                img = g.sect_image()
                phi32, want_img = oracle.sect_field(W, H, _occ(W, H, pos), sc.radius, sc.k,
                                                    sc.alpha, K, sc.periodic, image=True)
                want = (S + phi32.astype(np.float64)).astype(np.float32)
                assert _bits_equal(P, want), (name, K, t, "field")
                assert _bits_equal(img, want_img), (name, K, t, "sect image")
                r = oracle.step(st, pos, t, P=P.astype(np.float64))
                g.step(1)
                tgt, flags = g.last_moves()
                newpos = g.positions()
                live = pos >= 0
                won = (flags & sf.SF_FLAG_WON) != 0
                bad = live & ((tgt != r.target) | (won != (r.moved == 1)) | (newpos != r.pos))
                assert not bad.any(), (name, K, t, np.flatnonzero(bad)[:5])
                pos = newpos
        _say(f"[sect] {name} K={K}: {ticks} ticks identical to the oracle")


@pytest.mark.parametrize("K,refresh", [(8, 6), (2, 4), (16, 5)])
def test_sect_incremental_drift_matches_oracle(sf, K, refresh):
    """The incremental k-4/k-5 on the FP32 sect field: between full fields the
    oracle adds its own Algorithm 3 sums of the su entered and left, and the
    GPU's field, image and decisions follow it bit for bit."""
    sc = scenes.random_scene(160, 120, n_peds=3000, radius=5, seed=21, bernoulli=0.03,
                             exits=("E", "W", "N"), exit_width=10)
    st = oracle.statics(sc)
    W, H, R = sc.width, sc.height, sc.radius
    with sf.GpuScene(sc) as g:
        g.set_field_update(refresh)
        g.set_field_sect(K, image=True)
        pos = g.positions()
        phi32, img = oracle.sect_field(W, H, _occ(W, H, pos), R, sc.k, sc.alpha, K, image=True)
        drift = 0.0
        for i in range(3 * refresh + 2):
            t = sc.start_step + i
            P = g.field()
            want = (st.S + phi32.astype(np.float64)).astype(np.float32)
            assert _bits_equal(P, want), (K, t)
            assert _bits_equal(g.sect_image(), img), (K, t)
            r = oracle.step(st, pos, t, P=P.astype(np.float64))
            g.step(1)
            newpos = g.positions()
            assert np.array_equal(newpos, r.pos), (K, t)
            # the field after tick i is a full one every `refresh` ticks,
            # starting with the first tick
            if i % refresh == 0:
                phi32, img = oracle.sect_field(W, H, _occ(W, H, newpos), R, sc.k, sc.alpha, K,
                                               image=True)
            else:
                a, b = _occ(W, H, pos), _occ(W, H, newpos)
                phi32, img = oracle.sect_update(W, H, b & (1 - a), a & (1 - b), R, sc.k,
                                                sc.alpha, K, phi32, img)
                exact = oracle.source_field(W, H, b, R, sc.k, sc.alpha)
                drift = max(drift, float(np.max(np.abs(phi32 - exact))))
            pos = newpos
    _say(f"[sect update] K={K} refresh={refresh}: largest FP32 drift {drift:.3g}")


def test_sect_off_returns_to_the_exact_field(sf):
    sc = scenes.random_scene(120, 80, n_peds=1200, radius=6, seed=31, exits=("E",),
                             exit_width=6)
    st = oracle.statics(sc)
    with sf.GpuScene(sc) as g:
        g.step(3)
        exact = g.field()
        g.set_field_sect(4)
        g.set_field_sect(0)
        assert _bits_equal(g.field(), exact)
        assert _bits_equal(exact, oracle.total_field(st, g.positions()).astype(np.float32))
        with pytest.raises(sf.SfError):
            g.sect_image()  # no image kept
        with pytest.raises(sf.SfError):
            g.set_field_sect(3)


def test_sect_scene_cannot_join_a_batch(sf):
    sc = scenes.random_scene(64, 64, n_peds=100, radius=2, seed=1)
    with sf.GpuScene(sc) as g:
        g.set_field_sect(8)
        with pytest.raises(sf.SfError):
            sf.Batch([g])
