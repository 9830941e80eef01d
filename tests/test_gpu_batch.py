"""GPU tests of batches (sf_batch_*): many scenes advanced by one decide,
commit and field launch per tick, replayed from captured HIP graphs.

Bar: every member scene evolves bit for bit as the same scene stepped alone
with sf_step (same kernels per scene, field summation order independent of
the launch), across graph replays with eager work between them, for every
tiling and after the autotuner; and a batch passes the lockstep comparison
with the FP64 oracle (parity.py: the field bit for bit, no mismatched
decision).
"""
import os

import numpy as np
import pytest

import oracle
from paper_1803_04782_amd import scenes

pytestmark = pytest.mark.gpu

from parity import (THREADS, Report, assert_parity, classify, field_bits_differ,  # noqa: E402
                    field_rel_err)


@pytest.fixture(scope="module")
def sf():
    from paper_1803_04782_amd import sf as _sf

    _sf.load()
    return _sf


def _say(*a):
    print(*a, flush=True)


def _mixed_scenes():
    """Uneven sizes, crowds and radii, including an empty scene and R = 0."""
    out = [
        scenes.random_scene(64, 64, n_peds=300, radius=4, seed=1, exits=("E",), exit_width=4),
        scenes.random_scene(203, 117, n_peds=2500, radius=16, seed=2, bernoulli=0.03,
                            exits=("W", "E"), exit_width=8),
        scenes.random_scene(90, 250, n_peds=1800, radius=32, seed=3, bernoulli=0.02,
                            exits=("N", "S"), exit_width=6),
        scenes.random_scene(33, 29, n_peds=0, radius=8, seed=4, exits=("E",)),
        scenes.random_scene(150, 140, n_peds=8000, radius=8, seed=5, bernoulli=0.04,
                            exits=("E", "N"), exit_width=10),
        scenes.random_scene(47, 301, n_peds=900, radius=0, seed=6, exits=("S",), exit_width=5),
        scenes.random_scene(129, 65, n_peds=1200, radius=12, seed=7, exits=("W",), exit_width=4),
        scenes.random_scene(257, 190, n_peds=3000, radius=4, seed=8, bernoulli=0.06,
                            exits=("W", "E", "N", "S"), exit_width=12),
    ]
    return out


def _state(g):
    t, f = g.last_moves()
    return g.positions(), g.field(), t, f, g.stats()


def _assert_same(a, b, what):
    for x, y, name in zip(a, b, ("positions", "field", "targets", "flags", "stats")):
        if isinstance(x, dict):
            assert x == y, (what, name, x, y)
        else:
            assert np.array_equal(x, y), (what, name)


def test_batch_members_match_scenes_alone(sf):
    scs = _mixed_scenes()
    alone = [sf.GpuScene(s) for s in scs]
    member = [sf.GpuScene(s) for s in scs]
    _say(f"[batch] {len(scs)} scenes, graph replays of 5, 8, 3 and 13 ticks")
    with sf.Batch(member) as b:
        _say("   tiling", b.tiling())
        for n in (5, 8, 3, 13):
            b.step(n)
            for g in alone:
                g.step(n)
            # eager reads between replays
            totals = b.stats()
            for j, (a, m) in enumerate(zip(alone, member)):
                _assert_same(_state(a), _state(m), (n, j))
                assert totals[j] == m.stats(), (n, j)
    for g in alone + member:
        g.close()


@pytest.mark.parametrize("tiling", [
    dict(tw=16, hl=2, vec=2, nw=4),
    dict(tw=32, hl=4, vec=2, nw=4, items_per_block=1),
    dict(tw=8, hl=2, vec=2, nw=4, list_cap=4096, items_per_block=64),
    dict(tw=16, hl=4, vec=2, nw=8, blocks_per_cu=1),
    dict(tw=16, hl=4, vec=4, nw=4),
    dict(tw=32, hl=4, vec=4, nw=4, items_per_block=1),
    dict(tw=8, hl=4, vec=4, nw=4, list_cap=1024, items_per_block=64),
    dict(tw=16, hl=4, vec=4, nw=16, blocks_per_cu=1),
    dict(groups=2, split_radius=8,
         group=[dict(tw=32, hl=8, vec=4, nw=4), dict(tw=16, hl=8, vec=4, nw=4, list_cap=1024)]),
    dict(groups=1),
    dict(groups=2, split_radius=16,
         group=[dict(tw=32, hl=4, vec=2, nw=4), dict(tw=16, hl=2, vec=2, nw=8)]),
    dict(groups=2, split_radius=8,
         group=[dict(tw=16, hl=4, vec=4, nw=8), dict(tw=16, hl=4, vec=4, nw=4)]),
    dict(groups=3),
    dict(groups=4, split_radius=[4, 8, 16],
         group=[dict(tw=32, hl=4, vec=4, nw=4), dict(tw=16, hl=4, vec=4, nw=4),
                dict(tw=16, hl=2, vec=2, nw=8), dict(tw=16, hl=4, vec=4, nw=16)]),
])
def test_batch_tilings_identical(sf, tiling):
    scs = _mixed_scenes()[:5]
    alone = [sf.GpuScene(s) for s in scs]
    member = [sf.GpuScene(s) for s in scs]
    _say(f"[batch tiling] {tiling}")
    with sf.Batch(member, tiling=tiling) as b:
        b.step(9)
        for g in alone:
            g.step(9)
        for j, (a, m) in enumerate(zip(alone, member)):
            _assert_same(_state(a), _state(m), j)
    for g in alone + member:
        g.close()


def test_batch_extreme_radii(sf):
    """Members at the largest radius (48, bounded and periodic) beside R = 1
    and R = 47, under the default tiling: every member evolves as alone."""
    scs = [scenes.random_scene(210, 160, n_peds=2000, radius=48, seed=51, bernoulli=0.02,
                               exits=("E", "W"), exit_width=8),
           scenes.random_scene(120, 90, n_peds=3000, radius=1, seed=52, exits=("N",),
                               exit_width=6),
           scenes.flow_scene(128, 100, 0.3, 8, radius=48, seed=53),
           scenes.random_scene(70, 50, n_peds=200, radius=47, seed=54, exits=("S",))]
    alone = [sf.GpuScene(s) for s in scs]
    member = [sf.GpuScene(s) for s in scs]
    with sf.Batch(member) as b:
        _say("[batch extreme radii] tiling", b.tiling())
        b.step(7)
        for g in alone:
            g.step(7)
        for j, (a, m) in enumerate(zip(alone, member)):
            _assert_same(_state(a), _state(m), j)
    for g in alone + member:
        g.close()


def test_batch_tune_keeps_state_and_results(sf):
    scs = _mixed_scenes()
    alone = [sf.GpuScene(s) for s in scs]
    member = [sf.GpuScene(s) for s in scs]
    with sf.Batch(member) as b:
        b.step(4)
        before = [m.field() for m in member]
        chosen = b.tune(reps=2)
        _say("   tuned", chosen)
        assert chosen == b.tiling()
        for f, m in zip(before, member):
            assert np.array_equal(f, m.field())
        b.step(6)
        for g in alone:
            g.step(10)
        for j, (a, m) in enumerate(zip(alone, member)):
            _assert_same(_state(a), _state(m), j)
    for g in alone + member:
        g.close()


def test_batch_lockstep_against_oracle(sf):
    scs = _mixed_scenes()
    sts = [oracle.statics(s) for s in scs]
    member = [sf.GpuScene(s) for s in scs]
    reps = [Report() for _ in scs]
    with sf.Batch(member) as b:
        for t in range(12):
            before = []
            for st, g, sc in zip(sts, member, scs):
                pos = g.positions()
                r = oracle.step(st, pos, sc.start_step + t, threads=THREADS)
                before.append((pos, g.field(), r))
            b.step(1)
            for (pos, P_gpu, r), st, g, rep in zip(before, sts, member, reps):
                tgt_g, flags_g = g.last_moves()
                pos_g = g.positions()
                untied, tied = classify(pos, r, tgt_g, flags_g, pos_g)
                rep.steps += 1
                rep.max_field_err = max(rep.max_field_err, field_rel_err(P_gpu, r.P, st.obstacle))
                rep.field_mismatch += field_bits_differ(P_gpu, r.P)
                rep.untied += len(untied)
                rep.tied_mismatch += len(tied)
                rep.decisions += int((pos >= 0).sum())
    for sc, rep in zip(scs, reps):
        _say("   ", sc.name, rep)
        assert_parity(rep)
    for g in member:
        g.close()


def test_ensemble_sample_matches_alone(sf):
    # a few scenes of the uneven ensemble distribution (smaller sides)
    scs = scenes.ensemble(n_scenes=12, seed=3, side=(128, 384))
    alone = [sf.GpuScene(s) for s in scs]
    member = [sf.GpuScene(s) for s in scs]
    with sf.Batch(member) as b:
        b.tune(reps=1)
        b.step(20)
        for g in alone:
            g.step(20)
        for j, (a, m) in enumerate(zip(alone, member)):
            _assert_same(_state(a), _state(m), j)
    for g in alone + member:
        g.close()


def test_batch_membership_rules(sf):
    scs = _mixed_scenes()[:3]
    gs = [sf.GpuScene(s) for s in scs]
    b = sf.Batch(gs[:2])
    with pytest.raises(sf.SfError) as e:
        gs[0].step(1)
    assert e.value.code == sf.SF_EINVAL
    with pytest.raises(sf.SfError):
        gs[1].set_state(gs[1].positions(), 0)
    with pytest.raises(sf.SfError):
        sf.Batch([gs[1], gs[2]])  # already a member
    with pytest.raises(sf.SfError):
        sf.Batch([gs[2], gs[2]])  # listed twice
    with pytest.raises(sf.SfError):
        sf.Batch([])
    with pytest.raises(sf.SfError):
        sf.Batch([gs[2]], tiling=dict(tw=12, hl=2, vec=2, nw=4))  # not a compiled shape
    with pytest.raises(sf.SfError):
        sf.Batch([gs[2]], tiling=dict(tw=16, hl=2, vec=4, nw=4))  # 16-byte loads need HL 4
    with pytest.raises(sf.SfError):
        sf.Batch([gs[2]], tiling=dict(groups=2))  # one radius: the second group is empty
    with pytest.raises(sf.SfError):
        sf.Batch([gs[2]], tiling=dict(groups=5))
    b.step(2)
    b.close()
    gs[0].step(1)  # back on its own
    # destroying a member first disables the batch
    b2 = sf.Batch([gs[1], gs[2]])
    gs[2].close()
    with pytest.raises(sf.SfError):
        b2.step(1)
    b2.close()
    gs[1].step(1)
    for g in gs:
        g.close()


@pytest.mark.skipif(os.environ.get("SF_SKIP_ENSEMBLE") == "1", reason="disabled by env")
def test_ensemble256_full_size(sf):
    """The 256-scene ensemble at full size in the benchmark's launch
    configuration (autotuned two-group tiling, graph replays): every scene
    matches itself stepped alone, and the three largest scenes match the
    oracle in full for one tick: every su of the field (bit for bit) and
    every pedestrian's target, election and position."""
    import time

    scs = scenes.ensemble(n_scenes=256, seed=3)
    _say(f"[ensemble256] {sum(s.width * s.height for s in scs):.3g} su, "
         f"{sum(s.n_peds for s in scs)} pedestrians")
    alone = [sf.GpuScene(s) for s in scs]
    member = [sf.GpuScene(s) for s in scs]
    largest = [int(j) for j in np.argsort([s.width * s.height for s in scs])[-3:]]
    t0 = time.time()
    sts = {j: oracle.statics(scs[j], threads=THREADS) for j in largest}
    _say(f"   oracle statics of the 3 largest scenes: {time.time() - t0:.1f} s")
    with sf.Batch(member) as b:
        _say("   tuned", b.tune(reps=1))
        b.step(11)  # a graph of 8 ticks, then one of 3
        for g in alone:
            g.step(11)
        totals = b.stats()
        for j, (a, m) in enumerate(zip(alone, member)):
            assert np.array_equal(a.positions(), m.positions()), j
            assert totals[j] == a.stats(), j
        _say("   positions and totals of all 256 scenes identical")
        before = {}
        for j in largest:
            g = member[j]
            pos, P = g.positions(), g.field()
            r = oracle.step(sts[j], pos, totals[j]["step"], threads=THREADS)
            before[j] = (pos, P, r)
        b.step(1)
        for j in largest:
            pos, P, r = before[j]
            rep = Report()
            rep.steps = 1
            rep.max_field_err = field_rel_err(P, r.P, sts[j].obstacle)
            rep.field_mismatch = field_bits_differ(P, r.P)
            tgt_g, flags_g = member[j].last_moves()
            untied, tied = classify(pos, r, tgt_g, flags_g, member[j].positions())
            rep.untied, rep.tied_mismatch = len(untied), len(tied)
            rep.decisions = int((pos >= 0).sum())
            _say(f"   scene {j} {scs[j].width}x{scs[j].height} R={scs[j].radius}:", rep)
            assert_parity(rep)
        _say(f"   full oracle ticks of the 3 largest scenes passed ({time.time() - t0:.1f} s)")
    for g in alone + member:
        g.close()
