"""Host logic of the serving loop (admission by footprint, slot limit, arrival
order, retirement) with stand-in scene and batch objects: no device."""
import time
import types

import numpy as np
import pytest

from paper_1803_04782_amd import serve


class _FakeScene:
    def __init__(self, width, height, n, life):
        self.width, self.height = width, height
        self.pos = np.zeros(n, np.int32)
        self.life = life


class _Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


def _fake_sf(clock, log):
    class GpuScene:
        live_objects = 0

        def __init__(self, scene, stream=None):
            self.scene = scene
            self.ticks = 0
            GpuScene.live_objects += 1
            log.append(("create", scene))

        def close(self):
            GpuScene.live_objects -= 1

        def positions(self):
            return self.scene.pos

    class Batch:
        def __init__(self, members, tiling=None, stream=None):
            self.members = members

        def step(self, n):
            clock.t += 0.001 * n
            for m in self.members:
                m.ticks += n

        def stats(self):
            return [{"live": max(0, m.scene.life - m.ticks), "ped_steps": m.ticks}
                    for m in self.members]

        def close(self):
            pass

    return types.SimpleNamespace(GpuScene=GpuScene, Batch=Batch)


def test_admission_respects_budget_slots_and_order(monkeypatch):
    clock = _Clock()
    log = []
    fake = _fake_sf(clock, log)
    monkeypatch.setattr(serve, "sf", fake)
    rng = np.random.default_rng(0)
    reqs = []
    for i in range(30):
        sc = _FakeScene(int(rng.integers(50, 400)), int(rng.integers(50, 400)), 100,
                        life=int(rng.integers(3, 40)))
        reqs.append(serve.Request(i, arrival=0.002 * i, make_scene=(lambda s=sc: s),
                                  max_steps=25))
    budget = 4 * serve.footprint_bytes(_FakeScene(400, 400, 100, 1))
    srv = serve.Server(budget, max_scenes=3, clock=clock, background_builds=False)
    out = srv.run(reqs)
    assert out["finished"] == 30
    assert out["max_used_bytes"] <= budget
    assert out["max_resident"] <= 3
    # first-come first-served: admission in arrival order
    created = [e[1] for e in log if e[0] == "create"]
    assert created == [r.make_scene() for r in reqs]
    for f in out["results"]:
        r = reqs[f.rid]
        assert f.steps == min(r.make_scene().life, 25)
        assert f.admitted >= f.arrival
    assert fake.GpuScene.live_objects == 0


def test_request_larger_than_budget_is_an_error(monkeypatch):
    clock = _Clock()
    monkeypatch.setattr(serve, "sf", _fake_sf(clock, []))
    big = _FakeScene(1000, 1000, 10, 5)
    for bg in (False, True):
        srv = serve.Server(serve.footprint_bytes(big) - 1, clock=clock, background_builds=bg,
                           create_stream="builder")
        with pytest.raises(ValueError):
            srv.run([serve.Request(0, 0.0, lambda: big)])


def test_poisson_arrivals_rate():
    t = serve.poisson_arrivals(200.0, 50.0, seed=4)
    assert np.all(np.diff(t) > 0) and t[-1] < 50.0
    assert abs(len(t) / 50.0 - 200.0) < 200.0 * 0.05


def test_admissions_per_tick_are_bounded(monkeypatch):
    clock = _Clock()
    log = []
    fake = _fake_sf(clock, log)
    monkeypatch.setattr(serve, "sf", fake)
    reqs = [serve.Request(i, arrival=0.0, make_scene=(lambda: _FakeScene(60, 60, 10, 50)),
                          max_steps=5) for i in range(12)]
    created_per_tick = []

    class Counting(fake.Batch):
        def __init__(self, members, tiling=None, stream=None):
            super().__init__(members, tiling, stream)
            created_per_tick.append(sum(1 for e in log if e[0] == "create"))

    monkeypatch.setattr(fake, "Batch", Counting)
    out = serve.Server(1 << 40, max_scenes=8, clock=clock, max_admit_per_tick=2,
                       background_builds=False).run(reqs)
    assert out["finished"] == 12
    # the first batch takes every scene it can; later ones at most 2 newcomers
    steps = [b - a for a, b in zip(created_per_tick, created_per_tick[1:])]
    assert max(steps) <= 2


def test_background_builds_hold_budget_and_slots(monkeypatch):
    clock = _Clock()
    log = []
    fake = _fake_sf(clock, log)
    monkeypatch.setattr(serve, "sf", fake)
    base_init = fake.GpuScene.__init__
    streams = []

    def slow_init(self, scene, stream=None):
        time.sleep(0.002)  # the build overlaps the ticks of the resident scenes
        streams.append(stream)
        base_init(self, scene, stream)

    monkeypatch.setattr(fake.GpuScene, "__init__", slow_init)
    rng = np.random.default_rng(1)
    reqs = []
    for i in range(20):
        sc = _FakeScene(int(rng.integers(50, 300)), int(rng.integers(50, 300)), 50,
                        life=int(rng.integers(2, 30)))
        reqs.append(serve.Request(i, arrival=0.001 * i, make_scene=(lambda s=sc: s),
                                  max_steps=20))
    budget = 3 * serve.footprint_bytes(_FakeScene(300, 300, 50, 1))
    srv = serve.Server(budget, max_scenes=3, clock=clock, create_stream="builder",
                       max_building=2)
    out = srv.run(reqs)
    assert out["finished"] == 20
    assert out["max_used_bytes"] <= budget and out["max_resident"] <= 3
    created = [e[1] for e in log if e[0] == "create"]
    assert created == [r.make_scene() for r in reqs]  # one builder: arrival order
    assert set(streams) == {"builder"}
    for f in out["results"]:
        assert f.steps == min(reqs[f.rid].make_scene().life, 20)
    assert fake.GpuScene.live_objects == 0


def test_background_build_failure_is_raised_and_cleaned_up(monkeypatch):
    clock = _Clock()
    fake = _fake_sf(clock, [])
    monkeypatch.setattr(serve, "sf", fake)
    base_init = fake.GpuScene.__init__

    def failing_init(self, scene, stream=None):
        if scene.life == 13:
            raise RuntimeError("build failed")
        base_init(self, scene, stream)

    monkeypatch.setattr(fake.GpuScene, "__init__", failing_init)
    reqs = [serve.Request(i, arrival=0.0, make_scene=(lambda i=i: _FakeScene(60, 60, 5, 10 + i)),
                          max_steps=50) for i in range(6)]
    srv = serve.Server(1 << 40, max_scenes=4, clock=clock, create_stream="builder")
    with pytest.raises(RuntimeError, match="build failed"):
        srv.run(reqs)
    assert fake.GpuScene.live_objects == 0
