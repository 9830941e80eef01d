"""GPU test of the serving loop: requests arrive while others run, are admitted
as memory and slots free up, and share batched ticks; every result must be
the same as the scene run alone with sf_step for the same number of ticks, and
the same as the FP64 oracle's free run of that scene."""
import functools

import numpy as np
import pytest

from paper_1803_04782_amd import scenes, serve

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sf():
    from paper_1803_04782_amd import sf as _sf

    _sf.load()
    return _sf


def _request_scene(i):
    rng = np.random.default_rng([7, i])
    W = int(rng.integers(40, 140))
    H = int(rng.integers(40, 140))
    R = int(rng.choice([0, 2, 4, 8, 16]))
    walls = tuple(rng.permutation(["W", "E", "N", "S"])[: int(rng.integers(1, 3))])
    occ = float(rng.uniform(0.02, 0.12))
    return scenes.build_scene(W, H, exits=walls, exit_width=6, n_peds=0, radius=R,
                              seed=int(rng.integers(0, 2**31 - 1)), bernoulli=0.03,
                              occupancy=occ, name=f"req{i}")


@functools.lru_cache(maxsize=None)
def _oracle_run(rid, steps):
    """Final positions and evacuations of the oracle's free run of request rid."""
    import oracle

    sc = _request_scene(rid)
    st = oracle.statics(sc)
    pos = sc.pos.copy()
    left = 0
    for t in range(sc.start_step, sc.start_step + steps):
        r = oracle.step(st, pos, t)
        pos, left = r.pos, left + r.left
    return pos, left


@pytest.mark.parametrize("background", [True, False], ids=["background-builds", "sync-builds"])
def test_serving_results_match_scenes_alone(sf, background):
    n = 24
    arrivals = serve.poisson_arrivals(400.0, 0.5, seed=4)[:n]
    reqs = [serve.Request(i, float(a), (lambda i=i: _request_scene(i)), max_steps=120)
            for i, a in enumerate(arrivals)]
    # a budget of about five mid-sized scenes forces queueing and turnover
    budget = 5 * serve.footprint_bytes(_request_scene(0))
    import torch

    # admitted scenes are built on a stream of their own (on a worker thread,
    # or between ticks) while the others tick on the default stream
    srv = serve.Server(budget, max_scenes=6, keep_positions=True,
                       create_stream=torch.cuda.Stream(), background_builds=background)
    out = srv.run(reqs)
    print({k: v for k, v in out.items() if k != "results"}, flush=True)
    assert out["finished"] == len(reqs)
    assert out["max_used_bytes"] <= budget and out["max_resident"] <= 6
    for f in out["results"]:
        sc = _request_scene(f.rid)
        with sf.GpuScene(sc) as g:
            g.step(f.steps)
            assert np.array_equal(g.positions(), f.positions), f.rid
            alone = g.stats()
        for k in ("step", "live", "evacuated", "ped_steps", "movers", "moved", "tied"):
            assert alone[k] == f.stats[k], (f.rid, k, alone[k], f.stats[k])
        assert f.stats["live"] == 0 or f.steps == 120
        # the field is the oracle's rounded once and both sides decide on the
        # same FP32 numbers, so a served run follows the oracle's free run
        # tick for tick: same positions, same evacuations
        opos, oleft = _oracle_run(f.rid, f.steps)
        assert np.array_equal(opos, f.positions), (f.rid, "served run differs from the oracle")
        assert oleft == f.stats["evacuated"], (f.rid, oleft, f.stats["evacuated"])
