"""The C-ABI library loads, exports every symbol include/sf.h declares, and
rejects bad descriptors on the host before touching the device."""
import math
import os
import re
from dataclasses import replace

import numpy as np
import pytest

from paper_1803_04782_amd import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def sf():
    from paper_1803_04782_amd import build as _build
    from paper_1803_04782_amd import sf as _sf

    if not os.path.exists(_sf.LIB_PATH):
        _build.build()
    _sf.load()
    return _sf


def _declared():
    txt = open(os.path.join(ROOT, "include", "sf.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return set(re.findall(r"\b(sf_[a-z_]+)\s*\(", txt))


def test_exports_every_declared_symbol(sf):
    lib = sf.load()
    names = _declared()
    assert names == set(sf.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def test_binds_to_the_one_hip_runtime_of_the_process(sf):
    # the library must share torch's HIP runtime: a second copy in the
    # process leaves whichever starts second without a device
    runtimes = sf._hip_runtimes()
    assert len(runtimes) == 1, runtimes
    import torch

    assert os.path.dirname(runtimes[0]) == os.path.join(os.path.dirname(torch.__file__), "lib")
    assert sf.device_count() >= 0


def _base():
    return scenes.random_scene(16, 12, n_peds=10, radius=2, seed=1, bernoulli=0.0)


def _mut(**kw):
    sc = _base()
    for k, v in kw.items():
        setattr(sc, k, v)
    return sc


def test_validation_errors(sf):
    base = _base()
    W = base.width
    free_exit = int(np.flatnonzero(base.exit)[0])
    obst = int(np.flatnonzero(base.obstacle)[0])
    cases = {
        "zero width": _mut(width=0),
        "radius too large": _mut(radius=sf.SF_MAX_RADIUS + 1),
        "negative radius": _mut(radius=-1),
        "radius_obs": _mut(radius_obs=-2),
        "nan k": _mut(k=math.nan),
        "inf w_dest": _mut(w_dest=math.inf),
        "negative start": _mut(start_step=-3),
        # strengths spread too far for exact FP64 sums (1 down to about 1e-11)
        "steep law": _mut(alpha=-6.0, radius=48),
        "steep obstacle law": _mut(alpha_obs=-6.0, radius_obs=40),
        "strength overflows FP32": _mut(k=1e39),
    }
    p = base.pos.copy()
    p[0] = obst
    cases["ped on obstacle"] = _mut(pos=p)
    p = base.pos.copy()
    p[0] = free_exit
    cases["ped on exit"] = _mut(pos=p)
    p = base.pos.copy()
    p[1] = p[0]
    cases["duplicate"] = _mut(pos=p)
    p = base.pos.copy()
    p[2] = W * base.height
    cases["out of range"] = _mut(pos=p)
    ob = base.obstacle.copy()
    ob[free_exit] = 1
    cases["exit on obstacle"] = _mut(obstacle=ob)
    cases["no exit"] = _mut(exit=np.zeros_like(base.exit))
    hd = np.ones(base.n_peds, np.uint8)
    hd[3] = 9
    cases["heading above 8"] = _mut(heading=hd)
    cases["nan w_heading"] = _mut(w_heading=math.nan)
    wk = np.ones(base.n_peds, np.uint8)
    wk[2] = 0
    cases["walk period 0"] = _mut(walk_period=wk)
    flow = scenes.flow_scene(80, 70, 0.2, 4, radius=3, seed=1)
    ob = flow.obstacle.copy()
    ob[5] = 1
    cases["periodic with obstacle"] = replace(flow, obstacle=ob)
    ex = flow.exit.copy()
    ex[5] = 1
    cases["periodic with exit"] = replace(flow, exit=ex)
    narrow = scenes.flow_scene(60, 70, 0.2, 4, radius=3, seed=1)
    cases["periodic narrower than a word"] = narrow
    cases["periodic window wider than the grid"] = replace(
        scenes.flow_scene(64, 20, 0.2, 1, radius=3, seed=1), radius=10)
    for name, sc in cases.items():
        rc, msg = sf.create_error(sc)
        assert rc == sf.SF_EINVAL, (name, rc, msg)
        assert msg, name


def test_pedestrian_count_limit(sf):
    """n_peds above SF_MAX_PEDS is refused before any array is read."""
    import ctypes

    desc, keep = sf.make_desc(_base())
    desc.n_peds = sf.SF_MAX_PEDS + 1
    h = ctypes.c_void_p()
    rc = sf.load().sf_create_scene(ctypes.byref(desc), None, ctypes.byref(h))
    assert rc == sf.SF_EINVAL and "above" in sf.load().sf_last_error().decode()
    del keep


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_1803_04782_amd import sf as _sf

    monkeypatch.setattr(_sf, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(_sf, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        _sf.load()
