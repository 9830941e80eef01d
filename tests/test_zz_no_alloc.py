"""GPU test of sf_superpose_noalloc, the superposition whose scratch lives in a
static device array: through the C ABI it must give sf_superpose's field bit
for bit, call after call (the second call smaller than the first, so that
what the first left in the shared array must not leak into it), and refuse
grids beyond its static bitmap before any device work."""
import ctypes

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sf():
    from paper_1803_04782_amd import sf as _sf

    _sf.load()
    return _sf


def _inputs(W, H, dens, seed):
    rng = np.random.default_rng([23, W, H, seed])
    n_su = W * H
    S = rng.uniform(-20.0, 300.0, n_su)
    S[rng.random(n_su) < 0.02] = np.inf
    occ = rng.choice(n_su, size=int(dens * n_su), replace=False).astype(np.int32)
    pos = np.concatenate([occ, np.array([-1, n_su, -3], dtype=np.int32)])
    rng.shuffle(pos)
    mask = np.zeros(n_su, dtype=np.uint8)
    mask[occ] = 1
    return S, pos, mask


# a large dense call, then a smaller one (bounded, then a torus), then the first again
CALLS = [(640, 480, 20, 1.0, -0.5, False, 0.2), (129, 97, 7, -1.5, -0.5, True, 0.3),
         (640, 480, 20, 1.0, -0.5, False, 0.2)]


def test_noalloc_matches_superpose_call_after_call(sf):
    import torch

    dev = torch.device("cuda:0")
    for i, (W, H, R, k, alpha, periodic, dens) in enumerate(CALLS):
        print(f"call {i}: {W}x{H} R={R} periodic={periodic}", flush=True)
        S, pos, mask = _inputs(W, H, dens, seed=i)
        S_d = torch.from_numpy(S).to(dev)
        pos_d = torch.from_numpy(pos).to(dev)
        P_alloc = sf.superpose(S_d, pos_d, W, H, R, k, alpha, periodic)
        P_na = sf.superpose(S_d, pos_d, W, H, R, k, alpha, periodic, noalloc=True)
        torch.cuda.synchronize()
        a = P_alloc.cpu().numpy()
        b = P_na.cpu().numpy()
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), i
        want = (S + oracle.source_field(W, H, mask, R, k, alpha, periodic)).astype(np.float32)
        assert np.array_equal(b.view(np.uint32), want.view(np.uint32)), i


def test_noalloc_refuses_grids_beyond_its_scratch(sf):
    import torch

    lib = sf.load()
    small = torch.zeros(16, dtype=torch.float64, device="cuda:0")
    out = torch.zeros(16, dtype=torch.float32, device="cuda:0")
    # ceil(8256/64) * 8192 bitmap words > 2^20: refused before any device work
    rc = lib.sf_superpose_noalloc(8256, 8192, 0, 4, 1.0, -0.5, ctypes.c_void_p(small.data_ptr()),
                                  None, 0, ctypes.c_void_p(out.data_ptr()), None)
    assert rc == sf.SF_EINVAL
    assert b"static scratch" in lib.sf_last_error()
