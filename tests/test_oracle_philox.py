"""Pin of the oracle's Philox4x32-10 against an independent implementation:
rocRAND's philox4x32_10_engine (a library routine, compiled here for the host).
Philox is the counter-based generator of Salmon, Moraes, Dror and Shaw
(SC'11); the election keys of the tick are built from its first output word.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_ref")
    subprocess.run([hipcc, "-O1", os.path.join(HERE, "golden", "philox_rocrand_ref.cpp"), "-o",
                    exe], check=True, capture_output=True)

    def run(rows):
        txt = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
        out = subprocess.run([exe], input=txt, capture_output=True, text=True, check=True)
        return np.array([[int(v) for v in ln.split()] for ln in out.stdout.strip().splitlines()],
                        dtype=np.uint64)

    return run


def test_philox_matches_rocrand(orc, rocrand_ref):
    rng = np.random.default_rng(123)
    M = 2**32 - 1
    rows = [[0, 0, 0, 0, 0, 0], [M, M, M, M, M, M], [1, 0, 0, 0, 0, 0], [0, 1, 0, 0, 0, 0],
            [0, 0, 1, 0, 0, 0], [0, 0, 0, 1, 0, 0], [0, 0, 0, 0, 1, 0], [0, 0, 0, 0, 0, 1]]
    rows += rng.integers(0, 2**32, size=(400, 6), dtype=np.uint64).tolist()
    # the tick's counter layout: (id, t_lo, t_hi, 0)
    rows += [[i, t, 0, 0, 12345, 0] for i in (0, 1, 999_999) for t in (0, 1, 199, 2**31)]
    ref = rocrand_ref(rows)
    got = np.array([orc.philox4x32_10(r[:4], r[4:]) for r in rows], dtype=np.uint64)
    assert np.array_equal(got, ref)


def test_claim_key_layout(orc, rocrand_ref):
    seed = (77 << 32) | 5
    for pid, t in [(0, 0), (3, 11), (123456, 7), (2**31 - 1, 2**33 + 5)]:
        r = rocrand_ref([[pid, t & M32, t >> 32, 0, seed & M32, seed >> 32]])[0]
        assert orc.claim_key(pid, t, seed) == (int(r[0]) << 32) | pid


M32 = 2**32 - 1
