"""FP64 CPU oracle of the social-field pedestrian step -- TEST INFRASTRUCTURE.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never routes
through it.  The arithmetic lives in ``sf_oracle.c`` (plain C, FP64, compiled
with gcc, no fast-math); this module only marshals numpy arrays.

Every function follows the model readings stated at the top of
``sf_oracle.c``: field law phi(d) = fl32(k*|d|^alpha) on the (2R+1)^2 window
with phi(0) = 0 (section 3.1, Fig. 1 caption and Table I's 1x1 entry; the
strengths are FP32 numbers like the float caches of Algorithms 2 and 3, and
every sum of them is formed exactly in FP64), the
destination field as 8-neighbour BFS distance to the openings, linear
superposition of all fields (Algorithms 2/3: only the total matters), the
tick of Algorithm 1 (decide, register-and-elect, move), and Philox4x32-10 keys
for the election; for the periodic workloads of section 5, a torus without
openings and per-pedestrian headings (a uniform destination slope).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sf_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_liboracle.so")
_lib = None

TIE_RTOL = 1e-5


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (plain -O2, IEEE arithmetic)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                        "-fno-fast-math", "-Wall", "-pthread", "-o", tmp, _SRC, "-lm"],
                       check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i32, i64, u64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    lib.orc_phi.restype = f64
    lib.orc_phi.argtypes = [i32, i32, i32, f64, f64]
    lib.orc_phi_table.restype = None
    lib.orc_phi_table.argtypes = [i32, f64, f64, P]
    lib.orc_bfs_distance.restype = i64
    lib.orc_bfs_distance.argtypes = [i32, i32, P, P, P]
    lib.orc_source_field.restype = None
    lib.orc_source_field.argtypes = [i32, i32, P, i32, f64, f64, i32, P]
    lib.orc_total_field.restype = None
    lib.orc_total_field.argtypes = [i32, i32, P, P, P, f64, i32, P, i32, f64, f64, i32, i32, P]
    lib.orc_source_field_mt.restype = None
    lib.orc_source_field_mt.argtypes = [i32, i32, P, i32, f64, f64, i32, i32, P]
    lib.orc_philox4x32_10.restype = None
    lib.orc_philox4x32_10.argtypes = [P, P, P]
    lib.orc_claim_key.restype = u64
    lib.orc_claim_key.argtypes = [i32, i64, u64]
    lib.orc_step.restype = i64
    lib.orc_step.argtypes = [i32, i32, P, P, P, i32, f64, f64, i32, P, f64, P, i32, i32, u64, i64,
                             i32, P, P, P, P]
    lib.orc_body_map.restype = i64
    lib.orc_body_map.argtypes = [i32, i32, i32, P, i32, i32, i32, P]
    lib.orc_field_at.restype = f64
    lib.orc_field_at.argtypes = [i32, i32, P, P, P, f64, i32, f64, f64, i32, f64, f64, i32, i64]
    lib.orc_decide_at.restype = None
    lib.orc_decide_at.argtypes = [i32, i32, P, P, P, f64, i32, f64, f64, i32, f64, f64, i32, i32,
                                  f64, i32, P, P, P]
    lib.orc_sect.restype = i32
    lib.orc_sect.argtypes = [i32, i32]
    lib.orc_fan_out.restype = i32
    lib.orc_fan_out.argtypes = [i32, i32]
    lib.orc_sect_field.restype = i32
    lib.orc_sect_field.argtypes = [i32, i32, P, P, i32, f64, f64, i32, i32, P, P]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# ---- field law ---------------------------------------------------------------

def phi(dx: int, dy: int, R: int, k: float, alpha: float) -> float:
    return float(_load().orc_phi(int(dx), int(dy), int(R), float(k), float(alpha)))


def phi_table(R: int, k: float, alpha: float) -> np.ndarray:
    """(2R+1, 2R+1) stamp indexed [dy+R, dx+R]."""
    out = np.empty((2 * R + 1) * (2 * R + 1), dtype=np.float64)
    _load().orc_phi_table(int(R), float(k), float(alpha), _ptr(out))
    return out.reshape(2 * R + 1, 2 * R + 1)


# ---- static fields -----------------------------------------------------------

def bfs_distance(W: int, H: int, obstacle, exitm):
    """(D int32[H*W], number of unreachable free su)."""
    ob, ex = _c(obstacle, np.uint8), _c(exitm, np.uint8)
    D = np.empty(W * H, dtype=np.int32)
    unreach = _load().orc_bfs_distance(W, H, _ptr(ob), _ptr(ex), _ptr(D))
    return D, int(unreach)


def source_field(W: int, H: int, src_mask, R: int, k: float, alpha: float,
                 periodic: bool = False, threads: int = 1) -> np.ndarray:
    """Superposed field of the sources (serial scatter, or row bands on
    `threads` threads: the same bits)."""
    src = _c(src_mask, np.uint8)
    out = np.empty(W * H, dtype=np.float64)
    if threads > 1:
        _load().orc_source_field_mt(W, H, _ptr(src), int(R), float(k), float(alpha),
                                    int(periodic), int(threads), _ptr(out))
    else:
        _load().orc_source_field(W, H, _ptr(src), int(R), float(k), float(alpha),
                                 int(periodic), _ptr(out))
    return out


# ---- the paper's own field path: sects, fan-out, K slots (Algorithm 3) --------

SECT_KS = (2, 4, 8, 16)


def sect_of(dx: int, dy: int) -> int:
    """Sect (0..7) of a nonzero offset: floor(angle / 45 deg), the angle of d
    from +x toward +y in [0, 360)."""
    return int(_load().orc_sect(int(dx), int(dy)))


def fan_out(wd: int, ht: int) -> int:
    """Strength fan-out of a wd x ht geometry: most window offsets in one sect."""
    return int(_load().orc_fan_out(int(wd), int(ht)))


def sect_field(W: int, H: int, src_mask, R: int, k: float, alpha: float, K: int,
               periodic: bool = False, image: bool = False):
    """Algorithm 3's FP32 field of the sources with K slots: (phi float32
    [H*W], image float32 [8, H*W] or None)."""
    src = _c(src_mask, np.uint8)
    phi = np.empty(W * H, dtype=np.float32)
    img = np.empty((8, W * H), dtype=np.float32) if image else None
    n = _load().orc_sect_field(W, H, _ptr(src), None, int(R), float(k), float(alpha),
                               int(periodic), int(K), _ptr(phi),
                               None if img is None else _ptr(img))
    if n < 0:
        raise ValueError(f"K = {K} is not one of {SECT_KS}")
    return phi, img


def sect_update(W: int, H: int, entered, left, R: int, k: float, alpha: float, K: int,
                phi, image=None, periodic: bool = False):
    """The incremental form: phi (float32 [H*W]) and image (float32 [8, H*W]
    or None) add Algorithm 3's FP32 sums of +strength at the su entered and
    -strength at the su left.  Returns new arrays."""
    phi = np.array(phi, dtype=np.float32, copy=True)
    img = None if image is None else np.array(image, dtype=np.float32, copy=True)
    n = _load().orc_sect_field(W, H, _ptr(_c(entered, np.uint8)), _ptr(_c(left, np.uint8)),
                               int(R), float(k), float(alpha), int(periodic), int(K), _ptr(phi),
                               None if img is None else _ptr(img))
    if n < 0:
        raise ValueError(f"K = {K} is not one of {SECT_KS}")
    return phi, img


def host_threads() -> int:
    """Host cores this process may use (the threaded field's default)."""
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        return max(1, os.cpu_count() or 1)


@dataclass
class Statics:
    """Static part of a scene as the oracle sees it."""

    W: int
    H: int
    obstacle: np.ndarray
    exit: np.ndarray
    D: np.ndarray
    O: np.ndarray
    R: int
    k: float
    alpha: float
    R_obs: int
    k_obs: float
    alpha_obs: float
    w_dest: float
    seed: int
    unreachable: int
    periodic: bool = False
    heading: Optional[np.ndarray] = None  # uint8 [N] by pedestrian id, or None
    w_heading: float = 1.0
    walk_period: Optional[np.ndarray] = None  # uint8 [N] by pedestrian id, or None
    body_w: int = 1  # body width and height in su (odd; 1 x 1 = one su)
    body_h: int = 1

    def acts(self, i: int, t: int) -> bool:
        """Whether pedestrian i decides on tick t (walk period)."""
        if self.walk_period is None or self.walk_period[i] <= 1:
            return True
        return (int(t) + int(i)) % int(self.walk_period[i]) == 0

    def heading_of(self, i: int) -> int:
        return 0 if self.heading is None else int(self.heading[i])

    @property
    def S(self) -> np.ndarray:
        """w_D*D + O in FP64, +inf on obstacles."""
        s = self.w_dest * self.D.astype(np.float64) + self.O
        s[self.obstacle != 0] = np.inf
        return s


def statics(scene, with_obstacle_field: bool = True, threads: int = 1) -> Statics:
    """Static fields of a scene (any object with the Scene attributes); the
    obstacle field on `threads` threads (the same bits)."""
    W, H = int(scene.width), int(scene.height)
    ob = _c(scene.obstacle, np.uint8)
    ex = _c(scene.exit, np.uint8)
    periodic = bool(getattr(scene, "periodic", False))
    if periodic:
        # a torus without openings: no destination field
        D, unreach = np.zeros(W * H, dtype=np.int32), 0
    else:
        D, unreach = bfs_distance(W, H, ob, ex)
    R_obs = int(scene.radius if getattr(scene, "radius_obs", -1) < 0 else scene.radius_obs)
    O = (source_field(W, H, ob, R_obs, scene.k_obs, scene.alpha_obs, periodic, threads)
         if with_obstacle_field else None)
    hd = getattr(scene, "heading", None)
    wp = getattr(scene, "walk_period", None)
    return Statics(W, H, ob, ex, D, O, int(scene.radius), float(scene.k), float(scene.alpha),
                   R_obs, float(scene.k_obs), float(scene.alpha_obs), float(scene.w_dest),
                   int(scene.seed), unreach, periodic,
                   None if hd is None else _c(hd, np.uint8),
                   float(getattr(scene, "w_heading", 1.0)),
                   None if wp is None else _c(wp, np.uint8),
                   int(getattr(scene, "body_w", 1)), int(getattr(scene, "body_h", 1)))


def total_field(st: Statics, pos, threads: int = 1) -> np.ndarray:
    """P = w_D*D + O + Phi(pos) in FP64, +inf on obstacles (Phi on `threads`
    threads: the same bits)."""
    p = _c(pos, np.int32)
    P = np.empty(st.W * st.H, dtype=np.float64)
    _load().orc_total_field(st.W, st.H, _ptr(st.obstacle), _ptr(st.D), _ptr(_c(st.O, np.float64)),
                            st.w_dest, p.shape[0], _ptr(p), st.R, st.k, st.alpha,
                            int(st.periodic), int(threads), _ptr(P))
    return P


# ---- generator ---------------------------------------------------------------

def philox4x32_10(ctr, key) -> np.ndarray:
    c = _c(ctr, np.uint32)
    kk = _c(key, np.uint32)
    out = np.empty(4, dtype=np.uint32)
    _load().orc_philox4x32_10(_ptr(c), _ptr(kk), _ptr(out))
    return out


def claim_key(pid: int, t: int, seed: int) -> int:
    return int(_load().orc_claim_key(int(pid), int(t), int(seed) & (2**64 - 1)))


# ---- ticks -------------------------------------------------------------------

@dataclass
class StepResult:
    P: np.ndarray  # FP64 field of the step-start state
    target: np.ndarray  # int32 chosen su (own su when staying, -1 when evacuated)
    moved: np.ndarray  # uint8 won the election and moved
    tied: np.ndarray  # uint8 two best candidates within TIE_RTOL
    pos: np.ndarray  # int32 positions after the tick
    left: int  # pedestrians that left through an exit


def step(st: Statics, pos, t: int, P: Optional[np.ndarray] = None,
         threads: int = 1) -> StepResult:
    """One tick from (pos, t).  `pos` is not modified.  The step-start field is
    computed on `threads` threads unless given (the same bits)."""
    newpos = np.array(pos, dtype=np.int32, copy=True)
    if P is None:
        P = total_field(st, newpos, threads)
    n = newpos.shape[0]
    target = np.empty(n, dtype=np.int32)
    moved = np.empty(n, dtype=np.uint8)
    tied = np.empty(n, dtype=np.uint8)
    hd = None if st.heading is None else _ptr(st.heading)
    wp = None if st.walk_period is None else _ptr(st.walk_period)
    left = _load().orc_step(st.W, st.H, _ptr(st.obstacle), _ptr(st.exit), _ptr(P), st.R,
                            st.k, st.alpha, int(st.periodic), hd, st.w_heading, wp,
                            st.body_w, st.body_h, st.seed & (2**64 - 1), int(t), n,
                            _ptr(newpos), _ptr(target), _ptr(moved), _ptr(tied))
    return StepResult(P, target, moved, tied, newpos, int(left))


def run(st: Statics, pos, t0: int, n_steps: int):
    """Free run; returns the list of StepResults."""
    out = []
    cur = np.array(pos, dtype=np.int32, copy=True)
    for s in range(n_steps):
        r = step(st, cur, t0 + s)
        out.append(r)
        cur = r.pos
    return out


def body_map(st: Statics, pos):
    """(owner int32 [W*H]: the pedestrian whose body covers each su, else -1;
    0 or 1 + the first pedestrian whose body leaves a bounded grid or overlaps
    another)."""
    p = _c(pos, np.int32)
    owner = np.empty(st.W * st.H, dtype=np.int32)
    bad = _load().orc_body_map(st.W, st.H, p.shape[0], _ptr(p), st.body_w, st.body_h,
                               int(st.periodic), _ptr(owner))
    return owner, int(bad)


# ---- point evaluation (large grids) ------------------------------------------

def occupancy(W: int, H: int, pos) -> np.ndarray:
    occ = np.zeros(W * H, dtype=np.uint8)
    p = np.asarray(pos)
    occ[p[p >= 0]] = 1
    return occ


def field_at(st: Statics, occ: np.ndarray, cells) -> np.ndarray:
    lib = _load()
    out = np.empty(len(cells), dtype=np.float64)
    for j, c in enumerate(np.asarray(cells, dtype=np.int64)):
        out[j] = lib.orc_field_at(st.W, st.H, _ptr(st.obstacle), _ptr(occ), _ptr(st.D),
                                  st.w_dest, st.R, st.k, st.alpha, st.R_obs, st.k_obs,
                                  st.alpha_obs, int(st.periodic), int(c))
    return out


def decide_at(st: Statics, occ: np.ndarray, p: int, heading: int = 0):
    """(target su, tied, P on the 3x3 block by direction) for the pedestrian at
    p with the given heading."""
    t = np.empty(1, dtype=np.int32)
    tied = np.empty(1, dtype=np.uint8)
    P9 = np.empty(9, dtype=np.float64)
    _load().orc_decide_at(st.W, st.H, _ptr(st.obstacle), _ptr(occ), _ptr(st.D), st.w_dest,
                          st.R, st.k, st.alpha, st.R_obs, st.k_obs, st.alpha_obs,
                          int(st.periodic), int(heading), st.w_heading, int(p), _ptr(t),
                          _ptr(tied), _ptr(P9))
    return int(t[0]), bool(tied[0]), P9


DIRS = ((0, 0), (1, 0), (1, 1), (0, 1), (-1, 1), (-1, 0), (-1, -1), (0, -1), (1, -1))


def outcome_at(st: Statics, occ: np.ndarray, owner: np.ndarray, pos, i: int, t: int):
    """Full tick outcome of pedestrian i from point evaluations only:
    (target, moved, tied).  `owner[c]` is the id at su c or -1."""
    p = int(pos[i])
    if not st.acts(i, t):
        return p, False, False
    tgt, tied, _ = decide_at(st, occ, p, st.heading_of(i))
    if tgt == p:
        return tgt, False, tied
    # every live pedestrian that can register at tgt stands next to it
    W, H = st.W, st.H
    tx, ty = tgt % W, tgt // W
    best = None
    for dx, dy in DIRS[1:]:
        x, y = tx + dx, ty + dy
        if st.periodic:
            x, y = x % W, y % H
        elif not (0 <= x < W and 0 <= y < H):
            continue
        j = int(owner[y * W + x])
        if j < 0 or not st.acts(j, t):
            continue
        tj = tgt if j == i else decide_at(st, occ, y * W + x, st.heading_of(j))[0]
        if tj != tgt:
            continue
        key = claim_key(j, t, st.seed)
        if best is None or key < best[0]:
            best = (key, j)
    return tgt, best is not None and best[1] == i, tied
