"""Seeded synthetic scenes for the social-field pedestrian step.

This module only builds inputs: obstacle and exit masks, initial pedestrian
positions and the scalar parameters of a scene.  It holds none of the model's
arithmetic (no field, no distance, no move rule), so both the HIP library and
the FP64 oracle can be fed from it.

Scene geometry follows the paper's discrete model: a rectangular grid of space
units (su), one su per pedestrian (1x1 footprint, section 5 experiments),
openings (exits) where pedestrians leave, and static obstacles.  The paper's
experiments use a periodic boundary; most scenes here use walls with exits
instead, so that the static destination field is defined, and `flow_scene`
builds the paper's own workload: a torus with headed flows.

Recipe (all random draws from numpy PCG64 with the stated seed):
  * the border ring of su is obstacle (walls);
  * each exit is a run of border su centred on its wall, cleared from the wall;
  * interior obstacles: i.i.d. Bernoulli mask, or axis-aligned rectangles with
    sides uniform in [side_min, side_max] and uniform top-left corner, added
    until their union covers the requested fraction of the interior;
  * a clearance box (exit width x 8 su) in front of each exit is kept free;
  * free su that cannot reach any exit through 8-connected free su are filled
    as obstacles (connectivity by scipy.ndimage.label; no distances involved);
  * pedestrians are drawn uniformly without replacement from the free interior
    su that are not exits; pedestrian id = array index.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence

import numpy as np

# Walls a scene can carry exits on.
WALLS = ("W", "E", "N", "S")


@dataclass
class Scene:
    """Inputs of one scene.  Arrays are row-major [height, width], x fastest."""

    width: int
    height: int
    obstacle: np.ndarray  # uint8 [H*W], 1 = obstacle (walls included)
    exit: np.ndarray  # uint8 [H*W], 1 = exit su (never an obstacle)
    pos: np.ndarray  # int32 [N], linear su index y*W + x
    radius: int  # pedestrian field half-width R, window (2R+1)^2
    k: float = 1.0  # pedestrian field strength
    alpha: float = -0.5  # pedestrian field exponent
    k_obs: float = 1.0  # obstacle field strength
    alpha_obs: float = -0.5  # obstacle field exponent
    radius_obs: int = -1  # obstacle field half-width; -1 means "same as radius"
    w_dest: float = 1.0  # weight of the destination (distance) field
    seed: int = 0  # key of the counter-based generator used for elections
    start_step: int = 0  # step index of the initial state
    steps: int = 0  # number of steps the workload runs
    name: str = ""
    meta: dict = field(default_factory=dict)
    periodic: bool = False  # both axes wrap (a torus; no walls or exits)
    heading: Optional[np.ndarray] = None  # uint8 [N]: direction index 1..8, 0 = none
    w_heading: float = 1.0  # weight of the heading slope
    walk_period: Optional[np.ndarray] = None  # uint8 [N]: acts on ticks t with (t+id) % p == 0
    body_w: int = 1  # pedestrian body width in su (odd; section 2), centred on pos
    body_h: int = 1  # pedestrian body height in su (odd)

    @property
    def n_peds(self) -> int:
        return int(self.pos.shape[0])

    @property
    def r_obs(self) -> int:
        return self.radius if self.radius_obs < 0 else self.radius_obs

    def with_params(self, **kw) -> "Scene":
        return replace(self, **kw)


def _exit_span(length: int, width: int) -> range:
    lo = (length - width) // 2
    return range(lo, lo + width)


def _place_exits(obst2d: np.ndarray, exit2d: np.ndarray, walls: Sequence[str],
                 width: int) -> List[tuple]:
    """Clear `width` su centred on each named wall; returns clearance boxes."""
    H, W = obst2d.shape
    boxes = []
    for wall in walls:
        if wall in ("W", "E"):
            ys = _exit_span(H, width)
            x = 0 if wall == "W" else W - 1
            for y in ys:
                obst2d[y, x] = 0
                exit2d[y, x] = 1
            x_lo, x_hi = (1, min(W - 1, 9)) if wall == "W" else (max(1, W - 9), W - 1)
            boxes.append((ys.start, ys.stop, x_lo, x_hi))
        else:
            xs = _exit_span(W, width)
            y = 0 if wall == "N" else H - 1
            for x in xs:
                obst2d[y, x] = 0
                exit2d[y, x] = 1
            y_lo, y_hi = (1, min(H - 1, 9)) if wall == "N" else (max(1, H - 9), H - 1)
            boxes.append((y_lo, y_hi, xs.start, xs.stop))
    return boxes


def _fill_pockets(obst2d: np.ndarray, exit2d: np.ndarray) -> None:
    """Turn free su with no 8-connected free path to an exit into obstacles."""
    from scipy import ndimage

    free = obst2d == 0
    labels, _ = ndimage.label(free, structure=np.ones((3, 3), dtype=bool))
    keep = np.unique(labels[(exit2d == 1) & free])
    keep = keep[keep > 0]
    reachable = np.isin(labels, keep)
    obst2d[free & ~reachable] = 1


def _rectangles(obst2d: np.ndarray, rng: np.random.Generator, coverage: float,
                side_min: int, side_max: int) -> None:
    H, W = obst2d.shape
    interior = np.zeros_like(obst2d, dtype=bool)
    interior[1:H - 1, 1:W - 1] = True
    target = coverage * interior.sum()
    covered = 0
    rect = np.zeros_like(obst2d, dtype=bool)
    while covered < target:
        h = int(rng.integers(side_min, side_max + 1))
        w = int(rng.integers(side_min, side_max + 1))
        y = int(rng.integers(1, max(2, H - 1 - h + 1)))
        x = int(rng.integers(1, max(2, W - 1 - w + 1)))
        sl = rect[y:min(y + h, H - 1), x:min(x + w, W - 1)]
        covered += int((~sl).sum())
        sl[...] = True
    obst2d[rect] = 1


def build_scene(width: int, height: int, *, exits: Sequence[str], exit_width: int,
                n_peds: int, radius: int, seed: int, bernoulli: float = 0.0,
                rect_coverage: float = 0.0, rect_sides=(4, 32), steps: int = 0,
                name: str = "", occupancy: float | None = None, **params) -> Scene:
    """Generate a scene per the module recipe.  `occupancy` (fraction of free
    interior su) overrides `n_peds` when given."""
    rng = np.random.Generator(np.random.PCG64(seed))
    H, W = int(height), int(width)
    obst2d = np.zeros((H, W), dtype=np.uint8)
    obst2d[0, :] = obst2d[-1, :] = 1
    obst2d[:, 0] = obst2d[:, -1] = 1
    exit2d = np.zeros((H, W), dtype=np.uint8)
    if bernoulli > 0:
        mask = rng.random((H - 2, W - 2), dtype=np.float32) < bernoulli
        obst2d[1:H - 1, 1:W - 1][mask] = 1
        del mask
    if rect_coverage > 0:
        _rectangles(obst2d, rng, rect_coverage, *rect_sides)
    boxes = _place_exits(obst2d, exit2d, exits, exit_width)
    for (y0, y1, x0, x1) in boxes:
        obst2d[y0:y1, x0:x1] = 0
    # keep the wall ring intact outside the exits
    ring = np.zeros_like(obst2d, dtype=bool)
    ring[0, :] = ring[-1, :] = True
    ring[:, 0] = ring[:, -1] = True
    obst2d[ring & (exit2d == 0)] = 1
    _fill_pockets(obst2d, exit2d)
    cand = np.flatnonzero((obst2d.ravel() == 0) & (exit2d.ravel() == 0))
    if occupancy is not None:
        n_peds = int(round(occupancy * cand.size))
    if n_peds > cand.size:
        raise ValueError(f"{n_peds} pedestrians do not fit in {cand.size} free su")
    pick = rng.choice(cand.size, size=n_peds, replace=False)
    pos = cand[pick].astype(np.int32)
    return Scene(width=W, height=H, obstacle=obst2d.ravel().copy(),
                 exit=exit2d.ravel().copy(), pos=pos, radius=int(radius), seed=int(seed),
                 steps=int(steps), name=name, **params)


# --- the named workloads -------------------------------------------------------

def room64() -> Scene:
    """64x64 room, border walls, one 4-su exit centred on the east wall,
    200 pedestrians, R = 4, 200 steps, seed 0."""
    return build_scene(64, 64, exits=("E",), exit_width=4, n_peds=200, radius=4, seed=0,
                       steps=200, name="room64")


def hall1024() -> Scene:
    """1024x1024 hall, rectangles of side 4..32 covering 5% of the interior,
    two 16-su exits on the west and east walls, 50,000 pedestrians, R = 16,
    500 steps, seed 1."""
    return build_scene(1024, 1024, exits=("W", "E"), exit_width=16, n_peds=50_000,
                       radius=16, seed=1, rect_coverage=0.05, rect_sides=(4, 32),
                       steps=500, name="hall1024")


def plaza8192() -> Scene:
    """8192x8192 plaza, i.i.d. 2% obstacle su, four 64-su exits (one per wall),
    1,000,000 pedestrians, R = 32, 200 steps, seed 2."""
    return build_scene(8192, 8192, exits=("W", "E", "N", "S"), exit_width=64,
                       n_peds=1_000_000, radius=32, seed=2, bernoulli=0.02, steps=200,
                       name="plaza8192")


def flow1000() -> Scene:
    """The paper's baseline experiment scenario: 1000x1000 torus, density 0.5
    (500,000 pedestrians), 8-directional flow, 7x7 fields, 1000 ticks, seed 0."""
    return replace(flow_scene(1000, 1000, 0.5, 8, radius=3, seed=0, steps=1000), name="flow1000")


WORKLOADS = {"room64": room64, "hall1024": hall1024, "plaza8192": plaza8192,
             "flow1000": flow1000}


def ensemble(n_scenes: int = 256, seed: int = 3, side=(128, 2048), steps: int = 300):
    """Uneven ensemble: per scene, W and H uniform in `side`, rectangle
    coverage uniform in [0, 0.10], 1-4 exits on distinct walls (16 su wide),
    occupancy uniform in [1%, 10%] of free su, R drawn from {4, 8, 16, 32}."""
    out = []
    for s in range(n_scenes):
        rng = np.random.Generator(np.random.PCG64([seed, s]))
        W = int(rng.integers(side[0], side[1] + 1))
        H = int(rng.integers(side[0], side[1] + 1))
        cov = float(rng.uniform(0.0, 0.10))
        n_ex = int(rng.integers(1, 5))
        walls = tuple(rng.permutation(WALLS)[:n_ex])
        occ = float(rng.uniform(0.01, 0.10))
        R = int(rng.choice([4, 8, 16, 32]))
        sc_seed = int(rng.integers(0, 2**31 - 1))
        out.append(build_scene(W, H, exits=walls, exit_width=16, n_peds=0, radius=R,
                               seed=sc_seed, rect_coverage=cov, occupancy=occ, steps=steps,
                               name=f"ens{s}"))
    return out


# Headings of the flows of section 5 (indices into the direction list e1..e8:
# 1 east, 2 south-east, 3 south, ..., 8 north-east).
FLOW_HEADINGS = {1: (1,), 2: (1, 5), 4: (1, 3, 5, 7), 8: (1, 2, 3, 4, 5, 6, 7, 8)}


def flow_scene(width: int, height: int, density: float, directions: int, *, radius: int = 3,
               seed: int = 0, steps: int = 1000, w_heading: float = 1.0,
               max_walk_period: int = 1) -> Scene:
    """The paper's experiment workload: a width x height torus (periodic
    boundary, no obstacles or exits), round(density * su) pedestrians drawn
    uniformly without replacement, split evenly over the `directions` (1, 2,
    4 or 8) headings in random order, fields of half-width `radius` (3: the
    7x7 geometry), `steps` ticks; walk periods uniform in 1..max_walk_period
    (1: everyone acts every tick)."""
    if directions not in FLOW_HEADINGS:
        raise ValueError(f"directions must be one of {sorted(FLOW_HEADINGS)}")
    rng = np.random.Generator(np.random.PCG64([seed, width, height, directions]))
    n = width * height
    N = int(round(density * n))
    pos = np.sort(rng.choice(n, size=N, replace=False)).astype(np.int32)
    hs = np.array(FLOW_HEADINGS[directions], dtype=np.uint8)
    heading = rng.permutation(np.resize(hs, N)).astype(np.uint8)
    seed_sc = int(rng.integers(0, 2**63 - 1))
    walk = None
    if max_walk_period > 1:
        walk = np.random.Generator(np.random.PCG64([seed, 7, max_walk_period])).integers(
            1, max_walk_period + 1, size=N).astype(np.uint8)
    return Scene(width=width, height=height, obstacle=np.zeros(n, np.uint8),
                 exit=np.zeros(n, np.uint8), pos=pos, radius=radius, seed=seed_sc, steps=steps,
                 name=f"flow{width}x{height}d{density:g}k{directions}", periodic=True,
                 heading=heading, w_heading=w_heading, walk_period=walk)


def lattice_bodies(width: int, height: int, bw: int, bh: int, n: int, rng,
                   allowed=None, offset=(0, 0)) -> np.ndarray:
    """Centres of n non-overlapping bw x bh bodies: a random subset of the
    cells of the lattice of bw x bh blocks anchored at `offset` (whole blocks
    inside the grid only), keeping blocks whose su are all `allowed` (a bool
    [H*W] mask, None = all).  Sorted linear centre indices."""
    a, b = (bw - 1) // 2, (bh - 1) // 2
    xs = np.arange(offset[0] + a, width - a, bw)
    ys = np.arange(offset[1] + b, height - b, bh)
    cx, cy = np.meshgrid(xs, ys)
    cx, cy = cx.ravel(), cy.ravel()
    if allowed is not None:
        ok = np.ones(cx.size, bool)
        al = np.asarray(allowed, bool).reshape(height, width)
        for j in range(-b, b + 1):
            for i in range(-a, a + 1):
                ok &= al[cy + j, cx + i]
        cx, cy = cx[ok], cy[ok]
    if n > cx.size:
        raise ValueError(f"{n} bodies of {bw}x{bh} do not fit ({cx.size} lattice cells)")
    pick = rng.choice(cx.size, size=n, replace=False)
    return np.sort(cy[pick] * width + cx[pick]).astype(np.int32)


def body_flow_scene(width: int, height: int, cover: float, directions: int, body: int, *,
                    radius: int = 3, seed: int = 0, steps: int = 1000, w_heading: float = 1.0,
                    max_walk_period: int = 1) -> Scene:
    """The paper's footprint experiment (Table VI): a width x height torus
    whose pedestrians have body x body su bodies covering `cover` of the su
    (round(cover * su / body^2) pedestrians, on a random subset of the blocks
    of a body x body lattice), headed flows as in flow_scene, fields of
    half-width `radius`, walk periods uniform in 1..max_walk_period."""
    if directions not in FLOW_HEADINGS:
        raise ValueError(f"directions must be one of {sorted(FLOW_HEADINGS)}")
    rng = np.random.Generator(np.random.PCG64([seed, width, height, directions, body]))
    n = width * height
    N = int(round(cover * n / (body * body)))
    pos = lattice_bodies(width, height, body, body, N, rng)
    hs = np.array(FLOW_HEADINGS[directions], dtype=np.uint8)
    heading = rng.permutation(np.resize(hs, N)).astype(np.uint8)
    seed_sc = int(rng.integers(0, 2**63 - 1))
    walk = None
    if max_walk_period > 1:
        walk = np.random.Generator(np.random.PCG64([seed, 7, max_walk_period])).integers(
            1, max_walk_period + 1, size=N).astype(np.uint8)
    return Scene(width=width, height=height, obstacle=np.zeros(n, np.uint8),
                 exit=np.zeros(n, np.uint8), pos=pos, radius=radius, seed=seed_sc, steps=steps,
                 name=f"bodyflow{width}x{height}b{body}k{directions}", periodic=True,
                 heading=heading, w_heading=w_heading, walk_period=walk, body_w=body,
                 body_h=body)


def body_room(width: int, height: int, bw: int, bh: int, n_peds: int, radius: int, seed: int, *,
              exits=("E",), exit_width: int = 9, bernoulli: float = 0.0, **params) -> Scene:
    """A walled room (build_scene recipe, no pedestrians) with n_peds bodies
    of bw x bh su on a random subset of lattice blocks that cover only free
    interior su that are not exits."""
    sc = build_scene(width, height, exits=exits, exit_width=exit_width, n_peds=0,
                     radius=radius, seed=seed, bernoulli=bernoulli,
                     name=f"bodyroom{width}x{height}b{bw}x{bh}s{seed}", **params)
    rng = np.random.Generator(np.random.PCG64([seed, 91, bw, bh]))
    allowed = (sc.obstacle == 0) & (sc.exit == 0)
    sc.pos = lattice_bodies(width, height, bw, bh, n_peds, rng, allowed=allowed,
                            offset=(int(rng.integers(0, bw)), int(rng.integers(0, bh))))
    sc.body_w, sc.body_h = bw, bh
    return sc


def random_scene(width: int, height: int, n_peds: int, radius: int, seed: int, *,
                 bernoulli: float = 0.05, exits=("E",), exit_width: int = 2,
                 **params) -> Scene:
    """Small random scene for tests (ragged sizes, any radius)."""
    exit_width = max(1, min(exit_width, min(width, height) - 2))
    return build_scene(width, height, exits=exits, exit_width=exit_width, n_peds=n_peds,
                       radius=radius, seed=seed, bernoulli=bernoulli,
                       name=f"rand{width}x{height}s{seed}", **params)
