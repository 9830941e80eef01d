"""Pins of the oracle's static fields.

Destination field: BFS distance to the openings over 8-connected free su,
checked against scipy's unweighted shortest paths on an explicitly built
8-neighbour graph, and against the closed form (Chebyshev distance to the
nearest exit su) in an obstacle-free room.

Superposed fields: the scatter of every source's window, checked against
scipy.signal.convolve2d of the source mask with the stamp (the definition of
linear superposition of translated copies), plus linearity, single-source
and mirror properties.
"""
import numpy as np
import pytest
from scipy import signal
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import shortest_path

from paper_1803_04782_amd import scenes


def _grid_graph(W, H, obst):
    rows, cols = [], []
    for y in range(H):
        for x in range(W):
            c = y * W + x
            if obst[c]:
                continue
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    if dx == 0 and dy == 0:
                        continue
                    nx, ny = x + dx, y + dy
                    if 0 <= nx < W and 0 <= ny < H and not obst[ny * W + nx]:
                        rows.append(c)
                        cols.append(ny * W + nx)
    n = W * H
    return coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(n, n)).tocsr()


@pytest.mark.parametrize("W,H,seed,frac", [(13, 9, 0, 0.15), (20, 17, 1, 0.3), (7, 31, 2, 0.1),
                                          (33, 5, 3, 0.25)])
def test_bfs_matches_library_shortest_paths(orc, W, H, seed, frac):
    rng = np.random.default_rng(seed)
    obst = (rng.random(W * H) < frac).astype(np.uint8)
    exitm = np.zeros(W * H, np.uint8)
    free = np.flatnonzero(obst == 0)
    exitm[rng.choice(free, size=3, replace=False)] = 1
    D, unreach = orc.bfs_distance(W, H, obst, exitm)
    g = _grid_graph(W, H, obst)
    dist = shortest_path(g, unweighted=True, indices=np.flatnonzero(exitm)).min(axis=0)
    ref = np.where(np.isfinite(dist), dist, -1).astype(np.int64)
    ref[obst == 1] = -1
    assert np.array_equal(D.astype(np.int64), ref)
    assert unreach == int(((obst == 0) & (ref < 0)).sum())


def test_bfs_closed_form_empty_room(orc):
    W, H = 23, 15
    obst = np.zeros(W * H, np.uint8)
    exitm = np.zeros(W * H, np.uint8)
    ex = [(22, 7), (0, 3), (10, 0)]
    for x, y in ex:
        exitm[y * W + x] = 1
    D, unreach = orc.bfs_distance(W, H, obst, exitm)
    ys, xs = np.divmod(np.arange(W * H), W)
    cheb = np.min([np.maximum(np.abs(xs - x), np.abs(ys - y)) for x, y in ex], axis=0)
    assert unreach == 0
    assert np.array_equal(D, cheb)


def test_bfs_unreachable_marked(orc):
    W, H = 9, 7
    obst = np.zeros((H, W), np.uint8)
    obst[:, 4] = 1  # a wall splits the room
    exitm = np.zeros((H, W), np.uint8)
    exitm[3, 8] = 1
    D, unreach = orc.bfs_distance(W, H, obst.ravel(), exitm.ravel())
    D = D.reshape(H, W)
    assert unreach == H * 4
    assert (D[:, :4] == -1).all() and (D[:, 4] == -1).all()
    assert D[3, 7] == 1 and D[0, 5] == 3


def _stamp(orc, R, k, alpha):
    return orc.phi_table(R, k, alpha)


@pytest.mark.parametrize("W,H,R,seed", [(12, 12, 3, 0), (19, 11, 2, 1), (8, 21, 5, 2),
                                        (30, 7, 4, 3), (5, 5, 7, 4)])
def test_source_field_matches_convolution(orc, W, H, R, seed):
    rng = np.random.default_rng(seed)
    src = (rng.random(W * H) < 0.2).astype(np.uint8)
    k, alpha = 1.3, -0.7
    out = orc.source_field(W, H, src, R, k, alpha).reshape(H, W)
    ref = signal.convolve2d(src.reshape(H, W).astype(np.float64), _stamp(orc, R, k, alpha),
                            mode="same")
    if 2 * R + 1 > min(W, H):
        # 'same' centres a kernel larger than the grid differently: use 'full' and crop
        full = signal.convolve2d(src.reshape(H, W).astype(np.float64),
                                 _stamp(orc, R, k, alpha), mode="full")
        ref = full[R:R + H, R:R + W]
    np.testing.assert_allclose(out, ref, rtol=1e-13, atol=1e-13)


def test_source_field_single_source_is_translated_stamp(orc):
    W, H, R = 15, 12, 3
    src = np.zeros((H, W), np.uint8)
    src[1, 13] = 1  # near the north-east corner: stamp is clipped
    out = orc.source_field(W, H, src.ravel(), R, 1.0, -0.5).reshape(H, W)
    st = _stamp(orc, R, 1.0, -0.5)
    ref = np.zeros((H, W))
    for dy in range(-R, R + 1):
        for dx in range(-R, R + 1):
            y, x = 1 + dy, 13 + dx
            if 0 <= y < H and 0 <= x < W:
                ref[y, x] = st[dy + R, dx + R]
    assert np.array_equal(out, ref)
    assert out[1, 13] == 0.0


def test_source_field_linear_and_mirrored(orc):
    W, H, R = 17, 13, 4
    rng = np.random.default_rng(7)
    a = (rng.random((H, W)) < 0.15).astype(np.uint8)
    b = ((rng.random((H, W)) < 0.15) & (a == 0)).astype(np.uint8)
    fa = orc.source_field(W, H, a.ravel(), R, 1.0, -0.5)
    fb = orc.source_field(W, H, b.ravel(), R, 1.0, -0.5)
    fab = orc.source_field(W, H, (a | b).ravel(), R, 1.0, -0.5)
    np.testing.assert_allclose(fab, fa + fb, rtol=1e-13, atol=1e-13)
    fm = orc.source_field(W, H, a[:, ::-1].copy().ravel(), R, 1.0, -0.5).reshape(H, W)
    np.testing.assert_allclose(fm, fa.reshape(H, W)[:, ::-1], rtol=1e-13, atol=1e-13)
    fv = orc.source_field(W, H, a[::-1, :].copy().ravel(), R, 1.0, -0.5).reshape(H, W)
    np.testing.assert_allclose(fv, fa.reshape(H, W)[::-1, :], rtol=1e-13, atol=1e-13)


def test_radius_zero_field_vanishes(orc):
    W, H = 10, 6
    src = np.ones(W * H, np.uint8)
    assert not orc.source_field(W, H, src, 0, 1.0, -0.5).any()


def test_total_field_composition(orc):
    sc = scenes.random_scene(21, 14, n_peds=25, radius=3, seed=5, bernoulli=0.1,
                             k_obs=0.8, alpha_obs=-1.0, radius_obs=2, w_dest=1.7)
    st = orc.statics(sc)
    P = orc.total_field(st, sc.pos)
    W, H = sc.width, sc.height
    occ = np.zeros(W * H)
    occ[sc.pos] = 1
    phi_ped = signal.convolve2d(occ.reshape(H, W), _stamp(orc, 3, 1.0, -0.5), mode="same")
    obs = signal.convolve2d(sc.obstacle.reshape(H, W).astype(float),
                            _stamp(orc, 2, 0.8, -1.0), mode="same")
    ref = 1.7 * st.D.reshape(H, W) + obs + phi_ped
    ref[sc.obstacle.reshape(H, W) == 1] = np.inf
    np.testing.assert_allclose(P.reshape(H, W), ref, rtol=1e-13, atol=1e-12)
    assert np.isinf(P[sc.obstacle == 1]).all()


@pytest.mark.parametrize("W,H,R,periodic,threads", [(61, 47, 5, False, 4), (64, 40, 7, True, 8),
                                                    (33, 9, 12, False, 3), (70, 70, 3, True, 16)])
def test_threaded_field_is_the_serial_field(orc, W, H, R, periodic, threads):
    # the row-band threads give the serial scatter's field bit for bit: each
    # su gets the same terms, and every sum of FP32 strengths is exact
    rng = np.random.default_rng(W * H + R)
    src = (rng.random(W * H) < 0.35).astype(np.uint8)
    for k, alpha in ((1.0, -0.5), (-0.3, -1.0), (0.2, 1.0)):
        a = orc.source_field(W, H, src, R, k, alpha, periodic)
        b = orc.source_field(W, H, src, R, k, alpha, periodic, threads=threads)
        assert np.array_equal(a, b)
    sc = scenes.random_scene(W + 5, H + 5, n_peds=200, radius=R, seed=7, bernoulli=0.05)
    st = orc.statics(sc)
    st4 = orc.statics(sc, threads=threads)
    assert np.array_equal(st.O, st4.O)
    assert np.array_equal(orc.total_field(st, sc.pos), orc.total_field(st, sc.pos, threads))
