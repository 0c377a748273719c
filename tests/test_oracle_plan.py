"""Pins of the oracle's path search through the slices (Sec. III-D).

The oracle computes Dijkstra distances over the slice graph and reads a path
back from them.  Its pins do not come from itself:
  - closed form: on one layer of uniform cost c the distance to a cell dx, dy
    away is the diagonal (octile) count of straight and diagonal steps, each
    costing c + 1 or c + sqrt 2;
  - library: the same graph handed to scipy's Dijkstra gives the same
    distances;
  - the section's rules on hand-made one-row maps: node cost merged over
    layers with equal ground, gateways only to a strictly cheaper layer (up
    and down), barriers never entered;
  - path validity: consecutive nodes are linked and the edge costs add up to
    the goal's distance exactly.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import dijkstra

import oracle
import scenes

CB = 50.0
DX8 = [(-1, -1), (0, -1), (1, -1), (-1, 0), (1, 0), (-1, 1), (0, 1), (1, 1)]


def scipy_distances(cT, eG, start):
    """Distances from scipy's Dijkstra on the graph of Sec. III-D built with
    numpy (an independent construction of the same graph)."""
    cT = np.asarray(cT, np.float32)
    eG = np.asarray(eG, np.float32)
    L, ny, nx = cT.shape
    c64 = cT.astype(np.float64)
    cn = c64.copy()
    same_up = np.zeros(cT.shape, bool)
    same_dn = np.zeros(cT.shape, bool)
    same_up[:-1] = eG[1:] == eG[:-1]
    same_dn[1:] = eG[:-1] == eG[1:]
    cn[:-1] = np.where(same_up[:-1], np.minimum(cn[:-1], c64[1:]), cn[:-1])
    cn[1:] = np.where(same_dn[1:], np.minimum(cn[1:], c64[:-1]), cn[1:])
    idx = np.arange(L * ny * nx).reshape(L, ny, nx)
    rows, cols, wts = [], [], []
    for dx, dy in DX8:
        step = math.sqrt(2.0) if dx and dy else 1.0
        ys = slice(max(0, -dy), ny - max(0, dy))
        xs = slice(max(0, -dx), nx - max(0, dx))
        yt = slice(max(0, dy), ny - max(0, -dy))
        xt = slice(max(0, dx), nx - max(0, -dx))
        u = idx[:, ys, xs]
        v = idx[:, yt, xt]
        c = cn[:, yt, xt]
        ok = c < CB
        rows.append(u[ok])
        cols.append(v[ok])
        wts.append(c[ok] + step)
    up = same_up[:-1] & (cT[1:] < cT[:-1])      # gateway l -> l+1
    rows.append(idx[:-1][up])
    cols.append(idx[1:][up])
    wts.append(np.zeros(int(up.sum())))
    dn = same_dn[1:] & (cT[:-1] < cT[1:])       # gateway l -> l-1
    rows.append(idx[1:][dn])
    cols.append(idx[:-1][dn])
    wts.append(np.zeros(int(dn.sum())))
    r, c, w = (np.concatenate(a) for a in (rows, cols, wts))
    n = L * ny * nx
    # keep the cheapest of parallel edges (none arise here, but csr would add them)
    m = sp.coo_matrix((w, (r, c)), shape=(n, n)).tocsr()
    s = int(idx[start[2], start[1], start[0]])
    return dijkstra(m, indices=s).reshape(L, ny, nx)


def check_path(path, dist, cT, eG, start, goal):
    """Consecutive nodes are linked by an edge of the graph and the edge
    costs summed in order give the goal's distance bit for bit."""
    cT = np.asarray(cT, np.float32)
    eG = np.asarray(eG, np.float32)
    L = cT.shape[0]
    assert tuple(path[0]) == tuple(start) and tuple(path[-1]) == tuple(goal)

    def ncost(x, y, l):
        c = float(cT[l, y, x])
        for m in (l - 1, l + 1):
            if 0 <= m < L and eG[m, y, x] == eG[l, y, x]:
                c = min(c, float(cT[m, y, x]))
        return c

    d = 0.0
    for (x0, y0, l0), (x1, y1, l1) in zip(path[:-1], path[1:]):
        if l0 == l1:
            assert max(abs(x1 - x0), abs(y1 - y0)) == 1
            c = ncost(x1, y1, l1)
            assert c < CB
            d = d + (c + (math.sqrt(2.0) if x1 != x0 and y1 != y0 else 1.0))
        else:
            assert (x0, y0) == (x1, y1) and abs(l1 - l0) == 1
            assert eG[l1, y1, x1] == eG[l0, y0, x0] and cT[l1, y1, x1] < cT[l0, y0, x0]
            d = d + 0.0
    assert d == dist[goal[2], goal[1], goal[0]]


@pytest.mark.parametrize("c", [0.0, 3.0, 17.25])
def test_uniform_layer_closed_form(c):
    nx, ny = 23, 17
    cT = np.full((1, ny, nx), c, np.float32)
    eG = np.zeros((1, ny, nx), np.float32)
    s = (5, 11, 0)
    d = oracle.plan(cT, eG, CB, s)[0]
    x = np.abs(np.arange(nx)[None, :] - s[0])
    y = np.abs(np.arange(ny)[:, None] - s[1])
    nd = np.minimum(x, y)
    ns = np.maximum(x, y) - nd
    ref = ns * (c + 1.0) + nd * (c + math.sqrt(2.0))
    np.testing.assert_allclose(d, ref, rtol=1e-13, atol=0)
    p = oracle.plan_path(cT, eG, CB, oracle.plan(cT, eG, CB, s), s, (22, 0, 0))
    assert len(p) == 1 + max(22 - 5, 11)   # an octile path takes max(dx, dy) steps
    check_path(p, oracle.plan(cT, eG, CB, s), cT, eG, s, (22, 0, 0))


@pytest.mark.parametrize("seed,L,ny,nx", [(1, 1, 9, 13), (2, 3, 21, 17), (3, 4, 40, 37), (4, 2, 1, 30)])
def test_matches_scipy_dijkstra(seed, L, ny, nx):
    cT, eG = scenes.plan_layers(seed, L, ny, nx)
    rng = np.random.default_rng(100 + seed)
    s = (int(rng.integers(nx)), int(rng.integers(ny)), int(rng.integers(L)))
    d = oracle.plan(cT, eG, CB, s)
    ref = scipy_distances(cT, eG, s)
    np.testing.assert_array_equal(np.isinf(d), np.isinf(ref))
    np.testing.assert_array_equal(d, ref)
    reach = np.argwhere(np.isfinite(d))
    assert len(reach) > 1
    for t in range(5):
        l, y, x = reach[int(rng.integers(len(reach)))]
        g = (int(x), int(y), int(l))
        p = oracle.plan_path(cT, eG, CB, d, s, g)
        check_path(p, d, cT, eG, s, g)


def one_row(c0, c1, e1):
    """Two layers over a 6 x 1 map: layer 0 a floor at height 0, layer 1 an
    upper floor at height 3 except cells whose ground is the floor's."""
    cT = np.array([[c0], [c1]], np.float32)
    eG = np.array([[[0, 0, 0, 0, 0, 0]], [e1]], np.float32)
    return cT, eG


def test_gateway_up_merged_cost():
    # cell 2 of layer 1 lies on the floor with a lower cost: a gateway
    cT, eG = one_row([5, 5, 5, 5, 5, 5], [2, 2, 1, 2, 2, 2], [3, 3, 0, 3, 3, 3])
    d = oracle.plan(cT, eG, CB, (0, 0, 0))
    # floor: 5+1, then cell 2 at the merged cost min(5, 1) + 1; gateway; upper floor 2+1 per cell
    assert d[0, 0, 1] == 6.0 and d[0, 0, 2] == 8.0 and d[1, 0, 2] == 8.0
    assert list(d[1, 0, 3:]) == [11.0, 14.0, 17.0]
    assert list(d[1, 0, :2]) == [14.0, 11.0]   # reached on layer 1 from the gateway, not from below
    p = oracle.plan_path(cT, eG, CB, d, (0, 0, 0), (5, 0, 1))
    assert [tuple(r) for r in p] == [(0, 0, 0), (1, 0, 0), (2, 0, 0), (2, 0, 1), (3, 0, 1), (4, 0, 1), (5, 0, 1)]
    check_path(p, d, cT, eG, (0, 0, 0), (5, 0, 1))


def test_gateway_needs_strictly_lower_cost():
    cT, eG = one_row([5, 5, 5, 5, 5, 5], [2, 2, 5, 2, 2, 2], [3, 3, 0, 3, 3, 3])
    d = oracle.plan(cT, eG, CB, (0, 0, 0))
    assert np.isinf(d[1]).all()
    assert oracle.plan_path(cT, eG, CB, d, (0, 0, 0), (5, 0, 1)) is None


def test_gateway_down():
    cT, eG = one_row([5, 5, 0.5, 5, 5, 5], [2, 2, 1, 2, 2, 2], [3, 3, 0, 3, 3, 3])
    d = oracle.plan(cT, eG, CB, (5, 0, 1))
    assert list(d[1, 0, 2:]) == [7.5, 6.0, 3.0, 0.0]      # merged cost min(1, 0.5) at cell 2
    assert d[0, 0, 2] == 7.5 and d[0, 0, 1] == 13.5 and d[0, 0, 0] == 19.5
    check_path(oracle.plan_path(cT, eG, CB, d, (5, 0, 1), (0, 0, 0)), d, cT, eG, (5, 0, 1), (0, 0, 0))


def test_barriers_and_start_on_barrier():
    nx, ny = 12, 9
    cT = np.full((1, ny, nx), 1.0, np.float32)
    eG = np.zeros((1, ny, nx), np.float32)
    cT[0, :, 6] = CB                      # a wall
    d = oracle.plan(cT, eG, CB, (0, 4, 0))
    assert np.isinf(d[0, :, 6:]).all() and np.isfinite(d[0, :, :6]).all()
    cT[0, 8, 6] = 1.0                     # a gap at the bottom row
    d = oracle.plan(cT, eG, CB, (0, 4, 0))
    assert np.isfinite(d).sum() == d.size - (ny - 1) and np.isinf(d[0, :8, 6]).all()
    p = oracle.plan_path(cT, eG, CB, d, (0, 4, 0), (11, 4, 0))
    assert (6, 8, 0) in [tuple(r) for r in p]
    check_path(p, d, cT, eG, (0, 4, 0), (11, 4, 0))
    cT[0, 4, 0] = CB                      # the start itself may be a barrier
    d2 = oracle.plan(cT, eG, CB, (0, 4, 0))
    assert d2[0, 4, 0] == 0.0 and d2[0, 4, 1] == 2.0


def test_start_equals_goal_and_bad_nodes():
    cT = np.ones((2, 3, 4), np.float32)
    eG = np.zeros((2, 3, 4), np.float32)
    d = oracle.plan(cT, eG, CB, (1, 1, 1))
    p = oracle.plan_path(cT, eG, CB, d, (1, 1, 1), (1, 1, 1))
    assert [tuple(r) for r in p] == [(1, 1, 1)]
    with pytest.raises(ValueError):
        oracle.plan(cT, eG, CB, (4, 0, 0))
    assert oracle.plan_path(cT, eG, CB, d, (1, 1, 1), (0, 0, 0)) is None   # equal costs: no gateway
    with pytest.raises(ValueError):
        oracle.plan_path(cT, eG, CB, d, (1, 1, 1), (0, 0, 1), max_len=1)
