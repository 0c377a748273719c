"""GPU checks of the path search through the slices (Sec. III-D), through
the C ABI.

Distances are FP64 least rounded path sums, which every order of
relaxations reaches, so the library's must equal the oracle's Dijkstra bit
for bit; paths, read back with the same tie rule, must be identical.  At the
benchmark's size, where the oracle is not run here, the distance field is
checked against the Bellman equations of the graph at every node (no edge
can lower a node; every reached node but the start has an edge that gives
its value exactly): with positive planar steps and gateways only to
cheaper layers, that holds for the least fixed point alone."""
import math
import sys

import numpy as np
import pytest

import scenes

pytestmark = pytest.mark.gpu
CB = 50.0


def say(msg):
    print(f"[gpu] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2403_07631_amd as P
    P.lib()
    return P


def extent_of(N):
    import paper_2403_07631_amd as P
    return P.pct_extent(0.0, 1.0, N, 0, 0, 0)


def grid_of(ny, nx):
    return dict(x0=0.0, y0=0.0, res=0.1, nx=nx, ny=ny, slice_dz=0.3)


def robot_cb(P, cb=CB):
    r = P.robot_from_physical(scenes.ROBOT_CONFIG0, 0.1).as_dict()
    r["c_barrier"] = cb
    return r


def gpu_plan(P, cT, eG, layers, start, goals, cb=CB):
    import torch
    N, ny, nx = cT.shape
    c = torch.from_numpy(np.ascontiguousarray(cT, np.float32)).cuda()
    e = torch.from_numpy(np.ascontiguousarray(eG, np.float32)).cuda()
    g = grid_of(ny, nx)
    dist, ws, info = P.pct_plan_distance(c, e, g, extent_of(N), robot_cb(P, cb), layers, start)
    paths = [P.pct_plan_path(dist, g, start, goal, ws) for goal in goals]
    torch.cuda.synchronize()
    return dist.cpu().numpy(), [None if p is None else p.cpu().numpy() for p in paths], info


def check_against_oracle(P, oracle_lib, cT, eG, layers, start, goals, what, cb=CB):
    say(f"plan {what}: {len(layers)} x {cT.shape[1]} x {cT.shape[2]}")
    d, paths, info = gpu_plan(P, cT, eG, layers, start, goals, cb)
    ref = oracle_lib.plan(cT[layers], eG[layers], cb, start)
    np.testing.assert_array_equal(d.view(np.uint64), ref.view(np.uint64))
    n = 0
    for goal, p in zip(goals, paths):
        rp = oracle_lib.plan_path(cT[layers], eG[layers], cb, ref, start, goal)
        if rp is None:
            assert p is None
            continue
        rp[:, 2] = np.asarray(layers)[rp[:, 2]]
        np.testing.assert_array_equal(p, rp)
        n += 1
    say(f"plan {what}: bit-exact, {int(np.isfinite(ref).sum())} reachable, {info['rounds']} rounds, "
        f"{info['tiles']} tiles, {n} paths")
    return d, ref


def test_random_layers(P, oracle_lib):
    cT, eG = scenes.plan_layers(11, 3, 150, 130)
    rng = np.random.default_rng(5)
    goals = [(int(rng.integers(130)), int(rng.integers(150)), int(rng.integers(3))) for _ in range(6)]
    check_against_oracle(P, oracle_lib, cT, eG, [0, 1, 2], (7, 140, 0), goals, "random layers")


def test_many_tiles_and_subsets(P, oracle_lib):
    # hundreds of tiles per round in parallel; a subset of the slices
    cT, eG = scenes.plan_layers(21, 6, 700, 517, p_block=0.25, p_same=0.4)
    rng = np.random.default_rng(6)
    layers = [0, 1, 3, 4, 5]
    goals = [(int(rng.integers(517)), int(rng.integers(700)), int(rng.integers(5))) for _ in range(8)]
    check_against_oracle(P, oracle_lib, cT, eG, layers, (258, 350, 2), goals, "700x517, 5 of 6 slices")


def test_serpentine_and_edges(P, oracle_lib):
    cT, eG = scenes.plan_serpentine(13, 300, 257, pitch=6)
    check_against_oracle(P, oracle_lib, cT, eG, [0], (0, 0, 0), [(0, 299, 0), (256, 150, 0)], "serpentine")
    cT, eG = scenes.plan_layers(14, 2, 64, 64, p_block=0.6)
    cT[0, 10, 10] = CB
    check_against_oracle(P, oracle_lib, cT, eG, [0, 1], (10, 10, 0), [(63, 63, 1), (0, 0, 0)], "barrier start")
    cT = np.full((1, 1, 1), 3.0, np.float32)
    check_against_oracle(P, oracle_lib, cT, np.zeros_like(cT), [0], (0, 0, 0), [(0, 0, 0)], "single cell")
    cT = np.full((2, 1, 300), 2.0, np.float32)
    eG = np.zeros_like(cT)
    eG[1] += 1.0
    check_against_oracle(P, oracle_lib, cT, eG, [0, 1], (299, 0, 0), [(0, 0, 0), (5, 0, 1)], "one row")


def test_tomogram_building(P, oracle_lib):
    """The section's setting: slices kept by the oracle's slice test of a
    three-storey building with stairs, Table I quadruped; the path climbs
    through the layers by gateways."""
    sc = scenes.multistorey_scene(41, 20.0, 15.0, 396_000, n_floors=3)
    g = sc.grid
    tm = oracle_lib.tomogram(sc.points, g)
    r = dict(scenes.ROBOT_TABLE1)
    cT = oracle_lib.evaluate(tm["ground"], tm["ceil"], g["res"], r).astype(np.float32)
    layers = [int(v) for v in np.flatnonzero(oracle_lib.simplify(tm["ground"], cT.astype(np.float64), r["c_barrier"]))]
    eG = tm["ground"]
    trav = cT[layers] < r["c_barrier"]

    def pick(li, zlo, zhi):
        gl = eG[layers[li]]
        m = trav[li] & (gl > zlo) & (gl < zhi)
        ys, xs = np.nonzero(m)
        k = np.argmin((ys - g["ny"] / 2) ** 2 + (xs - g["nx"] / 2) ** 2)
        return (int(xs[k]), int(ys[k]), li)

    s = pick(0, -1.0, 0.5)
    goal = pick(len(layers) - 1, 5.5, 6.5)
    d, ref = check_against_oracle(P, oracle_lib, cT, eG, layers, s, [goal], "three-storey building",
                                  cb=r["c_barrier"])
    assert np.isfinite(ref[goal[2], goal[1], goal[0]])


def bellman_check(d, cT, eG, layers, start, cb):
    """Every edge satisfies d(v) <= d(u) + w(u, v), and every reached node
    but the start meets one with equality (vectorised over the map)."""
    cL = cT[layers].astype(np.float64)
    gL = eG[layers]
    L, ny, nx = cL.shape
    cn = cL.copy()
    same_up = np.zeros(cL.shape, bool)
    same_dn = np.zeros(cL.shape, bool)
    same_up[:-1] = gL[1:] == gL[:-1]
    same_dn[1:] = gL[:-1] == gL[1:]
    cn[:-1] = np.where(same_up[:-1], np.minimum(cn[:-1], cL[1:]), cn[:-1])
    cn[1:] = np.where(same_dn[1:], np.minimum(cn[1:], cL[:-1]), cn[1:])
    best = np.full(d.shape, np.inf)
    ok = cn < np.float64(np.float32(cb))
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dx == 0 and dy == 0:
                continue
            w = cn + (math.sqrt(2.0) if dx and dy else 1.0)
            src = np.full(d.shape, np.inf)
            ys = slice(max(0, -dy), ny - max(0, dy))
            yt = slice(max(0, dy), ny - max(0, -dy))
            xs = slice(max(0, -dx), nx - max(0, dx))
            xt = slice(max(0, dx), nx - max(0, -dx))
            src[:, yt, xt] = d[:, ys, xs]
            cand = np.where(ok, src + w, np.inf)
            np.minimum(best, cand, out=best)
    up = same_up[:-1] & (cL[1:] < cL[:-1])   # gateway l -> l+1 lands on l+1
    best[1:] = np.where(up, np.minimum(best[1:], d[:-1] + 0.0), best[1:])
    dn = same_dn[1:] & (cL[:-1] < cL[1:])    # gateway l+1 -> l lands on l
    best[:-1] = np.where(dn, np.minimum(best[:-1], d[1:] + 0.0), best[:-1])
    assert not (best < d).any(), "an edge lowers a node"
    reached = np.isfinite(d)
    reached[start[2], start[1], start[0]] = False
    assert (best[reached] == d[reached]).all(), "a reached node has no tight in-edge"
    assert d[start[2], start[1], start[0]] == 0.0


def test_full_size_building(P):
    """The benchmark's map (100 m x 100 m, six storeys without beams, 4 points
    per cell and storey, Table I quadruped): the GPU pipeline builds, evaluates and keeps
    slices; the path search from the ground-floor centre is checked against
    the Bellman equations at all nodes, and the path to the farthest reached
    node is valid with the exact cost."""
    import torch
    sc = scenes.plan_building()
    g = sc.grid
    say(f"full-size building: {len(sc.points)} points, {g['nx']}x{g['ny']}")
    xyz = torch.from_numpy(sc.points).cuda()
    ext = P.pct_tomogram_extent(xyz, g)
    G, Cc, _, _ = P.pct_build_tomogram(xyz, g, ext, with_ids=False)
    r = dict(scenes.ROBOT_TABLE1)
    cost, keep = P.pct_eval_traversability(G, Cc, g, ext, [r])
    cost = cost[0].contiguous()
    layers = [int(v) for v in np.flatnonzero(keep[0].cpu().numpy())]
    cT, eG = cost.cpu().numpy(), G.cpu().numpy()
    trav = cT[layers[0]] < r["c_barrier"]
    ys, xs = np.nonzero(trav & (eG[layers[0]] < 0.5))
    k = np.argmin((ys - g["ny"] / 2) ** 2 + (xs - g["nx"] / 2) ** 2)
    s = (int(xs[k]), int(ys[k]), 0)
    say(f"full-size building: {len(layers)} layers, start {s}")
    dist, ws, info = P.pct_plan_distance(cost, G, g, ext, r, layers, s)
    d = dist.cpu().numpy()
    say(f"full-size building: {int(np.isfinite(d).sum())} reached, {info['rounds']} rounds, {info['tiles']} tiles")
    bellman_check(d, cT, eG, layers, s, r["c_barrier"])
    fin = np.where(np.isfinite(d), d, -1.0)
    l, y, x = np.unravel_index(int(np.argmax(fin)), d.shape)
    goal = (int(x), int(y), int(l))
    p = P.pct_plan_path(dist, g, s, goal, ws).cpu().numpy()
    # rows are slice indices; walk the path with the layer positions
    pos = {v: i for i, v in enumerate(layers)}
    pl = np.column_stack([p[:, 0], p[:, 1], [pos[v] for v in p[:, 2]]])
    assert tuple(pl[0]) == s and tuple(pl[-1]) == goal
    tot = 0.0
    cL, gL = cT[layers], eG[layers]
    for (x0, y0, l0), (x1, y1, l1) in zip(pl[:-1], pl[1:]):
        if l0 == l1:
            c = float(cL[l1, y1, x1])
            for m in (l1 - 1, l1 + 1):
                if 0 <= m < len(layers) and gL[m, y1, x1] == gL[l1, y1, x1]:
                    c = min(c, float(cL[m, y1, x1]))
            tot = tot + (c + (math.sqrt(2.0) if x1 != x0 and y1 != y0 else 1.0))
        else:
            assert gL[l1, y1, x1] == gL[l0, y0, x0] and cL[l1, y1, x1] < cL[l0, y0, x0]
            tot = tot + 0.0
    assert tot == d[goal[2], goal[1], goal[0]]
    say(f"full-size building: path of {len(p)} nodes to the farthest node, cost {tot:.3f}")
    # the benchmark's single query: a goal 26.5 m away on the start layer
    ys, xs = np.nonzero(np.isfinite(d[0]))
    kq = int(np.argmin(np.abs(np.hypot(xs - s[0], ys - s[1]) - 265.0)))
    qgoal = (int(xs[kq]), int(ys[kq]), 0)
    dq, wq, qi = P.pct_plan_query(cost, G, g, ext, r, layers, s, qgoal)
    dqn = dq.cpu().numpy()
    settled = dqn < qi["settled"]
    assert qi["goal_dist"] == d[0, qgoal[1], qgoal[0]]
    np.testing.assert_array_equal(dqn[settled].view(np.uint64), d[settled].view(np.uint64))
    assert np.all(dqn[~settled] >= d[~settled])
    pq = P.pct_plan_path(dq, g, s, qgoal, wq).cpu().numpy()
    np.testing.assert_array_equal(pq, P.pct_plan_path(dist, g, s, qgoal, ws).cpu().numpy())
    say(f"full-size building: query to {qgoal} in {qi['rounds']} rounds, same cost and path as the full field")


def check_query(P, oracle_lib, cT, eG, layers, start, goals, what, cb=CB):
    """Goal-directed queries: the goal's distance and path equal the oracle's
    full search; every label below the settled bound equals the oracle's;
    the query takes no more rounds than the full search."""
    import torch
    N, ny, nx = cT.shape
    c = torch.from_numpy(np.ascontiguousarray(cT, np.float32)).cuda()
    e = torch.from_numpy(np.ascontiguousarray(eG, np.float32)).cuda()
    g = grid_of(ny, nx)
    ref = oracle_lib.plan(cT[layers], eG[layers], cb, start)
    _, _, full = P.pct_plan_distance(c, e, g, extent_of(N), robot_cb(P, cb), layers, start)
    for goal in goals:
        dist, ws, info = P.pct_plan_query(c, e, g, extent_of(N), robot_cb(P, cb), layers, start, goal)
        d = dist.cpu().numpy()
        want = ref[goal[2], goal[1], goal[0]]
        assert np.float64(info["goal_dist"]).view(np.uint64) == np.float64(want).view(np.uint64)
        settled = d < info["settled"]
        np.testing.assert_array_equal(d[settled].view(np.uint64), ref[settled].view(np.uint64))
        assert np.all(d[~settled] >= ref[~settled])
        assert info["rounds"] <= full["rounds"]
        p = P.pct_plan_path(dist, g, start, goal, ws)
        rp = oracle_lib.plan_path(cT[layers], eG[layers], cb, ref, start, goal)
        if rp is None:
            assert p is None
        else:
            rp[:, 2] = np.asarray(layers)[rp[:, 2]]
            np.testing.assert_array_equal(p.cpu().numpy(), rp)
        say(f"query {what} to {goal}: distance and path equal the full search's, {info['rounds']} of "
            f"{full['rounds']} rounds, {int(settled.sum())} labels settled")


def test_goal_directed_queries(P, oracle_lib):
    cT, eG = scenes.plan_layers(21, 6, 700, 517, p_block=0.25, p_same=0.4)
    layers = [0, 1, 3, 4, 5]
    check_query(P, oracle_lib, cT, eG, layers, (258, 350, 2),
                [(270, 360, 2), (300, 420, 0), (10, 10, 4), (258, 350, 2)], "700x517")
    cT, eG = scenes.plan_serpentine(13, 300, 257, pitch=6)
    check_query(P, oracle_lib, cT, eG, [0], (0, 0, 0), [(0, 40, 0), (256, 150, 0)], "serpentine")
    cT, eG = scenes.plan_layers(14, 2, 64, 64, p_block=0.6)
    check_query(P, oracle_lib, cT, eG, [0, 1], (10, 10, 0), [(63, 63, 1), (11, 10, 0)], "sparse")
