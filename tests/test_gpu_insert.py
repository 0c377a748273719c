"""GPU checks of incremental updates (streaming scans), through the C ABI.

An insertion into an existing tomogram must equal the build of the union of
old and new points bit for bit (heights and point ids; the oracle's literal
construction of the union agrees), and re-evaluating the window around the
new points must leave the cost map and keep flags equal to a whole-map
evaluation of the union."""
import sys

import numpy as np
import pytest

import scenes

pytestmark = pytest.mark.gpu


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


def bits(t):
    a = t.detach().cpu().numpy() if hasattr(t, "detach") else np.asarray(t)
    return a.view(np.uint32) if a.dtype == np.float32 else a


def box_scan(seed, x, y, z, m):
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(np.column_stack([rng.uniform(*x, m), rng.uniform(*y, m), rng.uniform(*z, m)]),
                                np.float32)


def insert_and_check(P, pts, new, g, robot, oracle_lib=None):
    import torch
    dev = torch.device("cuda")
    xyz = torch.from_numpy(pts).to(dev)
    ext = P.pct_tomogram_extent(xyz, g)
    G, Cc, aG, aC = P.pct_build_tomogram(xyz, g, ext, with_ids=True)
    cost, keep = P.pct_eval_traversability(G, Cc, g, ext, [robot])
    cost, keep = cost[0].contiguous(), keep[0].contiguous()
    bb = P.pct_tomogram_insert(torch.from_numpy(new).to(dev), g, ext, G, Cc, aG, aC, id_base=len(pts))
    grow = P.pct_kernel_radius(robot, g["res"]) + 2
    win = (bb[0] - grow, bb[1] - grow, bb[2] + 1 + grow, bb[3] + 1 + grow)
    P.pct_eval_traversability_window(G, Cc, g, ext, robot, win, cost, keep)
    union = np.ascontiguousarray(np.concatenate([pts, new]), np.float32)
    xu = torch.from_numpy(union).to(dev)
    eu = P.pct_tomogram_extent(xu, g)
    Gu, Cu, aGu, aCu = P.pct_build_tomogram(xu, g, eu, with_ids=True)
    cu, ku = P.pct_eval_traversability(Gu, Cu, g, eu, [robot])
    torch.cuda.synchronize()
    assert (ext.n_slices, ext.n_used, ext.n_dropped) == (eu.n_slices, eu.n_used, eu.n_dropped)
    assert np.float32(ext.z_max) == np.float32(eu.z_max)
    for a, b in ((G, Gu), (Cc, Cu), (aG, aGu), (aC, aCu), (cost, cu[0]), (keep, ku[0])):
        np.testing.assert_array_equal(bits(a), bits(b))
    if oracle_lib is not None:
        tm = oracle_lib.tomogram(union, g)
        np.testing.assert_array_equal(bits(G), bits(tm["ground"]))
        np.testing.assert_array_equal(bits(Cc), bits(tm["ceil"]))
        np.testing.assert_array_equal(aG.cpu().numpy(), tm["arg_ground"])
        np.testing.assert_array_equal(aC.cpu().numpy(), tm["arg_ceil"])
    return bb, win


def test_insert_matches_union(P, oracle_lib):
    sc = scenes.multistorey_scene(45, 13.3, 9.7, 300_000, n_floors=2)
    r = P.robot_from_physical(sc.robot, sc.grid["res"])
    new = box_scan(10, (3.0, 4.7), (2.0, 3.3), (0.0, 0.9), 40_000)
    bb, win = insert_and_check(P, sc.points, new, sc.grid, r, oracle_lib)
    say(f"insert: box {bb}, window {win}: equal to the union's build and evaluation and the oracle's")
    # a scan along the map edge, with points outside the grid and duplicates of old heights
    new = box_scan(11, (-1.0, 2.0), (-0.5, 9.7), (0.0, 2.5), 30_000)
    new[:1000] = sc.points[:1000]
    insert_and_check(P, sc.points, new, sc.grid, r, oracle_lib)


def test_insert_refuses_new_planes(P):
    import torch
    sc = scenes.multistorey_scene(46, 6.3, 5.7, 80_000, n_floors=2)
    g = sc.grid
    xyz = torch.from_numpy(sc.points).cuda()
    ext = P.pct_tomogram_extent(xyz, g)
    G, Cc, _, _ = P.pct_build_tomogram(xyz, g, ext)
    before = G.clone()
    for z in (ext.z_min - 0.5, ext.z_min + ext.n_slices * g["slice_dz"] + 1.0):
        with pytest.raises(P.PctError) as e:
            P.pct_tomogram_insert(torch.tensor([[1.0, 1.0, z]], device="cuda"), g, ext, G, Cc)
        assert e.value.status == P.PCT_ERR_ARG
    torch.cuda.synchronize()
    np.testing.assert_array_equal(bits(G), bits(before))


def test_insert_full_size_building(P):
    """A 200 k-point scan into the 26.4 M-point building: the updated
    tomogram, costs and keep flags equal the union's, bit for bit."""
    sc = scenes.plan_building()
    r = dict(scenes.ROBOT_TABLE1)
    new = box_scan(12, (40.0, 46.0), (55.0, 61.0), (0.0, 14.0), 200_000)
    bb, win = insert_and_check(P, sc.points, new, sc.grid, r)
    say(f"full-size insert: box {bb}, window {win}: equal to the union's")


def test_insert_degenerate_cases(P):
    """No points, points outside the grid only, a window outside the grid and
    a whole-map window."""
    import torch
    sc = scenes.multistorey_scene(47, 6.3, 5.7, 80_000, n_floors=2)
    g = sc.grid
    r = P.robot_from_physical(sc.robot, g["res"])
    xyz = torch.from_numpy(sc.points).cuda()
    ext = P.pct_tomogram_extent(xyz, g)
    G, Cc, aG, aC = P.pct_build_tomogram(xyz, g, ext, with_ids=True)
    cost, keep = P.pct_eval_traversability(G, Cc, g, ext, [r])
    cost, keep = cost[0].contiguous(), keep[0].contiguous()
    before = [t.clone() for t in (G, Cc, aG, aC, cost, keep)]
    n_used, n_dropped = ext.n_used, ext.n_dropped
    bb = P.pct_tomogram_insert(torch.zeros((0, 3), device="cuda"), g, ext, G, Cc, aG, aC, id_base=len(sc.points))
    assert bb[2] < bb[0] and (ext.n_used, ext.n_dropped) == (n_used, n_dropped)
    outside = torch.tensor([[-5.0, 1.0, 0.5], [1.0, 100.0, 0.5], [float("nan"), 1.0, 0.5]], device="cuda")
    bb = P.pct_tomogram_insert(outside, g, ext, G, Cc, aG, aC, id_base=len(sc.points))
    assert bb[2] < bb[0] and (ext.n_used, ext.n_dropped) == (n_used, n_dropped + 3)
    P.pct_eval_traversability_window(G, Cc, g, ext, r, (-50, -50, -10, -10), cost, keep)
    P.pct_eval_traversability_window(G, Cc, g, ext, r, (g["nx"] + 5, 0, g["nx"] + 9, g["ny"]), cost, keep)
    torch.cuda.synchronize()
    for a, b in zip((G, Cc, aG, aC, cost, keep), before):
        np.testing.assert_array_equal(bits(a), bits(b))
    # a window covering the map (and more) equals the whole-map evaluation
    cost.fill_(-1.0)
    P.pct_eval_traversability_window(G, Cc, g, ext, r, (-3, -3, g["nx"] + 3, g["ny"] + 3), cost, keep)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(bits(cost), bits(before[4]))
    np.testing.assert_array_equal(bits(keep), bits(before[5]))
