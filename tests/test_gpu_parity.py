"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Tomograms must match bit for bit (heights and point ids).  Costs must lie in
[lo - 1e-5, hi + 1e-5], where lo/hi is the oracle's FP64 envelope (lo = hi =
the FP64 value except where an Eq. (1)-(4) predicate sits within rounding of
its threshold).  Keep lists must be admissible under the oracle's
three-valued slice test."""
import sys

import numpy as np
import pytest

import scenes

pytestmark = pytest.mark.gpu
TOL = 1e-5


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


def bits(a):
    a = np.ascontiguousarray(a)
    return a.view(np.uint32) if a.dtype == np.float32 else a


def gpu_tomogram(P, pts, grid, ids=True):
    import torch
    xyz = torch.from_numpy(np.ascontiguousarray(pts, np.float32)).cuda()
    ext = P.pct_tomogram_extent(xyz, grid)
    if ext.n_slices == 0:
        return ext, None
    g, c, ag, ac = P.pct_build_tomogram(xyz, grid, ext, with_ids=ids)
    torch.cuda.synchronize()
    out = [g.cpu().numpy(), c.cpu().numpy()]
    out += [ag.cpu().numpy(), ac.cpu().numpy()] if ids else [None, None]
    return ext, out


def check_tomogram(P, oracle_lib, pts, grid, ids=True):
    say(f"build n={len(pts)} grid={grid['nx']}x{grid['ny']} ids={ids}")
    ext, out = gpu_tomogram(P, pts, grid, ids)
    tm = oracle_lib.tomogram(pts, grid)
    assert ext.n_used == tm["n_used"]
    assert ext.n_dropped == len(pts) - tm["n_used"]
    assert ext.n_slices == len(tm["h"])
    if ext.n_slices == 0:
        return ext, tm, None
    assert np.float32(ext.z_min) == np.float32(tm["zmin"]) and np.float32(ext.z_max) == np.float32(tm["zmax"])
    np.testing.assert_array_equal(P.pct_plane_heights(ext, grid["slice_dz"]), tm["h"])
    np.testing.assert_array_equal(bits(out[0]), bits(tm["ground"]))
    np.testing.assert_array_equal(bits(out[1]), bits(tm["ceil"]))
    if ids:
        np.testing.assert_array_equal(out[2], tm["arg_ground"])
        np.testing.assert_array_equal(out[3], tm["arg_ceil"])
    return ext, tm, out


def crop_scene(seed=21, lx=31.7, ly=23.3, n=500_000):
    return scenes.multistorey_scene(seed, lx, ly, n, n_floors=6)


# --------------------------------------------------------------- construction


def test_tiny_golden(P, oracle_lib):
    from conftest import load_golden
    g = load_golden("tiny_tomogram.json")
    pts = np.array(g["points"], dtype=np.float32)
    ext, tm, out = check_tomogram(P, oracle_lib, pts, g["grid"])
    np.testing.assert_array_equal(out[0], np.array(g["ground"], np.float32))
    np.testing.assert_array_equal(out[3], np.array(g["arg_ceil"], np.int32))
    assert not np.signbit(out[0][0, 1, 2])




@pytest.mark.parametrize("name", ["config0", "crop", "dense"])
@pytest.mark.parametrize("ids", [True, False])
def test_build_parity(P, oracle_lib, name, ids):
    if name == "config0":
        sc = scenes.config0_scene()
    elif name == "crop":
        sc = crop_scene()
    else:
        sc = scenes.multistorey_scene(22, 13.3, 9.1, 600_000, n_floors=3)
    check_tomogram(P, oracle_lib, sc.points, sc.grid, ids)


def test_build_edge_cases(P, oracle_lib):
    rng = np.random.default_rng(5)
    grid = dict(x0=-1.0, y0=2.0, res=0.125, nx=130, ny=19, slice_dz=0.25)
    # nothing inside the grid
    pts = np.array([[-5, 3, 1], [100, 3, 1], [0, np.nan, 1], [0, 3, np.inf]], np.float32)
    say("edge: empty map")
    ext, _ = gpu_tomogram(P, pts, grid)
    assert ext.n_slices == 0 and ext.n_used == 0 and ext.n_dropped == 4
    # one point
    check_tomogram(P, oracle_lib, np.array([[0.0, 2.5, -0.0]], np.float32), grid)
    # a cell far beyond the LDS capacity, with heavy ties, plus a tile over
    # capacity spread over many cells, plus junk and -0
    huge = np.column_stack([np.full(20_000, 0.3), np.full(20_000, 2.3),
                            rng.choice([-0.0, 0.25, 0.5, 1.0, 1.75], 20_000)]).astype(np.float32)
    spread = np.column_stack([rng.uniform(-1.0, 7.0, 9000), rng.uniform(2.0, 3.0, 9000),
                              np.round(rng.uniform(-0.5, 2.0, 9000), 2)]).astype(np.float32)
    junk = np.array([[np.nan, 2.5, 0], [0, 2.5, np.nan], [1e30, 2.5, 0], [0.0, 2.0 + 19 * 0.125, 0.5]],
                    np.float32)
    pts = np.concatenate([spread[:4000], huge, junk, spread[4000:]])
    check_tomogram(P, oracle_lib, pts, grid)
    # points exactly on plane heights and cell edges
    e = np.column_stack([-1.0 + 0.125 * rng.integers(0, 130, 3000), 2.0 + 0.125 * rng.integers(0, 19, 3000),
                         0.25 * rng.integers(0, 12, 3000)]).astype(np.float32)
    check_tomogram(P, oracle_lib, e, grid)


def test_build_deterministic(P):
    sc = crop_scene(seed=23, n=300_000)
    say("determinism")
    _, a = gpu_tomogram(P, sc.points, sc.grid)
    _, b = gpu_tomogram(P, sc.points, sc.grid)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(bits(x), bits(y))


# --------------------------------------------------------------- evaluation

def gpu_eval(P, pts, grid, robots):
    import torch
    xyz = torch.from_numpy(np.ascontiguousarray(pts, np.float32)).cuda()
    ext = P.pct_tomogram_extent(xyz, grid)
    g, c, _, _ = P.pct_build_tomogram(xyz, grid, ext)
    cost, keep = P.pct_eval_traversability(g, c, grid, ext, robots)
    torch.cuda.synchronize()
    return ext, g.cpu().numpy(), c.cpu().numpy(), cost.cpu().numpy(), keep.cpu().numpy()


def check_eval(P, oracle_lib, pts, grid, robot_dicts, label=""):
    rbs = [P.robot_struct(r) for r in robot_dicts]
    say(f"eval {label} grid={grid['nx']}x{grid['ny']} robots={len(rbs)}")
    ext, eG, eC, cost, keep = gpu_eval(P, pts, grid, rbs)
    stats = []
    for i, rb in enumerate(rbs):
        r = rb.as_dict()
        lo, hi, n_amb = oracle_lib.envelope(eG, eC, grid["res"], r)
        c = cost[i].astype(np.float64)
        below = c < lo - TOL
        above = c > hi + TOL
        assert not below.any() and not above.any(), (
            f"robot {i}: {below.sum()} below, {above.sum()} above; worst "
            f"{np.max(np.maximum(lo - c, c - hi))}")
        exact = lo == hi
        err = float(np.max(np.abs(c[exact] - lo[exact]))) if exact.any() else 0.0
        bad = oracle_lib.simplify_check(eG, lo, hi, r["c_barrier"], TOL, keep[i])
        assert bad == -1, f"robot {i}: keep decision at slice {bad} contradicts the slice test"
        stats.append((err, n_amb, int(keep[i].sum()), int((c < r["c_barrier"]).sum())))
    say(f"  max|err| / ambiguous / kept / traversable: {stats}")
    return stats


def robot(**kw):
    import oracle
    r = oracle.robot_from_physical(scenes.ROBOT_CONFIG0, 0.1)
    r.update(kw)
    return r


def test_eval_config0(P, oracle_lib):
    sc = scenes.config0_scene()
    check_eval(P, oracle_lib, sc.points, sc.grid, [robot()], "config0")


def test_eval_dense_multistorey(P, oracle_lib):
    sc = scenes.multistorey_scene(31, 14.1, 10.3, 900_000, n_floors=3)
    stats = check_eval(P, oracle_lib, sc.points, sc.grid, [robot()], "dense")
    assert stats[0][3] > 1000     # plenty of traversable cells


@pytest.mark.parametrize("kw", [dict(), dict(d_inf=0.05, d_sm=0.15), dict(d_inf=0.8, d_sm=0.9),
                                dict(d_inf=1.2, d_sm=0.5), dict(patch_radius=2, theta_p=0.45),
                                dict(theta_p=1.0), dict(d_min=0.3, d_ref=0.65, theta_b=1.7, theta_s=0.36)])
def test_eval_robot_variants(P, oracle_lib, kw):
    sc = scenes.multistorey_scene(32, 9.7, 7.9, 500_000, n_floors=2)
    check_eval(P, oracle_lib, sc.points, sc.grid, [robot(**kw)], str(kw))


def test_eval_analytic_scenes(P, oracle_lib):
    res = 0.1
    for name, fn in [("ramp", lambda x, y: 0.17 * x), ("steps", lambda x, y: 0.15 * np.floor(x / 0.6)),
                     ("bowl", lambda x, y: 0.2 * ((x - 3) ** 2 + (y - 2) ** 2))]:
        sc = scenes.dense_surface_scene(70, 45, res, fn, per_cell=4, slice_dz=0.3)
        check_eval(P, oracle_lib, sc.points, sc.grid, [robot()], name)


def test_eval_many_robots_match_single(P, oracle_lib):
    sc = scenes.multistorey_scene(33, 8.3, 6.1, 300_000, n_floors=2)
    rs = [robot(), robot(d_min=0.7, theta_s=0.3), robot(d_inf=0.5, d_sm=0.7)]
    say("multi-robot")
    ext, eG, eC, cost, keep = gpu_eval(P, sc.points, sc.grid, [P.robot_struct(r) for r in rs])
    for i, r in enumerate(rs):
        _, _, _, c1, k1 = gpu_eval(P, sc.points, sc.grid, [P.robot_struct(r)])
        np.testing.assert_array_equal(bits(cost[i]), bits(c1[0]))
        np.testing.assert_array_equal(keep[i], k1[0])


def test_autotune_keeps_results(P):
    """Tuning the strip height changes no value of the evaluation, on a map
    with traversable cells."""
    import torch
    sc = scenes.multistorey_scene(24, 14.1, 10.3, 900_000, n_floors=3)
    xyz = torch.from_numpy(sc.points).cuda()
    ext = P.pct_tomogram_extent(xyz, sc.grid)
    g, c, _, _ = P.pct_build_tomogram(xyz, sc.grid, ext)
    rb = P.robot_struct(robot())
    say("autotune")
    before, kb = P.pct_eval_traversability(g, c, sc.grid, ext, [rb])
    best, cands = P.pct_autotune_traversability(g, c, sc.grid, ext, rb)
    after, ka = P.pct_eval_traversability(g, c, sc.grid, ext, [rb])
    torch.cuda.synchronize()
    P.pct_autotune_reset()
    assert best in cands and len(cands) >= 6
    assert int((before < rb.c_barrier).sum()) > 1000
    np.testing.assert_array_equal(bits(after.cpu().numpy()), bits(before.cpu().numpy()))
    np.testing.assert_array_equal(ka.cpu().numpy(), kb.cpu().numpy())


def test_building_every_strip_height(P, oracle_lib):
    """The benchmark building (26.4 M points, 1000 x 1000 cells, 51 slices)
    evaluated at every strip height the autotuner tries and at ragged ones,
    for the Table I quadruped (inflation radius 4) and for the large map's
    robot (radius 5, the benchmark's kernel): c^T equals the oracle's
    Eqs. (1)-(6) to 1e-5 on windows (interior, corner, edges) that each hold
    many traversable cells, every height gives the same bits, and the keep
    flags follow the slice test on the library's own arrays."""
    import torch
    sc = scenes.plan_building()
    grid = sc.grid
    say("building: build")
    xyz = torch.from_numpy(sc.points).cuda()
    ext = P.pct_tomogram_extent(xyz, grid)
    g, c, _, _ = P.pct_build_tomogram(xyz, grid, ext, with_ids=False)
    torch.cuda.synchronize()
    zmin, zmax, _ = oracle_lib.extent(sc.points, grid)
    h = oracle_lib.planes(zmin, zmax, grid["slice_dz"])
    assert ext.n_slices == len(h)
    M = 7   # margin: inflation radius 5 + patch radius 1 + stencil 1
    tomo = []
    for wx0, wy0, wn in [(500, 500, 48), (0, 0, 40), (980, 311, 20), (413, 975, 25)]:
        ex0, ey0 = max(0, wx0 - M), max(0, wy0 - M)
        ex1, ey1 = min(grid["nx"], wx0 + wn + M), min(grid["ny"], wy0 + wn + M)
        w = oracle_lib.build_window(sc.points, grid, h, ex0, ey0, ex1 - ex0, ey1 - ey0, ids=False)
        sl = (slice(None), slice(ey0, ey1), slice(ex0, ex1))
        np.testing.assert_array_equal(bits(g[sl].cpu().numpy()), bits(w[0]))
        np.testing.assert_array_equal(bits(c[sl].cpu().numpy()), bits(w[1]))
        tomo.append((wx0, wy0, wn, wy0 - ey0, wx0 - ex0, w))
    eG = g.cpu().numpy()
    for rname, rb in (("Table I", P.robot_struct(dict(scenes.ROBOT_TABLE1))),
                      ("large-map robot", P.robot_from_physical(scenes.ROBOT_CONFIG0, grid["res"]))):
        r = rb.as_dict()
        wins = []
        for wx0, wy0, wn, iy0, ix0, w in tomo:
            lo, hi, _ = oracle_lib.envelope(w[0], w[1], grid["res"], r)
            inner = (slice(None), slice(iy0, iy0 + wn), slice(ix0, ix0 + wn))
            assert int((lo[inner] < r["c_barrier"]).sum()) > 1000, (rname, wx0, wy0)
            wins.append((wx0, wy0, wn, lo[inner], hi[inner]))
        first = None
        try:
            for rows, waves in [(r_, w_) for w_ in (P.PCT_STRIP_WAVES, 2, 1)
                                for r_ in (32, 64, 128, 256, 512, 1024, 100, 1000)]:
                P.pct_autotune_set_traversability(grid, ext, rb, rows, waves)
                say(f"building, {rname}: strips of {rows} rows, {waves} wavefronts")
                cost, keep = P.pct_eval_traversability(g, c, grid, ext, [rb])
                torch.cuda.synchronize()
                for wx0, wy0, wn, lo, hi in wins:
                    cw = cost[0][:, wy0:wy0 + wn, wx0:wx0 + wn].cpu().numpy().astype(np.float64)
                    assert np.all(cw >= lo - TOL) and np.all(cw <= hi + TOL), (rname, rows, wx0, wy0)
                if first is None:
                    first = (cost, keep)
                    cT = cost[0].cpu().numpy().astype(np.float64)
                    assert oracle_lib.simplify_check(eG, cT, cT, r["c_barrier"], 0.0, keep[0].cpu().numpy()) == -1
                    assert 0 < int(keep.sum()) < ext.n_slices
                    del cT
                else:
                    assert torch.equal(cost.view(torch.int32), first[0].view(torch.int32)), (rname, rows, waves)
                    assert torch.equal(keep, first[1]), (rname, rows, waves)
        finally:
            P.pct_autotune_reset()


# --------------------------------------------------------------- full size


def test_full_size_config1_windows(P, oracle_lib):
    """The 20 M-point map at its full size, in the benchmark's launch
    configuration: the tomogram and the costs are compared exactly on
    windows (interior, edges, corner) that the oracle computes one by one;
    the keep list is checked for consistency with the slice test on the
    whole map."""
    import torch
    sc = scenes.config1_scene()
    grid = sc.grid
    rb = P.robot_from_physical(sc.robot, grid["res"])
    r = rb.as_dict()
    say("full-size config1: build + eval")
    xyz = torch.from_numpy(sc.points).cuda()
    ext = P.pct_tomogram_extent(xyz, grid)
    g, c, ag, ac = P.pct_build_tomogram(xyz, grid, ext, with_ids=True)
    cost, keep = P.pct_eval_traversability(g, c, grid, ext, [rb])
    torch.cuda.synchronize()
    zmin, zmax, used = oracle_lib.extent(sc.points, grid)
    assert (ext.z_min, ext.z_max, ext.n_used) == (np.float32(zmin), np.float32(zmax), used)
    h = oracle_lib.planes(zmin, zmax, grid["slice_dz"])
    assert ext.n_slices == len(h)
    M = 7   # margin: inflation radius 5 + patch radius 1 + stencil 1
    for wx0, wy0, wn in [(1000, 1000, 48), (0, 0, 40), (1980, 731, 20), (613, 1975, 25)]:
        ex0, ey0 = max(0, wx0 - M), max(0, wy0 - M)
        ex1, ey1 = min(grid["nx"], wx0 + wn + M), min(grid["ny"], wy0 + wn + M)
        w = oracle_lib.build_window(sc.points, grid, h, ex0, ey0, ex1 - ex0, ey1 - ey0)
        sl = (slice(None), slice(ey0, ey1), slice(ex0, ex1))
        np.testing.assert_array_equal(bits(g[sl].cpu().numpy()), bits(w[0]))
        np.testing.assert_array_equal(bits(c[sl].cpu().numpy()), bits(w[1]))
        np.testing.assert_array_equal(ag[sl].cpu().numpy(), w[2])
        np.testing.assert_array_equal(ac[sl].cpu().numpy(), w[3])
        lo, hi, _ = oracle_lib.envelope(w[0], w[1], grid["res"], r)
        iy0, ix0 = wy0 - ey0, wx0 - ex0
        inner = (slice(None), slice(iy0, iy0 + wn), slice(ix0, ix0 + wn))
        cw = cost[0][:, wy0:wy0 + wn, wx0:wx0 + wn].cpu().numpy().astype(np.float64)
        assert np.all(cw >= lo[inner] - TOL) and np.all(cw <= hi[inner] + TOL)
    # keep list: admissible under the slice test given the tomogram and costs
    # produced on the device (a consistency property at full size)
    eG = g.cpu().numpy()
    cT = cost[0].cpu().numpy().astype(np.float64)
    assert oracle_lib.simplify_check(eG, cT, cT, r["c_barrier"], 0.0, keep[0].cpu().numpy()) == -1


def test_extent_on_device_matches_host(P):
    """The capturable extent record equals the host call's, also for no
    points, points outside the grid only, and when captured in a graph."""
    import torch
    sc = scenes.config0_scene()
    xyz = torch.from_numpy(sc.points).cuda()
    want = P.pct_tomogram_extent(xyz, sc.grid)
    got = P.extent_from_bytes(P.pct_tomogram_extent_device(xyz, sc.grid))
    for f in ("z_min", "z_max", "n_slices", "n_used", "n_dropped"):
        assert getattr(got, f) == getattr(want, f), f
    empty = P.extent_from_bytes(P.pct_tomogram_extent_device(xyz[:0], sc.grid))
    assert (empty.n_slices, empty.n_used, empty.n_dropped) == (0, 0, 0) and empty.z_min == float("inf")
    far = torch.full((5, 3), -1000.0, device="cuda")
    out = P.extent_from_bytes(P.pct_tomogram_extent_device(far, sc.grid))
    assert (out.n_slices, out.n_used, out.n_dropped) == (0, 0, 5)
    # captured once, replayed after the points change
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    rec = torch.empty(32, dtype=torch.uint8, device="cuda")
    ws = torch.empty(P.lib().pct_extent_workspace_bytes(xyz.shape[0]), dtype=torch.uint8, device="cuda")
    pts = xyz.clone()
    with torch.cuda.stream(s):
        P.pct_tomogram_extent_device(pts, sc.grid, out=rec, workspace=ws)
        torch.cuda.synchronize()
        graph = P.Graph(s)
        with graph:
            P.pct_tomogram_extent_device(pts, sc.grid, out=rec, workspace=ws)
    pts[:, 2] += 1.5
    torch.cuda.synchronize()
    graph.launch(s)
    s.synchronize()
    moved = P.pct_tomogram_extent(pts, sc.grid)
    got = P.extent_from_bytes(rec)
    assert (got.z_min, got.z_max, got.n_slices, got.n_used) == (moved.z_min, moved.z_max, moved.n_slices, moved.n_used)
    del graph
