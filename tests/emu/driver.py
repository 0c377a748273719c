"""Runs libpct's kernels on the CPU (the AddressSanitizer build made by
build_emu.py) on small seeded cases and compares the results with the oracle.

Started by tests/test_emu.py in a child process with the sanitizer runtime
preloaded:  python tests/emu/driver.py CASE [CASE ...]
Each case prints one line when it passes; a failed comparison raises, and an
out-of-bounds access ends the process with the sanitizer's report."""
import ctypes as C
import importlib.util
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import build_emu  # noqa: E402
import oracle  # noqa: E402
import scenes  # noqa: E402

_spec = importlib.util.spec_from_file_location("pct_abi", os.path.join(ROOT, "paper_2403_07631_amd", "abi.py"))
abi = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(abi)

L = abi.load(build_emu.LIB)
L.emu_alloc.argtypes, L.emu_alloc.restype = [C.c_size_t], C.c_void_p
L.emu_free.argtypes, L.emu_free.restype = [C.c_void_p], None
TOL = 1e-5


def say(msg):
    print(f"[emu] {msg}", flush=True)


class Buf:
    """A "device" buffer: a heap block of exactly the requested size, filled
    with a garbage pattern like fresh device memory."""

    def __init__(self, nbytes, fill=0xCD):
        self.nbytes = int(nbytes)
        self.ptr = L.emu_alloc(max(1, self.nbytes))
        C.memset(self.ptr, fill, self.nbytes)

    @classmethod
    def of(cls, arr):
        arr = np.ascontiguousarray(arr)
        b = cls(arr.nbytes)
        C.memmove(b.ptr, arr.ctypes.data, arr.nbytes)
        return b

    def get(self, shape, dtype):
        out = np.empty(shape, dtype)
        assert out.nbytes <= self.nbytes
        C.memmove(out.ctypes.data, self.ptr, out.nbytes)
        return out

    def __del__(self):
        if getattr(self, "ptr", None):
            L.emu_free(self.ptr)
            self.ptr = None


def P(b):
    return None if b is None else C.c_void_p(b.ptr)


def check(fn, status):
    if status != abi.PCT_OK:
        raise RuntimeError(f"{fn}: status {status}: {L.pct_last_error().decode()}")


def grid_s(g):
    return abi.pct_grid(float(g["x0"]), float(g["y0"]), float(g["res"]), int(g["nx"]), int(g["ny"]),
                        float(g["slice_dz"]))


def robot_s(r):
    return abi.pct_robot(*[float(r[n]) for n in abi._ROBOT_FIELDS], int(r.get("patch_radius", 1)))


def robot(**kw):
    r = oracle.robot_from_physical(scenes.ROBOT_CONFIG0, 0.1)
    r.update(kw)
    return r


def bits(a):
    a = np.ascontiguousarray(a)
    return a.view(np.uint32) if a.dtype == np.float32 else a


# ------------------------------------------------------------ entry points

def extent(xyz_buf, n, grid):
    g = grid_s(grid)
    ws = Buf(L.pct_extent_workspace_bytes(n))
    e = abi.pct_extent()
    check("extent", L.pct_tomogram_extent(P(xyz_buf), n, C.byref(g), C.byref(e), P(ws), ws.nbytes, None))
    return e


def build(xyz_buf, n, grid, e, ids=True):
    g = grid_s(grid)
    N = e.n_slices
    cells = N * grid["nx"] * grid["ny"]
    G, Cc = Buf(4 * cells), Buf(4 * cells)
    aG, aC = (Buf(4 * cells), Buf(4 * cells)) if ids else (None, None)
    ws = Buf(L.pct_build_workspace_bytes(n, C.byref(g), C.byref(e)))
    check("build", L.pct_build_tomogram(P(xyz_buf), n, C.byref(g), C.byref(e), P(G), P(Cc), P(aG), P(aC), P(ws),
                                        ws.nbytes, None))
    return G, Cc, aG, aC


def evaluate(G, Cc, grid, e, robots, keep=True):
    g = grid_s(grid)
    rs = (abi.pct_robot * len(robots))(*[robot_s(r) for r in robots])
    cells = e.n_slices * grid["nx"] * grid["ny"]
    cost = Buf(4 * cells * len(robots))
    kp = Buf(e.n_slices * len(robots)) if keep else None
    ws = Buf(L.pct_eval_workspace_bytes(C.byref(g), C.byref(e), len(robots)))
    check("eval", L.pct_eval_traversability(P(G), P(Cc), C.byref(g), C.byref(e), rs, len(robots), P(cost), P(kp),
                                            P(ws), ws.nbytes, None))
    return cost, kp


def tomogram_case(pts, grid, ids=True, label=""):
    pts = np.ascontiguousarray(pts, np.float32)
    xb = Buf.of(pts)
    e = extent(xb, len(pts), grid)
    tm = oracle.tomogram(pts, grid)
    assert e.n_used == tm["n_used"], (e.n_used, tm["n_used"])
    assert e.n_slices == len(tm["h"])
    if e.n_slices == 0:
        return e, tm, None
    G, Cc, aG, aC = build(xb, len(pts), grid, e, ids)
    shape = (e.n_slices, grid["ny"], grid["nx"])
    out = [G.get(shape, np.float32), Cc.get(shape, np.float32)]
    np.testing.assert_array_equal(bits(out[0]), bits(tm["ground"]))
    np.testing.assert_array_equal(bits(out[1]), bits(tm["ceil"]))
    if ids:
        np.testing.assert_array_equal(aG.get(shape, np.int32), tm["arg_ground"])
        np.testing.assert_array_equal(aC.get(shape, np.int32), tm["arg_ceil"])
    say(f"tomogram {label} n={len(pts)} grid={grid['nx']}x{grid['ny']} N={e.n_slices} ids={ids}: bit-exact")
    return e, tm, (G, Cc)


def evaluate_window_whole(G, Cc, grid, e, r):
    """Evaluation of one robot through the window entry point with the whole
    map as the window: the same kernels, and a slice test that reads every
    slice (no slice marks)."""
    g = grid_s(grid)
    cells = e.n_slices * grid["nx"] * grid["ny"]
    cost = Buf(4 * cells)
    kp = Buf(e.n_slices)
    ws = Buf(L.pct_eval_workspace_bytes(C.byref(g), C.byref(e), 1))
    rb = robot_s(r)
    check("eval window", L.pct_eval_traversability_window(P(G), P(Cc), C.byref(g), C.byref(e), C.byref(rb), 0, 0,
                                                          grid["nx"], grid["ny"], P(cost), P(kp), P(ws), ws.nbytes,
                                                          None))
    return cost, kp


def eval_case(pts, grid, robots, label=""):
    e, tm, dev = tomogram_case(pts, grid, ids=False, label=label)
    cost, kp = evaluate(dev[0], dev[1], grid, e, robots)
    shape = (len(robots), e.n_slices, grid["ny"], grid["nx"])
    c = cost.get(shape, np.float32)
    keep = kp.get((len(robots), e.n_slices), np.uint8)
    for i, r in enumerate(robots):
        lo, hi, _ = oracle.envelope(tm["ground"], tm["ceil"], grid["res"], r)
        ci = c[i].astype(np.float64)
        assert np.all(ci >= lo - TOL) and np.all(ci <= hi + TOL), f"robot {i}: cost outside the oracle envelope"
        assert oracle.simplify_check(tm["ground"], lo, hi, r["c_barrier"], TOL, keep[i]) == -1
    say(f"eval {label} robots={len(robots)}: within envelope, keep admissible")
    return c, keep


# ------------------------------------------------------------------ cases

def case_tiny():
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from conftest import load_golden
    g = load_golden("tiny_tomogram.json")
    tomogram_case(np.array(g["points"], np.float32), g["grid"], True, "tiny golden")


def case_config0():
    sc = scenes.config0_scene()
    tomogram_case(sc.points, sc.grid, True, "config0")
    eval_case(sc.points, sc.grid, [robot()], "config0")


def case_edges():
    rng = np.random.default_rng(5)
    grid = dict(x0=-1.0, y0=2.0, res=0.125, nx=130, ny=19, slice_dz=0.25)
    pts = np.array([[-5, 3, 1], [100, 3, 1], [0, np.nan, 1], [0, 3, np.inf]], np.float32)
    e, _, _ = tomogram_case(pts, grid, True, "empty")
    assert e.n_slices == 0
    tomogram_case(np.array([[0.0, 2.5, -0.0]], np.float32), grid, True, "one point")
    huge = np.column_stack([np.full(20_000, 0.3), np.full(20_000, 2.3),
                            rng.choice([-0.0, 0.25, 0.5, 1.0, 1.75], 20_000)]).astype(np.float32)
    spread = np.column_stack([rng.uniform(-1.0, 7.0, 9000), rng.uniform(2.0, 3.0, 9000),
                              np.round(rng.uniform(-0.5, 2.0, 9000), 2)]).astype(np.float32)
    junk = np.array([[np.nan, 2.5, 0], [0, 2.5, np.nan], [1e30, 2.5, 0], [0.0, 2.0 + 19 * 0.125, 0.5]], np.float32)
    pts = np.concatenate([spread[:4000], huge, junk, spread[4000:]])
    tomogram_case(pts, grid, True, "huge cell")
    tomogram_case(pts, grid, False, "huge cell")


def case_slice_runs():
    """The slice test that passes over slices without a traversable cell
    equals the slice test that reads every slice (the window entry point over
    the whole map) on the same costs: a floor beside a ramp under fine slices
    (runs of equal ground longer than 64 slices whose costs take many values
    as the ramp's cells gain ground slice by slice, and slices high above
    the ramp with no traversable cell between slices that have one), and a
    multi-storey map."""
    ramp = scenes.dense_surface_scene(70, 50, 0.1, lambda x, y: np.where(x < 2.5, 0.0, 0.55 * (x - 2.5)),
                                      per_cell=4, slice_dz=0.04,
                                      extra=[np.array([[0.05, 0.05, 6.2], [6.95, 4.95, -0.3]], np.float32)])
    ms = scenes.multistorey_scene(35, 6.1, 4.3, 200_000, n_floors=3)
    # a floor, a solid block from 1 m to 2 m over most of it (its slices hold
    # no traversable cell) and a slab at 3.2 m over half: runs on the block's
    # top start after slices that are passed over
    xs, ys = np.meshgrid((np.arange(48) + 0.5) * 0.1, (np.arange(36) + 0.5) * 0.1)
    inside = (xs > 0.6) & (xs < 4.2) & (ys > 0.5) & (ys < 3.1)
    block = np.concatenate([np.column_stack([xs[inside], ys[inside], np.full(inside.sum(), z)])
                            for z in np.arange(1.0, 2.001, 0.05)])
    half = xs < 2.4
    slab = np.column_stack([xs[half], ys[half], np.full(half.sum(), 3.2)])
    blk = scenes.dense_surface_scene(48, 36, 0.1, lambda x, y: np.zeros_like(x), per_cell=4, slice_dz=0.1,
                                     extra=[block.astype(np.float32), slab.astype(np.float32)])
    for sc, rs, label in ((ramp, [robot(), robot(theta_s=0.7, d_inf=0.5, d_sm=0.7)], "floor and ramp"),
                          (ms, [robot(), dict(scenes.ROBOT_TABLE1)], "three storeys"),
                          (blk, [robot(), robot(d_min=0.3, d_inf=0.1, d_sm=0.3)], "floor, block and slab")):
        e, tm, dev = tomogram_case(sc.points, sc.grid, ids=False, label=label)
        shape = (len(rs), e.n_slices, sc.grid["ny"], sc.grid["nx"])
        cost, kp = evaluate(dev[0], dev[1], sc.grid, e, rs)
        c = cost.get(shape, np.float32)
        k1 = kp.get((len(rs), e.n_slices), np.uint8)
        for i, r in enumerate(rs):
            cost2, kp2 = evaluate_window_whole(dev[0], dev[1], sc.grid, e, r)
            c2 = cost2.get(shape[1:], np.float32)
            k2 = kp2.get((e.n_slices,), np.uint8)
            np.testing.assert_array_equal(bits(c[i]), bits(c2))
            np.testing.assert_array_equal(k1[i], k2)
            lo, hi, _ = oracle.envelope(tm["ground"], tm["ceil"], sc.grid["res"], r)
            ci = c[i].astype(np.float64)
            assert np.all(ci >= lo - TOL) and np.all(ci <= hi + TOL)
            assert oracle.simplify_check(tm["ground"], ci, ci, r["c_barrier"], 0.0, k1[i]) == -1
            trav = c[i] < r["c_barrier"]
            empty = int((~trav.reshape(e.n_slices, -1).any(axis=1)).sum())
            g = tm["ground"]
            run = np.ones(g.shape[1:], np.int32)
            longest = 1
            for k in range(1, e.n_slices):
                run = np.where(g[k] == g[k - 1], run + 1, 1)
                longest = max(longest, int(run[trav[k]].max(initial=0)))
            say(f"slice runs {label} robot {i}: N={e.n_slices}, {empty} slices without a traversable cell, "
                f"longest run over a traversable cell {longest}, {int(k1[i].sum())} kept; both slice tests agree")


def case_static_many_slices():
    """About a thousand slices on a small map: the static-scratch entry point
    then holds one copy of the run starts (its array is nearly filled by the
    N x N bit matrix) while a sized workspace holds sixteen; both give the
    same costs and keep flags, admissible under the oracle's slice test."""
    xs, ys = np.meshgrid((np.arange(16) + 0.5) * 0.1, (np.arange(12) + 0.5) * 0.1)
    shelves = np.concatenate([np.column_stack([xs.ravel(), ys.ravel(), np.full(xs.size, z)])
                              for z in (2.5, 5.0, 7.5)])
    sc = scenes.dense_surface_scene(16, 12, 0.1, lambda x, y: 0.02 * x, per_cell=4, slice_dz=0.01,
                                    extra=[shelves.astype(np.float32),
                                           np.array([[0.05, 0.05, 9.9]], np.float32)])
    e, tm, dev = tomogram_case(sc.points, sc.grid, ids=False, label="thousand slices")
    assert e.n_slices > 960, e.n_slices
    r = robot()
    cost, kp = evaluate(dev[0], dev[1], sc.grid, e, [r])
    cells = e.n_slices * sc.grid["nx"] * sc.grid["ny"]
    g = grid_s(sc.grid)
    rs = (abi.pct_robot * 1)(robot_s(r))
    cost2, kp2 = Buf(4 * cells), Buf(e.n_slices)
    check("eval static", L.pct_eval_traversability_static(P(dev[0]), P(dev[1]), C.byref(g), C.byref(e), rs, 1,
                                                          P(cost2), P(kp2), None))
    np.testing.assert_array_equal(bits(cost2.get(cells, np.float32)), bits(cost.get(cells, np.float32)))
    k1 = kp.get(e.n_slices, np.uint8)
    np.testing.assert_array_equal(kp2.get(e.n_slices, np.uint8), k1)
    c = cost.get((e.n_slices, sc.grid["ny"], sc.grid["nx"]), np.float32).astype(np.float64)
    assert oracle.simplify_check(tm["ground"], c, c, r["c_barrier"], 0.0, k1) == -1
    say(f"static scratch at N={e.n_slices}: the same costs and {int(k1.sum())} kept slices as a sized workspace")


def case_crowded_cells():
    """Four adjacent cells whose records fit in the tile reduce's LDS one by
    one but not together (1500 points each), beside ordinary cells, on a
    grid whose rows are 16-byte aligned and one whose rows are not."""
    rng = np.random.default_rng(17)
    for nx in (64, 61):
        grid = dict(x0=0.0, y0=0.0, res=0.1, nx=nx, ny=9, slice_dz=0.25)
        crowd = np.column_stack([rng.uniform(0.4, 0.8, 6000), rng.uniform(0.5, 0.6, 6000),
                                 np.round(rng.uniform(0.0, 3.0, 6000), 2)])
        rest = np.column_stack([rng.uniform(0.0, nx * 0.1, 4000), rng.uniform(0.0, 0.9, 4000),
                                rng.uniform(0.0, 3.0, 4000)])
        pts = np.concatenate([crowd, rest]).astype(np.float32)
        tomogram_case(pts, grid, True, f"crowded cells nx={nx}")
        tomogram_case(pts, grid, False, f"crowded cells nx={nx}")


class _Offset:
    """A view `off` bytes into a Buf (the Buf stays alive with it)."""

    def __init__(self, base, off):
        self.base, self.ptr, self.nbytes = base, base.ptr + off, base.nbytes - off


def case_unaligned_points():
    """Points whose array is not 16-byte aligned (the extent and binning
    kernels then read them point by point) and an aligned array whose length
    is not a multiple of four, over several binning chunks: the same
    tomograms as the oracle's."""
    rng = np.random.default_rng(29)
    grid = dict(x0=0.0, y0=0.0, res=0.1, nx=70, ny=33, slice_dz=0.25)
    n = 3 * 4096 + 1003
    pts = np.column_stack([rng.uniform(-0.3, 7.3, n), rng.uniform(-0.2, 3.5, n),
                           np.round(rng.uniform(0.0, 3.0, n), 2)]).astype(np.float32)
    tm = oracle.tomogram(pts, grid)
    for off in (4, 8, 0):
        raw = Buf(pts.nbytes + off)
        C.memmove(raw.ptr + off, pts.ctypes.data, pts.nbytes)
        xb = _Offset(raw, off)
        e = extent(xb, n, grid)
        assert e.n_used == tm["n_used"] and e.n_slices == len(tm["h"])
        G, Cc, aG, aC = build(xb, n, grid, e, True)
        shape = (e.n_slices, grid["ny"], grid["nx"])
        np.testing.assert_array_equal(bits(G.get(shape, np.float32)), bits(tm["ground"]))
        np.testing.assert_array_equal(bits(Cc.get(shape, np.float32)), bits(tm["ceil"]))
        np.testing.assert_array_equal(aG.get(shape, np.int32), tm["arg_ground"])
        np.testing.assert_array_equal(aC.get(shape, np.int32), tm["arg_ceil"])
        say(f"tomogram from points at byte offset {off}, n={n}: bit-exact")


def case_dense_tiles():
    """Tiles with more records on average than the tile reduce's floor
    capacity, so that the launch raises it (above 64 KB of LDS): 12 000
    points a tile (one pass) and 20 000 (above the largest capacity, two
    passes), as one map and in a batch beside a sparse submap."""
    rng = np.random.default_rng(23)
    grid = dict(x0=0.0, y0=0.0, res=0.1, nx=40, ny=6, slice_dz=0.3)
    maps = []
    for n in (36_000, 60_000):
        pts = np.column_stack([rng.uniform(0.0, 4.0, n), rng.uniform(0.0, 0.6, n),
                               rng.uniform(0.0, 3.0, n)]).astype(np.float32)
        tomogram_case(pts, grid, True, f"dense tiles, {n} points")
        tomogram_case(pts, grid, False, f"dense tiles, {n} points")
        maps.append(scenes.Scene(pts, grid))
    maps.append(scenes.multistorey_scene(24, 4.1, 3.3, 20_000, n_floors=2))
    pts, specs, off = [], [], 0
    for sc in maps:
        specs.append(dict(xyz_offset=off, n_points=len(sc.points), grid=sc.grid))
        pts.append(sc.points)
        off += len(sc.points)
    pts = np.ascontiguousarray(np.concatenate(pts))
    for ids in (True, False):
        check_batch(maps, pts, specs, [robot()], ids)


def case_multirobot():
    sc = scenes.multistorey_scene(33, 4.3, 3.1, 60_000, n_floors=2)
    rs = [robot(), robot(d_min=0.7, theta_s=0.3), robot(d_inf=0.5, d_sm=0.7)]
    eval_case(sc.points, sc.grid, rs, "multi-robot")


def case_fallback_eval():
    """Robots that take the tiled kernel (patch radius 2, radius > 8)."""
    sc = scenes.multistorey_scene(32, 4.7, 3.9, 60_000, n_floors=2)
    eval_case(sc.points, sc.grid, [robot(patch_radius=2, theta_p=0.45)], "patch radius 2")
    eval_case(sc.points, sc.grid, [robot(d_inf=1.2, d_sm=0.5)], "radius > 8")


def case_crop():
    sc = scenes.multistorey_scene(21, 31.7, 23.3, 500_000, n_floors=6)
    tomogram_case(sc.points, sc.grid, True, "crop")
    tomogram_case(sc.points, sc.grid, False, "crop")


def case_dense():
    sc = scenes.multistorey_scene(22, 13.3, 9.1, 600_000, n_floors=3)
    tomogram_case(sc.points, sc.grid, True, "dense")
    tomogram_case(sc.points, sc.grid, False, "dense")


def case_multirobot_large():
    sc = scenes.multistorey_scene(33, 8.3, 6.1, 300_000, n_floors=2)
    rs = [robot(), robot(d_min=0.7, theta_s=0.3), robot(d_inf=0.5, d_sm=0.7)]
    eval_case(sc.points, sc.grid, rs, "multi-robot 83x61")


def case_many_chunks():
    """More than 64 binning workgroups (several groups of the column scan)."""
    rng = np.random.default_rng(8)
    grid = dict(x0=0.0, y0=0.0, res=0.1, nx=300, ny=40, slice_dz=0.3)
    n = 1_300_000
    pts = np.column_stack([rng.uniform(-0.5, 30.5, n), rng.uniform(-0.2, 4.2, n),
                           rng.uniform(0.0, 3.0, n)]).astype(np.float32)
    tomogram_case(pts, grid, True, "1.3M points")


def case_two_level():
    """Enough tiles for two binning levels with several level-2 workgroups
    per super-tile, a ragged last super-tile and an empty band."""
    rng = np.random.default_rng(9)
    grid = dict(x0=0.0, y0=0.0, res=0.1, nx=1000, ny=606, slice_dz=0.3)
    n = 1_800_000
    x = rng.uniform(-1.0, 101.0, n)
    y = rng.uniform(0.0, 60.6, n)
    keep = ~((y > 20.0) & (y < 26.0))          # a band of tiles with no points
    pts = np.column_stack([x[keep], y[keep], rng.uniform(0.0, 4.0, keep.sum())]).astype(np.float32)
    tomogram_case(pts, grid, True, "two-level binning")


def case_autotune():
    """The autotuner tries every strip height; evaluations after tuning are
    bit-identical to those before."""
    sc = scenes.multistorey_scene(34, 4.9, 3.3, 60_000, n_floors=2)
    pts = np.ascontiguousarray(sc.points, np.float32)
    xb = Buf.of(pts)
    e = extent(xb, len(pts), sc.grid)
    G, Cc, _, _ = build(xb, len(pts), sc.grid, e, False)
    r = robot()
    before = evaluate(G, Cc, sc.grid, e, [r])[0].get(e.n_slices * sc.grid["nx"] * sc.grid["ny"], np.float32)
    g = grid_s(sc.grid)
    rb = robot_s(r)
    scratch = Buf(4 * e.n_slices * sc.grid["nx"] * sc.grid["ny"])
    best, bw, count = C.c_int32(), C.c_int32(), C.c_int32()
    rows, waves, ms = (C.c_int32 * 24)(), (C.c_int32 * 24)(), (C.c_float * 24)()
    check("autotune", L.pct_autotune_traversability(P(G), P(Cc), C.byref(g), C.byref(e), C.byref(rb), P(scratch),
                                                    C.byref(best), C.byref(bw), rows, waves, ms, 24, C.byref(count),
                                                    None))
    cands = [(rows[i], waves[i]) for i in range(count.value)]
    assert count.value >= 4 and (best.value, bw.value) in cands, (best.value, bw.value, cands)
    assert {w for _, w in cands} == {1, 2, 4}
    after = evaluate(G, Cc, sc.grid, e, [r])[0].get(e.n_slices * sc.grid["nx"] * sc.grid["ny"], np.float32)
    np.testing.assert_array_equal(bits(after), bits(before))
    # every candidate shape gives the same bits
    for rr, ww in cands:
        check("set", L.pct_autotune_set_traversability(C.byref(g), C.byref(e), C.byref(rb), rr, ww))
        got = evaluate(G, Cc, sc.grid, e, [r])[0].get(e.n_slices * sc.grid["nx"] * sc.grid["ny"], np.float32)
        np.testing.assert_array_equal(bits(got), bits(before))
    check("reset", L.pct_autotune_reset())
    say(f"autotune: candidates {cands}, chose {(best.value, bw.value)}; evaluation unchanged at every shape")


# ----------------------------------------------------------------- batches

def make_batch(seed, n_items, side_hi=160, pts_hi=120_000, extra_empty=True):
    items = scenes.submap_batch(seed, n_items, side_lo=20, side_hi=side_hi, pts_lo=2_000, pts_hi=pts_hi)
    if extra_empty:
        junk = scenes.Scene(np.array([[-50.0, -50.0, 1.0]], np.float32),
                            dict(x0=0.0, y0=0.0, res=0.1, nx=30, ny=20, slice_dz=0.3))
        none = scenes.Scene(np.zeros((0, 3), np.float32), dict(x0=0.0, y0=0.0, res=0.1, nx=7, ny=9, slice_dz=0.3))
        items = items[:2] + [junk] + items[2:] + [none]
    pts, specs, off = [], [], 0
    for sc in items:
        specs.append(dict(xyz_offset=off, n_points=len(sc.points), grid=sc.grid))
        pts.append(sc.points)
        off += len(sc.points)
    return items, np.ascontiguousarray(np.concatenate(pts)), specs


def batch_run(pts, specs, robots, ids):
    n_items = len(specs)
    items = (abi.pct_item * n_items)()
    for it, sp in zip(items, specs):
        it.xyz_offset, it.n_points = sp["xyz_offset"], sp["n_points"]
        it.grid = grid_s(sp["grid"])
    xb = Buf.of(pts)
    ws = Buf(L.pct_batch_workspace_bytes(items, n_items, len(robots), int(ids)))
    tc, ts = C.c_int64(), C.c_int64()
    check("extent_batched", L.pct_tomogram_extent_batched(P(xb), len(pts), items, n_items, C.byref(tc), C.byref(ts),
                                                          P(ws), ws.nbytes, None))
    ws = Buf(L.pct_batch_workspace_bytes(items, n_items, len(robots), int(ids)))
    cells, slices = max(1, tc.value), max(1, ts.value)
    G, Cc = Buf(4 * cells), Buf(4 * cells)
    aG, aC = (Buf(4 * cells), Buf(4 * cells)) if ids else (None, None)
    check("build_batched", L.pct_build_tomogram_batched(P(xb), len(pts), items, n_items, P(G), P(Cc), P(aG), P(aC), 0,
                                                        P(ws), ws.nbytes, None))
    rs = (abi.pct_robot * len(robots))(*[robot_s(r) for r in robots])
    cost = Buf(4 * cells * len(robots))
    kp = Buf(slices * len(robots))
    check("eval_batched", L.pct_eval_traversability_batched(P(G), P(Cc), items, n_items, rs, len(robots), P(cost),
                                                            P(kp), 0, P(ws), ws.nbytes, None))
    out = dict(G=G.get(cells, np.float32), C=Cc.get(cells, np.float32),
               cost=cost.get((len(robots), cells), np.float32), keep=kp.get((len(robots), slices), np.uint8))
    if ids:
        out["aG"], out["aC"] = aG.get(cells, np.int32), aC.get(cells, np.int32)
    return items, out


def check_batch(items_sc, pts, specs, robots, ids, n_oracle=3, step=1):
    items, out = batch_run(pts, specs, robots, ids)
    checked = 0
    for i in range(0, len(specs), step):
        it, sp = items[i], specs[i]
        sub = pts[sp["xyz_offset"]:sp["xyz_offset"] + sp["n_points"]]
        tm = oracle.tomogram(sub, sp["grid"])
        assert it.extent.n_used == tm["n_used"] and it.extent.n_slices == len(tm["h"]), i
        N = it.extent.n_slices
        if N == 0:
            continue
        nx, ny = sp["grid"]["nx"], sp["grid"]["ny"]
        sl = slice(it.out_offset, it.out_offset + N * nx * ny)
        np.testing.assert_array_equal(bits(out["G"][sl]), bits(tm["ground"].ravel()))
        np.testing.assert_array_equal(bits(out["C"][sl]), bits(tm["ceil"].ravel()))
        if ids:
            off = sp["xyz_offset"]
            np.testing.assert_array_equal(out["aG"][sl], np.where(tm["arg_ground"].ravel() >= 0,
                                                                  tm["arg_ground"].ravel() + off, -1))
            np.testing.assert_array_equal(out["aC"][sl], np.where(tm["arg_ceil"].ravel() >= 0,
                                                                  tm["arg_ceil"].ravel() + off, -1))
        if checked < n_oracle:
            for r, rb in enumerate(robots):
                lo, hi, _ = oracle.envelope(tm["ground"], tm["ceil"], sp["grid"]["res"], rb)
                c = out["cost"][r, sl].reshape(N, ny, nx).astype(np.float64)
                assert np.all(c >= lo - TOL) and np.all(c <= hi + TOL), (i, r)
                kp = out["keep"][r, it.keep_offset:it.keep_offset + N]
                assert oracle.simplify_check(tm["ground"], lo, hi, rb["c_barrier"], TOL, kp) == -1, (i, r)
        checked += 1
    say(f"batch of {len(specs)} items, {len(pts)} points, {len(robots)} robots, ids={ids}: "
        f"{checked} items checked")


def case_batch():
    items, pts, specs = make_batch(61, 6, side_hi=60, pts_hi=30_000)
    check_batch(items, pts, specs, [robot(), robot(d_min=0.7, theta_s=0.3)], True)


def case_batch_resident():
    """Eager extent, build and evaluation, then build and evaluation again
    with PCT_DESCRIPTORS_RESIDENT on the same workspace (the sequence a
    graph capture uses): the same outputs."""
    items_sc, pts, specs = make_batch(63, 5, side_hi=60, pts_hi=30_000, extra_empty=False)
    robots = [robot()]
    n_items = len(specs)
    items = (abi.pct_item * n_items)()
    for it, sp in zip(items, specs):
        it.xyz_offset, it.n_points = sp["xyz_offset"], sp["n_points"]
        it.grid = grid_s(sp["grid"])
    xb = Buf.of(pts)
    tc, ts = C.c_int64(), C.c_int64()
    ws = Buf(L.pct_batch_workspace_bytes(items, n_items, 1, 0))
    check("extent_batched", L.pct_tomogram_extent_batched(P(xb), len(pts), items, n_items, C.byref(tc), C.byref(ts),
                                                          P(ws), ws.nbytes, None))
    ws = Buf(L.pct_batch_workspace_bytes(items, n_items, 1, 0))
    cells, slices = tc.value, ts.value
    rs = (abi.pct_robot * 1)(robot_s(robots[0]))
    outs = []
    for flags in (0, abi.PCT_DESCRIPTORS_RESIDENT, abi.PCT_DESCRIPTORS_RESIDENT):
        G, Cc = Buf(4 * cells), Buf(4 * cells)
        cost, kp = Buf(4 * cells), Buf(slices)
        check("build_batched", L.pct_build_tomogram_batched(P(xb), len(pts), items, n_items, P(G), P(Cc), None, None,
                                                            flags, P(ws), ws.nbytes, None))
        check("eval_batched", L.pct_eval_traversability_batched(P(G), P(Cc), items, n_items, rs, 1, P(cost), P(kp),
                                                                flags, P(ws), ws.nbytes, None))
        outs.append([G.get(cells, np.float32), Cc.get(cells, np.float32), cost.get(cells, np.float32),
                     kp.get(slices, np.uint8)])
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            np.testing.assert_array_equal(bits(a), bits(b))
    say(f"batch with resident descriptors: {n_items} items, 2 replays equal the eager run")


def case_batch_mixed_radius():
    """Robots with different inflation radii: per-job launches."""
    items, pts, specs = make_batch(62, 3, side_hi=50, pts_hi=20_000, extra_empty=False)
    check_batch(items, pts, specs, [robot(), robot(d_inf=0.5, d_sm=0.7)], False)


def case_batch_tune():
    """The size-class tuner: every class gets one choice per stage, and
    batched outputs after tuning (and after loading other shapes) equal
    those before; resident tables of other shapes are refused; the tables
    survive a save and load, and a malformed file applies nothing."""
    import tempfile
    # small items (the tuner runs every distinct candidate four times per
    # class) and one wider than 128 cells, whose class tunes its tile height
    items_sc, pts, specs = make_batch(64, 2, side_hi=24, pts_hi=3_000, extra_empty=True)
    wide = scenes.multistorey_scene(66, 14.0, 1.2, 4_000, n_floors=2)
    assert wide.grid["nx"] > 128
    specs.append(dict(xyz_offset=len(pts), n_points=len(wide.points), grid=wide.grid))
    pts = np.ascontiguousarray(np.concatenate([pts, wide.points]))
    items_sc.append(wide)
    rb = robot()
    L.pct_autotune_reset()
    _, before = batch_run(pts, specs, [rb], True)
    items, _ = batch_run(pts, specs, [rb], False)      # items with extents
    xb = Buf.of(pts)
    n_items = len(specs)
    ent = (abi.pct_tune_entry * 256)()
    cnt = C.c_int32()
    rs = (abi.pct_robot * 1)(robot_s(rb))
    check("autotune_batched", L.pct_autotune_batched(P(xb), len(pts), items, n_items, rs, ent, 256, C.byref(cnt),
                                                     None))
    es = list(ent[:cnt.value])
    classes = {(e.stage, e.class_x, e.class_y, e.radius) for e in es}
    # three tile heights for the wide class only; strip shapes that launch
    # the same strips are timed once
    assert sum(e.stage == 0 for e in es) == 3 and all(e.class_x >= 8 for e in es if e.stage == 0)
    assert len(classes) >= 3
    for c in {(e.class_x, e.class_y, e.radius) for e in es if e.stage == 1}:
        shapes = [(e.rows, e.waves) for e in es if e.stage == 1 and (e.class_x, e.class_y, e.radius) == c]
        assert len(set(shapes)) == len(shapes), (c, shapes)
    for c in classes:
        assert sum(e.chosen for e in es if (e.stage, e.class_x, e.class_y, e.radius) == c) == 1, c
        assert all(e.ms > 0 for e in es if (e.stage, e.class_x, e.class_y, e.radius) == c)
    _, after = batch_run(pts, specs, [rb], True)
    for k in before:
        np.testing.assert_array_equal(bits(after[k]), bits(before[k]), err_msg=k)
    say(f"batch tuner: {cnt.value} timings over {len(classes)} (stage, class) pairs, outputs unchanged")
    # shapes unlike the defaults for every class, through a file
    tmp = tempfile.mkdtemp()
    path = os.path.join(tmp, "tune.txt")
    lines = ["# shapes for the test"]
    chosen = {(e.stage, e.class_x, e.class_y, e.radius): (e.rows, e.waves) for e in es if e.chosen}
    for st_, cx, cy, R in sorted(classes):
        ch = chosen[(st_, cx, cy, R)]
        if st_ == 0:
            lines.append(f"cpu-emulator batch_build {cx} {cy} {4 if ch[0] == 8 else 8}")
        else:
            lines.append(f"cpu-emulator batch_eval {cx} {cy} {R} " + ("32 1" if ch == (64, 4) else "64 4"))
    lines.append("otherarch batch_build 1 1 4")
    with open(path, "w") as fp:
        fp.write("\n".join(lines) + "\n")
    ws = Buf(L.pct_batch_workspace_bytes(items, n_items, 1, 1))
    tc = sum(it.extent.n_slices * it.grid.nx * it.grid.ny for it in items)
    G, Cc, aG, aC = Buf(4 * tc), Buf(4 * tc), Buf(4 * tc), Buf(4 * tc)
    cost1, kp1 = Buf(4 * tc), Buf(sum(it.extent.n_slices for it in items))
    build_args = lambda fl: (P(xb), len(pts), items, n_items, P(G), P(Cc), P(aG), P(aC), fl, P(ws), ws.nbytes, None)
    eval_args = lambda fl: (P(G), P(Cc), items, n_items, rs, 1, P(cost1), P(kp1), fl, P(ws), ws.nbytes, None)
    check("build_batched", L.pct_build_tomogram_batched(*build_args(0)))
    check("eval_batched", L.pct_eval_traversability_batched(*eval_args(0)))
    n_ap = C.c_int32()
    check("autotune_load", L.pct_autotune_load(path.encode(), C.byref(n_ap)))
    assert n_ap.value == len(classes)
    assert L.pct_build_tomogram_batched(*build_args(abi.PCT_DESCRIPTORS_RESIDENT)) == abi.PCT_ERR_ARG
    assert L.pct_eval_traversability_batched(*eval_args(abi.PCT_DESCRIPTORS_RESIDENT)) == abi.PCT_ERR_ARG
    check("build_batched", L.pct_build_tomogram_batched(*build_args(0)))
    check("build_batched", L.pct_build_tomogram_batched(*build_args(abi.PCT_DESCRIPTORS_RESIDENT)))
    np.testing.assert_array_equal(bits(G.get(tc, np.float32)), bits(before["G"][:tc]))
    np.testing.assert_array_equal(aG.get(tc, np.int32), before["aG"][:tc])
    _, loaded = batch_run(pts, specs, [rb], True)
    for k in before:
        np.testing.assert_array_equal(bits(loaded[k]), bits(before[k]), err_msg=k)
    # save, reset, load back: the same records
    path2 = os.path.join(tmp, "saved.txt")
    check("autotune_save", L.pct_autotune_save(path2.encode()))
    L.pct_autotune_reset()
    check("autotune_load", L.pct_autotune_load(path2.encode(), C.byref(n_ap)))
    assert n_ap.value == len(classes), n_ap.value
    with open(path2) as fp:
        saved = sorted(l for l in fp.read().splitlines() if not l.startswith("#"))
    assert saved == sorted(l for l in lines[1:] if l.startswith("cpu-emulator")), saved
    with open(path, "a") as fp:
        fp.write("cpu-emulator batch_eval 7 7 3 32 2\n")     # two-wave strips are not batch shapes
    L.pct_autotune_reset()
    assert L.pct_autotune_load(path.encode(), C.byref(n_ap)) == abi.PCT_ERR_ARG
    check("autotune_save", L.pct_autotune_save(path2.encode()))
    with open(path2) as fp:
        assert not [l for l in fp.read().splitlines() if not l.startswith("#")]
    L.pct_autotune_reset()
    say("batch tuning tables: loaded shapes change no output, stale resident tables refused, save/load round trip")


def case_config1_build():
    """The 20 M-point 2000 x 2000 map, tomogram with ids (slow: minutes)."""
    sc = scenes.config1_scene()
    tomogram_case(sc.points, sc.grid, True, "config1")


# ------------------------------------------------------- trajectory costs

def sample_fwd(cost, G, grid, e, rb, w_z, wpb, slb, T, W):
    g = grid_s(grid)
    r = robot_s(rb)
    f = Buf(4 * T)
    check("sample_fwd", L.pct_sample_cost_fwd(P(cost), P(G), C.byref(g), C.byref(e), C.byref(r), w_z, P(wpb), P(slb),
                                              T, W, P(f), None))
    return f.get(T, np.float32)


def traj_bwd(G, Cc, cost, aG, aC, grid, e, rb, w_z, wpb, slb, T, W, gfb, n_points, gz, flags):
    g = grid_s(grid)
    r = robot_s(rb)
    gwp = Buf(12 * T * W)
    check("traj_bwd", L.pct_trajectory_cost_bwd(P(G), P(Cc), P(cost), P(aG), P(aC), C.byref(g), C.byref(e),
                                                 C.byref(r), w_z, P(wpb), P(slb), T, W, P(gfb), n_points, P(gwp),
                                                 P(gz), flags, None))
    return gwp.get((T, W, 3), np.float32)


def close(a, ref, mask=None, rel=1e-3):
    a, ref = np.asarray(a, np.float64), np.asarray(ref, np.float64)
    bad = np.abs(a - ref) > rel * np.maximum(1.0, np.abs(ref))
    if mask is not None:
        bad &= mask
    assert not bad.any(), f"{bad.sum()} entries differ; worst {np.max(np.abs(a - ref)[bad])}"


def case_traj_value_grad():
    """Several profiles in one on-demand launch = the per-profile path
    (cost map, sampling, fused adjoint) bit for bit for f and dL/dwp, and
    the oracle within the gradient tolerance."""
    w_z = 1.0
    sc = scenes.multistorey_scene(51, 5.3, 4.1, 160_000, n_floors=2)
    grid = sc.grid
    pts = np.ascontiguousarray(sc.points, np.float32)
    n = len(pts)
    xb = Buf.of(pts)
    e = extent(xb, n, grid)
    G, Cc, aG, aC = build(xb, n, grid, e, True)
    shape = (e.n_slices, grid["ny"], grid["nx"])
    tm = oracle.tomogram(pts, grid)
    profiles = [oracle.robot_from_physical(p, grid["res"]) for p in scenes.robot_profiles(4, 3)]
    T, W = 6, 70
    wps, sls = [], []
    for i, r in enumerate(profiles):
        cT = oracle.evaluate(tm["ground"], tm["ceil"], grid["res"], r)
        lo, hi, _ = oracle.envelope(tm["ground"], tm["ceil"], grid["res"], r)
        mask = (cT < r["c_barrier"]) & (lo == hi)
        wp, sl = scenes.random_walks(20 + i, mask, tm["ground"], grid, T, W, r["d_ref"])
        wps.append(wp)
        sls.append(sl)
    wp_all = np.ascontiguousarray(np.stack(wps), np.float32)
    sl_all = np.ascontiguousarray(np.stack(sls), np.int32)
    gf_all = np.ascontiguousarray(np.linspace(-1.0, 1.5, len(profiles) * T).reshape(len(profiles), T), np.float32)
    # per-profile path: c^T map, sampling, fused adjoint accumulated over profiles
    gz1 = Buf(4 * n)
    f1, gwp1 = [], []
    for i, r in enumerate(profiles):
        cost, _ = evaluate(G, Cc, grid, e, [r], keep=False)
        wpb, slb, gfb = Buf.of(wp_all[i]), Buf.of(sl_all[i]), Buf.of(gf_all[i])
        f1.append(sample_fwd(cost, G, grid, e, r, w_z, wpb, slb, T, W))
        gwp1.append(traj_bwd(G, Cc, cost, aG, aC, grid, e, r, w_z, wpb, slb, T, W, gfb, n, gz1,
                             abi.PCT_ACCUMULATE if i else 0))
    # one launch for all profiles
    rs = (abi.pct_robot * len(profiles))(*[robot_s(r) for r in profiles])
    ws = Buf(L.pct_trajectory_multi_workspace_bytes(len(profiles)))
    wpb, slb, gfb = Buf.of(wp_all), Buf.of(sl_all), Buf.of(gf_all)
    f2, gwp2, gz2 = Buf(4 * len(profiles) * T), Buf(12 * wp_all[..., 0].size), Buf(4 * n)
    gG2, gC2 = Buf(4 * int(np.prod(shape))), Buf(4 * int(np.prod(shape)))
    g = grid_s(grid)
    check("multi", L.pct_trajectory_cost_multi(P(G), P(Cc), P(aG), P(aC), C.byref(g), C.byref(e), rs, len(profiles),
                                               w_z, P(wpb), P(slb), T, W, P(gfb), P(f2), P(gwp2), P(gG2), P(gC2), n,
                                               P(gz2), 0, P(ws), ws.nbytes, None))
    f2 = f2.get((len(profiles), T), np.float32)
    gwp2 = gwp2.get(wp_all.shape, np.float32)
    np.testing.assert_array_equal(bits(f2), bits(np.stack(f1)))
    np.testing.assert_array_equal(bits(gwp2), bits(np.stack(gwp1)))
    # float atomics add in a different order: a few ulps of the largest partial sums
    a, b = gz2.get(n, np.float32), gz1.get(n, np.float32)
    np.testing.assert_allclose(a, b, rtol=1e-5, atol=2e-5 * max(1.0, float(np.abs(b).max())))
    # fixed-point sums: the per-profile loop and the one launch give the same
    # integers whatever order the (shuffled) wavefronts add in
    gz1x = Buf(8 * n)
    for i, r in enumerate(profiles):
        cost, _ = evaluate(G, Cc, grid, e, [r], keep=False)
        wpb1, slb1, gfb1 = Buf.of(wp_all[i]), Buf.of(sl_all[i]), Buf.of(gf_all[i])
        traj_bwd(G, Cc, cost, aG, aC, grid, e, r, w_z, wpb1, slb1, T, W, gfb1, n, gz1x,
                 abi.PCT_FIXED_POINT | (abi.PCT_ACCUMULATE if i else 0))
    f2x, gwp2x, gz2x = Buf(4 * len(profiles) * T), Buf(12 * wp_all[..., 0].size), Buf(8 * n)
    gG2x, gC2x = Buf(8 * int(np.prod(shape))), Buf(8 * int(np.prod(shape)))
    check("multi fixed", L.pct_trajectory_cost_multi(P(G), P(Cc), P(aG), P(aC), C.byref(g), C.byref(e), rs,
                                                     len(profiles), w_z, P(wpb), P(slb), T, W, P(gfb), P(f2x),
                                                     P(gwp2x), P(gG2x), P(gC2x), n, P(gz2x), abi.PCT_FIXED_POINT,
                                                     P(ws), ws.nbytes, None))
    q1, q2 = gz1x.get(n, np.int64), gz2x.get(n, np.int64)
    np.testing.assert_array_equal(q1, q2)
    assert np.count_nonzero(q2) > 20 and np.abs(q2).max() < 2 ** 53
    np.testing.assert_array_equal(bits(gwp2x.get(wp_all.shape, np.float32)), bits(gwp2))
    zf = Buf(4 * n)
    check("fixed_to_float", L.pct_fixed_to_float(P(gz2x), n, P(zf), None))
    zf = zf.get(n, np.float32)
    np.testing.assert_array_equal(bits(zf), bits((q2.astype(np.float64) * 2.0 ** -32).astype(np.float32)))
    np.testing.assert_allclose(zf, a, rtol=1e-5, atol=2e-5 * max(1.0, float(np.abs(a).max())))
    for qx, fl in ((gG2x, gG2), (gC2x, gC2)):
        qv, fv = qx.get(int(np.prod(shape)), np.int64), fl.get(int(np.prod(shape)), np.float32)
        np.testing.assert_allclose(qv * 2.0 ** -32, fv, rtol=1e-5, atol=2e-5 * max(1.0, float(np.abs(fv).max())))
    assert L.pct_fixed_to_float(P(gz2x), n, P(gz2x), None) == abi.PCT_ERR_ARG
    # waypoints shuffled over each profile's trajectories and slices: rounds
    # whose windows do not share one box take the per-lane path; f and dL/dwp
    # still equal the per-profile path's
    rng = np.random.default_rng(5)
    wps_s = wp_all.reshape(len(profiles), -1, 3).copy()
    sls_s = sl_all.reshape(len(profiles), -1).copy()
    for i in range(len(profiles)):
        perm = rng.permutation(wps_s.shape[1])
        wps_s[i], sls_s[i] = wps_s[i][perm], sls_s[i][perm]
    wps_s = np.ascontiguousarray(wps_s.reshape(wp_all.shape))
    sls_s = np.ascontiguousarray(sls_s.reshape(sl_all.shape))
    f1s, gwp1s = [], []
    for i, r in enumerate(profiles):
        cost, _ = evaluate(G, Cc, grid, e, [r], keep=False)
        wpb1, slb1, gfb1 = Buf.of(wps_s[i]), Buf.of(sls_s[i]), Buf.of(gf_all[i])
        f1s.append(sample_fwd(cost, G, grid, e, r, w_z, wpb1, slb1, T, W))
        gz1s = Buf(8 * n)
        gwp1s.append(traj_bwd(G, Cc, cost, aG, aC, grid, e, r, w_z, wpb1, slb1, T, W, gfb1, n, gz1s,
                              abi.PCT_FIXED_POINT))
    f2s, gwp2s, gz2s = Buf(4 * len(profiles) * T), Buf(12 * wp_all[..., 0].size), Buf(8 * n)
    wpbs, slbs = Buf.of(wps_s), Buf.of(sls_s)   # named: a temporary would be freed before the call
    check("multi shuffled", L.pct_trajectory_cost_multi(P(G), P(Cc), P(aG), P(aC), C.byref(g), C.byref(e), rs,
                                                        len(profiles), w_z, P(wpbs), P(slbs), T, W, P(gfb), P(f2s),
                                                        P(gwp2s), None, None, n, P(gz2s), abi.PCT_FIXED_POINT, P(ws),
                                                        ws.nbytes, None))
    np.testing.assert_array_equal(bits(f2s.get((len(profiles), T), np.float32)), bits(np.stack(f1s)))
    np.testing.assert_array_equal(bits(gwp2s.get(wp_all.shape, np.float32)), bits(np.stack(gwp1s)))
    # values only: the same f, gradients untouched
    f3 = Buf(4 * len(profiles) * T)
    check("multi value", L.pct_trajectory_cost_multi(P(G), P(Cc), None, None, C.byref(g), C.byref(e), rs,
                                                     len(profiles), w_z, P(wpb), P(slb), T, W, None, P(f3), None,
                                                     None, None, 0, None, abi.PCT_DESCRIPTORS_RESIDENT, P(ws),
                                                     ws.nbytes, None))
    np.testing.assert_array_equal(bits(f3.get((len(profiles), T), np.float32)), bits(f2))
    # the oracle: FP64 values and gradients summed over the profiles
    rz = np.zeros(n)
    rG_all = np.zeros(shape)
    rC_all = np.zeros(shape)
    uz = np.zeros(n, bool)
    for i, r in enumerate(profiles):
        cT = oracle.evaluate(tm["ground"], tm["ceil"], grid["res"], r)
        fr = oracle.sample_fwd(cT, tm["ground"], grid, w_z, r["d_ref"], wp_all[i], sl_all[i])
        assert np.all(np.abs(f2[i] - fr) <= 2e-5 * W + 1e-6 * np.abs(fr))
        g64 = gf_all[i].astype(np.float64)
        rgwp, rgc, rgg = oracle.sample_bwd(cT, tm["ground"], grid, w_z, r["d_ref"], wp_all[i], sl_all[i], g64)
        close(gwp2[i], rgwp)
        rG, rC, unc = oracle.eval_bwd(tm["ground"], tm["ceil"], grid["res"], r, rgc)
        rG_all += rG + rgg
        rC_all += rC
        rz += oracle.route(rG + rgg, rC, tm["arg_ground"], tm["arg_ceil"], n)
        for arr in (tm["arg_ground"], tm["arg_ceil"]):
            m = (arr >= 0) & unc
            uz[arr[m]] = True
    assert np.count_nonzero(rz) > 20
    close(gz2.get(n, np.float32), rz, ~uz)
    close(gG2.get(shape, np.float32), rG_all)
    close(gC2.get(shape, np.float32), rC_all)
    say(f"multi-profile value+grad: {len(profiles)} profiles x {T} x {W}: equals the per-profile path, "
        "oracle within tolerance")


def plan_run(cT, eG, layers, start, goals, what, band=0.0):
    """Distances and paths of the library against the oracle's, bit for bit."""
    N, ny, nx = cT.shape
    g = grid_s(dict(x0=0.0, y0=0.0, res=0.1, nx=nx, ny=ny, slice_dz=0.3))
    e = abi.pct_extent(0.0, 1.0, N, 0, 0, 0)
    rb = robot_s(robot())
    cB = robot()["c_barrier"]
    Lc = len(layers)
    lay = (C.c_int32 * Lc)(*layers)
    cb, gb = Buf.of(np.ascontiguousarray(cT, np.float32)), Buf.of(np.ascontiguousarray(eG, np.float32))
    dist = Buf(8 * Lc * ny * nx)
    ws = Buf(L.pct_plan_workspace_bytes(nx, ny, Lc))
    rounds, tiles = C.c_int32(), C.c_int64()
    check("plan", L.pct_plan_distance(P(cb), P(gb), C.byref(g), C.byref(e), C.byref(rb), lay, Lc, start[0], start[1],
                                      start[2], band, P(dist), P(ws), ws.nbytes, C.byref(rounds), C.byref(tiles),
                                      None))
    d = dist.get((Lc, ny, nx), np.float64)
    ref = oracle.plan(cT[layers], eG[layers], cB, start)
    assert np.array_equal(d.view(np.uint64), ref.view(np.uint64)), f"{what}: distances differ"
    n_paths = 0
    for goal in goals:
        pb = Buf(4 * 3 * Lc * nx * ny)
        n = C.c_int32()
        check("path", L.pct_plan_path(P(dist), C.byref(g), Lc, start[0], start[1], start[2], goal[0], goal[1], goal[2],
                                      P(pb), Lc * nx * ny, C.byref(n), P(ws), ws.nbytes, None))
        rp = oracle.plan_path(cT[layers], eG[layers], cB, ref, start, goal)
        if rp is None:
            assert n.value == 0, f"{what}: goal {goal} should be unreachable"
            continue
        got = pb.get((n.value, 3), np.int32)
        rp = rp.copy()
        rp[:, 2] = np.asarray(layers)[rp[:, 2]]
        assert np.array_equal(got, rp), f"{what}: path to {goal} differs"
        n_paths += 1
    say(f"plan {what} {Lc}x{ny}x{nx}: distances bit-exact ({int(np.isfinite(ref).sum())} reachable, "
        f"{rounds.value} rounds, {tiles.value} tiles), {n_paths} paths identical")


def case_plan():
    """Path search through the slices: random layers over several tiles with
    ragged edges, a subset of slices, a winding single layer, a barrier
    start, an unreachable goal."""
    cT, eG = scenes.plan_layers(11, 3, 150, 130)
    rng = np.random.default_rng(5)
    goals = [(int(rng.integers(130)), int(rng.integers(150)), int(rng.integers(3))) for _ in range(6)]
    plan_run(cT, eG, [0, 1, 2], (7, 140, 0), goals, "random layers")
    plan_run(cT, eG, [0, 1, 2], (7, 140, 0), goals, "random layers, narrow band", band=16.0)
    plan_run(cT, eG, [0, 1, 2], (7, 140, 0), goals, "random layers, one band", band=1e300)
    cT, eG = scenes.plan_layers(12, 5, 70, 97, p_same=0.5)
    plan_run(cT, eG, [0, 2, 3], (96, 0, 1), [(0, 69, 0), (50, 30, 2), (96, 0, 1)], "slice subset")
    cT, eG = scenes.plan_serpentine(13, 90, 75)
    plan_run(cT, eG, [0], (0, 0, 0), [(0, 89, 0), (74, 45, 0)], "serpentine")
    cT, eG = scenes.plan_layers(14, 2, 64, 64, p_block=0.6)
    cT[0, 10, 10] = 50.0
    plan_run(cT, eG, [0, 1], (10, 10, 0), [(63, 63, 1), (0, 0, 0)], "barrier start, sparse map")
    cT = np.full((1, 1, 1), 3.0, np.float32)
    plan_run(cT, np.zeros_like(cT), [0], (0, 0, 0), [(0, 0, 0)], "single cell")


def case_plan_query():
    """Goal-directed queries: the goal's distance equals the oracle's full
    Dijkstra, labels below the settled bound are exact, the others upper
    bounds."""
    cT, eG = scenes.plan_layers(21, 3, 150, 130)
    layers, start = [0, 1, 2], (7, 140, 0)
    ref = oracle.plan(cT, eG, 50.0, start)
    N, ny, nx = cT.shape
    gs = grid_s(dict(x0=0.0, y0=0.0, res=0.1, nx=nx, ny=ny, slice_dz=0.3))
    e = abi.pct_extent(0.0, 1.0, N, 0, 0, 0)
    r = robot()
    r["c_barrier"] = 50.0
    rb = robot_s(r)
    cb, eb = Buf.of(np.ascontiguousarray(cT, np.float32)), Buf.of(np.ascontiguousarray(eG, np.float32))
    dist, ws = Buf(8 * N * ny * nx), Buf(L.pct_plan_workspace_bytes(nx, ny, N))
    lay = (C.c_int32 * 3)(*layers)
    for goal in [(20, 130, 0), (100, 20, 2), (7, 140, 0)]:
        gd, st, ro, ti = C.c_double(), C.c_double(), C.c_int32(), C.c_int64()
        check("plan_query", L.pct_plan_query(P(cb), P(eb), C.byref(gs), C.byref(e), C.byref(rb), lay, 3, *start,
                                             *goal, 0.0, P(dist), P(ws), ws.nbytes, C.byref(gd), C.byref(st),
                                             C.byref(ro), C.byref(ti), None))
        d = dist.get((N, ny, nx), np.float64)
        sm = d < st.value
        assert gd.value == ref[goal[2], goal[1], goal[0]], (goal, gd.value)
        assert np.array_equal(d[sm], ref[sm]) and np.all(d[~sm] >= ref[~sm])
        say(f"plan query to {goal}: distance {gd.value:.3f} exact, {ro.value} rounds, {int(sm.sum())} labels settled")


def unique_run(eG, eC, cT, keep, what):
    """Unique cells of the kept slices against the oracle's, bit for bit."""
    N, ny, nx = eG.shape
    g = grid_s(dict(x0=0.0, y0=0.0, res=0.1, nx=nx, ny=ny, slice_dz=0.3))
    e = abi.pct_extent(0.0, 1.0, N, 0, 0, 0)
    r = robot()
    rb = robot_s(r)
    bufs = [Buf.of(np.ascontiguousarray(a, np.float32)) for a in (eG, eC, cT)]
    kb = Buf.of(np.ascontiguousarray(np.asarray(keep, np.uint8)))
    ws = Buf(L.pct_unique_workspace_bytes(C.byref(g), C.byref(e)))
    off = np.zeros(N + 1, np.int64)
    m = C.c_int64()
    offp = off.ctypes.data_as(C.POINTER(C.c_int64))
    check("unique count", L.pct_unique_cells(*[P(b) for b in bufs], P(kb), C.byref(g), C.byref(e), C.byref(rb), 0,
                                             None, None, None, None, offp, C.byref(m), P(ws), ws.nbytes, None))
    M = m.value
    ref = oracle.unique_cells(eG, eC, cT, r["c_barrier"], keep)
    assert M == len(ref["cell"]), f"{what}: {M} unique cells, oracle {len(ref['cell'])}"
    assert np.array_equal(off, ref["slice_off"]), f"{what}: slice offsets differ"
    if M > 0:
        outs = [Buf(4 * M) for _ in range(4)]
        if M > 1:
            st = L.pct_unique_cells(*[P(b) for b in bufs], P(kb), C.byref(g), C.byref(e), C.byref(rb), M - 1,
                                    *[P(o) for o in outs], offp, C.byref(m), P(ws), ws.nbytes, None)
            assert st == abi.PCT_ERR_CAPACITY and m.value == M, f"{what}: capacity check"
        check("unique", L.pct_unique_cells(*[P(b) for b in bufs], P(kb), C.byref(g), C.byref(e), C.byref(rb), M,
                                           *[P(o) for o in outs], offp, C.byref(m), P(ws), ws.nbytes, None))
        assert np.array_equal(outs[0].get(M, np.int32), ref["cell"]), f"{what}: cells differ"
        for o, name in zip(outs[1:], ("ground", "ceil", "cost")):
            assert np.array_equal(bits(o.get(M, np.float32)), bits(ref[name])), f"{what}: {name} differs"
    say(f"unique cells {what} {N}x{ny}x{nx}: {M} cells in {int(np.count_nonzero(keep))} kept slices, bit-exact")


def case_unique():
    """Sparse storage of the kept slices' unique cells: an oracle-evaluated
    building (ragged last block), a random keep list, no kept slice."""
    sc = scenes.multistorey_scene(44, 9.3, 7.1, 250_000, n_floors=3)
    tm = oracle.tomogram(sc.points, sc.grid)
    r = robot()
    cT = oracle.evaluate(tm["ground"], tm["ceil"], sc.grid["res"], r)
    keep = oracle.simplify(tm["ground"], cT, r["c_barrier"])
    c32 = cT.astype(np.float32)
    unique_run(tm["ground"], tm["ceil"], c32, keep, "building")
    rng = np.random.default_rng(9)
    unique_run(tm["ground"], tm["ceil"], c32, rng.random(len(keep)) < 0.5, "random keep list")
    unique_run(tm["ground"], tm["ceil"], c32, np.zeros(len(keep), bool), "nothing kept")


def case_insert():
    """Insertion into an existing tomogram equals the build of the union
    (heights and ids, bit for bit, and the oracle's); the re-evaluated
    window makes the cost map equal a whole-map evaluation of the union;
    heights that would move the planes are refused."""
    sc = scenes.multistorey_scene(45, 13.3, 9.7, 300_000, n_floors=2)
    g = sc.grid
    pts = np.ascontiguousarray(sc.points, np.float32)
    rng = np.random.default_rng(10)
    # a scan of a box on the ground floor: new points within the height range
    m = 40_000
    bx = np.column_stack([rng.uniform(3.0, 4.7, m), rng.uniform(2.0, 3.3, m), rng.uniform(0.0, 0.9, m)])
    new = np.ascontiguousarray(bx, np.float32)
    xa = Buf.of(pts)
    e = extent(xa, len(pts), g)
    G, Cc, aG, aC = build(xa, len(pts), g, e, True)
    N = e.n_slices
    cells = N * g["nx"] * g["ny"]
    r = robot()
    cost, kp = evaluate(G, Cc, g, e, [r])
    gs = grid_s(g)
    xb = Buf.of(new)
    ws = Buf(L.pct_insert_workspace_bytes(len(new), C.byref(gs)))
    bb = (C.c_int32 * 4)()
    check("insert", L.pct_tomogram_insert(P(xb), len(new), len(pts), C.byref(gs), C.byref(e), P(G), P(Cc), P(aG),
                                          P(aC), bb, P(ws), ws.nbytes, None))
    union = np.ascontiguousarray(np.concatenate([pts, new]), np.float32)
    xu = Buf.of(union)
    eu = extent(xu, len(union), g)
    assert (eu.n_slices, eu.n_used, eu.n_dropped, np.float32(eu.z_max)) == (e.n_slices, e.n_used, e.n_dropped,
                                                                              np.float32(e.z_max)), "extent"
    Gu, Cu, aGu, aCu = build(xu, len(union), g, eu, True)
    for a, b, name in ((G, Gu, "ground"), (Cc, Cu, "ceil"), (aG, aGu, "ids"), (aC, aCu, "ceil ids")):
        dt = np.int32 if "ids" in name else np.float32
        assert np.array_equal(bits(a.get(cells, dt)), bits(b.get(cells, dt))), f"insert: {name} differs from the union"
    tm = oracle.tomogram(union, g)
    assert np.array_equal(bits(G.get(cells, np.float32)), bits(tm["ground"].ravel())), "insert: oracle ground"
    assert np.array_equal(aG.get(cells, np.int32), tm["arg_ground"].ravel()), "insert: oracle ids"
    # window re-evaluation
    rr = C.c_int32()
    check("radius", L.pct_kernel_radius(C.byref(robot_s(r)), C.c_float(g["res"]), C.byref(rr)))
    grow = rr.value + 2
    win = (bb[0] - grow, bb[1] - grow, bb[2] + 1 + grow, bb[3] + 1 + grow)
    rb = robot_s(r)
    ews = Buf(L.pct_eval_workspace_bytes(C.byref(gs), C.byref(e), 1))
    check("window", L.pct_eval_traversability_window(P(G), P(Cc), C.byref(gs), C.byref(e), C.byref(rb), *win, P(cost),
                                                     P(kp), P(ews), ews.nbytes, None))
    cu, ku = evaluate(Gu, Cu, g, eu, [r])
    assert np.array_equal(bits(cost.get(cells, np.float32)), bits(cu.get(cells, np.float32))), "window: cost"
    assert np.array_equal(kp.get(N, np.uint8), ku.get(N, np.uint8)), "window: keep"
    # a point below z_min would move the planes: refused, nothing written
    low = Buf.of(np.array([[5.0, 5.0, e.z_min - 1.0]], np.float32))
    st = L.pct_tomogram_insert(P(low), 1, len(union), C.byref(gs), C.byref(e), P(G), P(Cc), P(aG), P(aC),
                               bb, P(ws), ws.nbytes, None)
    assert st == abi.PCT_ERR_ARG, "insert below z_min must be refused"
    assert np.array_equal(bits(G.get(cells, np.float32)), bits(Gu.get(cells, np.float32)))
    say(f"insert: {len(new)} points into {len(pts)}, box {tuple(bb)}, window {win}: tomogram, ids, cost and keep "
        f"equal the union's")


TRAJ_PRM = dict(w_z=2.0, w_c=0.05, w_v=1.0, w_a=0.5, w_h=20.0, w_T=1.0, c_safe=5.0, v_max=1.2, a_max=2.0,
                d_ref=0.65, d_min=0.5, samples=8)


def traj_maps():
    """An oracle-built and oracle-evaluated three-storey map."""
    sc = scenes.multistorey_scene(44, 9.3, 7.1, 250_000, n_floors=3)
    tm = oracle.tomogram(sc.points, sc.grid)
    r = dict(scenes.ROBOT_TABLE1)
    cT = oracle.evaluate(tm["ground"], tm["ceil"], sc.grid["res"], r).astype(np.float32)
    return sc.grid, cT, tm["ground"], tm["ceil"]


def traj_run(grid, maps, prm, pr, iters=None, step=1e-3):
    cT, eG, eC = maps
    n, M = pr["slices"].shape
    gs = grid_s(grid)
    e = abi.pct_extent(0.0, 1.0, cT.shape[0], 0, 0, 0)
    tp = abi.pct_traj_params(*[float(prm[k]) for k in ("w_z", "w_c", "w_v", "w_a", "w_h", "w_T", "c_safe", "v_max",
                                                        "a_max", "d_ref", "d_min")], int(prm["samples"]))
    bufs = [Buf.of(np.ascontiguousarray(a)) for a in (cT, eG, eC)]
    bd, sl = Buf.of(pr["bound"]), Buf.of(pr["slices"])
    kn = Buf.of(pr["knots"]) if M > 1 else None
    ta = Buf.of(pr["tau"])
    phi = Buf(8 * n)
    if iters is None:
        gk, gt, cf = (Buf(8 * n * (M - 1) * 3) if M > 1 else None), Buf(8 * n * M), Buf(8 * n * M * 18)
        check("traj_eval", L.pct_traj_eval(P(bufs[0]), P(bufs[1]), P(bufs[2]), C.byref(gs), C.byref(e), C.byref(tp), n,
                                           M, P(bd), P(sl), P(kn), P(ta), P(phi), P(gk), P(gt), P(cf), None))
        return (phi.get(n, np.float64), gk.get((n, M - 1, 3), np.float64) if M > 1 else np.zeros((n, 0, 3)),
                gt.get((n, M), np.float64), cf.get((n, M, 6, 3), np.float64))
    done = Buf(4 * n)
    check("traj_optimize", L.pct_traj_optimize(P(bufs[0]), P(bufs[1]), P(bufs[2]), C.byref(gs), C.byref(e), C.byref(tp),
                                               n, M, P(bd), P(sl), P(kn), P(ta), int(iters), float(step), P(phi),
                                               P(done), None))
    return (phi.get(n, np.float64), kn.get((n, M - 1, 3), np.float64) if M > 1 else np.zeros((n, 0, 3)),
            ta.get((n, M), np.float64), done.get(n, np.int32))


def case_traj_opt():
    """Trajectory optimisation (Sec. III-E): objective, gradient and spline
    coefficients against the oracle's KKT solve and autograd, for one to 64
    pieces and 1 to 16 samples, slices outside the map included; then
    optimiser runs against the oracle's loop."""
    from oracle import traj as otraj
    grid, cT, eG, eC = traj_maps()
    maps = (cT, eG, eC)
    N = cT.shape[0]
    for M, K, n in ((1, 4, 2), (2, 1, 2), (5, 7, 3), (33, 3, 1), (64, 2, 1)):
        prm = dict(TRAJ_PRM, samples=K)
        pr = scenes.traj_problems(20 + M, n, M, (1.0, 8.0), (1.0, 6.0), 0.7, slices=(0, 3, N - 1, N + 2))
        phi, gk, gt, cf = traj_run(grid, maps, prm, pr)
        for t in range(n):
            args = (pr["knots"][t], pr["tau"][t], pr["bound"][t, 0], pr["bound"][t, 1], pr["slices"][t], maps, grid,
                    prm)
            p_o, gk_o, gt_o = otraj.objective(*args)
            c_o = otraj.coefficients(*args[:4])
            scale = max(1.0, abs(p_o))
            assert abs(phi[t] - p_o) <= 1e-9 * scale, (M, K, t, phi[t], p_o)
            np.testing.assert_allclose(cf[t], c_o, rtol=1e-8, atol=1e-8 * np.abs(c_o).max())
            gs_ = max(1.0, np.abs(np.concatenate([gk_o.ravel(), gt_o])).max())
            np.testing.assert_allclose(gk[t], gk_o, rtol=1e-7, atol=1e-8 * gs_)
            np.testing.assert_allclose(gt[t], gt_o, rtol=1e-7, atol=1e-8 * gs_)
        say(f"traj eval: M={M} K={K} n={n}: phi, gradients and coefficients equal the oracle's")
    for M, K, n, iters in ((1, 4, 1, 6), (4, 6, 2, 5)):
        prm = dict(TRAJ_PRM, samples=K)
        pr = scenes.traj_problems(40 + M, n, M, (1.0, 8.0), (1.0, 6.0), 0.7, slices=(0, 3))
        phi, kn, ta, done = traj_run(grid, maps, prm, pr, iters=iters, step=1e-3)
        for t in range(n):
            k_o, t_o, p_o, d_o = otraj.optimize(pr["knots"][t], pr["tau"][t], pr["bound"][t, 0], pr["bound"][t, 1],
                                                pr["slices"][t], maps, grid, prm, iters, 1e-3)
            assert done[t] == d_o, (done[t], d_o)
            assert abs(phi[t] - p_o) <= 1e-7 * max(1.0, abs(p_o)), (phi[t], p_o)
            np.testing.assert_allclose(kn[t], k_o, rtol=1e-7, atol=1e-9)
            np.testing.assert_allclose(ta[t], t_o, rtol=1e-7, atol=1e-9)
        say(f"traj optimise: M={M} K={K} {iters} iterations: iterates equal the oracle's")


CASES = {k[5:]: v for k, v in globals().items() if k.startswith("case_")}

if __name__ == "__main__":
    oracle.lib()
    names = sys.argv[1:] or list(CASES)
    for name in names:
        say(f"case {name}")
        CASES[name]()
    say("all passed")
