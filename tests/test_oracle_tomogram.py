"""Pins of the oracle's tomogram construction (Sec. III-A, Algorithm 1).

Each test checks the oracle against something other than itself: a
hand-enumerated fixture, the plane rule's invariants, or an independent
sort-and-search algorithm for the same definition."""
import math

import numpy as np
import pytest

import scenes
from conftest import load_golden


def _arr(v, dt):
    return np.array(v, dtype=dt)


def test_golden_tiny_tomogram(oracle_lib):
    g = load_golden("tiny_tomogram.json")
    pts = np.array(g["points"], dtype=np.float32)
    tm = oracle_lib.tomogram(pts, g["grid"])
    assert tm["zmin"] == g["zmin"] and tm["zmax"] == g["zmax"]
    assert tm["n_used"] == g["n_used"]
    np.testing.assert_array_equal(tm["h"], _arr(g["planes"], np.float32))
    np.testing.assert_array_equal(tm["ground"], _arr(g["ground"], np.float32))
    np.testing.assert_array_equal(tm["ceil"], _arr(g["ceil"], np.float32))
    np.testing.assert_array_equal(tm["arg_ground"], _arr(g["arg_ground"], np.int32))
    np.testing.assert_array_equal(tm["arg_ceil"], _arr(g["arg_ceil"], np.int32))
    # the -0.0 input is stored as +0.0
    assert not np.signbit(tm["ground"][0, 1, 2])


def test_planes_rule(oracle_lib):
    """First plane d_s above the lowest point; the last one above the highest,
    the one before it not (the count is the least that covers the cloud)."""
    for zmin, zmax, ds in [(0.0, 1.25, 0.5), (-0.0797, 3.0739, 0.4), (-0.1, 16.6, 0.3),
                           (12.5, 12.5, 0.3), (5.0, 5.2, 0.5)]:
        zmin, zmax, ds = (float(np.float32(v)) for v in (zmin, zmax, ds))
        h = oracle_lib.planes(zmin, zmax, ds)
        assert h[0] == np.float32(np.float32(zmin) + np.float32(ds))
        assert h[-1] > np.float32(zmax)
        if len(h) > 1:
            assert h[-2] <= np.float32(zmax)
        assert np.all(np.diff(h) > 0)
        # planes follow z_min + (k+1) d_s to FP32 rounding
        k = np.arange(1, len(h) + 1)
        np.testing.assert_allclose(h, zmin + k * ds, rtol=0, atol=4 * np.spacing(np.float32(abs(zmax) + ds)))


def test_flat_floor_gives_one_slice(oracle_lib):
    sc = scenes.dense_surface_scene(20, 12, 0.1, lambda x, y: 0.02 * np.sin(x) * np.cos(y), slice_dz=0.3)
    tm = oracle_lib.tomogram(sc.points, sc.grid)
    assert len(tm["h"]) == 1
    assert np.all(np.isfinite(tm["ground"][0]))
    assert np.all(np.isinf(tm["ceil"][0]))


def test_plane_collision_rejected(oracle_lib):
    with pytest.raises(ValueError):
        oracle_lib.planes(1.0e7, 1.0e7 + 10.0, 1e-4)


def _sorted_reference(points, grid, h):
    """Independent algorithm for the same definition: per cell, sort the
    heights once and binary-search each plane (ground = last height at or
    below the plane, ceiling = first height above it)."""
    pts = np.asarray(points, np.float32)
    ok = np.all(np.isfinite(pts), axis=1)
    qx = (pts[:, 0] - np.float32(grid["x0"])) / np.float32(grid["res"])
    qy = (pts[:, 1] - np.float32(grid["y0"])) / np.float32(grid["res"])
    ok &= (qx >= 0) & (qx < grid["nx"]) & (qy >= 0) & (qy < grid["ny"])
    ids = np.flatnonzero(ok)
    ix = np.floor(qx[ids]).astype(np.int64)
    iy = np.floor(qy[ids]).astype(np.int64)
    z = pts[ids, 2] + np.float32(0.0)
    cell = iy * grid["nx"] + ix
    order = np.lexsort((ids, z, cell))            # by cell, then z, then id
    cell, z, ids = cell[order], z[order], ids[order]
    N, plane = len(h), grid["nx"] * grid["ny"]
    eG = np.full((N, plane), -np.inf, np.float32)
    eC = np.full((N, plane), np.inf, np.float32)
    aG = np.full((N, plane), -1, np.int32)
    aC = np.full((N, plane), -1, np.int32)
    starts = np.searchsorted(cell, np.arange(plane), "left")
    ends = np.searchsorted(cell, np.arange(plane), "right")
    for c in np.flatnonzero(ends > starts):
        zs, idc = z[starts[c]:ends[c]], ids[starts[c]:ends[c]]
        for k in range(N):
            j = np.searchsorted(zs, h[k], "right")
            if j > 0:
                eG[k, c] = zs[j - 1]
                aG[k, c] = idc[np.searchsorted(zs, zs[j - 1], "left")]
            if j < len(zs):
                eC[k, c] = zs[j]
                aC[k, c] = idc[j]
    shp = (N, grid["ny"], grid["nx"])
    return eG.reshape(shp), eC.reshape(shp), aG.reshape(shp), aC.reshape(shp)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_matches_sort_and_search(oracle_lib, seed):
    rng = np.random.default_rng(100 + seed)
    sc = scenes.multistorey_scene(seed, 6.3, 4.1, 30_000, n_floors=3, slice_dz=0.3)
    pts = sc.points.copy()
    # ties: duplicate heights, points on plane heights and cell edges, junk
    dup = pts[rng.integers(0, len(pts), 500)]
    pts = np.concatenate([pts, dup, np.array([[np.nan, 1, 1], [1, np.inf, 1], [-5, 1, 1]], np.float32)])
    tm = oracle_lib.tomogram(pts, sc.grid)
    h = tm["h"]
    snap = pts[rng.integers(0, len(pts), 300)].copy()
    snap[:, 2] = h[rng.integers(0, len(h), 300)]
    snap[:150, 0] = np.float32(sc.grid["res"]) * rng.integers(0, sc.grid["nx"], 150)
    pts = np.concatenate([pts, snap])
    tm = oracle_lib.tomogram(pts, sc.grid)
    ref = _sorted_reference(pts, sc.grid, tm["h"])
    for a, b in zip((tm["ground"], tm["ceil"], tm["arg_ground"], tm["arg_ceil"]), ref):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("seed", range(6))
def test_invariants_random_clouds(oracle_lib, seed):
    """e^G_k <= h_k < e^C_k; both layers non-decreasing in k; every value is
    the height of a point of that cell, identified by the recorded id."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 400))
    grid = dict(x0=-0.3, y0=0.2, res=0.25, nx=int(rng.integers(1, 9)), ny=int(rng.integers(1, 9)),
                slice_dz=float(rng.uniform(0.05, 0.7)))
    pts = np.stack([rng.uniform(-0.5, 2.5, n), rng.uniform(0.0, 2.5, n),
                    np.round(rng.uniform(-1, 3, n), 1)], 1).astype(np.float32)
    tm = oracle_lib.tomogram(pts, grid)
    if tm["n_used"] == 0:
        return
    h, eG, eC = tm["h"], tm["ground"], tm["ceil"]
    assert np.all(eG <= h[:, None, None])
    assert np.all(eC > h[:, None, None])
    assert np.all(eG[1:] >= eG[:-1]) and np.all(eC[1:] >= eC[:-1])
    for arr, ids in ((eG, tm["arg_ground"]), (eC, tm["arg_ceil"])):
        v = np.isfinite(arr)
        assert np.array_equal(v, ids >= 0)
        np.testing.assert_array_equal(pts[ids[v], 2], arr[v])
        k, iy, ix = np.nonzero(v)
        p = pts[ids[v]]
        assert np.all(np.floor((p[:, 0] - np.float32(grid["x0"])) / np.float32(grid["res"])) == ix)
        assert np.all(np.floor((p[:, 1] - np.float32(grid["y0"])) / np.float32(grid["res"])) == iy)
    # a cell with points has ground or ceiling in every slice
    occupied = np.isfinite(eG) | np.isfinite(eC)
    assert np.all(occupied == occupied[0:1])


def test_window_build_equals_full_build(oracle_lib):
    """The windowed loop (used for full-size checks) is the full loop cut to
    the window, including windows at the grid edge."""
    sc = scenes.config0_scene()
    tm = oracle_lib.tomogram(sc.points, sc.grid)
    full = (tm["ground"], tm["ceil"], tm["arg_ground"], tm["arg_ceil"])
    for wx0, wy0, wnx, wny in [(37, 150, 50, 21), (0, 0, 7, 9), (190, 180, 10, 20)]:
        w = oracle_lib.build_window(sc.points, sc.grid, tm["h"], wx0, wy0, wnx, wny)
        for a, b in zip(w, full):
            np.testing.assert_array_equal(a, b[:, wy0:wy0 + wny, wx0:wx0 + wnx])
