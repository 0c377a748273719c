"""Pins of the oracle's tomogram simplification (Sec. III-C, Eqs. (7)-(9)).

Dense noise-free scenes with a known number of distinct walkable levels,
and the property the simplification exists for (Eq. (7)): every traversable
cell of a removed slice is still present, with the same ground and no higher
cost, in a slice that is kept."""
import numpy as np
import pytest

import scenes

CB = 50.0


def _wall(ix, iy0, iy1, res, top, step=0.1):
    zs = np.arange(step, top + 1e-9, step)
    pts = [(res * (ix + 0.5), res * (iy + 0.5), z) for iy in range(iy0, iy1) for z in zs]
    return np.array(pts, np.float32)


def _run(oracle_lib, sc):
    tm = oracle_lib.tomogram(sc.points, sc.grid)
    rb = oracle_lib.robot_from_physical(sc.robot, sc.grid["res"])
    cT = oracle_lib.evaluate(tm["ground"], tm["ceil"], sc.grid["res"], rb)
    keep = oracle_lib.simplify(tm["ground"], cT, CB)
    return tm, cT, keep


def _covered(eG, cT, keep):
    """Eq. (7): each traversable cell of each slice has a kept slice with the
    same ground and a cost no higher."""
    N = eG.shape[0]
    kept = np.flatnonzero(keep)
    for k in range(N):
        trav = cT[k] < CB
        ok = np.zeros_like(trav)
        for j in kept:
            ok |= (eG[j] == eG[k]) & (cT[j] <= cT[k])
        if not np.all(ok[trav]):
            return False
    return True


def test_single_floor_with_walls_one_layer(oracle_lib):
    res = 0.1
    wall = np.concatenate([_wall(20, 5, 25, res, 3.0), _wall(8, 2, 12, res, 2.0)])
    sc = scenes.dense_surface_scene(40, 30, res, lambda x, y: 0 * x, per_cell=1, slice_dz=0.3,
                                    extra=[wall])
    tm, cT, keep = _run(oracle_lib, sc)
    assert len(tm["h"]) >= 10
    assert (cT < CB).any()
    assert keep.sum() == 1
    assert _covered(tm["ground"], cT, keep)


def test_two_storeys_two_layers(oracle_lib):
    """Ground floor everywhere, an upper floor (slab underside 2.8 m, top
    3.0 m) over half the area: two walkable levels, two kept slices."""
    res = 0.1
    nx, ny = 40, 30
    xs, ys = np.meshgrid((np.arange(20, nx) + 0.5) * res, (np.arange(ny) + 0.5) * res)
    slab = [np.stack([xs.ravel(), ys.ravel(), np.full(xs.size, z)], 1) for z in (2.8, 3.0)]
    sc = scenes.dense_surface_scene(nx, ny, res, lambda x, y: 0 * x, per_cell=1, slice_dz=0.3,
                                    extra=slab)
    tm, cT, keep = _run(oracle_lib, sc)
    assert keep.sum() == 2
    assert _covered(tm["ground"], cT, keep)
    levels = {float(np.nanmax(np.where(cT[k] < CB, tm["ground"][k], np.nan))) for k in np.flatnonzero(keep)}
    assert levels == {0.0, 3.0}


def test_ramp_under_platform_drops_middle_slices(oracle_lib):
    """The slope example of the tomogram figure: a ramp climbs from the floor
    to a platform that overhangs the floor.  Slices cut through the ramp
    partway hold nothing that the floor slice and the platform slice do not
    hold, so only two slices survive."""
    res = 0.1
    nx, ny = 60, 30
    ramp0, ramp1, top, under = 10, 34, 1.5, 1.2

    def ground(x, y):
        ix = np.floor(x / res)
        z = np.where(ix < ramp0, 0.0, np.where(ix < ramp1, (ix - ramp0 + 0.5) / (ramp1 - ramp0) * top, np.nan))
        return np.where((y > 1.0) & (y < 2.0) | (ix < ramp0), z, np.where(ix >= ramp1, 0.0, np.nan))
    xs, ys = np.meshgrid((np.arange(ramp1, nx) + 0.5) * res, (np.arange(ny) + 0.5) * res)
    plat = [np.stack([xs.ravel(), ys.ravel(), np.full(xs.size, z)], 1) for z in (under, top)]
    sc = scenes.dense_surface_scene(nx, ny, res, ground, per_cell=1, slice_dz=0.3, extra=plat)
    tm, cT, keep = _run(oracle_lib, sc)
    N = len(tm["h"])
    assert N >= 5
    assert keep.sum() == 2
    assert _covered(tm["ground"], cT, keep)
    # kept: the last slice that still passes under the platform, and the top
    # slice; the slices between them cut the ramp part-way and are removed
    floor_slice = int(np.flatnonzero(tm["h"] < under)[-1])
    assert list(np.flatnonzero(keep)) == [floor_slice, N - 1]
    assert N - 1 - floor_slice >= 2


@pytest.mark.parametrize("seed", [11, 12])
def test_coverage_on_dense_multistorey(oracle_lib, seed):
    sc = scenes.multistorey_scene(seed, 9.0, 7.0, 400_000, n_floors=3, beam_cover=0.05)
    tm, cT, keep = _run(oracle_lib, sc)
    assert (cT < CB).any()
    assert 1 <= keep.sum() < len(keep)
    assert _covered(tm["ground"], cT, keep)


def test_three_valued_check(oracle_lib):
    """The check accepts the oracle's own decisions and rejects a flipped
    definite one."""
    sc = scenes.multistorey_scene(13, 9.0, 7.0, 400_000, n_floors=3)
    tm, cT, keep = _run(oracle_lib, sc)
    assert oracle_lib.simplify_check(tm["ground"], cT, cT, CB, 1e-5, keep) == -1
    bad = keep.copy()
    k = int(np.flatnonzero(keep)[0])
    bad[k] = False
    assert oracle_lib.simplify_check(tm["ground"], cT, cT, CB, 1e-5, bad) == k
