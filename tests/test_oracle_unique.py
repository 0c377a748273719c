"""Pins of the oracle's sparse storage of the simplified tomogram (the unique
cells of the kept slices, Sec. III-C, Eqs. (8)-(9)).

  - a hand-worked three-slice map: which cells are unique in which slice
    follows from the two conditions by hand (comments give each step);
  - a single floor: the floor is repeated in every slice, only the last
    slice is kept, and every traversable cell of it is unique;
  - the slice test: with the oracle's keep flags, a slice has unique cells
    exactly when it is kept (the slice test and the storage are separate
    loops of the oracle);
  - the stored values are the dense arrays' values at the stored cells, and
    the cells of a slice are in raster order.
"""
import numpy as np

import oracle
import scenes

CB = 50.0
INF = np.inf


def test_hand_worked_three_slices():
    # one row of four cells, three slices
    eG = np.array([[[0, 0, 0, -INF]],          # slice 0: floor everywhere but cell 3
                   [[0, 1, 0, -INF]],          # slice 1: cell 1 rises to 1 m
                   [[0, 1, 0, 2]]], np.float32)  # slice 2: cell 3 appears at 2 m
    eC = np.full_like(eG, INF)
    cT = np.array([[[5, 5, 4, 50]],
                   [[5, 3, 4, 50]],
                   [[5, 3, 1, 7]]], np.float32)
    keep = [1, 1, 1]
    out = oracle.unique_cells(eG, eC, cT, CB, keep)
    # slice 0 (no slice below): upper test against slice 1:
    #   cell 0: e1 = e0, c0 = c1 -> not unique; cell 1: e1 = 1 > 0 -> unique;
    #   cell 2: e1 = e0, 4 < 4 false -> not unique; cell 3: c = 50, not traversable.
    # slice 1 (below: slice 0): cell 0: equal to slice 0 -> no; cell 1: e 1 > 0 (lower),
    #   upper: e2 = e1, 3 < 3 false -> no; cell 2: lower 4 < 4 false -> no; cell 3: barrier.
    # slice 2 (below: slice 1, last slice): cell 0: equal -> no; cell 1: equal -> no;
    #   cell 2: 1 < 4 -> unique; cell 3: 2 > -inf and 7 < 50 -> unique.
    np.testing.assert_array_equal(out["slice_off"], [0, 1, 1, 3])
    np.testing.assert_array_equal(out["cell"], [1, 2, 3])
    np.testing.assert_array_equal(out["cost"], [5, 1, 7])
    np.testing.assert_array_equal(out["ground"], [0, 0, 2])
    # slice 1 removed: slice 2 is then compared with slice 0
    out = oracle.unique_cells(eG, eC, cT, CB, [1, 0, 1])
    # slice 2 against slice 0: cell 1: e 1 > 0 -> unique; cell 2: 1 < 4 -> unique; cell 3 unique
    np.testing.assert_array_equal(out["slice_off"], [0, 1, 1, 4])
    np.testing.assert_array_equal(out["cell"], [1, 1, 2, 3])


def test_single_floor():
    nx, ny = 37, 23
    sc = scenes.dense_surface_scene(nx, ny, 0.1, lambda x, y: 0.0 * x + 0.05)
    tm = oracle.tomogram(sc.points, sc.grid)
    r = oracle.robot_from_physical(scenes.ROBOT_CONFIG0, 0.1)
    cT = oracle.evaluate(tm["ground"], tm["ceil"], 0.1, r)
    keep = oracle.simplify(tm["ground"], cT, r["c_barrier"])
    c32 = cT.astype(np.float32)
    out = oracle.unique_cells(tm["ground"], tm["ceil"], c32, r["c_barrier"], keep)
    N = len(keep)
    assert keep.sum() == 1 and keep[-1]
    trav = np.flatnonzero((c32[-1] < np.float32(r["c_barrier"])).ravel())
    assert len(trav) > 0
    np.testing.assert_array_equal(out["cell"], trav)
    np.testing.assert_array_equal(out["slice_off"][:N], 0)
    assert out["slice_off"][N] == len(trav)


def test_kept_slices_have_unique_cells():
    sc = scenes.multistorey_scene(44, 9.3, 7.1, 250_000, n_floors=3)
    g = sc.grid
    tm = oracle.tomogram(sc.points, g)
    r = dict(scenes.ROBOT_TABLE1)
    cT = oracle.evaluate(tm["ground"], tm["ceil"], g["res"], r)
    keep = oracle.simplify(tm["ground"], cT, r["c_barrier"])
    c32 = cT.astype(np.float32)
    out = oracle.unique_cells(tm["ground"], tm["ceil"], c32, r["c_barrier"], keep)
    off = out["slice_off"]
    counts = np.diff(off)
    np.testing.assert_array_equal(counts > 0, keep)
    assert keep.sum() >= 3
    plane = g["nx"] * g["ny"]
    for k in np.flatnonzero(keep):
        cells = out["cell"][off[k]:off[k + 1]]
        assert np.all(np.diff(cells) > 0) and cells.min() >= 0 and cells.max() < plane
        for name, a in (("ground", tm["ground"]), ("ceil", tm["ceil"]), ("cost", c32)):
            np.testing.assert_array_equal(out[name][off[k]:off[k + 1]], a[k].ravel()[cells])
