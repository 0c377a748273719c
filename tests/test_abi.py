"""Host-side checks of libpct that need no GPU: the library loads, exports
every entry point include/pct.h declares, validates arguments before any
device call, and its host tables agree with the oracle's."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def P():
    import paper_2403_07631_amd as P
    P.lib()
    return P


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "pct.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pct_[a-z0-9_]+)\s*\(", txt)))


def test_exports_every_declared_symbol(P):
    syms = header_symbols()
    assert len(syms) >= 10
    L = C.CDLL(P.LIB_PATH)
    missing = [s for s in syms if not hasattr(L, s)]
    assert not missing, missing
    assert P.pct_abi_version() == 1


def test_binding_declares_what_the_header_declares(P):
    assert set(P.declared_symbols()) <= set(header_symbols())


def test_robot_from_physical(P, oracle_lib):
    r = P.robot_from_physical(scenes.ROBOT_CONFIG0, 0.1).as_dict()
    o = oracle_lib.robot_from_physical(scenes.ROBOT_CONFIG0, 0.1)
    for k, v in o.items():
        assert r[k] == pytest.approx(float(np.float32(v)), rel=1e-7), k
    with pytest.raises(P.PctError) as e:
        P.pct_robot_from_physical(0.5, 1.0, 95.0, 0.2, 0.3, 0.4, 0.1)
    assert e.value.status == P.PCT_ERR_ARG


@pytest.mark.parametrize("bad", [dict(res=0.0), dict(res=-0.1), dict(slice_dz=0.0), dict(nx=0),
                                 dict(ny=70000), dict(x0=float("nan"))])
def test_grid_validation(P, bad):
    g = dict(x0=0.0, y0=0.0, res=0.1, nx=10, ny=10, slice_dz=0.3)
    P.pct_validate_grid(g)
    g.update(bad)
    with pytest.raises(P.PctError) as e:
        P.pct_validate_grid(g)
    assert e.value.status == P.PCT_ERR_ARG


def test_robot_validation(P):
    r = P.robot_from_physical(scenes.ROBOT_CONFIG0, 0.1).as_dict()
    P.pct_validate_robot(r, 0.1)
    for bad, code in [(dict(d_sm=0.1), P.PCT_ERR_ARG), (dict(patch_radius=0), P.PCT_ERR_ARG),
                      (dict(patch_radius=5), P.PCT_ERR_ARG), (dict(c_barrier=0.0), P.PCT_ERR_ARG),
                      (dict(d_inf=2.0), P.PCT_ERR_CAPACITY), (dict(theta_s=float("inf")), P.PCT_ERR_ARG)]:
        rr = dict(r)
        rr.update(bad)
        with pytest.raises(P.PctError) as e:
            P.pct_validate_robot(rr, 0.1)
        assert e.value.status == code, bad
    # the step threshold theta_b * 2 res must stay finite in single precision
    rr = dict(r, d_inf=0.0, d_sm=5.0)
    P.pct_validate_robot(dict(rr, theta_b=1e37), 4.0)
    with pytest.raises(P.PctError) as e:
        P.pct_validate_robot(dict(rr, theta_b=3e38), 4.0)
    assert e.value.status == P.PCT_ERR_ARG


@pytest.mark.parametrize("d_inf,d_sm,res", [(0.3, 0.4, 0.1), (0.2, 0.4, 0.1), (0.0, 0.15, 0.1),
                                            (0.5, 0.9, 0.2), (1.1, 0.6, 0.1), (0.25, 0.1001, 0.1)])
def test_kernel_radius_matches_oracle(P, oracle_lib, d_inf, d_sm, res):
    r = P.robot_from_physical(scenes.ROBOT_CONFIG0, res).as_dict()
    r.update(d_inf=d_inf, d_sm=d_sm)
    _, R = oracle_lib.kernel(res, d_inf, d_sm)
    assert P.pct_kernel_radius(r, res) == R


@pytest.mark.parametrize("zmin,zmax,ds", [(0.0, 1.25, 0.5), (-0.0797, 3.0739, 0.4), (-0.1, 16.6, 0.3),
                                          (123.4, 130.0, 0.05), (-7.0, -6.99, 0.3)])
def test_plane_heights_match_oracle(P, oracle_lib, zmin, zmax, ds):
    zmin, zmax, ds = (float(np.float32(v)) for v in (zmin, zmax, ds))
    h = oracle_lib.planes(zmin, zmax, ds)
    e = P.pct_extent(zmin, zmax, len(h), 0, 1, 0)
    np.testing.assert_array_equal(P.pct_plane_heights(e, ds), h)


def _g(P):
    return P.pct_grid(0.0, 0.0, 0.1, 16, 16, 0.3)


def test_extent_rejects_before_launch(P):
    L = P.lib()
    g = _g(P)
    e = P.pct_extent()
    assert L.pct_tomogram_extent(None, 10, C.byref(g), None, None, 0, None) == P.PCT_ERR_ARG
    assert L.pct_tomogram_extent(None, -1, C.byref(g), C.byref(e), None, 0, None) == P.PCT_ERR_ARG
    assert L.pct_tomogram_extent(None, 10, C.byref(g), C.byref(e), None, 0, None) == P.PCT_ERR_ARG
    assert L.pct_tomogram_extent(C.c_void_p(0x1000), 10, C.byref(g), C.byref(e), None, 0, None) == P.PCT_ERR_WORKSPACE
    # an empty cloud is an empty map, no device work
    assert L.pct_tomogram_extent(None, 0, C.byref(g), C.byref(e), None, 0, None) == P.PCT_OK
    assert e.n_slices == 0 and e.n_used == 0
    assert L.pct_last_error() == b""


def test_build_rejects_before_launch(P):
    L = P.lib()
    g = _g(P)
    good = P.pct_extent(0.0, 1.0, 4, 0, 10, 0)       # planes 0.3, 0.6, 0.9, 1.2
    bad = P.pct_extent(0.0, 1.0, 7, 0, 10, 0)
    fake = C.c_void_p(0x1000)
    assert L.pct_build_tomogram(fake, 10, C.byref(g), C.byref(bad), fake, fake, None, None, fake, 1 << 30, None) == P.PCT_ERR_ARG
    assert L.pct_build_tomogram(fake, 10, C.byref(g), C.byref(good), fake, fake, fake, None, fake, 1 << 30, None) == P.PCT_ERR_ARG
    assert L.pct_build_tomogram(fake, 10, C.byref(g), C.byref(good), fake, fake, None, None, fake, 16, None) == P.PCT_ERR_WORKSPACE
    assert L.pct_build_tomogram(fake, 10, C.byref(g), C.byref(good), None, fake, None, None, fake, 1 << 30, None) == P.PCT_ERR_ARG
    over = P.pct_extent(0.0, 1.0, 2000, 0, 10, 0)
    assert L.pct_build_tomogram(fake, 10, C.byref(g), C.byref(over), fake, fake, None, None, fake, 1 << 30, None) == P.PCT_ERR_CAPACITY
    empty = P.pct_extent(0.0, 0.0, 0, 0, 0, 0)
    assert L.pct_build_tomogram(None, 0, C.byref(g), C.byref(empty), None, None, None, None, None, 0, None) == P.PCT_OK


def test_eval_rejects_before_launch(P):
    L = P.lib()
    g = _g(P)
    e = P.pct_extent(0.0, 1.0, 4, 0, 10, 0)
    rb = P.robot_from_physical(scenes.ROBOT_CONFIG0, 0.1)
    rs = (P.pct_robot * 1)(rb)
    fake = C.c_void_p(0x1000)
    assert L.pct_eval_traversability(fake, fake, C.byref(g), C.byref(e), rs, 0, fake, None, None, 0, None) == P.PCT_ERR_ARG
    assert L.pct_eval_traversability(fake, fake, C.byref(g), C.byref(e), rs, 1, fake, fake, None, 0, None) == P.PCT_ERR_WORKSPACE
    rb2 = P.pct_robot.from_buffer_copy(rb)
    rb2.d_sm = 0.05
    rs2 = (P.pct_robot * 1)(rb2)
    assert L.pct_eval_traversability(fake, fake, C.byref(g), C.byref(e), rs2, 1, fake, None, None, 0, None) == P.PCT_ERR_ARG
    assert b"d_sm" in L.pct_last_error()
    assert L.pct_eval_traversability(None, fake, C.byref(g), C.byref(e), rs, 1, fake, None, None, 0, None) == P.PCT_ERR_ARG


def test_workspace_sizes(P):
    g = P.pct_grid(0.0, 0.0, 0.1, 2000, 2000, 0.3)
    e = P.pct_extent(0.0, 16.0, 54, 0, 20_000_000, 0)
    L = P.lib()
    b = L.pct_build_workspace_bytes(20_000_000, C.byref(g), C.byref(e))
    assert 12 * 20_000_000 <= b <= 26 * 20_000_000   # two levels of records + per-workgroup counts
    assert L.pct_eval_workspace_bytes(C.byref(g), C.byref(e), 1) > 0
    assert L.pct_extent_workspace_bytes(1000) > 0


def test_library_resolves_all_symbols_at_load(P):
    """Loading with immediate binding catches an entry point that refers to
    an undefined internal function."""
    C.CDLL(P.LIB_PATH, mode=os.RTLD_NOW | os.RTLD_LOCAL)


def test_item_struct_layout(P):
    """pct_item as laid out by a C compiler on this ABI: 96 bytes, extent at 48."""
    assert C.sizeof(P.pct_item) == 96
    assert P.pct_item.extent.offset == 48 and P.pct_item.out_offset.offset == 80
    assert C.sizeof(P.pct_extent) == 32 and C.sizeof(P.pct_grid) == 24 and C.sizeof(P.pct_robot) == 48


def test_batch_rejects_before_launch(P):
    L = P.lib()
    items = (P.pct_item * 2)()
    for it in items:
        it.grid = P.pct_grid(0.0, 0.0, 0.1, 10, 10, 0.3)
        it.n_points = 5
    items[1].xyz_offset = 8
    tc, ts = C.c_int64(), C.c_int64()
    # item 1 reaches past the 10 points given
    assert L.pct_tomogram_extent_batched(C.c_void_p(0x1000), 10, items, 2, C.byref(tc), C.byref(ts),
                                         C.c_void_p(0x1000), 1 << 20, None) == P.PCT_ERR_ARG
    items[1].grid.res = 0.0
    items[1].xyz_offset = 5
    assert L.pct_tomogram_extent_batched(C.c_void_p(0x1000), 10, items, 2, C.byref(tc), C.byref(ts),
                                         C.c_void_p(0x1000), 1 << 20, None) == P.PCT_ERR_ARG
    assert b"item 1" in L.pct_last_error()


def test_plan_argument_checks(P):
    """The path search validates its arguments before touching the device."""
    import ctypes as C
    L = P.lib()
    g = P.grid_struct(dict(x0=0.0, y0=0.0, res=0.1, nx=100, ny=80, slice_dz=0.3))
    e = P.pct_extent(0.0, 1.0, 5, 0, 0, 0)
    rb = P.robot_struct(P.robot_from_physical(scenes.ROBOT_CONFIG0, 0.1))
    assert L.pct_plan_workspace_bytes(100, 80, 3) > 100 * 80 * 3 * 5
    assert L.pct_plan_workspace_bytes(0, 80, 3) == 0
    dummy = C.c_void_p(16)

    def call(layers, start, ws_bytes=1 << 30, ptr=dummy, band=0.0):
        lay = (C.c_int32 * max(1, len(layers)))(*layers)
        return L.pct_plan_distance(ptr, ptr, C.byref(g), C.byref(e), C.byref(rb), lay, len(layers), *start, band,
                                   ptr, ptr, ws_bytes, None, None, None)

    assert call([0, 2, 2], (0, 0, 0)) == P.PCT_ERR_ARG       # not strictly increasing
    assert call([0, 5], (0, 0, 0)) == P.PCT_ERR_ARG          # slice outside the extent
    assert call([], (0, 0, 0)) == P.PCT_ERR_ARG              # no layer
    assert call([0, 1], (100, 0, 0)) == P.PCT_ERR_ARG        # start outside the map
    assert call([0, 1], (0, 0, 2)) == P.PCT_ERR_ARG          # start layer outside
    assert call([0, 1], (0, 0, 0), ptr=None) == P.PCT_ERR_ARG
    assert call([0, 1], (0, 0, 0), ws_bytes=16) == P.PCT_ERR_WORKSPACE
    assert call([0, 1], (0, 0, 0), band=-1.0) == P.PCT_ERR_ARG
    n = C.c_int32()
    assert L.pct_plan_path(dummy, C.byref(g), 2, 0, 0, 0, 0, 0, 5, dummy, 10, C.byref(n), dummy, 1 << 30,
                           None) == P.PCT_ERR_ARG            # goal layer outside
    assert L.pct_plan_path(dummy, C.byref(g), 2, 0, 0, 0, 0, 0, 1, dummy, 0, C.byref(n), dummy, 1 << 30,
                           None) == P.PCT_ERR_ARG            # max_len 0


def test_traj_argument_checks(P):
    """The trajectory optimisation validates its arguments before touching
    the device."""
    import ctypes as C
    from paper_2403_07631_amd import abi
    L = P.lib()
    g = P.grid_struct(dict(x0=0.0, y0=0.0, res=0.1, nx=100, ny=80, slice_dz=0.3))
    e = P.pct_extent(0.0, 1.0, 5, 0, 0, 0)
    good = dict(w_z=1.0, w_c=1.0, w_v=1.0, w_a=1.0, w_h=1.0, w_T=1.0, c_safe=5.0, v_max=1.0, a_max=1.0,
                d_ref=0.5, d_min=0.3, samples=8)
    d = C.c_void_p(16)

    def ev(prm=good, n=4, M=8, ptr=d, knots=d):
        p = P.traj_params_struct(prm)
        return L.pct_traj_eval(ptr, ptr, ptr, C.byref(g), C.byref(e), C.byref(p), n, M, ptr, ptr, knots, ptr, ptr,
                               ptr, ptr, None, None)

    def opt(iters=5, step=1e-3):
        p = P.traj_params_struct(good)
        return L.pct_traj_optimize(d, d, d, C.byref(g), C.byref(e), C.byref(p), 4, 8, d, d, d, d, iters, step, d,
                                   None, None)

    assert abi.PCT_MAX_PIECES == 64 and abi.PCT_MAX_TRAJ_SAMPLES == 64
    assert ev(M=0) == P.PCT_ERR_ARG
    assert ev(M=65) == P.PCT_ERR_ARG
    assert ev(prm=dict(good, samples=0)) == P.PCT_ERR_ARG
    assert ev(prm=dict(good, samples=65)) == P.PCT_ERR_ARG
    assert ev(prm=dict(good, w_c=-1.0)) == P.PCT_ERR_ARG
    assert ev(prm=dict(good, w_T=float("inf"))) == P.PCT_ERR_ARG
    assert ev(prm=dict(good, v_max=0.0)) == P.PCT_ERR_ARG
    assert ev(prm=dict(good, d_ref=float("nan"))) == P.PCT_ERR_ARG
    assert ev(n=-1) == P.PCT_ERR_ARG
    assert ev(ptr=None) == P.PCT_ERR_ARG
    assert ev(knots=None) == P.PCT_ERR_ARG            # interior waypoints needed for M > 1
    assert opt(iters=-1) == P.PCT_ERR_ARG
    assert opt(step=0.0) == P.PCT_ERR_ARG
    assert opt(step=float("nan")) == P.PCT_ERR_ARG
    assert ev(n=0) == P.PCT_OK                        # nothing to do


def test_graph_helpers_reject_before_device_calls(P):
    import ctypes as C
    L = P.lib()
    assert L.pct_graph_begin(None) == P.PCT_ERR_ARG          # the null stream cannot be captured
    assert L.pct_graph_end(None, None) == P.PCT_ERR_ARG
    assert L.pct_graph_launch(None, None) == P.PCT_ERR_ARG
    assert L.pct_graph_destroy(None) == P.PCT_OK


def test_plan_query_argument_checks(P):
    import ctypes as C
    L = P.lib()
    g = P.grid_struct(dict(x0=0.0, y0=0.0, res=0.1, nx=100, ny=80, slice_dz=0.3))
    e = P.pct_extent(0.0, 1.0, 5, 0, 0, 0)
    rb = P.robot_struct(P.robot_from_physical(scenes.ROBOT_CONFIG0, 0.1))
    d = C.c_void_p(16)
    lay = (C.c_int32 * 2)(0, 2)
    gd, st, ro, ti = C.c_double(), C.c_double(), C.c_int32(), C.c_int64()

    def q(goal, start=(0, 0, 0), ws_bytes=1 << 30):
        return L.pct_plan_query(d, d, C.byref(g), C.byref(e), C.byref(rb), lay, 2, *start, *goal, 0.0, d, d,
                                ws_bytes, C.byref(gd), C.byref(st), C.byref(ro), C.byref(ti), None)

    assert q((100, 0, 0)) == P.PCT_ERR_ARG       # goal outside the map
    assert q((0, 0, 2)) == P.PCT_ERR_ARG         # goal layer outside
    assert q((0, 0, 1), start=(0, 80, 0)) == P.PCT_ERR_ARG
    assert q((0, 0, 1), ws_bytes=16) == P.PCT_ERR_WORKSPACE
