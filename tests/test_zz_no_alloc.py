"""The evaluation entry point that allocates nothing (its slice-test scratch
is the library's static device array), through the C ABI: its costs and
keep flags must equal pct_eval_traversability's (same kernels) and lie in
the oracle's 1e-5 envelope of Eqs. (1)-(6), on two calls in a row, the
second on a smaller map with fewer slices, so that a stale bit matrix or
run-start table left by the first call would show."""
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


def run_both(P, oracle_lib, sc, robots, what):
    import torch
    g = sc.grid
    xyz = torch.from_numpy(np.ascontiguousarray(sc.points, np.float32)).cuda()
    ext = P.pct_tomogram_extent(xyz, g)
    ground, ceil, _, _ = P.pct_build_tomogram(xyz, g, ext, with_ids=False)
    rbs = [P.robot_from_physical(r, g["res"]) if "max_slope_deg" in r else r for r in robots]
    say(f"no-alloc eval {what}: {g['nx']}x{g['ny']} cells, {ext.n_slices} slices, {len(rbs)} robots")
    cost_s, keep_s = P.pct_eval_traversability_static(ground, ceil, g, ext, rbs)
    cost_w, keep_w = P.pct_eval_traversability(ground, ceil, g, ext, rbs)
    torch.cuda.synchronize()
    cs, cw = cost_s.cpu().numpy(), cost_w.cpu().numpy()
    np.testing.assert_array_equal(cs.view(np.uint32), cw.view(np.uint32))
    np.testing.assert_array_equal(keep_s.cpu().numpy(), keep_w.cpu().numpy())
    tm_g, tm_c = ground.cpu().numpy(), ceil.cpu().numpy()
    for i, rb in enumerate(rbs):
        r = rb.as_dict() if hasattr(rb, "as_dict") else dict(rb)
        lo, hi, _ = oracle_lib.envelope(tm_g, tm_c, g["res"], r)
        c = cs[i].astype(np.float64)
        assert np.all(c >= lo - TOL) and np.all(c <= hi + TOL), "c^T outside the oracle's 1e-5 envelope"
        assert oracle_lib.simplify_check(tm_g, lo, hi, r["c_barrier"], TOL, keep_s[i].cpu().numpy()) == -1
        n_trav = int((c < r["c_barrier"]).sum())
        say(f"no-alloc eval {what}: robot {i}: {n_trav} traversable cell-slices, "
            f"{int(keep_s[i].sum())} of {ext.n_slices} slices kept")
    return ext


def test_static_scratch_matches_workspace_entry_point(P, oracle_lib):
    big = scenes.multistorey_scene(41, 20.0, 15.0, 396_000, n_floors=3)
    small = scenes.multistorey_scene(43, 6.4, 5.3, 60_000, n_floors=2)
    robots = [dict(scenes.ROBOT_TABLE1), scenes.ROBOT_CONFIG0]
    e1 = run_both(P, oracle_lib, big, robots, "first call")
    e2 = run_both(P, oracle_lib, small, robots[:1], "second call, smaller")
    assert e2.n_slices < e1.n_slices and small.grid["nx"] < big.grid["nx"]


def test_static_scratch_without_keep_and_empty(P):
    import torch
    sc = scenes.multistorey_scene(44, 5.0, 4.0, 30_000, n_floors=2)
    g = sc.grid
    xyz = torch.from_numpy(np.ascontiguousarray(sc.points, np.float32)).cuda()
    ext = P.pct_tomogram_extent(xyz, g)
    ground, ceil, _, _ = P.pct_build_tomogram(xyz, g, ext, with_ids=False)
    rb = P.robot_from_physical(scenes.ROBOT_CONFIG0, g["res"])
    cost_s, keep_s = P.pct_eval_traversability_static(ground, ceil, g, ext, [rb], keep=False)
    cost_w, _ = P.pct_eval_traversability(ground, ceil, g, ext, [rb], keep=False)
    assert keep_s is None
    np.testing.assert_array_equal(cost_s.cpu().numpy().view(np.uint32), cost_w.cpu().numpy().view(np.uint32))
    # no slices: nothing to do, no error
    e0 = P.pct_extent(0.0, 0.0, 0, 0, 0, 0)
    z = torch.empty((0, g["ny"], g["nx"]), dtype=torch.float32, device="cuda")
    c0, k0 = P.pct_eval_traversability_static(z, z, g, e0, [rb])
    torch.cuda.synchronize()
    assert c0.numel() == 0 and k0.numel() == 0
