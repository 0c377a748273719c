"""GPU checks of the multi-profile trajectory cost (several robot profiles on
one map in one launch, c^T evaluated only at the sampled corners).

Against the per-profile path on the device (cost map, sampling, fused
adjoint): per-trajectory values, waypoint gradients and the fixed-point
point gradients bit for bit (float-atomic point gradients to their rounding).  Against the FP64 oracle: values within
2e-5 per waypoint, gradients within the rel 1e-3 tolerance outside the
near-tie cells the oracle marks."""
import sys

import numpy as np
import pytest

import scenes

pytestmark = pytest.mark.gpu
W_Z = 1.0


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


def close(gpu, ref, mask=None, rel=1e-3):
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    bad = np.abs(gpu - ref) > rel * np.maximum(1.0, np.abs(ref))
    if mask is not None:
        bad &= mask
    assert not bad.any(), f"{bad.sum()} entries differ; worst {np.max(np.abs(gpu - ref)[bad])}"


def per_profile(P, G, Cc, aG, aC, g, ext, rbs, wp, sl, gf, n, deterministic=True):
    """The per-profile path: c^T map, sampling, fused adjoint; gz summed over
    the profiles in one fixed-point accumulator (or float atomics)."""
    import torch
    fs, gwps = [], []
    gz = torch.zeros(n, dtype=torch.int64 if deterministic else torch.float32, device="cuda")
    for i, rb in enumerate(rbs):
        cost, _ = P.pct_eval_traversability(G, Cc, g, ext, [rb], keep=False)
        cost = cost[0].contiguous()
        fs.append(P.pct_sample_cost_fwd(cost, G, g, ext, rb, W_Z, wp[i], sl[i]))
        gwp, _ = P.pct_trajectory_cost_bwd(G, Cc, cost, aG, aC, g, ext, rb, W_Z, wp[i], sl[i], gf[i], n, gz=gz,
                                           flags=P.PCT_ACCUMULATE)
        gwps.append(gwp)
    return torch.stack(fs), torch.stack(gwps), (P.pct_fixed_to_float(gz) if deterministic else gz)


def test_multi_equals_per_profile_and_oracle(P, oracle_lib):
    import torch
    sc = scenes.multistorey_scene(51, 12.3, 9.1, 1_200_000, n_floors=3)
    g = sc.grid
    say("multi-profile world: build")
    xyz = torch.from_numpy(sc.points).cuda()
    n = xyz.shape[0]
    ext = P.pct_tomogram_extent(xyz, g)
    G, Cc, aG, aC = P.pct_build_tomogram(xyz, g, ext, with_ids=True)
    torch.cuda.synchronize()
    tm = oracle_lib.tomogram(sc.points, g)
    profiles = [oracle_lib.robot_from_physical(p, g["res"]) for p in scenes.robot_profiles(4, 6)]
    rbs = [P.robot_struct(r) for r in profiles]
    T, W = 32, 100
    wps, sls, cTs = [], [], []
    for i, r in enumerate(profiles):
        cT = oracle_lib.evaluate(tm["ground"], tm["ceil"], g["res"], r)
        lo, hi, _ = oracle_lib.envelope(tm["ground"], tm["ceil"], g["res"], r)
        wp, sl = scenes.random_walks(30 + i, (cT < r["c_barrier"]) & (lo == hi), tm["ground"], g, T, W, r["d_ref"])
        wps.append(wp)
        sls.append(sl)
        cTs.append(cT)
    wp = torch.from_numpy(np.stack(wps)).cuda()
    sl = torch.from_numpy(np.stack(sls)).cuda()
    gf = torch.linspace(-1.0, 1.5, len(rbs) * T, device="cuda").reshape(len(rbs), T)
    say("multi-profile: per-profile path")
    f1, gwp1, gz1 = per_profile(P, G, Cc, aG, aC, g, ext, rbs, wp, sl, gf, n)
    say("multi-profile: one launch")
    f2, gwp2, gG2, gC2, gz2 = P.pct_trajectory_cost_multi(G, Cc, aG, aC, g, ext, rbs, W_Z, wp, sl, gf, n_points=n,
                                                          grids=True)
    fv, *_ = P.pct_trajectory_cost_multi(G, Cc, None, None, g, ext, rbs, W_Z, wp, sl)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(bits(f2), bits(f1))
    np.testing.assert_array_equal(bits(fv), bits(f1))
    np.testing.assert_array_equal(bits(gwp2), bits(gwp1))
    # fixed-point sums do not depend on the order of the additions
    np.testing.assert_array_equal(bits(gz2), bits(gz1))
    # float atomics add in a different order: a few ulps of the largest partial sums
    _, _, gz1f = per_profile(P, G, Cc, aG, aC, g, ext, rbs, wp, sl, gf, n, deterministic=False)
    *_, gz2f = P.pct_trajectory_cost_multi(G, Cc, aG, aC, g, ext, rbs, W_Z, wp, sl, gf, n_points=n,
                                           deterministic=False)
    z1 = gz1.cpu().numpy()
    atol = 2e-5 * max(1.0, float(np.abs(z1).max()))
    np.testing.assert_allclose(gz1f.cpu().numpy(), z1, rtol=1e-5, atol=atol)
    np.testing.assert_allclose(gz2f.cpu().numpy(), z1, rtol=1e-5, atol=atol)
    say("multi-profile: oracle")
    rz = np.zeros(n)
    uz = np.zeros(n, bool)
    rG_all = np.zeros(tm["ground"].shape)
    rC_all = np.zeros(tm["ground"].shape)
    unc_all = np.zeros(tm["ground"].shape, bool)
    f2h, gwp2h = f2.cpu().numpy(), gwp2.cpu().numpy()
    for i, r in enumerate(profiles):
        fr = oracle_lib.sample_fwd(cTs[i], tm["ground"], g, W_Z, r["d_ref"], wps[i], sls[i])
        assert np.all(np.abs(f2h[i] - fr) <= 2e-5 * W + 1e-6 * np.abs(fr))
        g64 = gf[i].cpu().numpy().astype(np.float64)
        rgwp, rgc, rgg = oracle_lib.sample_bwd(cTs[i], tm["ground"], g, W_Z, r["d_ref"], wps[i], sls[i], g64)
        close(gwp2h[i], rgwp)
        rG, rC, unc = oracle_lib.eval_bwd(tm["ground"], tm["ceil"], g["res"], r, rgc)
        rG_all += rG + rgg
        rC_all += rC
        unc_all |= unc
        rz += oracle_lib.route(rG + rgg, rC, tm["arg_ground"], tm["arg_ceil"], n)
        for a in (tm["arg_ground"], tm["arg_ceil"]):
            m = (a >= 0) & unc
            uz[a[m]] = True
    assert np.count_nonzero(rz) > 100
    close(gz2.cpu().numpy(), rz, ~uz)
    close(gG2.cpu().numpy(), rG_all, ~unc_all)
    close(gC2.cpu().numpy(), rC_all, ~unc_all)


def test_multi_full_size_profiles(P):
    """The 20 M-point map with 64 profiles and the same 64 walks x 256
    waypoints per profile (the batched workload's shape per profile, fewer
    walks): the one-launch result equals the per-profile path."""
    import torch
    sc = scenes.config1_scene()
    g = sc.grid
    say("multi full size: build")
    xyz = torch.from_numpy(sc.points).cuda()
    n = xyz.shape[0]
    ext = P.pct_tomogram_extent(xyz, g)
    G, Cc, aG, aC = P.pct_build_tomogram(xyz, g, ext, with_ids=True)
    Gh = G.cpu().numpy()
    rb0 = P.robot_from_physical(sc.robot, g["res"])
    wp0, sl0 = scenes.random_walks(2, np.isfinite(Gh), Gh, g, 64, 256, rb0.as_dict()["d_ref"])
    profiles = scenes.robot_profiles(4, 64)
    rbs = [P.robot_from_physical(p, g["res"]) for p in profiles]
    wp = torch.from_numpy(np.ascontiguousarray(np.broadcast_to(wp0, (64,) + wp0.shape))).cuda()
    sl = torch.from_numpy(np.ascontiguousarray(np.broadcast_to(sl0, (64,) + sl0.shape))).cuda()
    gf = torch.ones((64, 64), device="cuda")
    say("multi full size: per-profile path")
    f1, gwp1, gz1 = per_profile(P, G, Cc, aG, aC, g, ext, rbs, wp, sl, gf, n)
    say("multi full size: one launch")
    f2, gwp2, _, _, gz2 = P.pct_trajectory_cost_multi(G, Cc, aG, aC, g, ext, rbs, W_Z, wp, sl, gf, n_points=n)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(bits(f2), bits(f1))
    np.testing.assert_array_equal(bits(gwp2), bits(gwp1))
    np.testing.assert_array_equal(bits(gz2), bits(gz1))
