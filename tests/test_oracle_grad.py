"""Pins of the oracle's trajectory cost sampling and adjoints.

Every analytic gradient is checked against a central finite difference of
the oracle's own forward functions.  Inside one branch every quantity is at
most quadratic in the perturbed input (bilinear interpolation, squared
height error, squared central differences, linear interval cost, max over
fixed taps), so a central difference is exact up to rounding; a sample
counts only when no discrete decision (branch, maximising tap, clip, point
that holds a ground/ceiling value) changes between -h and +h."""
import numpy as np
import pytest

import scenes

W_Z = 1.0
H = 2.0 ** -12          # exact perturbation of float32 heights/coordinates below 2^11 m


@pytest.fixture(scope="module")
def setup(oracle_lib):
    sc = scenes.multistorey_scene(41, 6.4, 4.7, 260_000, n_floors=3)
    tm = oracle_lib.tomogram(sc.points, sc.grid)
    rb = oracle_lib.robot_from_physical(sc.robot, sc.grid["res"])
    cT = oracle_lib.evaluate(tm["ground"], tm["ceil"], sc.grid["res"], rb)
    mask = np.isfinite(tm["ground"]) & (cT < rb["c_barrier"])
    wp, sl = scenes.random_walks(3, mask, tm["ground"], sc.grid, 6, 24, rb["d_ref"])
    return sc, tm, rb, cT, wp, sl


def test_sample_wrt_waypoints(oracle_lib, setup):
    sc, tm, rb, cT, wp, sl = setup
    rng = np.random.default_rng(0)
    gf = rng.normal(size=sl.shape[0])
    gwp, _, _ = oracle_lib.sample_bwd(cT, tm["ground"], sc.grid, W_Z, rb["d_ref"], wp, sl, gf)

    def L(w):
        return float(gf @ oracle_lib.sample_fwd(cT, tm["ground"], sc.grid, W_Z, rb["d_ref"], w, sl))
    checked = 0
    for _ in range(60):
        t, w, a = rng.integers(0, wp.shape[0]), rng.integers(0, wp.shape[1]), rng.integers(0, 3)
        p, m = wp.copy(), wp.copy()
        p[t, w, a] += np.float32(H)
        m[t, w, a] -= np.float32(H)
        h2 = float(p[t, w, a]) - float(m[t, w, a])
        fd = (L(p) - L(m)) / h2
        assert fd == pytest.approx(gwp[t, w, a], rel=1e-6, abs=1e-7), (t, w, a)
        checked += 1
    assert checked == 60
    assert np.abs(gwp[..., 2]).max() > 0 and np.abs(gwp[..., :2]).max() > 0


def test_sample_wrt_grids(oracle_lib, setup):
    sc, tm, rb, cT, wp, sl = setup
    rng = np.random.default_rng(1)
    gf = rng.normal(size=sl.shape[0])
    _, gcT, gG = oracle_lib.sample_bwd(cT, tm["ground"], sc.grid, W_Z, rb["d_ref"], wp, sl, gf)

    def L(c, g):
        return float(gf @ oracle_lib.sample_fwd(c, g, sc.grid, W_Z, rb["d_ref"], wp, sl))
    touched = np.flatnonzero(gcT.ravel())
    assert touched.size > 20
    for i in rng.choice(touched, 25, replace=False):
        c1, c2 = cT.copy().ravel(), cT.copy().ravel()
        c1[i] += 1e-3
        c2[i] -= 1e-3
        fd = (L(c1.reshape(cT.shape), tm["ground"]) - L(c2.reshape(cT.shape), tm["ground"])) / 2e-3
        assert fd == pytest.approx(gcT.ravel()[i], rel=1e-7, abs=1e-9)
    tg = np.flatnonzero(gG.ravel())
    for i in rng.choice(tg, 25, replace=False):
        g1, g2 = tm["ground"].copy().ravel(), tm["ground"].copy().ravel()
        g1[i] += np.float32(H)
        g2[i] -= np.float32(H)
        h2 = float(g1[i]) - float(g2[i])
        fd = (L(cT, g1.reshape(cT.shape)) - L(cT, g2.reshape(cT.shape))) / h2
        assert fd == pytest.approx(gG.ravel()[i], rel=1e-6, abs=1e-8)
    # untouched cells get no gradient
    assert np.count_nonzero(gcT) <= 4 * sl.size


def _stepped(oracle_lib):
    """Dense terrain of risers along both axes (0.15 m every 0.5 m in x,
    0.12 m every 0.7 m in y) with small noise: step-branch cells of Eq. (4)
    with either axis dominant."""
    rng = np.random.default_rng(9)
    f = lambda x, y: 0.15 * np.floor(x / 0.5) + 0.12 * np.floor(y / 0.7) + rng.normal(0, 0.004, x.shape)
    sc = scenes.dense_surface_scene(48, 37, 0.1, f, per_cell=4, slice_dz=0.3)
    tm = oracle_lib.tomogram(sc.points, sc.grid)
    return sc, tm


@pytest.mark.parametrize("case", ["building", "building-dref1.6", "steps"])
def test_eval_adjoint(oracle_lib, setup, case):
    """The building as is; with d_ref = 1.6 m, where the 1.2 m beams put the
    interval cost of Eq. (1) in play (ceiling gradient); and a stepped
    terrain for the step cost of Eq. (4)."""
    sc, tm, rb, cT, wp, sl = setup
    if case == "building-dref1.6":
        rb = dict(rb, d_ref=1.6)
        cT = oracle_lib.evaluate(tm["ground"], tm["ceil"], sc.grid["res"], rb)
    elif case == "steps":
        # a one-tap kernel (R = 0): c^T = c^init, so no ties between the many
        # equal step costs along a riser hide the Eq. (4) gradient
        sc, tm = _stepped(oracle_lib)
        rb = dict(rb, d_inf=0.05, d_sm=0.11)
        cT = oracle_lib.evaluate(tm["ground"], tm["ceil"], sc.grid["res"], rb)
    d_ref = 1.6 if case == "building-dref1.6" else None
    eG, eC = tm["ground"], tm["ceil"]
    res = sc.grid["res"]
    rng = np.random.default_rng(2)
    gcT = np.zeros(cT.shape)
    trav = np.flatnonzero(cT.ravel() < rb["c_barrier"])
    idx = np.union1d(rng.choice(trav, min(300, trav.size), replace=False), rng.choice(cT.size, 100, replace=False))
    gcT.ravel()[idx] = rng.normal(size=idx.size)
    gG, gC, unc = oracle_lib.eval_bwd(eG, eC, res, rb, gcT)
    sig0 = oracle_lib.eval_signature(eG, eC, res, rb)

    def L(g, c):
        return float(np.sum(gcT * oracle_lib.evaluate(g, c, res, rb)))
    valid = nonzero = n_step_nb = 0
    nz_by = {"G": 0, "C": 0}
    near_nz = np.zeros(0, np.int64)
    for which, arr, grad in (("G", eG, gG), ("C", eC, gC)):
        cand = np.flatnonzero(np.isfinite(arr.ravel()) & ~unc.ravel())
        # entries with a gradient, stratified so that every term is sampled:
        # ground under an active interval cost, the stencil neighbours of
        # step-branch cells, any other non-zero entry, and random entries
        nz = np.flatnonzero(grad.ravel() != 0)
        strata = [nz]
        if which == "G":
            strata.append(np.flatnonzero((gC.ravel() != 0) & (grad.ravel() != 0)))
            step = (sig0 & 7) == 3
            near = np.zeros_like(step)
            near[:, :, 1:] |= step[:, :, :-1]
            near[:, :, :-1] |= step[:, :, 1:]
            near[:, 1:, :] |= step[:, :-1, :]
            near[:, :-1, :] |= step[:, 1:, :]
            near_nz = np.flatnonzero(near.ravel() & (grad.ravel() != 0))
            strata.append(near_nz)
        strata.append(cand)
        pick = np.concatenate([rng.choice(a, min(40, a.size), replace=False) for a in strata if a.size])
        for i in pick:
            if unc.ravel()[i]:
                continue
            a1, a2 = arr.copy().ravel(), arr.copy().ravel()
            a1[i] += np.float32(H)
            a2[i] -= np.float32(H)
            a1, a2 = a1.reshape(arr.shape), a2.reshape(arr.shape)
            args1 = (a1, eC) if which == "G" else (eG, a1)
            args2 = (a2, eC) if which == "G" else (eG, a2)
            if not (np.array_equal(oracle_lib.eval_signature(*args1, res, rb), sig0) and
                    np.array_equal(oracle_lib.eval_signature(*args2, res, rb), sig0)):
                continue
            h2 = float(a1.ravel()[i]) - float(a2.ravel()[i])
            fd = (L(*args1) - L(*args2)) / h2
            assert fd == pytest.approx(grad.ravel()[i], rel=1e-6, abs=1e-7), (which, i)
            valid += 1
            nonzero += grad.ravel()[i] != 0
            nz_by[which] += grad.ravel()[i] != 0
            n_step_nb += which == "G" and i in set(near_nz.tolist())
    assert valid >= 40 and nonzero >= 10, (valid, nonzero)
    if d_ref is not None:
        assert nz_by["C"] >= 5, nz_by
    if case == "steps":
        assert n_step_nb >= 3, n_step_nb


def test_full_chain_to_point_heights(oracle_lib):
    """z -> tomogram -> traversability -> trajectory cost; dL/dz routed
    through the recorded point ids matches a central difference."""
    sc = scenes.multistorey_scene(43, 4.1, 3.3, 90_000, n_floors=2)
    g = sc.grid
    res = g["res"]
    rb = oracle_lib.robot_from_physical(sc.robot, res)
    pts = sc.points

    def forward(p):
        tm = oracle_lib.tomogram(p, g)
        cT = oracle_lib.evaluate(tm["ground"], tm["ceil"], res, rb)
        return tm, cT
    tm, cT = forward(pts)
    mask = np.isfinite(tm["ground"]) & (cT < rb["c_barrier"])
    wp, sl = scenes.random_walks(5, mask, tm["ground"], g, 5, 20, rb["d_ref"])
    rng = np.random.default_rng(3)
    gf = rng.normal(size=sl.shape[0])
    _, gcT, gGs = oracle_lib.sample_bwd(cT, tm["ground"], g, W_Z, rb["d_ref"], wp, sl, gf)
    gGe, gCe, unc = oracle_lib.eval_bwd(tm["ground"], tm["ceil"], res, rb, gcT)
    gz = oracle_lib.route(gGs + gGe, gCe, tm["arg_ground"], tm["arg_ceil"], len(pts))
    uz = np.zeros(len(pts), bool)
    for a in (tm["arg_ground"], tm["arg_ceil"]):
        m = (a >= 0) & unc
        uz[a[m]] = True
    sig0 = oracle_lib.eval_signature(tm["ground"], tm["ceil"], res, rb)

    def L(p):
        t, c = forward(p)
        return float(gf @ oracle_lib.sample_fwd(c, t["ground"], g, W_Z, rb["d_ref"], wp, sl)), t, c
    cand = np.flatnonzero(gz != 0)
    assert cand.size > 10
    z = pts[:, 2]
    cand = cand[(z[cand] > z.min()) & (z[cand] < z.max()) & ~uz[cand]]
    valid = 0
    for i in rng.choice(cand, min(30, cand.size), replace=False):
        p1, p2 = pts.copy(), pts.copy()
        p1[i, 2] += np.float32(H)
        p2[i, 2] -= np.float32(H)
        L1, t1, _ = L(p1)
        L2, t2, _ = L(p2)
        same = all(np.array_equal(t[k], tm[k]) for t in (t1, t2) for k in ("arg_ground", "arg_ceil"))
        same = same and all(np.array_equal(oracle_lib.eval_signature(t["ground"], t["ceil"], res, rb), sig0)
                            for t in (t1, t2))
        if not same:
            continue
        h2 = float(p1[i, 2]) - float(p2[i, 2])
        assert (L1 - L2) / h2 == pytest.approx(gz[i], rel=1e-6, abs=1e-7), i
        valid += 1
    assert valid >= 8, valid


def test_invalid_waypoints_contribute_nothing(oracle_lib, setup):
    sc, tm, rb, cT, wp, sl = setup
    w2, s2 = wp.copy(), sl.copy()
    w2[0, 3] = np.nan
    s2[1, 5] = len(tm["h"])
    s2[2, 0] = -1
    f1 = oracle_lib.sample_fwd(cT, tm["ground"], sc.grid, W_Z, rb["d_ref"], wp, sl)
    f2 = oracle_lib.sample_fwd(cT, tm["ground"], sc.grid, W_Z, rb["d_ref"], w2, s2)
    one = lambda t, w: oracle_lib.sample_fwd(cT, tm["ground"], sc.grid, W_Z, rb["d_ref"],
                                             wp[t:t + 1, w:w + 1], sl[t:t + 1, w:w + 1])[0]
    assert f2[0] == pytest.approx(f1[0] - one(0, 3))
    assert f2[1] == pytest.approx(f1[1] - one(1, 5))
    assert f2[2] == pytest.approx(f1[2] - one(2, 0))
