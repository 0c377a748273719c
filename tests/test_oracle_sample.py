"""Value pins of the oracle's trajectory cost sampling (Sec. III-E, Eq. (11):
the travel cost C and the height reference Z_ref = e^G + d_ref).

The sampler is cell-centred bilinear interpolation clamped at the grid edge
(the paper defines no interpolation; this is the stated reading).  Bilinear
interpolation reproduces a map that is linear in the cell indices, so on
such maps the sampled cost and ground have closed forms in the waypoint
coordinates, written out here without the oracle's corner weights:
    u = (x - x0)/r - 1/2,  v = (y - y0)/r - 1/2   (clamped to [0, n-1])
    C = a + b u + c v,     G = g + p u + q v
    f = C + w_z (z - G - d_ref)^2.
The slopes differ in x and y and between the two maps, so a dropped
cell-centre offset, swapped corner weights, a transposed map or a flipped
sign of the height term each change the value.  The adjoint is pinned by
the same closed forms (its derivatives) and by hand-worked corner weights.
"""
import numpy as np
import pytest

NX, NY, N = 23, 17, 3
RES = 0.25
X0, Y0 = -1.5, 2.0
GRID = dict(x0=X0, y0=Y0, res=RES, nx=NX, ny=NY, slice_dz=0.3)
# per slice: (a, b, c) of the cost map and (g, p, q) of the ground map
COST = [(3.0, 0.5, -0.25), (1.0, -0.125, 0.75), (7.0, 0.0625, 0.375)]
GROUND = [(0.5, 0.03125, -0.0625), (3.25, -0.015625, 0.046875), (6.0, 0.0, 0.0)]
D_REF = 0.65


def maps():
    jj, ii = np.mgrid[0:NY, 0:NX].astype(np.float64)
    cT = np.stack([a + b * ii + c * jj for a, b, c in COST])
    eG = np.stack([g + p * ii + q * jj for g, p, q in GROUND]).astype(np.float32)
    # every value above is a short binary fraction: exact in float32
    assert np.array_equal(eG.astype(np.float64), np.stack([g + p * ii + q * jj for g, p, q in GROUND]))
    return cT, eG


def closed_form(wp, k, w_z, d_ref=D_REF):
    """(C, G, f) of one waypoint, from the linear maps directly."""
    x, y, z = (float(t) for t in wp)
    u = min(max((x - X0) / RES - 0.5, 0.0), NX - 1.0)
    v = min(max((y - Y0) / RES - 0.5, 0.0), NY - 1.0)
    a, b, c = COST[k]
    g, p, q = GROUND[k]
    C = a + b * u + c * v
    G = g + p * u + q * v
    return C, G, C + w_z * (z - G - d_ref) ** 2


def waypoints(rng, T, W, inside=True):
    lo = np.array([X0 + 0.5 * RES, Y0 + 0.5 * RES]) if inside else np.array([X0 - 2.0, Y0 - 2.0])
    hi = np.array([X0 + (NX - 0.5) * RES, Y0 + (NY - 0.5) * RES]) if inside else \
        np.array([X0 + NX * RES + 2.0, Y0 + NY * RES + 2.0])
    xy = lo + (hi - lo) * rng.random((T, W, 2))
    z = rng.uniform(0.0, 8.0, (T, W, 1))
    wp = np.concatenate([xy, z], axis=2).astype(np.float32)
    sl = rng.integers(0, N, (T, W)).astype(np.int32)
    return wp, sl


@pytest.mark.parametrize("inside", [True, False])
@pytest.mark.parametrize("w_z", [1.0, 2.5])
def test_linear_maps_closed_form(oracle_lib, inside, w_z):
    cT, eG = maps()
    rng = np.random.default_rng(5 if inside else 6)
    wp, sl = waypoints(rng, 7, 13, inside)
    f = oracle_lib.sample_fwd(cT, eG, GRID, w_z, D_REF, wp, sl)
    want = np.array([sum(closed_form(wp[t, w], sl[t, w], w_z)[2] for w in range(wp.shape[1]))
                     for t in range(wp.shape[0])])
    assert np.allclose(f, want, rtol=1e-12, atol=1e-12)


def test_single_waypoints_cost_and_height_terms(oracle_lib):
    """Each term alone: w_z = 0 leaves C; a zero cost map leaves the height
    term, checked against (z - G - d_ref)^2 with G written out."""
    cT, eG = maps()
    rng = np.random.default_rng(7)
    wp, sl = waypoints(rng, 40, 1)
    f_c = oracle_lib.sample_fwd(cT, eG, GRID, 0.0, D_REF, wp, sl)
    f_h = oracle_lib.sample_fwd(np.zeros_like(cT), eG, GRID, 1.0, D_REF, wp, sl)
    for t in range(40):
        C, G, _ = closed_form(wp[t, 0], sl[t, 0], 1.0)
        assert f_c[t] == pytest.approx(C, rel=1e-13, abs=1e-13)
        assert f_h[t] == pytest.approx((float(wp[t, 0, 2]) - G - D_REF) ** 2, rel=1e-12, abs=1e-12)


def test_constant_ground_height_term(oracle_lib):
    """A flat ground at height g gives w_z (z - g - d_ref)^2 wherever the
    waypoint is, inside the grid or beyond its edge."""
    g = 1.75
    cT = np.zeros((N, NY, NX))
    eG = np.full((N, NY, NX), g, np.float32)
    rng = np.random.default_rng(8)
    for inside in (True, False):
        wp, sl = waypoints(rng, 30, 1, inside)
        f = oracle_lib.sample_fwd(cT, eG, GRID, 3.0, D_REF, wp, sl)
        want = 3.0 * (wp[:, 0, 2].astype(np.float64) - g - D_REF) ** 2
        assert np.allclose(f, want, rtol=1e-13, atol=1e-13)
    # a waypoint at exactly body height costs nothing
    wp = np.array([[[X0 + 3.3 * RES, Y0 + 5.6 * RES, g + D_REF]]], np.float32)
    z = float(wp[0, 0, 2])
    assert oracle_lib.sample_fwd(cT, eG, GRID, 3.0, D_REF, wp, np.zeros((1, 1), np.int32))[0] == \
        pytest.approx(3.0 * (z - g - D_REF) ** 2, abs=1e-15)


def test_hand_worked_corner_weights(oracle_lib):
    """One waypoint at u = 3.25, v = 7.75 of slice 1: the cost of a map that
    is 1 at a single cell is that cell's bilinear weight, worked by hand:
    (3,7) 0.75*0.25, (4,7) 0.25*0.25, (3,8) 0.75*0.75, (4,8) 0.25*0.75, and
    0 at every other cell.  The adjoint scatters the same weights."""
    u, v = 3.25, 7.75
    wp = np.array([[[X0 + (u + 0.5) * RES, Y0 + (v + 0.5) * RES, 0.0]]], np.float32)
    sl = np.ones((1, 1), np.int32)
    eG = np.full((N, NY, NX), -np.inf, np.float32)   # no ground: the height term is dropped
    want = {(3, 7): 0.75 * 0.25, (4, 7): 0.25 * 0.25, (3, 8): 0.75 * 0.75, (4, 8): 0.25 * 0.75}
    for (i, j) in [(3, 7), (4, 7), (3, 8), (4, 8), (2, 7), (5, 8), (3, 6), (4, 9), (7, 3), (8, 4)]:
        cT = np.zeros((N, NY, NX))
        cT[1, j, i] = 1.0
        f = oracle_lib.sample_fwd(cT, eG, GRID, 1.0, D_REF, wp, sl)[0]
        assert f == want.get((i, j), 0.0), (i, j)
        cT[1, j, i] = 0.0
        cT[0, j, i] = cT[2, j, i] = 1.0     # other slices are not sampled
        assert oracle_lib.sample_fwd(cT, eG, GRID, 1.0, D_REF, wp, sl)[0] == 0.0
    _, gcT, gG = oracle_lib.sample_bwd(np.zeros((N, NY, NX)), eG, GRID, 1.0, D_REF, wp, sl, np.array([2.0]))
    got = {(int(i), int(j)): gcT[1, j, i] for j, i in zip(*np.nonzero(gcT[1]))}
    assert got == {c: 2.0 * w for c, w in want.items()}
    assert not gcT[0].any() and not gcT[2].any() and not gG.any()


def test_missing_ground_drops_height_term(oracle_lib):
    """A missing ground at any of the four corners drops the height term
    (C stays); a missing ground elsewhere changes nothing."""
    cT, eG = maps()
    u, v = 6.5, 4.25
    wp = np.array([[[X0 + (u + 0.5) * RES, Y0 + (v + 0.5) * RES, 5.0]]], np.float32)
    sl = np.zeros((1, 1), np.int32)
    C, G, full = closed_form(wp[0, 0], 0, 1.0)
    for (i, j), drop in [((6, 4), True), ((7, 4), True), ((6, 5), True), ((7, 5), True),
                         ((5, 4), False), ((8, 5), False), ((6, 6), False), ((7, 3), False)]:
        e = eG.copy()
        e[0, j, i] = -np.inf
        f = oracle_lib.sample_fwd(cT, e, GRID, 1.0, D_REF, wp, sl)[0]
        assert f == pytest.approx(C if drop else full, rel=1e-13), (i, j)


def test_invalid_waypoints_cost_nothing(oracle_lib):
    cT, eG = maps()
    wp = np.array([[[X0 + 1.0, Y0 + 1.0, 1.0], [np.nan, Y0 + 1.0, 1.0], [X0 + 1.0, np.inf, 1.0],
                    [X0 + 1.0, Y0 + 1.0, 1.0], [X0 + 1.0, Y0 + 1.0, 1.0]]], np.float32)
    sl = np.array([[0, 0, 0, -1, N]], np.int32)
    f = oracle_lib.sample_fwd(cT, eG, GRID, 1.0, D_REF, wp, sl)
    assert f[0] == pytest.approx(closed_form(wp[0, 0], 0, 1.0)[2], rel=1e-13)


def test_adjoint_on_linear_maps(oracle_lib):
    """Inside the grid (away from cell-centre lines) the waypoint gradient is
    the derivative of the closed form: df/dx = (b - 2 w_z e p)/r,
    df/dy = (c - 2 w_z e q)/r, df/dz = 2 w_z e with e = z - G - d_ref; beyond
    the clamp the x or y part is zero."""
    cT, eG = maps()
    rng = np.random.default_rng(9)
    w_z = 1.5
    for inside in (True, False):
        wp, sl = waypoints(rng, 5, 11, inside)
        gf = rng.normal(size=5)
        gwp, _, _ = oracle_lib.sample_bwd(cT, eG, GRID, w_z, D_REF, wp, sl, gf)
        for t in range(5):
            for w in range(11):
                x, y, z = (float(s) for s in wp[t, w])
                k = sl[t, w]
                a, b, c = COST[k]
                g, p, q = GROUND[k]
                u, v = (x - X0) / RES - 0.5, (y - Y0) / RES - 0.5
                inu, inv = 0.0 < u < NX - 1, 0.0 < v < NY - 1
                C, G, _ = closed_form(wp[t, w], k, w_z)
                e = z - G - D_REF
                want = np.array([(b - 2 * w_z * e * p) / RES if inu else 0.0,
                                 (c - 2 * w_z * e * q) / RES if inv else 0.0,
                                 2 * w_z * e]) * gf[t]
                assert np.allclose(gwp[t, w], want, rtol=1e-10, atol=1e-10), (t, w, gwp[t, w], want)
