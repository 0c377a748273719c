"""Pins of the oracle's traversability evaluation (Sec. III-B, Eqs. (1)-(6)).

Analytic ground/ceiling grids with known slopes, steps and intervals; the
inflation kernel against values worked out by hand from Eq. (6); inflation
against its impulse response and, for a 0/1 kernel, against
scipy.ndimage.grey_dilation; invariants stated in the paper."""
import math

import numpy as np
import pytest
from scipy import ndimage

import scenes
from conftest import load_golden

RES = 0.1
ROBOT0 = None


def robot0(oracle_lib, **kw):
    r = oracle_lib.robot_from_physical(scenes.ROBOT_CONFIG0, RES)
    r.update(kw)
    return r


def f32(a):
    return np.asarray(a, dtype=np.float32)


def interior(a, m=1):
    return a[m:-m, m:-m]


def test_robot_mapping(oracle_lib):
    r = robot0(oracle_lib)
    assert r["theta_b"] == pytest.approx(1.0)
    assert r["theta_s"] == pytest.approx(math.tan(math.radians(30)))
    t1 = load_golden("table1_params.json")
    for k in ("theta_p", "c_barrier", "alpha_d", "alpha_b", "alpha_s"):
        assert r[k] == t1[k]


def test_flat_ground_open_sky(oracle_lib):
    """Flat ground, no ceiling: zero slope, zero cost inside; a cell whose
    stencil leaves the grid has no slope estimate and is a barrier."""
    ny, nx = 7, 9
    eG = np.full((ny, nx), 0.7, np.float32)
    eC = np.full((ny, nx), np.inf, np.float32)
    L = oracle_lib.layers(eG, eC, RES, robot0(oracle_lib))
    assert np.all(interior(L["mgrad"]) == 0) and np.all(interior(L["mxy"]) == 0)
    assert np.all(interior(L["cG"]) == 0) and np.all(interior(L["cI"]) == 0)
    assert np.all(interior(L["cinit"]) == 0)
    border = np.ones((ny, nx), bool)
    border[1:-1, 1:-1] = False
    assert np.all(L["cinit"][border] == 50.0)
    assert np.all(L["branch"][border] == 1)


@pytest.mark.parametrize("gap,expect", [(1.0, 0.0), (0.8, 4.0), (0.5, 10.0), (0.25, 50.0), (1.5, 0.0)])
def test_interval_cost_eq1(oracle_lib, gap, expect):
    """Eq. (1) with d_min = 0.5, d_ref = 1.0, alpha_d = 20: a barrier below
    d_min (strict), 20 (d_ref - d^I) between, 0 above d_ref."""
    ny, nx = 5, 5
    eG = np.full((ny, nx), 0.5, np.float32)
    eC = np.full((ny, nx), np.float32(0.5) + np.float32(gap), np.float32)
    L = oracle_lib.layers(eG, eC, RES, robot0(oracle_lib))
    dI = float(np.float32(0.5) + np.float32(gap)) - 0.5
    assert L["cI"][2, 2] == pytest.approx(expect if dI >= 0.5 else 50.0, abs=2e-5)
    assert L["cinit"][2, 2] == pytest.approx(min(50.0, L["cI"][2, 2] + L["cG"][2, 2]))


@pytest.mark.parametrize("axis", ["x", "y", "xy"])
def test_ramp_gives_its_slope(oracle_lib, axis):
    """A plane of slope angle phi: m^grad = tan(phi) (along an axis m^xy is
    the same; along the diagonal with tan(phi) per axis, m^grad = sqrt(2) m^xy)
    and the gentle cost alpha_s (m^grad / theta_s)^2.  The grid is not
    square so that swapped axes show."""
    ny, nx = 6, 11
    s = math.tan(math.radians(10.0))
    iy, ix = np.mgrid[0:ny, 0:nx].astype(np.float64)
    z = {"x": ix, "y": iy, "xy": ix + iy}[axis] * RES * s
    eG = f32(z)
    eC = np.full((ny, nx), np.inf, np.float32)
    rb = robot0(oracle_lib)
    L = oracle_lib.layers(eG, eC, RES, rb)
    mg = s * (math.sqrt(2) if axis == "xy" else 1.0)
    np.testing.assert_allclose(interior(L["mgrad"]), mg, rtol=2e-6)
    np.testing.assert_allclose(interior(L["mxy"]), s, rtol=2e-6)
    np.testing.assert_allclose(interior(L["cG"]), 15.0 * (mg / rb["theta_s"]) ** 2, rtol=5e-6)
    assert np.all(interior(L["branch"]) == 2)


def test_step_central_difference_and_p_s(oracle_lib):
    """A step of height s along x: exactly the two columns beside it see
    m^xy = s / 2r (central difference).  With s = 0.15 m (m^xy = 0.75, between
    theta_s and theta_b) three of the eight neighbours are gentle, which
    beats floor(0.2 * 8) = 1, so Eq. (4) gives alpha_b (m^xy / theta_b)^2."""
    ny, nx = 7, 12
    for s, br, cg in [(0.15, 3, 20.0 * 0.75 ** 2), (0.25, 1, 50.0)]:
        eG = np.zeros((ny, nx), np.float32)
        eG[:, 6:] = s
        eC = np.full((ny, nx), np.inf, np.float32)
        L = oracle_lib.layers(eG, eC, RES, robot0(oracle_lib))
        col = interior(L["mxy"])[0]       # interior row, columns 1..nx-2
        expect = np.zeros(nx - 2)
        expect[[4, 5]] = float(np.float32(s)) / (2 * float(np.float32(RES)))
        np.testing.assert_allclose(col, expect, rtol=1e-12, atol=0)
        assert np.all(L["branch"][1:-1, 5:7] == br)
        np.testing.assert_allclose(L["cG"][1:-1, 5:7], cg, rtol=1e-6)
        # the wheeled robot (theta_p = 1) turns every step cell into a barrier
        W = oracle_lib.layers(eG, eC, RES, robot0(oracle_lib, theta_p=1.0))
        assert np.all(W["cG"][1:-1, 5:7] == 50.0)
        assert not np.any(W["branch"] == 3)


def test_patch_count_rule(oracle_lib):
    """Branch 3 (step, traversable) exactly where more than floor(theta_p * 8)
    of the 8 patch neighbours are gentle, with off-grid neighbours not gentle."""
    rng = np.random.default_rng(7)
    ny, nx = 14, 17
    eG = f32(np.round(rng.normal(0, 0.06, (ny, nx)), 3))
    eG[rng.random((ny, nx)) < 0.1] = -np.inf
    eC = np.full((ny, nx), np.inf, np.float32)
    for tp in (0.2, 0.45, 0.8, 1.0):
        L = oracle_lib.layers(eG, eC, RES, robot0(oracle_lib, theta_p=tp))
        g = np.pad(L["gentle"], 1)
        cnt = sum(np.roll(np.roll(g, dy, 0), dx, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
                  if dy or dx)[1:-1, 1:-1]
        kp = math.floor(float(np.float32(tp)) * 8)
        step = (L["branch"] == 3) | (L["branch"] == 4)
        assert np.array_equal(L["branch"][step] == 3, cnt[step] > kp)


def test_kernel_figure_example(oracle_lib):
    g = load_golden("inflation_kernel_fig.json")
    K, R = oracle_lib.kernel(g["res"], g["d_inf"], g["d_sm"])
    c = K.shape[0] // 2
    np.testing.assert_allclose(K[c, c + np.array(g["axis_distance_cells"])], g["axis_values"], atol=1e-6)
    for key, v in g["diag_values_cells"].items():
        m, n = map(int, key.split(","))
        assert K[c + n, c + m] == pytest.approx(v, abs=1e-6)
        assert K[c - m, c - n] == pytest.approx(v, abs=1e-6)
    assert R == g["support_radius"]
    assert (K > 0).sum() == g["support_taps"] and (K == 1).sum() == g["unit_taps"]


def test_kernel_config0_robot(oracle_lib):
    """d_inf = 0.3, d_sm = 0.4, r = 0.1: weight 1 within 3 cells, support
    m^2 + n^2 < 36 (R = 5, 109 taps, 29 of them at 1)."""
    K, R = oracle_lib.kernel(0.1, 0.3, 0.4)
    assert R == 5 and (K > 0).sum() == 109 and (K == 1).sum() == 29
    with pytest.raises(ValueError):
        oracle_lib.kernel(0.1, 0.3, 0.1)


@pytest.mark.parametrize("where", [(6, 7), (0, 0), (12, 3)])
def test_inflation_impulse_response(oracle_lib, where):
    K, R = oracle_lib.kernel(0.1, 0.3, 0.4)
    ny, nx = 13, 16
    ci = np.zeros((ny, nx))
    y0, x0 = where
    ci[y0, x0] = 50.0
    cT = oracle_lib.inflate(ci, K, R)
    c = K.shape[0] // 2
    for y in range(ny):
        for x in range(nx):
            dy, dx = y - y0, x - x0
            w = K[c + dy, c + dx] if abs(dy) <= c and abs(dx) <= c else 0.0
            assert cT[y, x] == pytest.approx(50.0 * w, abs=1e-12)


def test_binary_kernel_is_disk_dilation(oracle_lib):
    """With a margin narrower than any gap between lattice distances the
    kernel is 0/1 on a disk, and the weighted max is grey dilation by that
    disk (off-grid taps contribute nothing: costs are >= 0)."""
    K, R = oracle_lib.kernel(0.1, 0.25, 0.1001)
    rng = np.random.default_rng(3)
    ci = rng.random((23, 31)) * 50.0
    cT = oracle_lib.inflate(ci, K, R)
    m = np.arange(-R, R + 1)
    disk = (m[:, None] ** 2 + m[None, :] ** 2) <= 6
    assert np.array_equal(K[K.shape[0] // 2 + m][:, K.shape[0] // 2 + m] > 0, disk)
    ref = ndimage.grey_dilation(ci, footprint=disk, mode="constant", cval=0.0)
    np.testing.assert_array_equal(cT, ref)


def _c0_tomogram(oracle_lib):
    sc = scenes.config0_scene()
    return sc, oracle_lib.tomogram(sc.points, sc.grid)


def test_invariants_on_scenes(oracle_lib):
    """m^xy <= m^grad <= sqrt(2) m^xy; 0 <= c^init <= c^B; c^init <= c^T <= c^B."""
    sc = scenes.multistorey_scene(5, 8.0, 6.0, 120_000, n_floors=3)
    tm = oracle_lib.tomogram(sc.points, sc.grid)
    rb = oracle_lib.robot_from_physical(sc.robot, sc.grid["res"])
    K, R = oracle_lib.kernel(sc.grid["res"], rb["d_inf"], rb["d_sm"])
    for k in range(0, len(tm["h"]), 3):
        L = oracle_lib.layers(tm["ground"][k], tm["ceil"][k], sc.grid["res"], rb)
        f = np.isfinite(L["mxy"])
        assert np.all(L["mxy"][f] <= L["mgrad"][f] * (1 + 1e-12))
        assert np.all(L["mgrad"][f] <= math.sqrt(2) * L["mxy"][f] * (1 + 1e-12))
        assert np.all((L["cinit"] >= 0) & (L["cinit"] <= 50.0))
        cT = oracle_lib.inflate(L["cinit"], K, R)
        assert np.all(cT >= L["cinit"]) and np.all(cT <= 50.0)


def test_no_ground_is_barrier(oracle_lib):
    eG = np.zeros((6, 6), np.float32)
    eG[3, 3] = -np.inf
    eC = np.full((6, 6), np.inf, np.float32)
    L = oracle_lib.layers(eG, eC, RES, robot0(oracle_lib))
    assert L["cinit"][3, 3] == 50.0 and L["branch"][3, 3] == 0
    # its four stencil neighbours lose their slope estimate
    for y, x in [(2, 3), (4, 3), (3, 2), (3, 4)]:
        assert L["branch"][y, x] == 1


def test_envelope_brackets_and_flags_thresholds(oracle_lib):
    """Away from thresholds lo = hi = c^T; a step of exactly max_step sits on
    theta_b and is flagged, with lo (step cost) < hi (barrier)."""
    sc, tm = _c0_tomogram(oracle_lib)
    rb = oracle_lib.robot_from_physical(sc.robot, sc.grid["res"])
    cT = oracle_lib.evaluate(tm["ground"], tm["ceil"], sc.grid["res"], rb)
    lo, hi, n = oracle_lib.envelope(tm["ground"], tm["ceil"], sc.grid["res"], rb)
    assert np.all(lo <= cT) and np.all(cT <= hi)
    if n == 0:
        assert np.array_equal(lo, hi)
    eG = np.zeros((1, 25, 30), np.float32)
    eG[0, :, 15:] = 0.2
    eC = np.full_like(eG, np.inf)
    lo, hi, n = oracle_lib.envelope(eG, eC, RES, robot0(oracle_lib))
    assert n > 0
    # cells more than 5 cells from the (barrier) border are not inflated by it
    assert np.all(lo[0, 8:17, 14:16] == 20.0) and np.all(hi[0, 8:17, 14:16] == 50.0)
