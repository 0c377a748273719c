"""Pins of the oracle's trajectory optimisation (Sec. III-E, Eq. (10)).

  - one rest-to-rest piece is the textbook minimum-jerk profile
    Delta (10 s^3 - 15 s^4 + 6 s^5), with effort 720 |Delta|^2 / T^5;
  - waypoints on a line at constant speed give a straight, jerk-free spline;
  - the spline interpolates, is continuous in derivatives 0..3 (imposed) and
    also in the fourth derivative, which the constraints do not impose: the
    Euler-Lagrange condition of the minimum, so the KKT solve found it;
  - no other C2 spline through the same waypoints (quintic Hermite pieces
    with arbitrary knot velocities and accelerations) has less jerk effort;
  - on a flat map the penalties of a constant-velocity line have closed
    forms (the trapezoid rule is exact for constants);
  - missing ground drops the height terms; an open ceiling drops its term;
  - autograd gradients equal central differences of the forward on maps
    that are linear in x and y (the interpolation then has no kinks);
  - a cost map linear in the cell indices and the textbook profile's speed
    and acceleration give closed forms of the map and kinematic terms;
  - one piece with a time weight: the optimiser reaches the closed-form
    duration T* = (5 * 720 |Delta|^2 / w_T)^(1/6), and its objective never
    increases.
"""
import numpy as np
import pytest
import torch

from oracle import traj

REST = np.zeros((3, 3))
ZERO_W = dict(w_z=0.0, w_c=0.0, w_v=0.0, w_a=0.0, w_h=0.0, w_T=0.0, c_safe=0.0, v_max=1.0, a_max=1.0,
              d_ref=0.0, d_min=0.0, samples=4)


def state(p, v=(0, 0, 0), a=(0, 0, 0)):
    return np.array([p, v, a], np.float64)


def flat_maps(nx=40, ny=30, N=2, g=0.0, c=1.0, ceil=np.inf):
    eG = np.full((N, ny, nx), g, np.float32)
    cT = np.full((N, ny, nx), c, np.float32)
    eC = np.full((N, ny, nx), ceil, np.float32)
    return cT, eG, eC


GRID = dict(x0=0.0, y0=0.0, res=0.5, nx=40, ny=30)


def test_single_piece_rest_to_rest():
    d = np.array([3.0, -2.0, 0.5])
    T = 2.0
    coef = traj.coefficients(np.zeros((0, 3)), [np.log(T)], REST, state(d))
    want = np.zeros((6, 3))
    want[3], want[4], want[5] = 10 * d / T ** 3, -15 * d / T ** 4, 6 * d / T ** 5
    np.testing.assert_allclose(coef[0], want, atol=1e-12)
    phi, _, _ = traj.objective(np.zeros((0, 3)), [np.log(T)], REST, state(d), [0], flat_maps(), GRID, ZERO_W)
    assert phi == pytest.approx(720 * (d @ d) / T ** 5, rel=1e-12)


def test_constant_velocity_line():
    v = np.array([1.5, 0.5, 0.0])
    Ts = np.array([0.5, 0.5, 0.5, 0.5])
    p0 = np.array([1.0, 2.0, 0.3])
    knots = np.array([p0 + v * 0.5 * (i + 1) for i in range(3)])
    coef = traj.coefficients(knots, np.log(Ts), state(p0, v), state(p0 + 2.0 * v, v))
    for i in range(4):
        np.testing.assert_allclose(coef[i, 0], p0 + v * 0.5 * i, atol=1e-12)
        np.testing.assert_allclose(coef[i, 1], v, atol=1e-12)
        np.testing.assert_allclose(coef[i, 2:], 0.0, atol=1e-11)
    phi, _, _ = traj.objective(knots, np.log(Ts), state(p0, v), state(p0 + 2.0 * v, v), [0] * 4, flat_maps(),
                               GRID, ZERO_W)
    assert abs(phi) < 1e-18


def _deriv(c, d, t):
    return sum(np.prod(range(j - d + 1, j + 1)) * c[j] * t ** (j - d) for j in range(d, 6))


def test_interpolation_and_snap_continuity():
    rng = np.random.default_rng(0)
    M = 6
    knots = rng.uniform(-5, 5, (M - 1, 3))
    Ts = rng.uniform(0.4, 2.0, M)
    start = state(rng.uniform(-5, 5, 3), rng.uniform(-1, 1, 3), rng.uniform(-1, 1, 3))
    goal = state(rng.uniform(-5, 5, 3), rng.uniform(-1, 1, 3), rng.uniform(-1, 1, 3))
    coef = traj.coefficients(knots, np.log(Ts), start, goal)
    for d in range(3):
        np.testing.assert_allclose(_deriv(coef[0], d, 0.0), start[d], atol=1e-9)
        np.testing.assert_allclose(_deriv(coef[-1], d, Ts[-1]), goal[d], atol=1e-9)
    for i in range(M - 1):
        np.testing.assert_allclose(_deriv(coef[i], 0, Ts[i]), knots[i], atol=1e-9)
        for d in range(5):  # 0..3 imposed, 4 follows from optimality
            a, b = _deriv(coef[i], d, Ts[i]), _deriv(coef[i + 1], d, 0.0)
            np.testing.assert_allclose(a, b, atol=1e-7 * max(1.0, np.abs(a).max()))


def _hermite_piece(x0, x1, T):
    """Quintic through (p, v, a) at both ends, solved numerically."""
    A = np.array([[_deriv(np.eye(6)[j], d, t) for j in range(6)] for t in (0.0, T) for d in range(3)])
    return np.linalg.solve(A, np.concatenate([x0, x1]))


def _jerk_numeric(c, T):
    x, w = np.polynomial.legendre.leggauss(8)
    t = 0.5 * T * (x + 1)
    j = _deriv(c, 3, t)
    return 0.5 * T * float((w * j * j).sum())


def test_no_c2_spline_has_less_jerk():
    rng = np.random.default_rng(1)
    M = 5
    knots = rng.uniform(-3, 3, (M - 1, 3))
    Ts = rng.uniform(0.5, 1.5, M)
    start, goal = state(rng.uniform(-3, 3, 3)), state(rng.uniform(-3, 3, 3))
    coef = traj.coefficients(knots, np.log(Ts), start, goal)
    j_opt, _, _ = traj.objective(knots, np.log(Ts), start, goal, [0] * M, flat_maps(), GRID, ZERO_W)
    pts = [start[0]] + list(knots) + [goal[0]]

    def effort(vel, acc):
        tot = 0.0
        for i in range(M):
            for ax in range(3):
                x0 = [pts[i][ax], vel[i][ax], acc[i][ax]]
                x1 = [pts[i + 1][ax], vel[i + 1][ax], acc[i + 1][ax]]
                tot += _jerk_numeric(_hermite_piece(x0, x1, Ts[i]), Ts[i])
        return tot

    # the optimum's own knot states reproduce its effort
    vel = [start[1]] + [_deriv(coef[i], 1, Ts[i]) for i in range(M - 1)] + [goal[1]]
    acc = [start[2]] + [_deriv(coef[i], 2, Ts[i]) for i in range(M - 1)] + [goal[2]]
    assert effort(vel, acc) == pytest.approx(j_opt, rel=1e-9)
    for trial in range(20):
        dv = rng.normal(0, 0.3, (M + 1, 3))
        da = rng.normal(0, 0.3, (M + 1, 3))
        dv[0] = dv[-1] = da[0] = da[-1] = 0
        assert effort(np.array(vel) + dv, np.array(acc) + da) > j_opt


def test_flat_map_closed_forms():
    v = np.array([2.0, 0.0, 0.0])
    p0 = np.array([2.0, 3.0, 0.7])
    Ts = np.array([0.6, 0.9, 0.5])
    knots = np.array([p0 + v * Ts[:1].sum(), p0 + v * Ts[:2].sum()])
    goal = state(p0 + v * Ts.sum(), v)
    prm = dict(w_z=3.0, w_c=0.5, w_v=2.0, w_a=7.0, w_h=11.0, w_T=1.25, c_safe=1.0, v_max=1.5, a_max=1.0,
               d_ref=0.5, d_min=0.3, samples=6)
    g0, c0 = 0.25, 3.0
    maps = flat_maps(g=g0, c=c0, ceil=10.0)
    phi, _, _ = traj.objective(knots, np.log(Ts), state(p0, v), goal, [0, 1, 0], maps, GRID, prm)
    Tt = Ts.sum()
    f32 = lambda x: float(np.float32(x))
    want = (f32(prm["w_T"]) * Tt + f32(prm["w_v"]) * (4.0 - f32(1.5) ** 2) ** 3 * Tt
            + f32(prm["w_c"]) * (c0 - 1.0) ** 3 * Tt + f32(prm["w_z"]) * (0.7 - g0 - 0.5) ** 2 * Tt)
    assert phi == pytest.approx(want, rel=1e-10)
    # a body below H_g (ground + d_min) and above the ceiling
    for z, term in ((g0 + 0.1, (g0 + f32(0.3) - (g0 + 0.1)) ** 3), (10.5, 0.5 ** 3)):
        pz = p0.copy()
        pz[2] = z
        kz = knots.copy()
        kz[:, 2] = z
        gz = state(pz + v * Tt, v)
        phi_z, _, _ = traj.objective(kz, np.log(Ts), state(pz, v), gz, [0, 1, 0], maps, GRID, prm)
        base = (f32(prm["w_T"]) + f32(prm["w_v"]) * (4.0 - f32(1.5) ** 2) ** 3 + f32(prm["w_c"]) * 8.0
                + f32(prm["w_z"]) * (z - g0 - 0.5) ** 2) * Tt
        assert phi_z == pytest.approx(base + f32(11.0) * term * Tt, rel=1e-9)


def test_missing_ground_and_open_ceiling():
    p0 = np.array([2.0, 3.0, 0.7])
    goal = state(p0 + [3.0, 1.0, 0.0])
    prm = dict(w_z=3.0, w_c=0.0, w_v=0.0, w_a=0.0, w_h=11.0, w_T=0.0, c_safe=0.0, v_max=1.0, a_max=1.0,
               d_ref=0.5, d_min=0.3, samples=5)
    base, _, _ = traj.objective(np.zeros((0, 3)), [0.3], state(p0), goal, [0], flat_maps(), GRID, ZERO_W)
    cT, eG, eC = flat_maps(g=0.0, ceil=0.1)
    eG[:] = -np.inf
    phi, _, _ = traj.objective(np.zeros((0, 3)), [0.3], state(p0), goal, [0], (cT, eG, eC), GRID, prm)
    # no ground: only the ceiling term remains besides the jerk
    assert phi > base
    eC[:] = np.inf
    phi, _, _ = traj.objective(np.zeros((0, 3)), [0.3], state(p0), goal, [0], (cT, eG, eC), GRID, prm)
    assert phi == pytest.approx(base, rel=1e-12)


def linear_maps(nx=40, ny=30, N=2):
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    cT = np.stack([0.2 * x + 0.1 * y + 1.0 + k for k in range(N)]).astype(np.float32)
    eG = np.stack([0.03 * x - 0.02 * y + 0.5 * k for k in range(N)]).astype(np.float32)
    eC = np.stack([0.01 * x + 0.02 * y + 2.0 + k for k in range(N)]).astype(np.float32)
    return cT, eG, eC


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    M = 4
    prm = dict(w_z=2.0, w_c=0.3, w_v=0.7, w_a=0.2, w_h=5.0, w_T=0.8, c_safe=3.0, v_max=1.0, a_max=1.5,
               d_ref=0.6, d_min=0.45, samples=5)
    start = state([4.0, 4.0, 0.9], [0.5, 0.2, 0.0])
    goal = state([14.0, 9.0, 1.1])
    knots = np.array([[6.5, 5.0, 1.0], [9.0, 6.5, 0.5], [11.5, 7.5, 2.4]]) + rng.normal(0, 0.05, (3, 3))
    tau = np.log(rng.uniform(0.8, 1.6, M))
    maps = linear_maps()
    sl = [0, 1, 1, 0]
    phi, gk, gt = traj.objective(knots, tau, start, goal, sl, maps, GRID, prm)
    h = 1e-6
    for idx in np.ndindex(knots.shape):
        kp, km = knots.copy(), knots.copy()
        kp[idx] += h
        km[idx] -= h
        fp = traj.objective(kp, tau, start, goal, sl, maps, GRID, prm, grad=False)[0]
        fm = traj.objective(km, tau, start, goal, sl, maps, GRID, prm, grad=False)[0]
        assert gk[idx] == pytest.approx((fp - fm) / (2 * h), rel=1e-5, abs=1e-6 * abs(phi))
    for i in range(M):
        tp, tm = tau.copy(), tau.copy()
        tp[i] += h
        tm[i] -= h
        fp = traj.objective(knots, tp, start, goal, sl, maps, GRID, prm, grad=False)[0]
        fm = traj.objective(knots, tm, start, goal, sl, maps, GRID, prm, grad=False)[0]
        assert gt[i] == pytest.approx((fp - fm) / (2 * h), rel=1e-5, abs=1e-6 * abs(phi))


def test_optimizer_reaches_closed_form_duration():
    d = np.array([2.0, 1.0, 0.0])
    prm = dict(ZERO_W, w_T=3.0)
    wT = float(np.float32(3.0))
    t_star = (5 * 720 * (d @ d) / wT) ** (1 / 6)
    seen = []
    tau = np.array([np.log(1.0)])
    for _ in range(6):
        _, tau, phi, n = traj.optimize(np.zeros((0, 3)), tau, REST, state(d), [0], flat_maps(), GRID, prm,
                                       iters=10, step=1e-4)
        seen.append(phi)
    assert all(b <= a for a, b in zip(seen, seen[1:]))
    assert np.exp(tau[0]) == pytest.approx(t_star, rel=1e-6)


def test_linear_cost_map_closed_form():
    """Bilinear interpolation reproduces a map that is linear in the cell
    indices, so on a straight constant-velocity line the cost term is the
    trapezoid sum of (C(q(t)) - C_safe)^3 with C written out directly."""
    nx, ny, res = 40, 30, 0.5
    a0, bx, by = 2.0, 0.25, -0.125
    jj, ii = np.mgrid[0:ny, 0:nx].astype(np.float64)
    cT = np.stack([a0 + bx * ii + by * jj] * 2).astype(np.float32)
    eG = np.full_like(cT, -np.inf)
    eC = np.full_like(cT, np.inf)
    grid = dict(x0=0.0, y0=0.0, res=res, nx=nx, ny=ny)
    v = np.array([1.5, 0.75, 0.0])
    p0 = np.array([3.1, 4.2, 1.0])
    Ts = np.array([1.25, 0.75])
    knots = np.array([p0 + v * Ts[0]])
    goal = state(p0 + v * Ts.sum(), v)
    K = 5
    prm = dict(ZERO_W, w_c=1.0, c_safe=-1.0, samples=K)
    phi, _, _ = traj.objective(knots, np.log(Ts), state(p0, v), goal, [1, 0], (cT, eG, eC), grid, prm)
    want, t0 = 0.0, 0.0
    for T in Ts:
        for j in range(K + 1):
            t = T * j / K
            q = p0 + v * (t0 + t)
            C = a0 + bx * (q[0] / res - 0.5) + by * (q[1] / res - 0.5)
            want += (T / K) * (0.5 if j in (0, K) else 1.0) * (C + 1.0) ** 3
        t0 += T
    assert phi == pytest.approx(want, rel=1e-12)


def test_kinematic_terms_on_textbook_profile():
    """Speed and acceleration penalties along the rest-to-rest profile, with
    its velocity Delta (30 s^2 - 60 s^3 + 30 s^4) / T and acceleration
    Delta (60 s - 180 s^2 + 120 s^3) / T^2 written out."""
    d = np.array([3.0, -2.0, 0.5])
    T, K = 2.0, 7
    f32 = lambda x: float(np.float32(x))
    prm = dict(ZERO_W, w_v=0.3, v_max=0.5, w_a=0.2, a_max=0.4, samples=K)
    phi, _, _ = traj.objective(np.zeros((0, 3)), [np.log(T)], REST, state(d), [0], flat_maps(), GRID, prm)
    want = 720 * (d @ d) / T ** 5
    for j in range(K + 1):
        s = j / K
        v = d * (30 * s ** 2 - 60 * s ** 3 + 30 * s ** 4) / T
        a = d * (60 * s - 180 * s ** 2 + 120 * s ** 3) / T ** 2
        w = T / K * (0.5 if j in (0, K) else 1.0)
        want += w * (f32(0.3) * max(0.0, v @ v - f32(0.5) ** 2) ** 3 + f32(0.2) * max(0.0, a @ a - f32(0.4) ** 2) ** 3)
    assert phi == pytest.approx(want, rel=1e-11)
