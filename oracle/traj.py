"""Trajectory optimisation through the tomogram (Sec. III-E, Eq. (10)), FP64.

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and
by the benchmark's CPU-baseline leg, never by the product path.  It shares no
code with the HIP library.  Plain PyTorch CPU operations in float64; the
gradients come from autograd through the forward definitions.

Readings of the paper:
  - A trajectory is M quintic pieces per axis (degree N = 5), piece i on its
    own local time [0, T_i], with fixed start and goal states (position,
    velocity, acceleration).  For given interior waypoints and durations the
    pieces are the minimum-jerk spline: the quadratic program "minimise the
    jerk effort J_c subject to the boundary states, the waypoints and
    continuity of the derivatives 0..3 at the interior knots" (the
    constraints of Eq. (10)), solved here through its KKT system.  This is
    the minimum-control parametrisation the section follows.
  - Eq. (10)'s constraints enter as penalties sampled at K + 1 evenly spaced
    times per piece, summed with trapezoid weights T_i / K (halved at the
    two ends of a piece):
        w_z (q_z - Z_ref)^2                       Z_ref = G + d_ref
        w_c max(0, C - C_safe)^3                  C: travel cost c^T
        w_v max(0, |q'|^2 - v_max^2)^3            kinematic limits
        w_a max(0, |q''|^2 - a_max^2)^3
        w_h max(0, G + d_min - q_z)^3             H_g = e^G + d_min
        w_h max(0, q_z - H_c)^3                   H_c: the ceiling e^C
    The cost constraint is read as C <= C_safe (the printed inequality
    direction would reward high cost).  The heading-rate limit is not
    modelled (it is undefined at rest, where both ends of a trajectory are).
  - Maps are the piece's slice of c^T, e^G, e^C, interpolated bilinearly at
    cell centres and clamped to the grid edge with zero slope across the
    clamp.  Terms that use G are dropped where any of the four e^G corners
    is missing; the ceiling term where any e^C corner is open (+inf).  A
    piece whose slice lies outside [0, N) has no map terms (the kinematic
    terms remain).
  - Durations are T_i = exp(tau_i); the objective adds w_T * sum T_i.  The
    variables are the interior waypoints and the tau_i.
  - The optimiser: gradient descent with Armijo backtracking (sufficient
    decrease 1e-4, halving up to 30 times, the step doubled after each
    accepted iteration); an iteration whose search fails ends the run.  A
    trial point with a non-finite duration, coefficient or sample has the
    value +inf (it is rejected).
"""
from __future__ import annotations

import numpy as np
import torch

DT = torch.float64


def _jerk_gram(T):
    """W[j, k] = integral over [0, T] of (d^3 t^j / dt^3)(d^3 t^k / dt^3)."""
    W = torch.zeros(6, 6, dtype=DT)
    for j in range(3, 6):
        for k in range(3, 6):
            cj = j * (j - 1) * (j - 2)
            ck = k * (k - 1) * (k - 2)
            e = j + k - 5
            W[j, k] = cj * ck * T ** e / e
    return W


def _deriv_row(d, t):
    """Row r with r . c = d-th derivative of sum_j c_j t^j at time t."""
    row = []
    for j in range(6):
        if j < d:
            row.append(torch.zeros((), dtype=DT) * t)
            continue
        f = 1
        for m in range(d):
            f *= j - m
        row.append(f * t ** (j - d))
    return torch.stack([torch.as_tensor(x, dtype=DT) for x in row])


def minjerk_coeffs(knots, T, start, goal):
    """Monomial coefficients [M, 6, 3] (local time) of the minimum-jerk spline.

    knots: interior waypoints [M-1, 3]; T: durations [M]; start, goal: [3, 3]
    rows position, velocity, acceleration.  Tensors (autograd flows)."""
    M = T.shape[0]
    n = 6 * M
    W = torch.zeros(n, n, dtype=DT)
    for i in range(M):
        W[6 * i:6 * i + 6, 6 * i:6 * i + 6] = _jerk_gram(T[i])
    rows, rhs = [], []
    zero = torch.zeros(3, dtype=DT)

    def con(entries, b):
        r = torch.zeros(n, dtype=DT)
        for col, vec in entries:
            r = r.index_add(0, torch.arange(col, col + 6), vec)
        rows.append(r)
        rhs.append(b)

    t0 = torch.zeros((), dtype=DT)
    for d in range(3):  # start state
        con([(0, _deriv_row(d, t0))], start[d])
    for i in range(M - 1):  # waypoint and continuity of derivatives 0..3
        con([(6 * i, _deriv_row(0, T[i]))], knots[i])
        for d in range(4):
            con([(6 * i, _deriv_row(d, T[i])), (6 * i + 6, -_deriv_row(d, t0))], zero)
    for d in range(3):  # goal state
        con([(6 * (M - 1), _deriv_row(d, T[M - 1]))], goal[d])
    A = torch.stack(rows)
    b = torch.stack(rhs)
    m = A.shape[0]
    K = torch.zeros(n + m, n + m, dtype=DT)
    K[:n, :n] = 2 * W
    K[:n, n:] = A.T
    K[n:, :n] = A
    R = torch.cat([torch.zeros(n, 3, dtype=DT), b])
    sol = torch.linalg.solve(K, R)
    return sol[:n].reshape(M, 6, 3)


def jerk_effort(coef, T):
    """J_c = sum over pieces and axes of the integral of the squared jerk."""
    J = torch.zeros((), dtype=DT)
    for i in range(T.shape[0]):
        W = _jerk_gram(T[i])
        c = coef[i]
        J = J + torch.einsum("ja,jk,ka->", c, W, c)
    return J


def _axis(q, n):
    """Clamped cell-centred coordinate: (i0, i1, fraction), fraction carrying
    the gradient (zero across the clamp)."""
    if n == 1:
        return 0, 0, q * 0.0
    qc = torch.clamp(q, 0.0, float(n - 1))
    a = min(int(torch.floor(qc.detach())), n - 2)
    return a, a + 1, qc - a


def _bilinear(grid_vals, k, i0, i1, j0, j1, fu, fv):
    g00, g10 = float(grid_vals[k, j0, i0]), float(grid_vals[k, j0, i1])
    g01, g11 = float(grid_vals[k, j1, i0]), float(grid_vals[k, j1, i1])
    corners = (g00, g10, g01, g11)
    if not all(np.isfinite(corners)):
        return None
    return (1 - fu) * (1 - fv) * g00 + fu * (1 - fv) * g10 + (1 - fu) * fv * g01 + fu * fv * g11


def penalty_terms(coef, T, slices, maps, grid, prm):
    """Sum over pieces and samples of the weighted penalties (trapezoid)."""
    cT, eG, eC = maps
    ny, nx = cT.shape[1], cT.shape[2]
    K = int(prm["samples"])
    r = float(np.float32(grid["res"]))
    x0, y0 = float(np.float32(grid["x0"])), float(np.float32(grid["y0"]))
    F = torch.zeros((), dtype=DT)
    relu3 = lambda s: torch.clamp(s, min=0.0) ** 3
    for i in range(T.shape[0]):
        c = coef[i]
        k = int(slices[i])
        for j in range(K + 1):
            t = T[i] * j / K
            w = T[i] / K * (0.5 if j in (0, K) else 1.0)
            q = sum(c[m] * t ** m for m in range(6))
            v = sum(m * c[m] * t ** (m - 1) for m in range(1, 6))
            a = sum(m * (m - 1) * c[m] * t ** (m - 2) for m in range(2, 6))
            if not bool(torch.isfinite(q).all() & torch.isfinite(v).all() & torch.isfinite(a).all()):
                return torch.full((), float("inf"), dtype=DT)
            f = prm["w_v"] * relu3((v * v).sum() - prm["v_max"] ** 2)
            f = f + prm["w_a"] * relu3((a * a).sum() - prm["a_max"] ** 2)
            if 0 <= k < cT.shape[0]:
                u = (q[0] - x0) / r - 0.5
                vv = (q[1] - y0) / r - 0.5
                i0, i1, fu = _axis(u, nx)
                j0, j1, fv = _axis(vv, ny)
                f = f + prm["w_c"] * relu3(_bilinear(cT, k, i0, i1, j0, j1, fu, fv) - prm["c_safe"])
                G = _bilinear(eG, k, i0, i1, j0, j1, fu, fv)
                if G is not None:
                    f = f + prm["w_z"] * (q[2] - G - prm["d_ref"]) ** 2
                    f = f + prm["w_h"] * relu3(G + prm["d_min"] - q[2])
                H = _bilinear(eC, k, i0, i1, j0, j1, fu, fv)
                if H is not None:
                    f = f + prm["w_h"] * relu3(q[2] - H)
            F = F + w * f
    return F


def _as_param(prm):
    """Parameters as the library holds them: float32 values widened to FP64."""
    out = {k: float(np.float32(v)) for k, v in prm.items() if k != "samples"}
    out["samples"] = int(prm["samples"])
    return out


def objective(knots, tau, start, goal, slices, maps, grid, prm, grad=True):
    """(phi, d phi / d knots [M-1, 3], d phi / d tau [M]) in FP64.

    knots [M-1, 3], tau [M], start / goal [3, 3] (position, velocity,
    acceleration), slices [M] (slice of each piece), maps = (c^T, e^G, e^C)
    arrays [N, ny, nx]; prm: weights and limits (see the module text)."""
    prm = _as_param(prm)
    kn = torch.tensor(np.asarray(knots, np.float64).reshape(-1, 3), dtype=DT, requires_grad=grad)
    ta = torch.tensor(np.asarray(tau, np.float64), dtype=DT, requires_grad=grad)
    st = torch.tensor(np.asarray(start, np.float64), dtype=DT)
    go = torch.tensor(np.asarray(goal, np.float64), dtype=DT)
    T = torch.exp(ta)
    if not bool(torch.isfinite(T).all() & (T > 0).all()):
        # a trial point of the line search far outside the useful range
        return float("inf"), None, None
    coef = minjerk_coeffs(kn, T, st, go)
    phi = jerk_effort(coef, T) + prm["w_T"] * T.sum() + penalty_terms(coef, T, slices, maps, grid, prm)
    if not grad:
        return float(phi), None, None
    gk, gt = torch.autograd.grad(phi, [kn, ta], allow_unused=True)
    gk = torch.zeros_like(kn) if gk is None else gk
    return float(phi.detach()), gk.numpy().copy(), gt.numpy().copy()


def coefficients(knots, tau, start, goal):
    """Monomial coefficients [M, 6, 3] of the minimum-jerk spline (numpy)."""
    kn = torch.tensor(np.asarray(knots, np.float64).reshape(-1, 3), dtype=DT)
    T = torch.exp(torch.tensor(np.asarray(tau, np.float64), dtype=DT))
    st = torch.tensor(np.asarray(start, np.float64), dtype=DT)
    go = torch.tensor(np.asarray(goal, np.float64), dtype=DT)
    return minjerk_coeffs(kn, T, st, go).numpy()


def optimize(knots, tau, start, goal, slices, maps, grid, prm, iters, step):
    """Gradient descent with Armijo backtracking from (knots, tau).

    Returns (knots, tau, phi, iterations taken)."""
    x_k = np.asarray(knots, np.float64).reshape(-1, 3).copy()
    x_t = np.asarray(tau, np.float64).copy()
    alpha = float(step)
    phi, gk, gt = objective(x_k, x_t, start, goal, slices, maps, grid, prm)
    done = 0
    if not np.isfinite(phi):
        return x_k, x_t, phi, done
    for _ in range(iters):
        g2 = float((gk * gk).sum() + (gt * gt).sum())
        if g2 == 0.0:
            break
        ok = False
        for _ls in range(30):
            nk, nt = x_k - alpha * gk, x_t - alpha * gt
            p_new, _, _ = objective(nk, nt, start, goal, slices, maps, grid, prm, grad=False)
            if p_new <= phi - 1e-4 * alpha * g2:
                ok = True
                break
            alpha *= 0.5
        if not ok:
            break
        x_k, x_t = nk, nt
        phi, gk, gt = objective(x_k, x_t, start, goal, slices, maps, grid, prm)
        alpha *= 2.0
        done += 1
    return x_k, x_t, phi, done
