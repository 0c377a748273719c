"""ctypes binding of the CPU oracle (``oracle/pct_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and
by the benchmark's CPU-baseline leg, never by the product path.  It shares no
code with the HIP library.  ``compile_library()`` compiles the C source with gcc; the
library is otherwise loaded from ``oracle/libpct_oracle.so``.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pct_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libpct_oracle.so")
_lib = None

RMAX = 24  # kernel half-width of the oracle's table (O_RMAX in the C source)


def compile_library(openmp: bool = True) -> str:
    cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-std=c11", "-shared", "-fPIC",
           "-Wall", "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
    if openmp:
        cmd.insert(1, "-fopenmp")
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class Grid(C.Structure):
    _fields_ = [("x0", C.c_float), ("y0", C.c_float), ("res", C.c_float),
                ("nx", C.c_int32), ("ny", C.c_int32), ("slice_dz", C.c_float)]


class Robot(C.Structure):
    _fields_ = [(n, C.c_float) for n in ("d_min", "d_ref", "theta_b", "theta_s", "theta_p",
                                         "c_barrier", "alpha_d", "alpha_b", "alpha_s",
                                         "d_inf", "d_sm")] + [("patch_radius", C.c_int32)]


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            compile_library()
        L = C.CDLL(_LIB_PATH)
        f32p, f64p = C.POINTER(C.c_float), C.POINTER(C.c_double)
        i32p, u8p = C.POINTER(C.c_int32), C.POINTER(C.c_uint8)
        L.o_omp_threads.restype = C.c_int
        L.o_set_threads.argtypes = [C.c_int]
        L.o_extent.argtypes = [f32p, C.c_int64, C.POINTER(Grid), f32p, f32p]
        L.o_extent.restype = C.c_int64
        L.o_planes.argtypes = [C.c_float, C.c_float, C.c_float, C.c_int, f32p]
        L.o_planes.restype = C.c_int
        L.o_build.argtypes = [f32p, C.c_int64, C.POINTER(Grid), f32p, C.c_int, f32p, f32p, i32p, i32p]
        L.o_build_window.argtypes = [f32p, C.c_int64, C.POINTER(Grid), f32p, C.c_int, C.c_int, C.c_int,
                                     C.c_int, C.c_int, f32p, f32p, i32p, i32p]
        L.o_layers.argtypes = [f32p, f32p, C.c_int, C.c_int, C.c_double, C.POINTER(Robot),
                               f64p, f64p, f64p, f64p, f64p, u8p, i32p]
        L.o_kernel.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int, f64p]
        L.o_kernel.restype = C.c_int
        L.o_inflate.argtypes = [f64p, C.c_int, C.c_int, f64p, C.c_int, C.c_int, f64p]
        L.o_eval.argtypes = [f32p, f32p, C.c_int, C.c_int, C.c_int, C.c_double, C.POINTER(Robot), f64p]
        L.o_eval.restype = C.c_int
        L.o_simplify.argtypes = [f32p, f64p, C.c_int, C.c_int, C.c_int, C.c_double, u8p]
        L.o_eval_envelope.argtypes = [f32p, f32p, C.c_int, C.c_int, C.c_int, C.c_double,
                                      C.POINTER(Robot), C.c_double, f64p, f64p]
        L.o_eval_envelope.restype = C.c_int64
        L.o_simplify_check.argtypes = [f32p, f64p, f64p, C.c_int, C.c_int, C.c_int, C.c_double,
                                       C.c_double, u8p]
        L.o_simplify_check.restype = C.c_int
        _register_grad(L)
        L.o_plan.argtypes = [f32p, f32p, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int, C.c_int, C.c_int, f64p]
        L.o_plan.restype = C.c_int64
        L.o_plan_path.argtypes = [f32p, f32p, C.c_int, C.c_int, C.c_int, C.c_double, f64p, C.c_int, C.c_int,
                                  C.c_int, C.c_int, C.c_int, C.c_int, i32p, C.c_int]
        L.o_plan_path.restype = C.c_int
        i64p = C.POINTER(C.c_int64)
        L.o_unique_cells.argtypes = [f32p, f32p, f32p, C.c_int, C.c_int, C.c_int, C.c_double, u8p, C.c_int64, i32p,
                                     f32p, f32p, f32p, i64p]
        L.o_unique_cells.restype = C.c_int64
        _lib = L
    return _lib


def _register_grad(L):
    """Signatures of the sampling and adjoint functions."""
    f32p, f64p = C.POINTER(C.c_float), C.POINTER(C.c_double)
    i32p, u8p = C.POINTER(C.c_int32), C.POINTER(C.c_uint8)
    L.o_sample_fwd.argtypes = [f64p, f32p, C.c_int, C.c_int, C.c_int, C.POINTER(Grid), C.c_double, C.c_double,
                               f32p, i32p, C.c_int, C.c_int, f64p]
    L.o_sample_bwd.argtypes = [f64p, f32p, C.c_int, C.c_int, C.c_int, C.POINTER(Grid), C.c_double, C.c_double,
                               f32p, i32p, C.c_int, C.c_int, f64p, f64p, f64p, f64p]
    L.o_eval_bwd.argtypes = [f32p, f32p, C.c_int, C.c_int, C.c_int, C.c_double, C.POINTER(Robot), f64p, f64p,
                             f64p, u8p, C.c_double]
    L.o_eval_bwd.restype = C.c_int
    L.o_route.argtypes = [f64p, f64p, i32p, i32p, C.c_int64, C.c_int64, f64p]
    L.o_eval_signature.argtypes = [f32p, f32p, C.c_int, C.c_int, C.c_int, C.c_double, C.POINTER(Robot), i32p]
    L.o_eval_signature.restype = C.c_int


def threads() -> int:
    return int(lib().o_omp_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops (results do not depend on it)."""
    lib().o_set_threads(int(n))


def grid_struct(g: dict) -> Grid:
    return Grid(g["x0"], g["y0"], g["res"], g["nx"], g["ny"], g["slice_dz"])


def robot_from_physical(phys: dict, res: float) -> dict:
    """The oracle's mapping from a physical robot description to the
    thresholds of Eqs. (1)-(6).  theta_s = tan(max slope) (a gradient
    magnitude is the tangent of the slope angle); theta_b = max step / 2r (the
    central difference across a step of height s is s / 2r); d_min and d_ref
    are the minimum and nominal body heights; theta_p, c^B and the scaling
    factors are Table I's values; d_inf is the inflation radius and d_sm the
    safe margin."""
    return dict(d_min=phys["min_interval"], d_ref=phys["nominal_height"],
                theta_b=phys["max_step"] / (2.0 * res),
                theta_s=math.tan(math.radians(phys["max_slope_deg"])),
                theta_p=0.20, c_barrier=50.0, alpha_d=20.0, alpha_b=20.0, alpha_s=15.0,
                d_inf=phys["inflation_radius"], d_sm=phys["safe_margin"], patch_radius=1)


def robot_struct(r: dict) -> Robot:
    return Robot(*[float(r[n]) for n in ("d_min", "d_ref", "theta_b", "theta_s", "theta_p",
                                         "c_barrier", "alpha_d", "alpha_b", "alpha_s",
                                         "d_inf", "d_sm")], int(r.get("patch_radius", 1)))


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


# ---------------------------------------------------------------------------
# tomogram construction

def extent(points, grid):
    pts = _f32(points).reshape(-1, 3)
    lo, hi = C.c_float(), C.c_float()
    g = grid_struct(grid)
    n = lib().o_extent(_p(pts, C.c_float), pts.shape[0], C.byref(g), C.byref(lo), C.byref(hi))
    return float(np.float32(lo.value)), float(np.float32(hi.value)), int(n)


def planes(zmin, zmax, ds, cap=1024):
    h = np.zeros(cap, dtype=np.float32)
    n = lib().o_planes(C.c_float(zmin), C.c_float(zmax), C.c_float(ds), cap, _p(h, C.c_float))
    if n == -1:
        raise ValueError("consecutive planes coincide in FP32")
    if n == -2:
        raise ValueError("too many slices")
    return h[:n].copy()


def build(points, grid, h, ids=True):
    pts = _f32(points).reshape(-1, 3)
    h = _f32(h)
    N, ny, nx = len(h), grid["ny"], grid["nx"]
    eG = np.empty((N, ny, nx), np.float32)
    eC = np.empty((N, ny, nx), np.float32)
    aG = np.empty((N, ny, nx), np.int32) if ids else None
    aC = np.empty((N, ny, nx), np.int32) if ids else None
    g = grid_struct(grid)
    lib().o_build(_p(pts, C.c_float), pts.shape[0], C.byref(g), _p(h, C.c_float), N,
                  _p(eG, C.c_float), _p(eC, C.c_float),
                  _p(aG, C.c_int32) if ids else None, _p(aC, C.c_int32) if ids else None)
    return eG, eC, aG, aC


def build_window(points, grid, h, wx0, wy0, wnx, wny, ids=True):
    """Algorithm 1 for the cells of one window of the grid; [N, wny, wnx]."""
    pts = _f32(points).reshape(-1, 3)
    h = _f32(h)
    N = len(h)
    eG = np.empty((N, wny, wnx), np.float32)
    eC = np.empty((N, wny, wnx), np.float32)
    aG = np.empty((N, wny, wnx), np.int32) if ids else None
    aC = np.empty((N, wny, wnx), np.int32) if ids else None
    g = grid_struct(grid)
    lib().o_build_window(_p(pts, C.c_float), pts.shape[0], C.byref(g), _p(h, C.c_float), N,
                         wx0, wy0, wnx, wny, _p(eG, C.c_float), _p(eC, C.c_float),
                         _p(aG, C.c_int32) if ids else None, _p(aC, C.c_int32) if ids else None)
    return eG, eC, aG, aC


def tomogram(points, grid, ids=True):
    """Extent, planes and Algorithm 1's construction loop in one call."""
    zmin, zmax, used = extent(points, grid)
    if used == 0:
        z = np.zeros((0, grid["ny"], grid["nx"]), np.float32)
        return dict(zmin=zmin, zmax=zmax, n_used=0, h=np.zeros(0, np.float32),
                    ground=z, ceil=z.copy(), arg_ground=None, arg_ceil=None)
    h = planes(zmin, zmax, grid["slice_dz"])
    eG, eC, aG, aC = build(points, grid, h, ids)
    return dict(zmin=zmin, zmax=zmax, n_used=used, h=h, ground=eG, ceil=eC,
                arg_ground=aG, arg_ceil=aC)


# ---------------------------------------------------------------------------
# traversability

def layers(eG2, eC2, res, robot):
    """Per-cell layers of one slice: c^I, c^G, c^init, m^xy, m^grad, gentle, branch."""
    eG2, eC2 = _f32(eG2), _f32(eC2)
    ny, nx = eG2.shape
    out = {k: np.empty((ny, nx), np.float64) for k in ("cI", "cG", "cinit", "mxy", "mgrad")}
    gentle = np.empty((ny, nx), np.uint8)
    branch = np.empty((ny, nx), np.int32)
    rb = robot_struct(robot)
    lib().o_layers(_p(eG2, C.c_float), _p(eC2, C.c_float), nx, ny, float(np.float32(res)), C.byref(rb),
                   *[_p(out[k], C.c_double) for k in ("cI", "cG", "cinit", "mxy", "mgrad")],
                   _p(gentle, C.c_uint8), _p(branch, C.c_int32))
    out["gentle"] = gentle.astype(bool)
    out["branch"] = branch
    return out


def kernel(res, d_inf, d_sm, rmax=RMAX):
    """Eq. (6) weights as a (2 rmax + 1)^2 array and the support radius R.
    Parameters are taken as FP32 values promoted to FP64."""
    w = 2 * rmax + 1
    K = np.zeros((w, w), np.float64)
    R = lib().o_kernel(float(np.float32(res)), float(np.float32(d_inf)), float(np.float32(d_sm)),
                       rmax, _p(K, C.c_double))
    if R == -1:
        raise ValueError("d_sm must exceed the grid resolution")
    if R == -2:
        raise ValueError("kernel support exceeds rmax")
    return K, R


def inflate(cinit, K, R, rmax=RMAX):
    ci = np.ascontiguousarray(cinit, dtype=np.float64)
    ny, nx = ci.shape
    out = np.empty_like(ci)
    Kc = np.ascontiguousarray(K, dtype=np.float64)
    lib().o_inflate(_p(ci, C.c_double), nx, ny, _p(Kc, C.c_double), rmax, R, _p(out, C.c_double))
    return out


def evaluate(eG, eC, res, robot):
    """c^T for all slices, FP64, shape [N, ny, nx]."""
    eG, eC = _f32(eG), _f32(eC)
    N, ny, nx = eG.shape
    out = np.empty((N, ny, nx), np.float64)
    rb = robot_struct(robot)
    R = lib().o_eval(_p(eG, C.c_float), _p(eC, C.c_float), N, nx, ny, float(np.float32(res)),
                     C.byref(rb), _p(out, C.c_double))
    if R < 0:
        raise ValueError("invalid inflation kernel parameters")
    return out


def simplify(eG, cT, c_barrier):
    eG = _f32(eG)
    cT = np.ascontiguousarray(cT, dtype=np.float64)
    N, ny, nx = eG.shape
    keep = np.zeros(N, np.uint8)
    lib().o_simplify(_p(eG, C.c_float), _p(cT, C.c_double), N, nx, ny, float(np.float32(c_barrier)),
                     _p(keep, C.c_uint8))
    return keep.astype(bool)


def envelope(eG, eC, res, robot, tau=4e-6):
    """(lo, hi, n_ambiguous) bracketing an FP32 evaluation of c^T."""
    eG, eC = _f32(eG), _f32(eC)
    N, ny, nx = eG.shape
    lo = np.empty((N, ny, nx), np.float64)
    hi = np.empty((N, ny, nx), np.float64)
    rb = robot_struct(robot)
    n = lib().o_eval_envelope(_p(eG, C.c_float), _p(eC, C.c_float), N, nx, ny, float(np.float32(res)),
                              C.byref(rb), tau, _p(lo, C.c_double), _p(hi, C.c_double))
    if n < 0:
        raise ValueError("invalid inflation kernel parameters")
    return lo, hi, int(n)


def simplify_check(eG, lo, hi, c_barrier, tol, keep):
    """-1 if ``keep`` is admissible under the three-valued rule, else the
    first offending slice."""
    eG = _f32(eG)
    lo = np.ascontiguousarray(lo, np.float64)
    hi = np.ascontiguousarray(hi, np.float64)
    kp = np.ascontiguousarray(np.asarray(keep, dtype=np.uint8))
    N, ny, nx = eG.shape
    return int(lib().o_simplify_check(_p(eG, C.c_float), _p(lo, C.c_double), _p(hi, C.c_double),
                                      N, nx, ny, float(np.float32(c_barrier)), tol, _p(kp, C.c_uint8)))


# ---------------------------------------------------------------------------
# trajectory cost sampling and adjoints

def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def sample_fwd(cT, eG, grid, w_z, d_ref, wp, slices):
    """Per-trajectory cost f [T] (FP64)."""
    cT, eG = _f64(cT), _f32(eG)
    wp = _f32(wp)
    sl = np.ascontiguousarray(slices, dtype=np.int32)
    T, W = sl.shape
    N, ny, nx = eG.shape
    f = np.empty(T, np.float64)
    g = grid_struct(grid)
    lib().o_sample_fwd(_p(cT, C.c_double), _p(eG, C.c_float), N, nx, ny, C.byref(g), float(w_z), float(d_ref),
                       _p(wp, C.c_float), _p(sl, C.c_int32), T, W, _p(f, C.c_double))
    return f


def sample_bwd(cT, eG, grid, w_z, d_ref, wp, slices, gf):
    """(gwp [T,W,3], gcT [N,ny,nx], gG [N,ny,nx]) for upstream gradient gf [T]."""
    cT, eG = _f64(cT), _f32(eG)
    wp = _f32(wp)
    sl = np.ascontiguousarray(slices, dtype=np.int32)
    T, W = sl.shape
    N, ny, nx = eG.shape
    gf = _f64(gf)
    gwp = np.zeros((T, W, 3), np.float64)
    gcT = np.zeros((N, ny, nx), np.float64)
    gG = np.zeros((N, ny, nx), np.float64)
    g = grid_struct(grid)
    lib().o_sample_bwd(_p(cT, C.c_double), _p(eG, C.c_float), N, nx, ny, C.byref(g), float(w_z), float(d_ref),
                       _p(wp, C.c_float), _p(sl, C.c_int32), T, W, _p(gf, C.c_double), _p(gwp, C.c_double),
                       _p(gcT, C.c_double), _p(gG, C.c_double))
    return gwp, gcT, gG


def eval_bwd(eG, eC, res, robot, gcT, tau=4e-6):
    """(gG, gC, uncertain) for upstream gradient gcT [N,ny,nx]."""
    eG, eC, gcT = _f32(eG), _f32(eC), _f64(gcT)
    N, ny, nx = eG.shape
    gG = np.zeros((N, ny, nx), np.float64)
    gC = np.zeros((N, ny, nx), np.float64)
    unc = np.zeros((N, ny, nx), np.uint8)
    rb = robot_struct(robot)
    R = lib().o_eval_bwd(_p(eG, C.c_float), _p(eC, C.c_float), N, nx, ny, float(np.float32(res)), C.byref(rb),
                         _p(gcT, C.c_double), _p(gG, C.c_double), _p(gC, C.c_double), _p(unc, C.c_uint8), tau)
    if R < 0:
        raise ValueError("invalid inflation kernel parameters")
    return gG, gC, unc.astype(bool)


def route(gG, gC, aG, aC, n_points):
    """dL/dz per point from dL/de^G, dL/de^C and the recorded point ids."""
    gG, gC = _f64(gG), _f64(gC)
    aG = np.ascontiguousarray(aG, np.int32)
    aC = np.ascontiguousarray(aC, np.int32)
    gz = np.zeros(n_points, np.float64)
    lib().o_route(_p(gG, C.c_double), _p(gC, C.c_double), _p(aG, C.c_int32), _p(aC, C.c_int32), gG.size,
                  n_points, _p(gz, C.c_double))
    return gz


def eval_signature(eG, eC, res, robot):
    eG, eC = _f32(eG), _f32(eC)
    N, ny, nx = eG.shape
    sig = np.empty((N, ny, nx), np.int32)
    rb = robot_struct(robot)
    lib().o_eval_signature(_p(eG, C.c_float), _p(eC, C.c_float), N, nx, ny, float(np.float32(res)), C.byref(rb),
                           _p(sig, C.c_int32))
    return sig


# ---------------------------------------------------------------------------
# path search through the slices (Sec. III-D)

def plan(cT, eG, c_barrier, start):
    """Distances [L, ny, nx] (FP64, +inf unreachable) from ``start`` = (x, y,
    layer) over the layers given as FP32 c^T and e^G arrays [L, ny, nx]."""
    cT, eG = _f32(cT), _f32(eG)
    L, ny, nx = cT.shape
    dist = np.empty((L, ny, nx), np.float64)
    n = lib().o_plan(_p(cT, C.c_float), _p(eG, C.c_float), L, nx, ny, float(np.float32(c_barrier)),
                     int(start[0]), int(start[1]), int(start[2]), _p(dist, C.c_double))
    if n < 0:
        raise ValueError("bad start node")
    return dist


def plan_path(cT, eG, c_barrier, dist, start, goal, max_len=None):
    """(x, y, layer) rows of the least-cost path from start to goal read
    back from ``dist``; None if the goal is unreachable."""
    cT, eG = _f32(cT), _f32(eG)
    dist = np.ascontiguousarray(dist, np.float64)
    L, ny, nx = cT.shape
    max_len = max_len or L * nx * ny
    path = np.empty((max_len, 3), np.int32)
    n = lib().o_plan_path(_p(cT, C.c_float), _p(eG, C.c_float), L, nx, ny, float(np.float32(c_barrier)),
                          _p(dist, C.c_double), int(start[0]), int(start[1]), int(start[2]), int(goal[0]),
                          int(goal[1]), int(goal[2]), _p(path, C.c_int32), int(max_len))
    if n == -2:
        raise ValueError("path longer than max_len")
    if n < 0:
        raise ValueError("bad node or not a distance field")
    return None if n == 0 else path[:n].copy()


# ---------------------------------------------------------------------------
# sparse storage of the unique cells of the kept slices (Sec. III-C)

def unique_cells(eG, eC, cT, c_barrier, keep):
    """Unique cells of the kept slices: dict of cell [M] int32, ground, ceil,
    cost [M] float32 and slice_off [N+1] int64 (slice k's cells are
    slice_off[k] .. slice_off[k+1])."""
    eG, eC, cT = _f32(eG), _f32(eC), _f32(cT)
    N, ny, nx = eG.shape
    kp = np.ascontiguousarray(np.asarray(keep, dtype=np.uint8))
    off = np.zeros(N + 1, np.int64)
    args = (_p(eG, C.c_float), _p(eC, C.c_float), _p(cT, C.c_float), N, nx, ny, float(np.float32(c_barrier)),
            _p(kp, C.c_uint8))
    m = int(lib().o_unique_cells(*args, 0, None, None, None, None, _p(off, C.c_int64)))
    out = dict(cell=np.empty(m, np.int32), ground=np.empty(m, np.float32), ceil=np.empty(m, np.float32),
               cost=np.empty(m, np.float32), slice_off=off)
    lib().o_unique_cells(*args, m, _p(out["cell"], C.c_int32), _p(out["ground"], C.c_float),
                         _p(out["ceil"], C.c_float), _p(out["cost"], C.c_float), _p(off, C.c_int64))
    return out
