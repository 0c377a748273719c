"""Python binding of libpct, the MI355X (gfx950) point-cloud-tomography library.

The functions carry the C ABI's names (see ``include/pct.h``) and only
marshal arguments: torch CUDA tensors are passed by ``data_ptr()`` with the
current stream, outputs and workspaces are allocated as torch tensors.  Every
step of the computation runs in the library's HIP kernels; if the library is
missing, importing this package raises.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpct.so")

from .abi import (PCT_ACCUMULATE, PCT_DESCRIPTORS_RESIDENT, PCT_ERR_ARG, PCT_ERR_CAPACITY,  # noqa: F401
                  PCT_ERR_DEVICE, PCT_ERR_WORKSPACE, PCT_FIXED_POINT, PCT_MAX_SLICES, PCT_OK, PCT_STRIP_WAVES,
                  _ROBOT_FIELDS,
                  pct_extent, pct_grid,
                  pct_item, pct_robot)
from . import abi as _abi


class PctError(RuntimeError):
    def __init__(self, fn, status, msg):
        super().__init__(f"{fn} failed (status {status}): {msg}")
        self.status = status


_lib = None


def lib():
    """Load libpct.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libpct.so not found at {LIB_PATH}; build it with "
                          "`python -m paper_2403_07631_amd.build`")
    _lib = _abi.load(LIB_PATH)
    return _lib


def declared_symbols():
    """Names of the entry points the binding declares (for export checks)."""
    lib()
    return sorted(n for n in dir(_lib) if n.startswith("pct_"))


def _check(fn, status):
    if status != PCT_OK:
        raise PctError(fn, status, lib().pct_last_error().decode())


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def grid_struct(grid) -> pct_grid:
    if isinstance(grid, pct_grid):
        return grid
    return pct_grid(float(grid["x0"]), float(grid["y0"]), float(grid["res"]), int(grid["nx"]),
                    int(grid["ny"]), float(grid["slice_dz"]))


def robot_struct(r) -> pct_robot:
    if isinstance(r, pct_robot):
        return r
    return pct_robot(*[float(r[n]) for n in _ROBOT_FIELDS], int(r.get("patch_radius", 1)))


def _workspace(nbytes, device):
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


# --------------------------------------------------------------------- host

def pct_abi_version() -> int:
    return int(lib().pct_abi_version())


def pct_robot_from_physical(min_interval, nominal_height, max_slope_deg, max_step,
                            inflation_radius, safe_margin, res) -> pct_robot:
    out = pct_robot()
    _check("pct_robot_from_physical",
           lib().pct_robot_from_physical(min_interval, nominal_height, max_slope_deg, max_step,
                                         inflation_radius, safe_margin, res, C.byref(out)))
    return out


def robot_from_physical(phys: dict, res: float) -> pct_robot:
    return pct_robot_from_physical(phys["min_interval"], phys["nominal_height"], phys["max_slope_deg"],
                                   phys["max_step"], phys["inflation_radius"], phys["safe_margin"], res)


def pct_validate_grid(grid) -> None:
    g = grid_struct(grid)
    _check("pct_validate_grid", lib().pct_validate_grid(C.byref(g)))


def pct_validate_robot(robot, res) -> None:
    r = robot_struct(robot)
    _check("pct_validate_robot", lib().pct_validate_robot(C.byref(r), res))


def pct_kernel_radius(robot, res) -> int:
    r = robot_struct(robot)
    out = C.c_int32()
    _check("pct_kernel_radius", lib().pct_kernel_radius(C.byref(r), res, C.byref(out)))
    return int(out.value)


def pct_plane_heights(extent: pct_extent, slice_dz: float):
    import numpy as np
    h = np.zeros(max(1, extent.n_slices), np.float32)
    _check("pct_plane_heights", lib().pct_plane_heights(C.byref(extent), slice_dz,
                                                        h.ctypes.data_as(C.c_void_p), len(h)))
    return h[:extent.n_slices]


# --------------------------------------------------------------------- device

def _points(xyz):
    if not (xyz.is_cuda and xyz.dtype == torch.float32 and xyz.dim() == 2 and xyz.shape[1] == 3):
        raise ValueError("points must be a CUDA float32 tensor of shape [n, 3]")
    return xyz.contiguous()


def pct_tomogram_extent(xyz, grid) -> pct_extent:
    xyz = _points(xyz)
    g = grid_struct(grid)
    n = xyz.shape[0]
    ws = _workspace(lib().pct_extent_workspace_bytes(n), xyz.device)
    out = pct_extent()
    _check("pct_tomogram_extent",
           lib().pct_tomogram_extent(_ptr(xyz), n, C.byref(g), C.byref(out), _ptr(ws), ws.numel(),
                                     _stream(xyz.device)))
    return out


def pct_tomogram_extent_device(xyz, grid, out=None, workspace=None):
    """The extent record written to device memory without a host
    synchronisation: a uint8 tensor of sizeof(pct_extent) bytes (decode with
    ``extent_from_bytes``)."""
    xyz = _points(xyz)
    g = grid_struct(grid)
    n = xyz.shape[0]
    need = lib().pct_extent_workspace_bytes(n)
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, xyz.device)
    if out is None:
        out = torch.empty(C.sizeof(pct_extent), dtype=torch.uint8, device=xyz.device)
    _check("pct_tomogram_extent_device",
           lib().pct_tomogram_extent_device(_ptr(xyz) if n else None, n, C.byref(g), _ptr(out), _ptr(ws), ws.numel(),
                                            _stream(xyz.device)))
    return out


def extent_from_bytes(t) -> pct_extent:
    """Decodes the record written by pct_tomogram_extent_device."""
    return pct_extent.from_buffer_copy(bytes(t.cpu().numpy().tobytes()))


def pct_build_tomogram(xyz, grid, extent: pct_extent, with_ids: bool = False, workspace=None):
    """Returns (ground, ceil, arg_ground, arg_ceil); the ids are None unless
    ``with_ids``.  Shapes [N, ny, nx]."""
    xyz = _points(xyz)
    g = grid_struct(grid)
    n, N = xyz.shape[0], extent.n_slices
    dev = xyz.device
    ground = torch.empty((N, g.ny, g.nx), dtype=torch.float32, device=dev)
    ceil = torch.empty_like(ground)
    ag = torch.empty((N, g.ny, g.nx), dtype=torch.int32, device=dev) if with_ids else None
    ac = torch.empty_like(ag) if with_ids else None
    need = lib().pct_build_workspace_bytes(n, C.byref(g), C.byref(extent))
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, dev)
    _check("pct_build_tomogram",
           lib().pct_build_tomogram(_ptr(xyz), n, C.byref(g), C.byref(extent), _ptr(ground), _ptr(ceil),
                                    _ptr(ag), _ptr(ac), _ptr(ws), ws.numel(), _stream(dev)))
    return ground, ceil, ag, ac


def pct_eval_traversability(ground, ceil, grid, extent: pct_extent, robots, keep: bool = True,
                            workspace=None):
    """Returns (cost [R, N, ny, nx] float32, keep [R, N] uint8 or None)."""
    if isinstance(robots, (pct_robot, dict)):
        robots = [robots]
    rs = (pct_robot * len(robots))(*[robot_struct(r) for r in robots])
    g = grid_struct(grid)
    N = extent.n_slices
    dev = ground.device
    for t in (ground, ceil):
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and tuple(t.shape) == (N, g.ny, g.nx)):
            raise ValueError("ground/ceil must be contiguous CUDA float32 [N, ny, nx]")
    cost = torch.empty((len(robots), N, g.ny, g.nx), dtype=torch.float32, device=dev)
    kp = torch.empty((len(robots), N), dtype=torch.uint8, device=dev) if keep else None
    need = lib().pct_eval_workspace_bytes(C.byref(g), C.byref(extent), len(robots))
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, dev)
    _check("pct_eval_traversability",
           lib().pct_eval_traversability(_ptr(ground), _ptr(ceil), C.byref(g), C.byref(extent), rs,
                                         len(robots), _ptr(cost), _ptr(kp), _ptr(ws), ws.numel(),
                                         _stream(dev)))
    return cost, kp


def pct_eval_traversability_static(ground, ceil, grid, extent: pct_extent, robots, keep: bool = True,
                                   cost=None, keep_out=None):
    """pct_eval_traversability with the slice test's scratch in the library's
    static device array (the call allocates nothing on the device itself).
    ``cost`` [R, N, ny, nx] float32 and ``keep_out`` [R, N] uint8 may be
    given; otherwise they are allocated here, before the call.
    Returns (cost, keep or None)."""
    if isinstance(robots, (pct_robot, dict)):
        robots = [robots]
    rs = (pct_robot * len(robots))(*[robot_struct(r) for r in robots])
    g = grid_struct(grid)
    N = extent.n_slices
    dev = ground.device
    for t in (ground, ceil):
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and tuple(t.shape) == (N, g.ny, g.nx)):
            raise ValueError("ground/ceil must be contiguous CUDA float32 [N, ny, nx]")
    shape = (len(robots), N, g.ny, g.nx)
    if cost is None:
        cost = torch.empty(shape, dtype=torch.float32, device=dev)
    elif not (cost.is_cuda and cost.dtype == torch.float32 and cost.is_contiguous() and tuple(cost.shape) == shape):
        raise ValueError("cost must be contiguous CUDA float32 %s" % (shape,))
    kp = None
    if keep:
        kp = keep_out if keep_out is not None else torch.empty((len(robots), N), dtype=torch.uint8, device=dev)
        if not (kp.is_cuda and kp.dtype == torch.uint8 and kp.is_contiguous() and tuple(kp.shape) == (len(robots), N)):
            raise ValueError("keep_out must be contiguous CUDA uint8 [R, N]")
    _check("pct_eval_traversability_static",
           lib().pct_eval_traversability_static(_ptr(ground), _ptr(ceil), C.byref(g), C.byref(extent), rs,
                                                len(robots), _ptr(cost), _ptr(kp), _stream(dev)))
    return cost, kp


def pct_autotune_traversability(ground, ceil, grid, extent, robot, scratch=None):
    """Tune the evaluation's strip shape for this map shape (synchronous).
    Returns ((best_rows, best_waves), {(rows, waves): ms}); best_rows is 0
    when the robot's evaluation does not use strips.  waves = 1: one
    wavefront per strip; waves = PCT_STRIP_WAVES: a workgroup per strip."""
    g, rb = grid_struct(grid), robot_struct(robot)
    N = extent.n_slices
    cost = scratch if scratch is not None else torch.empty((max(N, 1), g.ny, g.nx), dtype=torch.float32,
                                                           device=ground.device)
    best, bw, count = C.c_int32(), C.c_int32(), C.c_int32()
    rows = (C.c_int32 * 24)()
    waves = (C.c_int32 * 24)()
    ms = (C.c_float * 24)()
    _check("pct_autotune_traversability",
           lib().pct_autotune_traversability(_ptr(ground), _ptr(ceil), C.byref(g), C.byref(extent), C.byref(rb),
                                             _ptr(cost), C.byref(best), C.byref(bw), rows, waves, ms, 24,
                                             C.byref(count), _stream(ground.device)))
    return ((int(best.value), int(bw.value)),
            {(int(rows[i]), int(waves[i])): float(ms[i]) for i in range(count.value)})


def pct_autotune_reset():
    _check("pct_autotune_reset", lib().pct_autotune_reset())


def pct_autotune_set_traversability(grid, extent, robot, rows: int, waves: int = PCT_STRIP_WAVES):
    """Record (rows > 0) or forget (rows = 0) the strip shape used for maps
    of this shape and this robot's inflation radius."""
    g, rb = grid_struct(grid), robot_struct(robot)
    _check("pct_autotune_set_traversability",
           lib().pct_autotune_set_traversability(C.byref(g), C.byref(extent), C.byref(rb), int(rows), int(waves)))


# --------------------------------------------------------------------- path search

def pct_plan_distance(cost, ground, grid, extent: pct_extent, robot, layers, start, workspace=None, dist=None,
                      band=0.0):
    """Least path costs from ``start`` = (x, y, layer index) over the slices
    ``layers`` (strictly increasing slice indices) of one robot's c^T
    [N, ny, nx] and e^G.  Returns (dist [L, ny, nx] float64, workspace,
    {"rounds", "tiles"}); pass the workspace on to ``pct_plan_path``."""
    g, rb = grid_struct(grid), robot_struct(robot)
    N = extent.n_slices
    for t in (cost, ground):
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and tuple(t.shape) == (N, g.ny, g.nx)):
            raise ValueError("cost/ground must be contiguous CUDA float32 [N, ny, nx]")
    lay = (C.c_int32 * len(layers))(*[int(v) for v in layers])
    L = len(layers)
    dev = cost.device
    if dist is None:
        dist = torch.empty((L, g.ny, g.nx), dtype=torch.float64, device=dev)
    need = lib().pct_plan_workspace_bytes(g.nx, g.ny, max(L, 1))
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, dev)
    rounds, tiles = C.c_int32(), C.c_int64()
    _check("pct_plan_distance",
           lib().pct_plan_distance(_ptr(cost), _ptr(ground), C.byref(g), C.byref(extent), C.byref(rb), lay, L,
                                   int(start[0]), int(start[1]), int(start[2]), float(band), _ptr(dist), _ptr(ws),
                                   ws.numel(),
                                   C.byref(rounds), C.byref(tiles), _stream(dev)))
    return dist, ws, {"rounds": int(rounds.value), "tiles": int(tiles.value)}


def pct_plan_query(cost, ground, grid, extent: pct_extent, robot, layers, start, goal, workspace=None, dist=None,
                   band=0.0):
    """Goal-directed search: stops once the goal's distance is final.
    Returns (dist, workspace, {"rounds", "tiles", "goal_dist", "settled"});
    labels below ``settled`` are final."""
    g, rb = grid_struct(grid), robot_struct(robot)
    N = extent.n_slices
    for t in (cost, ground):
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and tuple(t.shape) == (N, g.ny, g.nx)):
            raise ValueError("cost/ground must be contiguous CUDA float32 [N, ny, nx]")
    lay = (C.c_int32 * len(layers))(*[int(v) for v in layers])
    L = len(layers)
    dev = cost.device
    if dist is None:
        dist = torch.empty((L, g.ny, g.nx), dtype=torch.float64, device=dev)
    need = lib().pct_plan_workspace_bytes(g.nx, g.ny, max(L, 1))
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, dev)
    rounds, tiles, gd, st = C.c_int32(), C.c_int64(), C.c_double(), C.c_double()
    _check("pct_plan_query",
           lib().pct_plan_query(_ptr(cost), _ptr(ground), C.byref(g), C.byref(extent), C.byref(rb), lay, L,
                                int(start[0]), int(start[1]), int(start[2]), int(goal[0]), int(goal[1]),
                                int(goal[2]), float(band), _ptr(dist), _ptr(ws), ws.numel(), C.byref(gd), C.byref(st),
                                C.byref(rounds), C.byref(tiles), _stream(dev)))
    return dist, ws, {"rounds": int(rounds.value), "tiles": int(tiles.value), "goal_dist": float(gd.value),
                      "settled": float(st.value)}


def pct_plan_path(dist, grid, start, goal, workspace, max_len=None):
    """Least-cost path as int32 [n, 3] rows (x, y, slice index), start
    first, on the device; None if the goal is unreachable."""
    g = grid_struct(grid)
    L = dist.shape[0]
    max_len = int(max_len or min(L * g.nx * g.ny, 1 << 24))
    path = torch.empty((max_len, 3), dtype=torch.int32, device=dist.device)
    n = C.c_int32()
    _check("pct_plan_path",
           lib().pct_plan_path(_ptr(dist), C.byref(g), L, int(start[0]), int(start[1]), int(start[2]), int(goal[0]),
                               int(goal[1]), int(goal[2]), _ptr(path), max_len, C.byref(n), _ptr(workspace),
                               workspace.numel(), _stream(dist.device)))
    return None if n.value == 0 else path[:n.value]


# --------------------------------------------------------------------- incremental updates

def pct_tomogram_insert(xyz, grid, extent: pct_extent, ground, ceil, arg_ground=None, arg_ceil=None, id_base=0,
                        workspace=None):
    """Adds the points ``xyz`` [n, 3] (ids id_base ..) to the tomogram in
    place; ``extent`` is updated.  Returns the cell box (x_min, y_min,
    x_max, y_max) of the new points (x_max < x_min when none)."""
    g = grid_struct(grid)
    if not (xyz.is_cuda and xyz.dtype == torch.float32 and xyz.is_contiguous() and xyz.dim() == 2
            and xyz.shape[1] == 3):
        raise ValueError("xyz must be a contiguous CUDA float32 [n, 3] tensor")
    n = xyz.shape[0]
    need = lib().pct_insert_workspace_bytes(n, C.byref(g))
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, xyz.device)
    bb = (C.c_int32 * 4)()
    _check("pct_tomogram_insert",
           lib().pct_tomogram_insert(_ptr(xyz), n, int(id_base), C.byref(g), C.byref(extent), _ptr(ground), _ptr(ceil),
                                     _ptr(arg_ground), _ptr(arg_ceil), bb, _ptr(ws), ws.numel(),
                                     _stream(xyz.device)))
    return tuple(int(v) for v in bb)


def pct_eval_traversability_window(ground, ceil, grid, extent: pct_extent, robot, window, cost, keep=None,
                                   workspace=None):
    """Re-evaluates c^T of one robot on the cells window = (x0, y0, x1, y1)
    (half-open) of every slice into ``cost`` [N, ny, nx]; with ``keep``
    (uint8 [N]) the slice test runs again on the whole map."""
    g, rb = grid_struct(grid), robot_struct(robot)
    need = lib().pct_eval_workspace_bytes(C.byref(g), C.byref(extent), 1)
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, ground.device)
    x0, y0, x1, y1 = (int(v) for v in window)
    _check("pct_eval_traversability_window",
           lib().pct_eval_traversability_window(_ptr(ground), _ptr(ceil), C.byref(g), C.byref(extent), C.byref(rb), x0,
                                                y0, x1, y1, _ptr(cost), _ptr(keep), _ptr(ws), ws.numel(),
                                                _stream(ground.device)))


# --------------------------------------------------------------------- sparse storage

def pct_unique_cells(ground, ceil, cost, keep, grid, extent: pct_extent, robot, workspace=None):
    """The unique cells of the kept slices (Sec. III-C): returns dict of
    cell int32 [M], ground, ceil, cost float32 [M] (on the device) and
    slice_off int64 [N+1] (host numpy)."""
    import numpy as np
    g, rb = grid_struct(grid), robot_struct(robot)
    N = extent.n_slices
    dev = cost.device
    for t in (ground, ceil, cost):
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and tuple(t.shape) == (N, g.ny, g.nx)):
            raise ValueError("ground/ceil/cost must be contiguous CUDA float32 [N, ny, nx]")
    if not (keep.is_cuda and keep.dtype == torch.uint8 and keep.numel() == N):
        raise ValueError("keep must be a CUDA uint8 [N] tensor")
    need = lib().pct_unique_workspace_bytes(C.byref(g), C.byref(extent))
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, dev)
    off = np.zeros(N + 1, np.int64)
    offp = off.ctypes.data_as(C.POINTER(C.c_int64))
    m = C.c_int64()
    keep = keep.contiguous()
    _check("pct_unique_cells",
           lib().pct_unique_cells(_ptr(ground), _ptr(ceil), _ptr(cost), _ptr(keep), C.byref(g), C.byref(extent),
                                  C.byref(rb), 0, None, None, None, None, offp, C.byref(m), _ptr(ws), ws.numel(),
                                  _stream(dev)))
    M = int(m.value)
    out = dict(cell=torch.empty(M, dtype=torch.int32, device=dev), ground=torch.empty(M, dtype=torch.float32, device=dev),
               ceil=torch.empty(M, dtype=torch.float32, device=dev), cost=torch.empty(M, dtype=torch.float32, device=dev))
    if M > 0:
        _check("pct_unique_cells",
               lib().pct_unique_cells(_ptr(ground), _ptr(ceil), _ptr(cost), _ptr(keep), C.byref(g), C.byref(extent),
                                      C.byref(rb), M, _ptr(out["cell"]), _ptr(out["ground"]), _ptr(out["ceil"]),
                                      _ptr(out["cost"]), offp, C.byref(m), _ptr(ws), ws.numel(), _stream(dev)))
    out["slice_off"] = off
    return out


# --------------------------------------------------------------------- graphs

class Graph:
    """A graph captured through the library's own helpers
    (pct_graph_begin / pct_graph_end) on a torch stream."""

    def __init__(self, stream):
        self.stream = stream
        self.handle = C.c_void_p()

    def __enter__(self):
        _check("pct_graph_begin", lib().pct_graph_begin(C.c_void_p(self.stream.cuda_stream)))
        return self

    def __exit__(self, exc_type, exc, tb):
        st = lib().pct_graph_end(C.c_void_p(self.stream.cuda_stream), C.byref(self.handle))
        if exc_type is None:
            _check("pct_graph_end", st)
        return False

    def launch(self, stream=None):
        s = stream if stream is not None else torch.cuda.current_stream()
        _check("pct_graph_launch", lib().pct_graph_launch(self.handle, C.c_void_p(s.cuda_stream)))

    def __del__(self):
        if getattr(self, "handle", None) and self.handle.value:
            lib().pct_graph_destroy(self.handle)
            self.handle = C.c_void_p()


# --------------------------------------------------------------------- trajectory optimisation

_TRAJ_FIELDS = ("w_z", "w_c", "w_v", "w_a", "w_h", "w_T", "c_safe", "v_max", "a_max", "d_ref", "d_min")


def traj_params_struct(prm):
    """pct_traj_params from a dict with the weights, limits and samples."""
    if isinstance(prm, _abi.pct_traj_params):
        return prm
    return _abi.pct_traj_params(*[float(prm[n]) for n in _TRAJ_FIELDS], int(prm["samples"]))


def _traj_inputs(cost, ground, ceil, grid, extent, bound, slices, knots, tau):
    g = grid_struct(grid)
    N = extent.n_slices
    for t in (cost, ground, ceil):
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.numel() == N * g.nx * g.ny):
            raise ValueError("cost/ground/ceil must be contiguous CUDA float32 [N, ny, nx]")
    n, M = slices.shape
    if not (slices.is_cuda and slices.dtype == torch.int32 and slices.is_contiguous()):
        raise ValueError("slices must be a contiguous CUDA int32 [n, M] tensor")
    if not (bound.is_cuda and bound.dtype == torch.float64 and bound.is_contiguous() and tuple(bound.shape) == (n, 2, 3, 3)):
        raise ValueError("bound must be a contiguous CUDA float64 [n, 2, 3, 3] tensor")
    if not (tau.is_cuda and tau.dtype == torch.float64 and tau.is_contiguous() and tuple(tau.shape) == (n, M)):
        raise ValueError("tau must be a contiguous CUDA float64 [n, M] tensor")
    if not (knots.is_cuda and knots.dtype == torch.float64 and knots.is_contiguous()
            and tuple(knots.shape) == (n, M - 1, 3)):
        raise ValueError("knots must be a contiguous CUDA float64 [n, M-1, 3] tensor")
    return g, n, M


def pct_traj_eval(cost, ground, ceil, grid, extent: pct_extent, prm, bound, slices, knots, tau, coefficients=False):
    """Objective of Eq. (10) (penalty form) for n trajectories of M pieces:
    returns (phi [n], d phi / d knots [n, M-1, 3], d phi / d tau [n, M]) and,
    with ``coefficients``, the monomial coefficients [n, M, 6, 3]."""
    g, n, M = _traj_inputs(cost, ground, ceil, grid, extent, bound, slices, knots, tau)
    dev = tau.device
    f64 = dict(dtype=torch.float64, device=dev)
    phi, gk, gt = torch.empty(n, **f64), torch.empty(n, M - 1, 3, **f64), torch.empty(n, M, **f64)
    coef = torch.empty(n, M, 6, 3, **f64) if coefficients else None
    p = traj_params_struct(prm)
    _check("pct_traj_eval",
           lib().pct_traj_eval(_ptr(cost), _ptr(ground), _ptr(ceil), C.byref(g), C.byref(extent), C.byref(p), n, M,
                               _ptr(bound), _ptr(slices), _ptr(knots) if M > 1 else None, _ptr(tau), _ptr(phi),
                               _ptr(gk) if M > 1 else None, _ptr(gt), _ptr(coef), _stream(dev)))
    return (phi, gk, gt, coef) if coefficients else (phi, gk, gt)


def pct_traj_optimize(cost, ground, ceil, grid, extent: pct_extent, prm, bound, slices, knots, tau, iters, step):
    """Gradient descent with Armijo backtracking on ``knots`` / ``tau`` in
    place; returns (phi [n], iterations accepted [n])."""
    g, n, M = _traj_inputs(cost, ground, ceil, grid, extent, bound, slices, knots, tau)
    dev = tau.device
    phi = torch.empty(n, dtype=torch.float64, device=dev)
    done = torch.empty(n, dtype=torch.int32, device=dev)
    p = traj_params_struct(prm)
    _check("pct_traj_optimize",
           lib().pct_traj_optimize(_ptr(cost), _ptr(ground), _ptr(ceil), C.byref(g), C.byref(extent), C.byref(p), n,
                                   M, _ptr(bound), _ptr(slices), _ptr(knots) if M > 1 else None, _ptr(tau),
                                   int(iters), float(step), _ptr(phi), _ptr(done), _stream(dev)))
    return phi, done


# --------------------------------------------------------------------- trajectory cost

def _wp(wp, slices):
    if not (wp.is_cuda and wp.dtype == torch.float32 and wp.dim() == 3 and wp.shape[2] == 3):
        raise ValueError("waypoints must be a CUDA float32 tensor [T, W, 3]")
    if not (slices.is_cuda and slices.dtype == torch.int32 and tuple(slices.shape) == tuple(wp.shape[:2])):
        raise ValueError("slice ids must be a CUDA int32 tensor [T, W]")
    return wp.contiguous(), slices.contiguous()


def pct_sample_cost_fwd(cost, ground, grid, extent, robot, w_z, wp, slices):
    """f [T]: per-trajectory sum of c^T + w_z (z - e^G - d_ref)^2 (bilinear)."""
    wp, slices = _wp(wp, slices)
    g, rb = grid_struct(grid), robot_struct(robot)
    T, W = slices.shape
    f = torch.empty(T, dtype=torch.float32, device=wp.device)
    _check("pct_sample_cost_fwd",
           lib().pct_sample_cost_fwd(_ptr(cost), _ptr(ground), C.byref(g), C.byref(extent), C.byref(rb), float(w_z),
                                     _ptr(wp), _ptr(slices), T, W, _ptr(f), _stream(wp.device)))
    return f


def pct_fixed_to_float(acc):
    """Fixed-point gradient sums (int64, units of 2^-32) as float32."""
    if not (acc.is_cuda and acc.dtype == torch.int64 and acc.is_contiguous()):
        raise ValueError("acc must be a contiguous CUDA int64 tensor")
    out = torch.empty(acc.shape, dtype=torch.float32, device=acc.device)
    _check("pct_fixed_to_float", lib().pct_fixed_to_float(_ptr(acc), acc.numel(), _ptr(out), _stream(acc.device)))
    return out


def _sum_outputs(*ts):
    """PCT_FIXED_POINT when the given gradient sums are int64, 0 when float32."""
    kinds = {t.dtype for t in ts if t is not None}
    if kinds <= {torch.float32}:
        return 0
    if kinds == {torch.int64}:
        return PCT_FIXED_POINT
    raise ValueError("gradient sums must all be float32 or all int64 (fixed point)")


def _sum_dtype(deterministic):
    return torch.int64 if deterministic else torch.float32


def pct_sample_cost_bwd(cost, ground, grid, extent, robot, w_z, wp, slices, gf, grids=True, deterministic=True):
    """(gwp [T, W, 3], gcost, gground) - the grid gradients are [N, ny, nx]
    (None unless ``grids``), summed in fixed point unless not
    ``deterministic`` (then float atomics, order-dependent in the last bits)."""
    wp, slices = _wp(wp, slices)
    g, rb = grid_struct(grid), robot_struct(robot)
    T, W = slices.shape
    dev = wp.device
    gwp = torch.empty_like(wp)
    dt = _sum_dtype(deterministic)
    gcost = torch.empty(cost.shape, dtype=dt, device=dev) if grids else None
    gground = torch.empty(ground.shape, dtype=dt, device=dev) if grids else None
    _check("pct_sample_cost_bwd",
           lib().pct_sample_cost_bwd(_ptr(cost), _ptr(ground), C.byref(g), C.byref(extent), C.byref(rb), float(w_z),
                                     _ptr(wp), _ptr(slices), T, W, _ptr(gf.contiguous()), _ptr(gwp), _ptr(gcost),
                                     _ptr(gground), _sum_outputs(gcost, gground), _stream(dev)))
    if deterministic and grids:
        gcost, gground = pct_fixed_to_float(gcost), pct_fixed_to_float(gground)
    return gwp, gcost, gground


def pct_eval_traversability_bwd(ground, ceil, grid, extent, robot, gcost, deterministic=True):
    """(dL/de^G, dL/de^C) [N, ny, nx] for dL/dc^T = gcost (one robot),
    summed in fixed point unless not ``deterministic``."""
    g, rb = grid_struct(grid), robot_struct(robot)
    dt = _sum_dtype(deterministic)
    gG = torch.empty(ground.shape, dtype=dt, device=ground.device)
    gC = torch.empty(ceil.shape, dtype=dt, device=ground.device)
    _check("pct_eval_traversability_bwd",
           lib().pct_eval_traversability_bwd(_ptr(ground), _ptr(ceil), C.byref(g), C.byref(extent), C.byref(rb),
                                             _ptr(gcost.contiguous()), _ptr(gG), _ptr(gC), _sum_outputs(gG, gC),
                                             _stream(ground.device)))
    if deterministic:
        gG, gC = pct_fixed_to_float(gG), pct_fixed_to_float(gC)
    return gG, gC


def pct_route_grad_to_points(gground, gceil, arg_ground, arg_ceil, grid, extent, n_points):
    """dL/dz [n_points] from grid gradients and the recorded point ids (each
    point's sum is formed by the one thread of its cell, in slice order)."""
    g = grid_struct(grid)
    gz = torch.empty(n_points, dtype=torch.float32, device=gground.device)
    _check("pct_route_grad_to_points",
           lib().pct_route_grad_to_points(_ptr(gground), _ptr(gceil), _ptr(arg_ground), _ptr(arg_ceil), C.byref(g),
                                          C.byref(extent), n_points, _ptr(gz), 0, _stream(gground.device)))
    return gz


def pct_trajectory_cost_bwd(ground, ceil, cost, arg_ground, arg_ceil, grid, extent, robot, w_z, wp, slices, gf,
                            n_points, gwp=None, gz=None, flags=0, deterministic=True):
    """(gwp [T, W, 3], gz [n_points]) in one pass (no dense gradient grids).
    gwp/gz may be passed in; with ``flags=PCT_ACCUMULATE`` gz is added to.
    A gz passed in as int64 holds fixed-point sums (units of 2^-32) and is
    returned as it is, so that calls accumulate exactly; an allocated gz is
    summed in fixed point and returned as float32 unless not
    ``deterministic``."""
    wp, slices = _wp(wp, slices)
    g, rb = grid_struct(grid), robot_struct(robot)
    T, W = slices.shape
    gwp = torch.empty_like(wp) if gwp is None else gwp
    convert = gz is None and deterministic
    if gz is None:
        gz = torch.empty(n_points, dtype=_sum_dtype(deterministic), device=wp.device)
    _check("pct_trajectory_cost_bwd",
           lib().pct_trajectory_cost_bwd(_ptr(ground), _ptr(ceil), _ptr(cost), _ptr(arg_ground), _ptr(arg_ceil),
                                         C.byref(g), C.byref(extent), C.byref(rb), float(w_z), _ptr(wp),
                                         _ptr(slices), T, W, _ptr(gf.contiguous()), n_points, _ptr(gwp), _ptr(gz),
                                         int(flags) | _sum_outputs(gz), _stream(wp.device)))
    return gwp, (pct_fixed_to_float(gz) if convert else gz)


def pct_trajectory_cost_multi(ground, ceil, arg_ground, arg_ceil, grid, extent, robots, w_z, wp, slices, gf=None,
                              n_points=0, grids=False, flags=0, workspace=None, out=None, deterministic=True):
    """Several robot profiles on one map in one launch, c^T evaluated only at
    the sampled corners.  wp [P, T, W, 3], slices [P, T, W], gf [P, T] or
    None.  Returns (f [P, T], gwp [P, T, W, 3], gground, gceil, gz); the
    gradients are None without gf, the grids None unless ``grids``, gz None
    unless n_points > 0.  ``out`` passes preallocated (f, gwp, gground,
    gceil, gz) and ``workspace`` a preallocated workspace (for graphs);
    gradient sums passed in as int64 are fixed point (units of 2^-32) and
    returned as they are.  Allocated sums are formed in fixed point and
    returned as float32 unless not ``deterministic``."""
    if isinstance(robots, (pct_robot, dict)):
        robots = [robots]
    rs = (pct_robot * len(robots))(*[robot_struct(r) for r in robots])
    Pn = len(robots)
    if not (wp.is_cuda and wp.dtype == torch.float32 and wp.dim() == 4 and wp.shape[0] == Pn and wp.shape[3] == 3):
        raise ValueError("waypoints must be a CUDA float32 tensor [P, T, W, 3]")
    if not (slices.is_cuda and slices.dtype == torch.int32 and tuple(slices.shape) == tuple(wp.shape[:3])):
        raise ValueError("slice ids must be a CUDA int32 tensor [P, T, W]")
    wp, slices = wp.contiguous(), slices.contiguous()
    T, W = int(wp.shape[1]), int(wp.shape[2])
    g = grid_struct(grid)
    dev = wp.device
    if gf is not None:
        gf = gf.contiguous()
        if tuple(gf.shape) != (Pn, T):
            raise ValueError("gf must be [P, T]")
    convert = out is None and deterministic and gf is not None
    if out is None:
        dt = _sum_dtype(deterministic)
        f = torch.empty((Pn, T), dtype=torch.float32, device=dev)
        gwp = torch.empty_like(wp) if gf is not None else None
        gground = torch.empty(ground.shape, dtype=dt, device=dev) if (gf is not None and grids) else None
        gceil = torch.empty(ceil.shape, dtype=dt, device=dev) if (gf is not None and grids) else None
        gz = torch.empty(n_points, dtype=dt, device=dev) if (gf is not None and n_points > 0) else None
    else:
        f, gwp, gground, gceil, gz = out
    need = lib().pct_trajectory_multi_workspace_bytes(Pn)
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, dev)
    _check("pct_trajectory_cost_multi",
           lib().pct_trajectory_cost_multi(_ptr(ground), _ptr(ceil), _ptr(arg_ground), _ptr(arg_ceil), C.byref(g),
                                           C.byref(extent), rs, Pn, float(w_z), _ptr(wp), _ptr(slices), T, W,
                                           _ptr(gf), _ptr(f), _ptr(gwp), _ptr(gground), _ptr(gceil), int(n_points),
                                           _ptr(gz), int(flags) | _sum_outputs(gground, gceil, gz), _ptr(ws),
                                           ws.numel(), _stream(dev)))
    if convert:
        gground, gceil, gz = (None if t is None else pct_fixed_to_float(t) for t in (gground, gceil, gz))
    return f, gwp, gground, gceil, gz


# --------------------------------------------------------------------- autograd

class BuildTomogram(torch.autograd.Function):
    """points [n, 3] -> (ground, ceil) [N, ny, nx]; the backward routes the
    grid gradients to the z of the points that hold the values."""

    @staticmethod
    def forward(ctx, xyz, grid, extent):
        ground, ceil, ag, ac = pct_build_tomogram(xyz.detach(), grid, extent, with_ids=True)
        ctx.save_for_backward(ag, ac)
        ctx.grid, ctx.extent, ctx.n = grid, extent, xyz.shape[0]
        ctx.mark_non_differentiable(ag, ac)
        return ground, ceil, ag, ac

    @staticmethod
    def backward(ctx, g_ground, g_ceil, _ga, _gc):
        ag, ac = ctx.saved_tensors
        gG = g_ground.contiguous() if g_ground is not None else torch.zeros_like(ag, dtype=torch.float32)
        gC = g_ceil.contiguous() if g_ceil is not None else None
        gz = pct_route_grad_to_points(gG, gC, ag, ac if gC is not None else None, ctx.grid, ctx.extent, ctx.n)
        gxyz = torch.zeros((ctx.n, 3), dtype=torch.float32, device=gz.device)
        gxyz[:, 2] = gz
        return gxyz, None, None


class EvalTraversability(torch.autograd.Function):
    """(ground, ceil) -> c^T [N, ny, nx] for one robot."""

    @staticmethod
    def forward(ctx, ground, ceil, grid, extent, robot):
        cost, _ = pct_eval_traversability(ground.detach().contiguous(), ceil.detach().contiguous(), grid, extent,
                                          [robot], keep=False)
        ctx.save_for_backward(ground, ceil)
        ctx.grid, ctx.extent, ctx.robot = grid, extent, robot
        return cost[0]

    @staticmethod
    def backward(ctx, g_cost):
        ground, ceil = ctx.saved_tensors
        gG, gC = pct_eval_traversability_bwd(ground.detach().contiguous(), ceil.detach().contiguous(), ctx.grid,
                                             ctx.extent, ctx.robot, g_cost.contiguous())
        return gG, gC, None, None, None


class TrajectoryCost(torch.autograd.Function):
    """(cost, ground, waypoints) -> f [T]: the Eq. (11) cost and height
    terms summed along each trajectory."""

    @staticmethod
    def forward(ctx, cost, ground, wp, slices, grid, extent, robot, w_z):
        f = pct_sample_cost_fwd(cost.detach().contiguous(), ground.detach().contiguous(), grid, extent, robot, w_z,
                                wp.detach(), slices)
        ctx.save_for_backward(cost, ground, wp, slices)
        ctx.grid, ctx.extent, ctx.robot, ctx.w_z = grid, extent, robot, w_z
        return f

    @staticmethod
    def backward(ctx, gf):
        cost, ground, wp, slices = ctx.saved_tensors
        gwp, gcost, gground = pct_sample_cost_bwd(cost.detach().contiguous(), ground.detach().contiguous(), ctx.grid,
                                                  ctx.extent, ctx.robot, ctx.w_z, wp.detach(), slices, gf)
        return gcost, gground, gwp, None, None, None, None, None


# --------------------------------------------------------------------- batches

class Batch:
    """A batch of submaps sharing one point array: item table, packed sizes
    and a workspace sized for the batched calls."""

    def __init__(self, xyz, specs, n_robots=1, with_ids=False):
        self.xyz = _points(xyz)
        self.items = (pct_item * len(specs))()
        for it, sp in zip(self.items, specs):
            it.xyz_offset, it.n_points = int(sp["xyz_offset"]), int(sp["n_points"])
            it.grid = grid_struct(sp["grid"])
        self.n = len(specs)
        self.n_robots, self.with_ids = n_robots, with_ids
        self.ws = None
        self._size_workspace()
        self.total_cells = 0
        self.total_slices = 0

    def _size_workspace(self):
        nb = lib().pct_batch_workspace_bytes(self.items, self.n, self.n_robots, int(self.with_ids))
        if nb == 0:
            raise PctError("pct_batch_workspace_bytes", PCT_ERR_ARG, lib().pct_last_error().decode())
        if self.ws is None or self.ws.numel() < nb:
            self.ws = _workspace(nb, self.xyz.device)

    def item_view(self, flat, i):
        """Item i's [N, ny, nx] view of a packed grid output."""
        it = self.items[i]
        n = it.extent.n_slices * it.grid.nx * it.grid.ny
        return flat[it.out_offset:it.out_offset + n].view(it.extent.n_slices, it.grid.ny, it.grid.nx)


def pct_tomogram_extent_batched(batch: Batch):
    tc, ts = C.c_int64(), C.c_int64()
    _check("pct_tomogram_extent_batched",
           lib().pct_tomogram_extent_batched(_ptr(batch.xyz), batch.xyz.shape[0], batch.items, batch.n, C.byref(tc),
                                             C.byref(ts), _ptr(batch.ws), batch.ws.numel(),
                                             _stream(batch.xyz.device)))
    batch.total_cells, batch.total_slices = int(tc.value), int(ts.value)
    batch._size_workspace()     # the evaluation scratch depends on the slice counts
    return batch


def pct_build_tomogram_batched(batch: Batch, with_ids=False, flags=0, out=None):
    """Packed (ground, ceil, arg_ground, arg_ceil) of every item."""
    dev = batch.xyz.device
    if out is None:
        ground = torch.empty(max(1, batch.total_cells), dtype=torch.float32, device=dev)
        ceil = torch.empty_like(ground)
        ag = torch.empty(max(1, batch.total_cells), dtype=torch.int32, device=dev) if with_ids else None
        ac = torch.empty_like(ag) if with_ids else None
    else:
        ground, ceil, ag, ac = out
    _check("pct_build_tomogram_batched",
           lib().pct_build_tomogram_batched(_ptr(batch.xyz), batch.xyz.shape[0], batch.items, batch.n, _ptr(ground),
                                            _ptr(ceil), _ptr(ag), _ptr(ac), flags, _ptr(batch.ws),
                                            batch.ws.numel(), _stream(dev)))
    return ground, ceil, ag, ac


def pct_eval_traversability_batched(batch: Batch, ground, ceil, robots, keep=True, flags=0, out=None):
    """Packed (cost [R, total_cells], keep [R, total_slices]) of every
    (item, robot) pair."""
    if isinstance(robots, (pct_robot, dict)):
        robots = [robots]
    rs = (pct_robot * len(robots))(*[robot_struct(r) for r in robots])
    dev = ground.device
    if out is None:
        cost = torch.empty((len(robots), max(1, batch.total_cells)), dtype=torch.float32, device=dev)
        kp = torch.empty((len(robots), max(1, batch.total_slices)), dtype=torch.uint8, device=dev) if keep else None
    else:
        cost, kp = out
    _check("pct_eval_traversability_batched",
           lib().pct_eval_traversability_batched(_ptr(ground), _ptr(ceil), batch.items, batch.n, rs, len(robots),
                                                 _ptr(cost), _ptr(kp), flags, _ptr(batch.ws), batch.ws.numel(),
                                                 _stream(dev)))
    return cost, kp


def pct_autotune_batched(batch: Batch, robot, n_max=1024):
    """Times construction tile heights and evaluation strip shapes per size
    class of the batch's items (after pct_tomogram_extent_batched) and
    records the fastest for later batched calls; returns the timings as
    dicts (stage "build" or "eval", class_x, class_y, radius, rows, waves,
    n_items, chosen, ms).  The batch's next calls must upload their
    descriptor tables again (no PCT_DESCRIPTORS_RESIDENT)."""
    rb = robot_struct(robot)
    ent = (_abi.pct_tune_entry * n_max)()
    cnt = C.c_int32()
    _check("pct_autotune_batched",
           lib().pct_autotune_batched(_ptr(batch.xyz), batch.xyz.shape[0], batch.items, batch.n, C.byref(rb), ent,
                                      n_max, C.byref(cnt), _stream(batch.xyz.device)))
    out = []
    for e in ent[:min(cnt.value, n_max)]:
        out.append(dict(stage="build" if e.stage == 0 else "eval", class_x=e.class_x, class_y=e.class_y,
                        radius=e.radius, rows=e.rows, waves=e.waves, n_items=e.n_items, chosen=bool(e.chosen),
                        ms=float(e.ms)))
    return out


def pct_autotune_save(path):
    """Writes every recorded tuning shape to a text file (for this device's
    architecture)."""
    _check("pct_autotune_save", lib().pct_autotune_save(os.fsencode(path)))


def pct_autotune_load(path):
    """Adds the shapes a file records for this device's architecture;
    returns how many were added."""
    n = C.c_int32()
    _check("pct_autotune_load", lib().pct_autotune_load(os.fsencode(path), C.byref(n)))
    return int(n.value)
