"""The C ABI of libpct (include/pct.h) described with ctypes: status codes,
flags, the parameter structs and the argument types of every entry point.
Free of torch, so that host-only tools can load the library with it."""
from __future__ import annotations

import ctypes as C

PCT_OK, PCT_ERR_ARG, PCT_ERR_WORKSPACE, PCT_ERR_CAPACITY, PCT_ERR_DEVICE = 0, -1, -2, -3, -4
PCT_MAX_SLICES = 1024
PCT_MAX_PIECES = 64
PCT_MAX_TRAJ_SAMPLES = 64
PCT_ACCUMULATE = 1
PCT_DESCRIPTORS_RESIDENT = 2
PCT_FIXED_POINT = 4
PCT_FIXED_FRAC_BITS = 32
PCT_STRIP_WAVES = 4


class pct_grid(C.Structure):
    _fields_ = [("x0", C.c_float), ("y0", C.c_float), ("res", C.c_float),
                ("nx", C.c_int32), ("ny", C.c_int32), ("slice_dz", C.c_float)]


class pct_extent(C.Structure):
    _fields_ = [("z_min", C.c_float), ("z_max", C.c_float), ("n_slices", C.c_int32),
                ("reserved", C.c_int32), ("n_used", C.c_int64), ("n_dropped", C.c_int64)]


_ROBOT_FIELDS = ("d_min", "d_ref", "theta_b", "theta_s", "theta_p", "c_barrier", "alpha_d",
                 "alpha_b", "alpha_s", "d_inf", "d_sm")


class pct_item(C.Structure):
    _fields_ = [("xyz_offset", C.c_int64), ("n_points", C.c_int64), ("grid", pct_grid), ("reserved", C.c_int32),
                ("extent", pct_extent), ("out_offset", C.c_int64), ("keep_offset", C.c_int64)]


class pct_tune_entry(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("stage", "class_x", "class_y", "radius", "rows", "waves", "n_items",
                                         "chosen")] + [("ms", C.c_float)]


class pct_robot(C.Structure):
    _fields_ = [(n, C.c_float) for n in _ROBOT_FIELDS] + [("patch_radius", C.c_int32)]

    def as_dict(self):
        d = {n: float(getattr(self, n)) for n in _ROBOT_FIELDS}
        d["patch_radius"] = int(self.patch_radius)
        return d


class pct_traj_params(C.Structure):
    _fields_ = [(n, C.c_float) for n in ("w_z", "w_c", "w_v", "w_a", "w_h", "w_T", "c_safe", "v_max", "a_max",
                                          "d_ref", "d_min")] + [("samples", C.c_int32)]


def load(path):
    """Open the shared library at `path` and set the argument and result
    types of every entry point."""
    L = C.CDLL(path)
    vp, sz, i64, i32, f32 = C.c_void_p, C.c_size_t, C.c_int64, C.c_int32, C.c_float
    G, E, Rb = C.POINTER(pct_grid), C.POINTER(pct_extent), C.POINTER(pct_robot)
    It = C.POINTER(pct_item)
    Tp = C.POINTER(pct_traj_params)
    sig = {
        "pct_abi_version": ([], i32),
        "pct_last_error": ([], C.c_char_p),
        "pct_robot_from_physical": ([f32, f32, f32, f32, f32, f32, f32, Rb], i32),
        "pct_validate_grid": ([G], i32),
        "pct_validate_robot": ([Rb, f32], i32),
        "pct_kernel_radius": ([Rb, f32, C.POINTER(i32)], i32),
        "pct_plane_heights": ([E, f32, vp, i32], i32),
        "pct_extent_workspace_bytes": ([i64], sz),
        "pct_tomogram_extent": ([vp, i64, G, E, vp, sz, vp], i32),
        "pct_tomogram_extent_device": ([vp, i64, G, vp, vp, sz, vp], i32),
        "pct_build_workspace_bytes": ([i64, G, E], sz),
        "pct_build_tomogram": ([vp, i64, G, E, vp, vp, vp, vp, vp, sz, vp], i32),
        "pct_eval_workspace_bytes": ([G, E, i32], sz),
        "pct_eval_traversability": ([vp, vp, G, E, Rb, i32, vp, vp, vp, sz, vp], i32),
        "pct_eval_traversability_static": ([vp, vp, G, E, Rb, i32, vp, vp, vp], i32),
        "pct_autotune_traversability": ([vp, vp, G, E, Rb, vp, C.POINTER(i32), C.POINTER(i32), vp, vp, vp, i32,
                                         C.POINTER(i32), vp], i32),
        "pct_autotune_reset": ([], i32),
        "pct_autotune_set_traversability": ([G, E, Rb, i32, i32], i32),
        "pct_sample_cost_fwd": ([vp, vp, G, E, Rb, f32, vp, vp, i32, i32, vp, vp], i32),
        "pct_sample_cost_bwd": ([vp, vp, G, E, Rb, f32, vp, vp, i32, i32, vp, vp, vp, vp, i32, vp], i32),
        "pct_eval_traversability_bwd": ([vp, vp, G, E, Rb, vp, vp, vp, i32, vp], i32),
        "pct_route_grad_to_points": ([vp, vp, vp, vp, G, E, i64, vp, i32, vp], i32),
        "pct_trajectory_cost_bwd": ([vp, vp, vp, vp, vp, G, E, Rb, f32, vp, vp, i32, i32, vp, i64, vp, vp, i32,
                                     vp], i32),
        "pct_fixed_to_float": ([vp, i64, vp, vp], i32),
        "pct_autotune_batched": ([vp, i64, It, i32, Rb, C.POINTER(pct_tune_entry), i32, C.POINTER(i32), vp], i32),
        "pct_autotune_save": ([C.c_char_p], i32),
        "pct_autotune_load": ([C.c_char_p, C.POINTER(i32)], i32),
        "pct_trajectory_multi_workspace_bytes": ([i32], sz),
        "pct_trajectory_cost_multi": ([vp, vp, vp, vp, G, E, Rb, i32, f32, vp, vp, i32, i32, vp, vp, vp, vp, vp, i64, vp,
                                       i32, vp, sz, vp], i32),
        "pct_batch_workspace_bytes": ([It, i32, i32, i32], sz),
        "pct_tomogram_extent_batched": ([vp, i64, It, i32, C.POINTER(i64), C.POINTER(i64), vp, sz, vp], i32),
        "pct_build_tomogram_batched": ([vp, i64, It, i32, vp, vp, vp, vp, i32, vp, sz, vp], i32),
        "pct_eval_traversability_batched": ([vp, vp, It, i32, Rb, i32, vp, vp, i32, vp, sz, vp], i32),
        "pct_plan_workspace_bytes": ([i32, i32, i32], sz),
        "pct_plan_distance": ([vp, vp, G, E, Rb, vp, i32, i32, i32, i32, C.c_double, vp, vp, sz, C.POINTER(i32),
                               C.POINTER(i64), vp], i32),
        "pct_plan_query": ([vp, vp, G, E, Rb, vp, i32, i32, i32, i32, i32, i32, i32, C.c_double, vp, vp, sz,
                            C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(i32), C.POINTER(i64), vp], i32),
        "pct_plan_path": ([vp, G, i32, i32, i32, i32, i32, i32, i32, vp, i32, C.POINTER(i32), vp, sz, vp], i32),
        "pct_unique_workspace_bytes": ([G, E], sz),
        "pct_insert_workspace_bytes": ([i64, G], sz),
        "pct_tomogram_insert": ([vp, i64, i32, G, E, vp, vp, vp, vp, vp, vp, sz, vp], i32),
        "pct_eval_traversability_window": ([vp, vp, G, E, Rb, i32, i32, i32, i32, vp, vp, vp, sz, vp], i32),
        "pct_unique_cells": ([vp, vp, vp, vp, G, E, Rb, i64, vp, vp, vp, vp, vp, C.POINTER(i64), vp, sz, vp], i32),
        "pct_graph_begin": ([vp], i32),
        "pct_graph_end": ([vp, C.POINTER(vp)], i32),
        "pct_graph_launch": ([vp, vp], i32),
        "pct_graph_destroy": ([vp], i32),
        "pct_traj_eval": ([vp, vp, vp, G, E, Tp, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp], i32),
        "pct_traj_optimize": ([vp, vp, vp, G, E, Tp, i32, i32, vp, vp, vp, vp, i32, C.c_double, vp, vp, vp], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    return L
