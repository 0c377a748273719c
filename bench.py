"""Benchmark of the tomography hot path on one MI355X.

One step = the whole path over the 20 M-point six-storey map (2000 x 2000
cells at 0.1 m, slice interval 0.3 m): extent and slice count, tomogram
construction, traversability with inflation, and the slice test.  Inputs
are resident in HBM before timing starts.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 vector issue rate without packed math: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def eval_ops_per_cell(R):
    """Algorithmic FP32/integer operations per cell-slice of the evaluation:
    Eqs. (1)-(5) with the patch count and validity tests (40), and Eq. (6)
    in the folded row decomposition of radius R: R column maxima, (R+1)^2
    products and maxima, 3R row-pass maxima."""
    return 40 + 4 * R + 2 * (R + 1) ** 2
METRIC = "points/s tomogram + cells/s traversability (HBM GB/s %peak); batched fwd+bwd vs plain"

# Table III of the paper: its own method's map construction (T_p) and
# traversability estimation (T_e) times in ms on its scenes (which are not
# available here), on a desktop with an i9-12900KF and an RTX 3080 Ti ("PC"),
# a Jetson AGX Orin, and the same desktop's CPU alone.  Context, not targets.
PAPER_TABLE3 = {
    "source": "Table III of the paper (its own scenes, not available here); times in ms",
    "hardware": {"PC": "Intel i9-12900KF + NVIDIA RTX 3080 Ti", "Orin": "NVIDIA Jetson AGX Orin",
                 "CPU": "the PC's CPU alone"},
    "scenes": [
        {"scene": "factory 84x68x12 m, 0.2 m", "T_p": {"PC": 2.39, "Orin": 20.06, "CPU": 630.76},
         "T_e": {"PC": 2.41, "Orin": 12.53, "CPU": 785.68}},
        {"scene": "building 22x20x16 m, 0.1 m", "T_p": {"PC": 3.10, "Orin": 23.05, "CPU": 290.98},
         "T_e": {"PC": 3.42, "Orin": 17.69, "CPU": 234.95}},
        {"scene": "forest 40x40x7 m, 0.1 m", "T_p": {"PC": 1.42, "Orin": 12.50, "CPU": 293.43},
         "T_e": {"PC": 3.02, "Orin": 19.88, "CPU": 460.51}},
        {"scene": "overpass 155x95x30 m, 0.2 m", "T_p": {"PC": 18.11, "Orin": 123.55, "CPU": 1490.0},
         "T_e": {"PC": 14.35, "Orin": 81.78, "CPU": 3300.0}},
        {"scene": "stairs (real scan) 14x14x7 m", "T_p": {"PC": 0.42, "Orin": 3.23, "CPU": 55.41},
         "T_e": {"PC": 0.20, "Orin": 1.36, "CPU": 58.10}},
        {"scene": "boxes (real scan) 22x22x4 m", "T_p": {"PC": 0.37, "Orin": 2.93, "CPU": 107.55},
         "T_e": {"PC": 0.95, "Orin": 5.52, "CPU": 18.70}},
    ],
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_digest():
    h = hashlib.sha256()
    for f in ("eval.hip", "pct_internal.h"):
        with open(os.path.join(ROOT, "paper_2403_07631_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel, strip_shape):
    """HBM traffic per launch from committed rocprofv3 counter runs, if they
    were taken on the current kernel sources and at the strip shape
    (rows, waves) of the timed launch."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    e = d.get(kernel)
    if not e or e.get("source_digest") != kernel_source_digest():
        return None
    m = e.get("by_strip_shape", {}).get(f"{strip_shape[0]}x{strip_shape[1]}")
    return m.get("hbm_bytes_per_launch") if m else None


def _oracle_path(sc, window_cells):
    """The oracle's whole path (extent, construction, traversability, slice
    test) on the centred window of window_cells^2 cells; (points, seconds,
    slices)."""
    import numpy as np

    import oracle
    g = sc.grid
    cx = g["nx"] // 2 - window_cells // 2
    x0 = g["x0"] + cx * g["res"]
    x1 = x0 + window_cells * g["res"]
    p = sc.points
    sel = (p[:, 0] >= x0) & (p[:, 0] < x1) & (p[:, 1] >= x0) & (p[:, 1] < x1)
    sub = np.ascontiguousarray(p[sel])
    sg = dict(g, x0=float(x0), y0=float(x0), nx=window_cells, ny=window_cells)
    rb = oracle.robot_from_physical(sc.robot, g["res"])
    t = time.perf_counter()
    tm = oracle.tomogram(sub, sg, ids=False)
    cT = oracle.evaluate(tm["ground"], tm["ceil"], g["res"], rb)
    oracle.simplify(tm["ground"], cT, rb["c_barrier"])
    return len(sub), time.perf_counter() - t, len(tm["h"])


def cpu_baseline(sc, window_cells=2000, single_window=500):
    """The oracle, as it stands, on the same map: on all host cores over a
    centred window of window_cells^2 cells (the whole map by default), and
    on one core over a window of single_window^2 cells; end to end (extent,
    construction, traversability, slice test)."""
    import oracle
    cores = oracle.threads()
    n, dt, N = _oracle_path(sc, window_cells)
    oracle.set_threads(1)
    try:
        n1, dt1, N1 = _oracle_path(sc, single_window)
    finally:
        oracle.set_threads(cores)
    return dict(value=n / dt, unit="points/s", cores=cores, kind="oracle",
                sample=f"{n} points of a {window_cells}x{window_cells}-cell window at the map centre, {N} slices, "
                       f"full path (extent, construction, traversability, slice test) in {dt:.2f} s",
                single_core=dict(value=n1 / dt1, unit="points/s", cores=1, kind="oracle",
                                 sample=f"{n1} points of a {single_window}x{single_window}-cell window at the map "
                                        f"centre, {N1} slices, full path in {dt1:.2f} s"))


def bench_profiles(P, torch, sc, xyz, dev, steps, warmup, n_profiles=64, n_walks=1024, traversable=False,
                   map_name="the 20M-point map"):
    """Batched fwd+bwd against the plain path: n_profiles robot profiles on
    the map, each followed by the trajectory-cost forward and backward of
    the first n_walks of the 4096 x 256 random walks (values, waypoint
    gradients, point-height gradients).  The walks step over the cells that
    are traversable for the map's robot (traversable=True) or over the cells
    with ground.  Plain: per profile the cost map, the sampling forward and
    the fused backward (the same kernels, one profile at a time).  Batched:
    one launch for all profiles with c^T evaluated at the sampled corners
    only, replayed from a graph."""
    import numpy as np

    import scenes
    g = sc.grid
    ext = P.pct_tomogram_extent(xyz, g)
    G, Cc, aG, aC = P.pct_build_tomogram(xyz, g, ext, with_ids=True)
    n = xyz.shape[0]
    Gh = G.cpu().numpy()
    rb0 = P.robot_from_physical(sc.robot, g["res"])
    if traversable:
        c0, _ = P.pct_eval_traversability(G, Cc, g, ext, [rb0], keep=False)
        mask = c0[0].cpu().numpy() < rb0.c_barrier
        del c0
    else:
        mask = np.isfinite(Gh)
    log("random walks for the profile batch")
    wp0, sl0 = scenes.random_walks(2, mask, Gh, g, 4096, 256, rb0.as_dict()["d_ref"])
    n_mask = int(mask.sum())
    del Gh, mask
    wp0, sl0 = wp0[:n_walks], sl0[:n_walks]
    rbs = [P.robot_from_physical(p, g["res"]) for p in scenes.robot_profiles(4, n_profiles)]
    wp = torch.from_numpy(np.ascontiguousarray(np.broadcast_to(wp0, (n_profiles,) + wp0.shape))).to(dev)
    sl = torch.from_numpy(np.ascontiguousarray(np.broadcast_to(sl0, (n_profiles,) + sl0.shape))).to(dev)
    gf = torch.ones((n_profiles, n_walks), device=dev)
    f1 = torch.empty((n_profiles, n_walks), device=dev)
    gwp1 = torch.empty_like(wp)
    # point gradients are summed in fixed point (int64, 2^-32 units) and
    # converted to float32 once: both paths give the same bits
    gz1_acc = torch.empty(n, dtype=torch.int64, device=dev)
    gz1 = torch.empty(n, device=dev)

    def to_float(acc, dst):
        st = P.lib().pct_fixed_to_float(acc.data_ptr(), n, dst.data_ptr(), P._stream(dev))
        if st != P.PCT_OK:
            raise RuntimeError(P.lib().pct_last_error().decode())

    def plain():
        for i, rb in enumerate(rbs):
            cost, _ = P.pct_eval_traversability(G, Cc, g, ext, [rb], keep=False)
            cost = cost[0]
            f1[i] = P.pct_sample_cost_fwd(cost, G, g, ext, rb, 1.0, wp[i], sl[i])
            P.pct_trajectory_cost_bwd(G, Cc, cost, aG, aC, g, ext, rb, 1.0, wp[i], sl[i], gf[i], n, gwp=gwp1[i],
                                      gz=gz1_acc, flags=P.PCT_ACCUMULATE if i else 0)
        to_float(gz1_acc, gz1)

    f2 = torch.empty((n_profiles, n_walks), device=dev)
    gwp2 = torch.empty_like(wp)
    gz2_acc = torch.empty(n, dtype=torch.int64, device=dev)
    gz2 = torch.empty(n, device=dev)
    ws = torch.empty(P.lib().pct_trajectory_multi_workspace_bytes(n_profiles), dtype=torch.uint8, device=dev)
    out = (f2, gwp2, None, None, gz2_acc)

    def batched(flags=0):
        P.pct_trajectory_cost_multi(G, Cc, aG, aC, g, ext, rbs, 1.0, wp, sl, gf, n_points=n, flags=flags,
                                    workspace=ws, out=out)
        to_float(gz2_acc, gz2)

    s = torch.cuda.current_stream(dev)

    def timed(fn, reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record(s)
        for _ in range(reps):
            fn()
        b.record(s)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    log("profile batch: plain path")
    for _ in range(max(1, warmup)):
        plain()
    ms_plain = timed(plain, steps)
    log("profile batch: batched path, graph-captured")
    batched()                                   # uploads the profile table
    torch.cuda.synchronize()
    cs = torch.cuda.Stream(device=dev)
    cs.wait_stream(torch.cuda.current_stream(dev))
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(cs):
        batched(P.PCT_DESCRIPTORS_RESIDENT)
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=cs):
            batched(P.PCT_DESCRIPTORS_RESIDENT)
    torch.cuda.synchronize()
    for _ in range(max(1, warmup)):
        graph.replay()
    ms_batched = timed(graph.replay, steps)
    torch.cuda.synchronize()
    same_f = bool(torch.equal(f1.view(torch.int32), f2.view(torch.int32)))
    same_gwp = bool(torch.equal(gwp1.view(torch.int32), gwp2.view(torch.int32)))
    dz = float((gz1 - gz2).abs().max().item())
    zs = float(gz1.abs().max().item())
    wps = n_profiles * n_walks * wp.shape[2]
    return {"workload": f"{n_profiles} robot profiles (min interval 0.4-0.8 m, slope 20-40 deg, step 0.1-0.3 m) "
                        f"on {map_name}, each with {n_walks} walks x {int(wp.shape[2])} waypoints, "
                        "trajectory-cost forward + backward (waypoint and point-height gradients)",
            "walk_cells": ("cells traversable for the map's robot" if traversable else
                           "cells with ground (the map has almost no traversable cell)") + f", {n_mask} cell-slices",
            "plain": "per profile: cost map, sampling forward, fused backward",
            "batched": "one launch for all profiles, c^T evaluated at the sampled bilinear corners only, "
                       "graph replay",
            "plain_ms": ms_plain, "batched_ms": ms_batched, "ratio": ms_plain / ms_batched,
            "waypoints_per_s": wps / (ms_batched * 1e-3),
            "identical_f": same_f, "identical_gwp": same_gwp, "gz_max_abs_diff": dz, "gz_max_abs": zs}


def bench_submaps(P, torch, dev, steps, warmup, n_items=512):
    """Batched construction + evaluation of n_items submaps of uneven size
    (50-400 cells a side, 10k-1M points, 2-8 storeys) against the plain
    path.  Plain: per submap the extent (with its host read-back), the
    construction and the evaluation with the slice test.  Batched: one
    extent pass for all submaps (one read-back), then the construction and
    the evaluation of all submaps as one graph replay."""
    import numpy as np

    import scenes
    log(f"generating {n_items} submaps")
    items = scenes.submap_batch(3, n_items)
    pts, specs, off = [], [], 0
    for sc in items:
        specs.append(dict(xyz_offset=off, n_points=len(sc.points), grid=sc.grid))
        pts.append(sc.points)
        off += len(sc.points)
    xyz = torch.from_numpy(np.ascontiguousarray(np.concatenate(pts))).to(dev)
    del pts
    rb = P.robot_from_physical(scenes.ROBOT_CONFIG0, 0.1)
    subs = [xyz[sp["xyz_offset"]:sp["xyz_offset"] + sp["n_points"]] for sp in specs]

    def plain():
        outs = []
        for sub, sp in zip(subs, specs):
            ext = P.pct_tomogram_extent(sub, sp["grid"])
            if ext.n_slices == 0:
                continue
            g, c, _, _ = P.pct_build_tomogram(sub, sp["grid"], ext)
            outs.append(P.pct_eval_traversability(g, c, sp["grid"], ext, [rb]))
        return outs

    b = P.Batch(xyz, specs)
    P.pct_tomogram_extent_batched(b)
    G = torch.empty(max(1, b.total_cells), device=dev)
    Cc = torch.empty_like(G)
    cost = torch.empty((1, max(1, b.total_cells)), device=dev)
    keep = torch.empty((1, max(1, b.total_slices)), dtype=torch.uint8, device=dev)

    def build_eval(flags=0):
        P.pct_build_tomogram_batched(b, flags=flags, out=(G, Cc, None, None))
        P.pct_eval_traversability_batched(b, G, Cc, [rb], flags=flags, out=(cost, keep))

    s = torch.cuda.current_stream(dev)

    def timed(fn, reps):
        a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record(s)
        for _ in range(reps):
            fn()
        e.record(s)
        torch.cuda.synchronize()
        return a.elapsed_time(e) / reps

    log("submaps: plain path")
    for _ in range(max(1, warmup)):
        plain()
    ms_plain = timed(plain, steps)
    def capture():
        build_eval()                     # uploads the descriptor tables
        torch.cuda.synchronize()
        cs = torch.cuda.Stream(device=dev)
        cs.wait_stream(torch.cuda.current_stream(dev))
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.stream(cs):
            build_eval(P.PCT_DESCRIPTORS_RESIDENT)
            torch.cuda.synchronize()
            with torch.cuda.graph(graph, stream=cs):
                build_eval(P.PCT_DESCRIPTORS_RESIDENT)
        torch.cuda.synchronize()

        def batched():
            P.pct_tomogram_extent_batched(b)
            graph.replay()

        for _ in range(max(1, warmup)):
            batched()
        return graph, timed(batched, steps), timed(graph.replay, steps)

    log("submaps: batched path, default tile shapes")
    P.pct_autotune_reset()
    _, ms_default, ms_graph_default = capture()
    log("submaps: tuning tile shapes per size class")
    t0 = time.perf_counter()
    ent = P.pct_autotune_batched(b, rb)
    tune_s = time.perf_counter() - t0
    classes = {}
    for e in ent:
        key = f"2^{e['class_x']} x 2^{e['class_y']}"
        c = classes.setdefault(key, {"items": e["n_items"], "build_ms": {}, "eval_ms": {}})
        if e["stage"] == "build":
            c["build_ms"][f"th{e['rows']}"] = round(e["ms"], 4)
            if e["chosen"]:
                c["build_chosen"] = f"th{e['rows']}"
        else:
            name = "default" if e["rows"] == 0 else f"{e['rows']}x{e['waves']}"
            c["eval_ms"][name] = round(e["ms"], 4)
            if e["chosen"]:
                c["eval_chosen"] = name
    log("submaps: batched path, tuned tile shapes")
    graph, ms_batched, ms_graph = capture()
    # outputs: the plain results of every item equal the batched ones
    outs = plain()
    torch.cuda.synchronize()
    same = True
    j = 0
    for i, sp in enumerate(specs):
        it = b.items[i]
        if it.extent.n_slices == 0:
            continue
        cp, kp = outs[j]
        j += 1
        same &= bool(torch.equal(b.item_view(cost[0], i).view(torch.int32), cp[0].view(torch.int32)))
        same &= bool(torch.equal(keep[0, it.keep_offset:it.keep_offset + it.extent.n_slices], kp[0]))
    return {"workload": f"{n_items} submaps of 50-400 cells a side at 0.1 m (log-uniform), 10k-1M points, "
                        "2-8 storeys, slice interval 0.3 m, one robot: extent, construction, evaluation with the "
                        "slice test",
            "points": int(off), "cell_slices": int(b.total_cells),
            "plain": "per submap: extent with read-back, construction, evaluation",
            "batched": "one extent pass with one read-back, then construction + evaluation of all submaps "
                       "as one graph replay",
            "plain_ms": ms_plain, "batched_ms": ms_batched, "ratio": ms_plain / ms_batched,
            "graph_replay_ms": ms_graph, "identical": same,
            "batched_default_shapes_ms": ms_default, "graph_replay_default_shapes_ms": ms_graph_default,
            "tuning": {"what": "per size class (ceil(log2 nx), ceil(log2 ny)): construction tile height 2/4/8 and "
                               "evaluation strip rows x wavefronts, each timed on a batch of that class's items; "
                               "batched_ms uses the chosen shapes", "seconds": tune_s, "classes": classes}}


def bench_plan(P, torch, dev, steps, warmup, cpu=True):
    """Path search through the slices (Sec. III-D) on the six-storey
    building without beams (100 m x 100 m, 1000 x 1000 cells, 26.4 M
    points, Table I quadruped): the library's pipeline builds the tomogram, evaluates it and
    keeps slices; the search runs from the ground-floor cell nearest the
    centre over every kept slice, and a path is read back to the farthest
    reached node.  The oracle's Dijkstra is timed on the oracle's own
    pipeline output for the same map."""
    import numpy as np

    import scenes
    log("path search: generating the building")
    sc = scenes.plan_building()
    g = sc.grid
    xyz = torch.from_numpy(sc.points).to(dev)
    ext = P.pct_tomogram_extent(xyz, g)
    G, Cc, _, _ = P.pct_build_tomogram(xyz, g, ext)
    r = dict(scenes.ROBOT_TABLE1)
    cost, keep = P.pct_eval_traversability(G, Cc, g, ext, [r])
    cost = cost[0].contiguous()
    layers = [int(v) for v in np.flatnonzero(keep[0].cpu().numpy())]

    def centre_start(cT0, eG0):
        ys, xs = np.nonzero((cT0 < r["c_barrier"]) & (eG0 < 0.5))
        k = int(np.argmin((ys - g["ny"] / 2) ** 2 + (xs - g["nx"] / 2) ** 2))
        return (int(xs[k]), int(ys[k]), 0)

    # sparse storage of the kept slices' unique cells (Sec. III-C)
    kp = keep[0].contiguous()
    uq = P.pct_unique_cells(G, Cc, cost, kp, g, ext, r)
    uts = []
    for i in range(warmup + steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        uq = P.pct_unique_cells(G, Cc, cost, kp, g, ext, r)
        torch.cuda.synchronize()
        if i >= warmup:
            uts.append((time.perf_counter() - t0) * 1e3)
    m = int(uq["cell"].numel())
    plane = g["nx"] * g["ny"]
    unique = {"cells": m, "kept_slices": len(layers), "ms": float(np.median(uts)),
              "dense_bytes": len(layers) * plane * 12, "sparse_bytes": m * 16,
              "share_of_kept_cells": m / (len(layers) * plane),
              "bytes_moved": 2 * len(layers) * plane * 24 + m * 28}
    unique["moved_gbs"] = unique["bytes_moved"] / (unique["ms"] * 1e-3) / 1e9
    del uq

    s = centre_start(cost[layers[0]].cpu().numpy(), G[layers[0]].cpu().numpy())
    dist, ws, info = P.pct_plan_distance(cost, G, g, ext, r, layers, s)
    for _ in range(warmup):
        P.pct_plan_distance(cost, G, g, ext, r, layers, s, workspace=ws, dist=dist)
    torch.cuda.synchronize()
    times = []
    for _ in range(steps):
        t0 = time.perf_counter()
        _, _, info = P.pct_plan_distance(cost, G, g, ext, r, layers, s, workspace=ws, dist=dist)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
    ms_dist = float(np.median(times))
    d = dist.cpu().numpy()
    reached = int(np.isfinite(d).sum())
    l, y, x = np.unravel_index(int(np.argmax(np.where(np.isfinite(d), d, -1.0))), d.shape)
    goal = (int(x), int(y), int(l))
    ptimes = []
    for i in range(warmup + steps):
        t0 = time.perf_counter()
        path = P.pct_plan_path(dist, g, s, goal, ws)
        torch.cuda.synchronize()
        if i >= warmup:
            ptimes.append((time.perf_counter() - t0) * 1e3)
    # a single query as the paper times them: a goal 26.5 m from the start
    # (the reached ground-floor node nearest that planar distance)
    ys, xs = np.nonzero(np.isfinite(d[0]))
    kq = int(np.argmin(np.abs(np.hypot(xs - s[0], ys - s[1]) - 265.0)))
    qgoal = (int(xs[kq]), int(ys[kq]), 0)
    qts = []
    for i in range(warmup + steps):
        t0 = time.perf_counter()
        _, _, qinfo = P.pct_plan_query(cost, G, g, ext, r, layers, s, qgoal, workspace=ws, dist=dist)
        torch.cuda.synchronize()
        if i >= warmup:
            qts.append((time.perf_counter() - t0) * 1e3)
    query = {"goal": list(qgoal), "planar_distance_m": float(np.hypot(qgoal[0] - s[0], qgoal[1] - s[1]) * g["res"]),
             "ms": float(np.median(qts)), "rounds": qinfo["rounds"], "tiles": qinfo["tiles"],
             "goal_cost": qinfo["goal_dist"], "equals_full_search": bool(qinfo["goal_dist"] == float(d[0, qgoal[1], qgoal[0]]))}
    # trajectory optimisation (Sec. III-E) on the ground floor: 4096
    # trajectories of 32 quintic pieces, 16 samples per piece
    h = P.pct_plane_heights(ext, g["slice_dz"])
    k0 = int(np.searchsorted(h, 0.3))
    tprm = dict(w_z=2.0, w_c=0.05, w_v=1.0, w_a=0.5, w_h=20.0, w_T=1.0, c_safe=5.0, v_max=1.2, a_max=2.0,
                d_ref=0.65, d_min=0.5, samples=16)
    tp = scenes.traj_problems(60, 4096, 32, (5.0, 95.0), (5.0, 95.0), 0.65, slices=(k0,))
    td = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in tp.items()}
    t_iters = 10
    kn0, ta0 = td["knots"].clone(), td["tau"].clone()
    ev_ts, op_ts = [], []
    for i in range(warmup + steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        phi0, _, _ = P.pct_traj_eval(cost, G, Cc, g, ext, tprm, td["bound"], td["slices"], td["knots"], td["tau"])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        phi_t, done_t = P.pct_traj_optimize(cost, G, Cc, g, ext, tprm, td["bound"], td["slices"], td["knots"],
                                            td["tau"], t_iters, 1e-3)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        td["knots"].copy_(kn0)
        td["tau"].copy_(ta0)
        if i >= warmup:
            ev_ts.append((t1 - t0) * 1e3)
            op_ts.append((t2 - t1) * 1e3)
    ntr = int(tp["tau"].shape[0])
    done_mean = float(done_t.float().mean())
    traj = {"workload": "4096 trajectories of 32 quintic pieces on the building's ground floor, 16 samples per "
                        "piece, gradient descent with backtracking",
            "trajectories": ntr, "pieces": 32, "samples": 16, "eval_ms": float(np.median(ev_ts)),
            "optimize_iters": t_iters, "optimize_ms": float(np.median(op_ts)), "iterations_accepted_mean": done_mean,
            "objective_mean_before": float(phi0.mean()), "objective_mean_after": float(phi_t.mean())}
    traj["evals_per_s"] = ntr / (traj["eval_ms"] * 1e-3)
    if cpu:
        from oracle import traj as otraj
        maps = (cost.cpu().numpy(), G.cpu().numpy(), Cc.cpu().numpy())
        t0 = time.perf_counter()
        n_o = 4
        for t in range(n_o):
            otraj.objective(tp["knots"][t], tp["tau"][t], tp["bound"][t, 0], tp["bound"][t, 1], tp["slices"][t],
                            maps, g, tprm)
        dt = time.perf_counter() - t0
        del maps
        traj["cpu_oracle"] = {"evals_per_s": n_o / dt, "cores": 1, "kind": "oracle",
                              "sample": f"objective and gradient of the first {n_o} trajectories"}
    del td, kn0, ta0
    # a streaming scan: 200 k new points into the map, re-evaluated around
    # them, against rebuilding and re-evaluating the union
    rng = np.random.default_rng(12)
    scan = np.ascontiguousarray(np.column_stack([rng.uniform(40.0, 46.0, 200_000), rng.uniform(55.0, 61.0, 200_000),
                                                 rng.uniform(0.0, 14.0, 200_000)]), np.float32)
    scan_t = torch.from_numpy(scan).to(dev)
    union_t = torch.cat([xyz, scan_t]).contiguous()
    grow = P.pct_kernel_radius(r, g["res"]) + 2

    def incremental():
        ext_i = P.pct_extent(ext.z_min, ext.z_max, ext.n_slices, 0, ext.n_used, ext.n_dropped)
        bb = P.pct_tomogram_insert(scan_t, g, ext_i, G, Cc2, id_base=int(xyz.shape[0]))
        P.pct_eval_traversability_window(G, Cc2, g, ext_i, r, (bb[0] - grow, bb[1] - grow, bb[2] + 1 + grow,
                                                                bb[3] + 1 + grow), cost, kp)
        return bb

    def rebuild():
        eu = P.pct_tomogram_extent(union_t, g)
        Gu, Cu, _, _ = P.pct_build_tomogram(union_t, g, eu)
        P.pct_eval_traversability(Gu, Cu, g, eu, [r])

    def wall(fn):
        ts = []
        for i in range(warmup + steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            if i >= warmup:
                ts.append((time.perf_counter() - t0) * 1e3)
        return float(np.median(ts))

    Cc2 = Cc
    bb = incremental()
    insert = {"workload": "200 k points of a scan (6 m x 6 m x 14 m box) into the building",
              "points": int(scan.shape[0]), "cell_box": list(bb), "incremental_ms": wall(incremental),
              "rebuild_ms": wall(rebuild)}
    insert["ratio"] = insert["rebuild_ms"] / insert["incremental_ms"]
    nodes = len(layers) * g["nx"] * g["ny"]
    out = {"workload": "six-storey building without beams, 100 m x 100 m at 0.1 m (1000 x 1000 cells), 26.4 M points, "
                       "slice interval 0.3 m, Table I quadruped; search from the ground-floor centre over the "
                       "kept slices, path to the farthest reached node",
           "slices": int(ext.n_slices), "layers": len(layers), "nodes": nodes, "reached": reached,
           "rounds": info["rounds"], "tiles_processed": info["tiles"], "distance_ms": ms_dist,
           "nodes_per_s": nodes / (ms_dist * 1e-3), "path_ms": float(np.median(ptimes)),
           "path_nodes": int(path.shape[0]), "goal_cost": float(d[goal[2], goal[1], goal[0]]),
           "query": query, "unique_cells": unique, "insert": insert, "traj": traj}
    if cpu:
        import oracle
        log("path search: oracle pipeline and Dijkstra")
        tm = oracle.tomogram(sc.points, g, ids=False)
        cT = oracle.evaluate(tm["ground"], tm["ceil"], g["res"], r)
        lo = np.flatnonzero(oracle.simplify(tm["ground"], cT, r["c_barrier"]))
        c32 = np.ascontiguousarray(cT[lo], np.float32)
        e32 = np.ascontiguousarray(tm["ground"][lo])
        del cT
        so = centre_start(c32[0], e32[0])
        t0 = time.perf_counter()
        do = oracle.plan(c32, e32, r["c_barrier"], so)
        ms_cpu = (time.perf_counter() - t0) * 1e3
        out["cpu_oracle"] = {"distance_ms": ms_cpu, "cores": 1, "kind": "oracle",
                             "nodes": int(do.size), "reached": int(np.isfinite(do).sum()),
                             "sample": "Dijkstra over the oracle's own kept slices of the same map, whole map"}
    return out


def bench_step(P, torch, dev, sc, rb, steps, warmup, label, strip_shape=None):
    """The timed step on one map: extent (with its host read-back), tomogram
    construction, evaluation with inflation and the slice test, inputs
    resident in HBM; the evaluation's strip shape is autotuned first, or set
    to strip_shape = (rows, waves) when given.  Returns the timings and the
    last step's outputs."""
    import ctypes
    grid = sc.grid
    xyz = torch.from_numpy(sc.points).to(dev)
    torch.cuda.synchronize()
    ext0 = P.pct_tomogram_extent(xyz, grid)
    ws_b = torch.empty(P.lib().pct_build_workspace_bytes(xyz.shape[0], ctypes.byref(P.grid_struct(grid)),
                                                          ctypes.byref(ext0)), dtype=torch.uint8, device=dev)
    ws_e = torch.empty(P.lib().pct_eval_workspace_bytes(ctypes.byref(P.grid_struct(grid)), ctypes.byref(ext0), 1),
                       dtype=torch.uint8, device=dev)
    g0, c0, _, _ = P.pct_build_tomogram(xyz, grid, ext0, workspace=ws_b)
    if strip_shape:
        log(f"{label}: strip shape set to {strip_shape[0]} rows x {strip_shape[1]} wavefront(s)")
        P.pct_autotune_set_traversability(grid, ext0, rb, strip_shape[0], strip_shape[1])
        tuned, tune_ms = tuple(strip_shape), {}
    else:
        log(f"{label}: autotuning the evaluation's strip shape")
        tuned, tune_ms = P.pct_autotune_traversability(g0, c0, grid, ext0, rb)
    del g0, c0

    def step():
        ext = P.pct_tomogram_extent(xyz, grid)
        g, c, _, _ = P.pct_build_tomogram(xyz, grid, ext, workspace=ws_b)
        cost, keep = P.pct_eval_traversability(g, c, grid, ext, [rb], workspace=ws_e)
        return ext, g, c, cost, keep

    log(f"{label}: warmup {warmup}")
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    log(f"{label}: timing {steps} steps")
    s = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    e0.record(s)
    for _ in range(steps):
        ext, g, c, cost, keep = step()
    e1.record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    ms_step = e0.elapsed_time(e1) / steps

    # per-stage times on the stream the kernels run on (events around each
    # entry point; the evaluation without the slice test is one kernel)
    def timed(fn, reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record(s)
        for _ in range(reps):
            fn()
        b.record(s)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    reps = max(3, steps)
    ms_build = timed(lambda: P.pct_build_tomogram(xyz, grid, ext, workspace=ws_b), reps)
    ms_eval_kernel = timed(lambda: P.pct_eval_traversability(g, c, grid, ext, [rb], keep=False, workspace=ws_e), reps)
    ms_eval_full = timed(lambda: P.pct_eval_traversability(g, c, grid, ext, [rb], workspace=ws_e), reps)
    n = xyz.shape[0]
    N = ext.n_slices
    cells = grid["nx"] * grid["ny"] * N
    eval_bytes = 12 * cells                 # read e^G, e^C; write c^T (4 B each per cell-slice)
    build_bytes = 12 * n + 8 * cells        # read xyz; write e^G, e^C
    trav = int((cost < rb.c_barrier).sum().item())
    res = {"points": n, "nx": grid["nx"], "ny": grid["ny"], "slices": N, "kept_slices": int(keep.sum().item()),
           "traversable_cell_slices": trav, "ms_per_step": ms_step, "wall_s_timed": wall,
           "points_per_s": n / (ms_step * 1e-3), "cell_slices_per_s": cells / (ms_step * 1e-3),
           "stages_ms": {"build": ms_build, "eval_kernel": ms_eval_kernel, "eval_with_slice_test": ms_eval_full,
                         "slice_test": max(0.0, ms_eval_full - ms_eval_kernel),
                         "extent_and_sync": max(0.0, ms_step - ms_build - ms_eval_full)},
           "hbm_frac": {"eval_kernel": eval_bytes / (ms_eval_kernel * 1e-3) / 1e9 / HBM_PEAK_GBS,
                        "eval_with_slice_test": eval_bytes / (ms_eval_full * 1e-3) / 1e9 / HBM_PEAK_GBS,
                        "build": build_bytes / (ms_build * 1e-3) / 1e9 / HBM_PEAK_GBS,
                        "step": (eval_bytes + build_bytes) / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS},
           "alg_bytes": {"eval": eval_bytes, "build": build_bytes},
           "autotune": {"strip_rows": tuned[0], "strip_waves": tuned[1], "set_not_tuned": bool(strip_shape),
                        "candidates_ms": {f"{r}x{w}": v for (r, w), v in tune_ms.items()}}}
    return res, xyz, (ext, g, c, cost, keep)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-window", type=int, default=2000)
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-vs-plain measurements")
    ap.add_argument("--no-plan", action="store_true", help="skip the building (traversable map, path search, ...)")
    ap.add_argument("--plan-only", action="store_true",
                    help="run only the building's measurements (path search, unique cells, insertion, trajectories) "
                         "and print them, for profiling; no benchmark line")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for scaling HBM byte counters)")
    ap.add_argument("--strip-shape", type=lambda v: tuple(int(x) for x in v.split(",")), default=None,
                    metavar="ROWS,WAVES",
                    help="set the 20M-point map's evaluation strip shape instead of autotuning it (for counter runs, "
                         "whose instrumentation changes which shape the tuner picks)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU sharding is a design "
              "note, not a built path", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2403_07631_amd as P
    import scenes

    dev = torch.device("cuda:0")
    if args.plan_only:
        print(json.dumps({"plan": bench_plan(P, torch, dev, args.steps, args.warmup, cpu=False)}), flush=True)
        return
    log("generating the 20M-point map")
    sc = scenes.config1_scene()
    grid = sc.grid
    rb = P.robot_from_physical(sc.robot, grid["res"])
    c1, xyz, (ext, g, c, cost, keep) = bench_step(P, torch, dev, sc, rb, args.steps, args.warmup, "20M-point map",
                                                  strip_shape=args.strip_shape)
    n, N = c1["points"], c1["slices"]
    ms_eval_kernel = c1["stages_ms"]["eval_kernel"]
    eval_bytes = c1["alg_bytes"]["eval"]
    cells = grid["nx"] * grid["ny"] * N
    eval_gbs = eval_bytes / (ms_eval_kernel * 1e-3) / 1e9
    R = P.pct_kernel_radius(rb, grid["res"])
    eval_ops = eval_ops_per_cell(R) * cells
    eval_tops = eval_ops / (ms_eval_kernel * 1e-3) / 1e12
    at = c1["autotune"]
    traffic = load_traffic("k_eval_strip", (at["strip_rows"], at["strip_waves"]))
    if args.copy_calibration:
        log("copy calibration: 3 x 1 GiB device copy")
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    out = {
        "metric": METRIC,
        "value": c1["points_per_s"],
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": c1["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "20M-point six-storey map, 2000x2000 cells at 0.1 m, slice interval 0.3 m, "
                               "one robot (min interval 0.5 m, nominal 1.0 m, slope 30 deg, step 0.2 m, "
                               "inflation 0.3 m)",
                   "points": n, "nx": grid["nx"], "ny": grid["ny"], "slices": N,
                   "kept_slices": c1["kept_slices"], "robots": 1},
        "note": "at the workload's density (about 0.75 points per cell and surface) almost no cell of this map is "
                "traversable (traversable_cell_slices); the same step on a densely sampled building with "
                "traversable floors is reported under traversable_map",
        "cell_slices_per_s": c1["cell_slices_per_s"],
        "traversable_cell_slices": c1["traversable_cell_slices"],
        "stages_ms": c1["stages_ms"],
        "hbm_frac": c1["hbm_frac"],
        "build_points_per_s": n / (c1["stages_ms"]["build"] * 1e-3),
        "roofline": {"kernel": "k_eval_strip", "bound": "hbm", "achieved": eval_gbs, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": eval_gbs / HBM_PEAK_GBS, "traffic": traffic,
                     "alg_bytes_per_launch": eval_bytes, "bytes_per_cell_slice": 12, "kernel_ms": ms_eval_kernel,
                     "valu_counted_ops": {"note": "the method's FP32 operations counted per cell-slice, over the "
                                                  "non-packed FP32 issue rate of the chip; not a measure of the "
                                                  "kernel: it issues fewer instructions than counted (weights of "
                                                  "exactly 1 and 0 skip their multiplies, rows whose outputs are "
                                                  "known to be c^B skip their inflation), so this can exceed 1; "
                                                  "issued counts are in profiles/valu-config1-20M-map.txt",
                                          "ops_per_cell_slice": eval_ops_per_cell(R), "achieved_tops": eval_tops,
                                          "issue_peak_tops": VALU_PEAK_TOPS, "frac": eval_tops / VALU_PEAK_TOPS}},
        "wall_s_timed": c1["wall_s_timed"],
        "autotune": c1["autotune"],
        "paper_context": PAPER_TABLE3,
    }
    del g, c, cost, keep
    if not args.no_batched:
        out["batched_vs_plain"] = {"profiles": bench_profiles(P, torch, sc, xyz, dev, args.steps, args.warmup)}
        out["batched_vs_plain"]["submaps"] = bench_submaps(P, torch, dev, args.steps, args.warmup)
    del xyz
    torch.cuda.empty_cache()
    if not args.no_plan:
        log("generating the building")
        bsc = scenes.plan_building()
        bsc.robot = dict(sc.robot)
        tm, bxyz, outs = bench_step(P, torch, dev, bsc, rb, args.steps, args.warmup, "building")
        del outs
        tm["workload"] = ("the six-storey layout on 100 m x 100 m (1000 x 1000 cells at 0.1 m), 26.4 M points "
                          "(4 per cell and storey), slice interval 0.3 m, the same robot as the 20M-point map")
        out["traversable_map"] = tm
        if not args.no_batched:
            out["traversable_map"]["profiles"] = bench_profiles(P, torch, bsc, bxyz, dev, args.steps, args.warmup,
                                                                traversable=True, map_name="the building")
        del bxyz, bsc
        torch.cuda.empty_cache()
        out["plan"] = bench_plan(P, torch, dev, args.steps, args.warmup, cpu=not args.no_cpu_baseline)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on the map, all cores and one core)")
        out["cpu_baseline"] = cpu_baseline(sc, args.cpu_window)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
