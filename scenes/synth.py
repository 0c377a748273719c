"""Seeded synthetic scenes with the structure of the paper's workloads.

Every scene is a set of piecewise-horizontal surfaces (floors, slabs, stair
treads, beams, ramps, a bumpy ground).  Points are allocated to surfaces in
proportion to their xy area by one multinomial draw, placed uniformly in xy
on their surface, and given N(0, sigma) height noise.  All draws come from
``numpy.random.default_rng(seed)``; the same seed gives the same float32
array on every machine.

Nothing here slices, rasterises or costs anything: that is the method, and it
lives in the library and (independently) in the oracle.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Robot descriptions in physical units.  ``safe_margin`` is the width d_sm of
# the graded margin of the inflation kernel; the paper's kernel figure uses
# d_sm = 0.4 m, which is taken for every robot here.
ROBOT_CONFIG0 = dict(min_interval=0.5, nominal_height=1.0, max_slope_deg=30.0,
                     max_step=0.2, inflation_radius=0.3, safe_margin=0.4)

# Table I of the paper gives thresholds directly (quadruped).  d_inf and d_sm
# are not in Table I; the kernel-figure values are used.
ROBOT_TABLE1 = dict(d_min=0.50, d_ref=0.65, theta_b=1.70, theta_s=0.36,
                    theta_p=0.20, c_barrier=50.0, alpha_d=20.0, alpha_b=20.0,
                    alpha_s=15.0, d_inf=0.2, d_sm=0.4, patch_radius=1)


@dataclass
class Scene:
    points: np.ndarray                 # float32 [P, 3], C-contiguous
    grid: dict                         # x0, y0, res, nx, ny, slice_dz
    robot: dict = field(default_factory=lambda: dict(ROBOT_CONFIG0))
    name: str = ""
    meta: dict = field(default_factory=dict)


# --------------------------------------------------------------------------
# surfaces

def _rect_minus(rect, holes):
    """Split the xy rectangle ``rect`` minus ``holes`` into disjoint rectangles."""
    x0, x1, y0, y1 = rect
    hs = [(max(a, x0), min(b, x1), max(c, y0), min(d, y1)) for a, b, c, d in holes]
    hs = [h for h in hs if h[0] < h[1] and h[2] < h[3]]
    if not hs:
        return [rect]
    xs = sorted({x0, x1, *[h[0] for h in hs], *[h[1] for h in hs]})
    ys = sorted({y0, y1, *[h[2] for h in hs], *[h[3] for h in hs]})
    out = []
    for i in range(len(xs) - 1):
        for j in range(len(ys) - 1):
            cx = 0.5 * (xs[i] + xs[i + 1])
            cy = 0.5 * (ys[j] + ys[j + 1])
            if any(h[0] <= cx < h[1] and h[2] <= cy < h[3] for h in hs):
                continue
            out.append((xs[i], xs[i + 1], ys[j], ys[j + 1]))
    return out


def _surf(x0, x1, y0, y1, z0, kind="const", slope=0.0, bumps=None):
    return dict(rect=(float(x0), float(x1), float(y0), float(y1)), z0=float(z0),
                kind=kind, slope=float(slope), bumps=bumps)


def _bump_field(rng, lx, ly, spacing, sigma, amp):
    """One Gaussian bump per spacing x spacing square, jittered inside it."""
    gx = max(1, int(math.ceil(lx / spacing)))
    gy = max(1, int(math.ceil(ly / spacing)))
    cx = (np.arange(gx)[:, None] + rng.random((gx, gy))) * spacing
    cy = (np.arange(gy)[None, :] + rng.random((gx, gy))) * spacing
    return dict(cx=cx, cy=cy, spacing=spacing, sigma=sigma, amp=amp)


def _bump_height(b, x, y):
    sp, s2 = b["spacing"], 2.0 * b["sigma"] ** 2
    gx, gy = b["cx"].shape
    ix = np.floor(x / sp).astype(np.int64)
    iy = np.floor(y / sp).astype(np.int64)
    z = np.zeros_like(x)
    for di in (-1, 0, 1):
        for dj in (-1, 0, 1):
            jx = np.clip(ix + di, 0, gx - 1)
            jy = np.clip(iy + dj, 0, gy - 1)
            ok = (ix + di >= 0) & (ix + di < gx) & (iy + dj >= 0) & (iy + dj < gy)
            d2 = (x - b["cx"][jx, jy]) ** 2 + (y - b["cy"][jx, jy]) ** 2
            z += np.where(ok, b["amp"] * np.exp(-d2 / s2), 0.0)
    return z


def _sample_surfaces(rng, surfaces, n_points, noise):
    areas = np.array([(s["rect"][1] - s["rect"][0]) * (s["rect"][3] - s["rect"][2])
                      for s in surfaces], dtype=np.float64)
    counts = rng.multinomial(n_points, areas / areas.sum())
    out = np.empty((n_points, 3), dtype=np.float32)
    pos = 0
    for s, c in zip(surfaces, counts):
        if c == 0:
            continue
        x0, x1, y0, y1 = s["rect"]
        x = x0 + (x1 - x0) * rng.random(c)
        y = y0 + (y1 - y0) * rng.random(c)
        if s["kind"] == "const":
            z = np.full(c, s["z0"])
        elif s["kind"] == "ramp_y":
            z = s["z0"] + s["slope"] * (y - y0)
        elif s["kind"] == "ramp_x":
            z = s["z0"] + s["slope"] * (x - x0)
        elif s["kind"] == "bumps":
            z = s["z0"] + _bump_height(s["bumps"], x, y)
        else:
            raise ValueError(s["kind"])
        if noise > 0:
            z = z + rng.normal(0.0, noise, c)
        out[pos:pos + c, 0] = x
        out[pos:pos + c, 1] = y
        out[pos:pos + c, 2] = z
        pos += c
    return out


# --------------------------------------------------------------------------
# the paper-shaped workloads

def config0_scene(seed: int = 0, n_points: int = 60_000, noise: float = 0.02) -> Scene:
    """20 m x 20 m: ground floor at z=0, an upper storey over half the area
    (slab underside at 2.8 m, floor at 3.0 m), a 15 degree ramp 2 m wide and a
    landing joining the floors.  Grid 0.1 m (200 x 200), slice interval 0.4 m."""
    rng = np.random.default_rng(seed)
    t15 = math.tan(math.radians(15.0))
    run = 3.0 / t15                      # 11.196 m of ramp for 3 m of rise
    y_top = 2.0 + run
    surfaces = [
        _surf(0, 20, 0, 20, 0.0),                        # ground floor
        _surf(10, 20, 0, 20, 2.8),                       # slab underside
        _surf(10, 20, 0, 20, 3.0),                       # upper floor
        _surf(8, 10, 2.0, y_top, 0.0, "ramp_y", t15),    # ramp
        _surf(8, 10, y_top, y_top + 2.0, 3.0),           # landing
    ]
    pts = _sample_surfaces(rng, surfaces, n_points, noise)
    grid = dict(x0=0.0, y0=0.0, res=0.1, nx=200, ny=200, slice_dz=0.4)
    return Scene(pts, grid, dict(ROBOT_CONFIG0), "config0", dict(seed=seed))


def multistorey_scene(seed: int, lx: float, ly: float, n_points: int, n_floors: int = 6,
                      storey: float = 3.0, res: float = 0.1, slice_dz: float = 0.3,
                      beam_cover: float = 0.05, bumps: bool = True, noise: float = 0.02,
                      rng: np.random.Generator | None = None) -> Scene:
    """A building of ``n_floors`` storeys ``storey`` metres apart on [0,lx)x[0,ly).

    Each storey transition has two staircases 2 m wide (16 risers of 0.18 m,
    0.30 m treads, a 0.12 m top riser) with an opening in the floor above the
    run; each storey has 0.3 m wide beams (underside at floor+1.2 m, top at
    floor+1.5 m) until ``beam_cover`` of the area is covered; the ground floor
    carries Gaussian bumps (sigma 0.5 m, amplitude 0.1 m, one per 25 m^2).
    Staircases are left out where the footprint is too small to hold them."""
    rng = rng if rng is not None else np.random.default_rng(seed)
    nx = int(round(lx / res))
    ny = int(round(ly / res))
    width, tread, n_treads, riser = 2.0, 0.30, 16, 0.18
    run = n_treads * tread
    surfaces = []
    holes = [[] for _ in range(n_floors)]
    stairs_fit = lx >= width + 1.0 and ly >= run + 1.0
    for s in range(n_floors - 1):
        if not stairs_fit:
            break
        for _ in range(2):
            sx = rng.uniform(0.5, lx - width - 0.5)
            sy = rng.uniform(0.5, ly - run - 0.5)
            zb = s * storey
            for i in range(n_treads):
                surfaces.append(_surf(sx, sx + width, sy + i * tread, sy + (i + 1) * tread,
                                      zb + (i + 1) * riser))
            holes[s + 1].append((sx, sx + width, sy, sy + run))
    for s in range(n_floors):
        z = s * storey
        for r in _rect_minus((0.0, lx, 0.0, ly), holes[s]):
            if s == 0 and bumps:
                surfaces.append(_surf(*r, z, "bumps", bumps=None))
            else:
                surfaces.append(_surf(*r, z))
    if bumps:
        field = _bump_field(rng, lx, ly, 5.0, 0.5, 0.1)
        for sf in surfaces:
            if sf["kind"] == "bumps":
                sf["bumps"] = field
    # beams: full-length strips along x or y, until the covered area reaches
    # beam_cover of the footprint (measured on a coarse 0.1 m raster)
    if beam_cover > 0:
        for s in range(n_floors):
            z = s * storey
            cover = np.zeros((max(1, ny), max(1, nx)), dtype=bool)
            target = beam_cover * cover.size
            guard = 0
            while cover.sum() < target and guard < 10_000:
                guard += 1
                if rng.random() < 0.5:
                    c = rng.uniform(0.0, max(ly - 0.3, 1e-3))
                    r = (0.0, lx, c, c + 0.3)
                    cover[int(c / res):int(math.ceil((c + 0.3) / res)), :] = True
                else:
                    c = rng.uniform(0.0, max(lx - 0.3, 1e-3))
                    r = (c, c + 0.3, 0.0, ly)
                    cover[:, int(c / res):int(math.ceil((c + 0.3) / res))] = True
                surfaces.append(_surf(*r, z + 1.2))
                surfaces.append(_surf(*r, z + 1.5))
    pts = _sample_surfaces(rng, surfaces, n_points, noise)
    grid = dict(x0=0.0, y0=0.0, res=res, nx=nx, ny=ny, slice_dz=slice_dz)
    return Scene(pts, grid, dict(ROBOT_CONFIG0), "multistorey",
                 dict(seed=seed, n_floors=n_floors, lx=lx, ly=ly))


def config1_scene(seed: int = 1, n_points: int = 20_000_000, side: float = 200.0) -> Scene:
    """The large map: 200 m x 200 m, six storeys, 20 M points, grid 0.1 m
    (2000 x 2000), slice interval 0.3 m.  ``side``/``n_points`` scale it down
    with the same structure and density for the parity tests."""
    sc = multistorey_scene(seed, side, side, n_points, n_floors=6)
    sc.name = "config1" if (side == 200.0 and n_points == 20_000_000) else "config1-crop"
    return sc


def dense_surface_scene(nx: int, ny: int, res: float, height_fn, per_cell: int = 4,
                        x0: float = 0.0, y0: float = 0.0, slice_dz: float = 0.3,
                        extra=None) -> Scene:
    """Noise-free points on a regular sub-lattice: ``per_cell`` (a square
    number) points per cell at the sub-cell centres, with z = height_fn(x, y).
    ``extra`` is an optional list of further float32 [M,3] point arrays."""
    k = int(round(math.sqrt(per_cell)))
    off = (np.arange(k) + 0.5) / k
    ix = np.arange(nx)
    iy = np.arange(ny)
    xs = (x0 + res * (ix[:, None] + off[None, :])).reshape(-1)
    ys = (y0 + res * (iy[:, None] + off[None, :])).reshape(-1)
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    Z = height_fn(X, Y)
    pts = np.stack([X.reshape(-1), Y.reshape(-1), np.asarray(Z, dtype=np.float64).reshape(-1)], 1)
    pts = pts[np.isfinite(pts[:, 2])]
    arrs = [pts.astype(np.float32)]
    if extra:
        arrs += [np.asarray(e, dtype=np.float32) for e in extra]
    grid = dict(x0=float(x0), y0=float(y0), res=float(res), nx=int(nx), ny=int(ny),
                slice_dz=float(slice_dz))
    return Scene(np.ascontiguousarray(np.concatenate(arrs, 0)), grid, dict(ROBOT_CONFIG0), "dense")


# --------------------------------------------------------------------------
# trajectories, batches, robot profiles

def random_walks(seed: int, mask: np.ndarray, ground: np.ndarray, grid: dict,
                 n_traj: int, n_wp: int, d_ref: float, z_sigma: float = 0.05,
                 slices: np.ndarray | None = None):
    """Random walks over the cells where ``mask`` ([N, ny, nx] bool) holds.

    A walk starts on a uniformly chosen masked cell-slice and steps to a
    uniformly chosen masked 8-neighbour on the same slice (it stays put when
    none is masked).  Each waypoint sits at the cell centre offset by
    +-U(0.1, 0.4) cells per axis; its z is ground + d_ref + N(0, z_sigma),
    read from the caller's ``ground`` array.  Returns (wp float32 [T,W,3],
    slice int32 [T,W])."""
    rng = np.random.default_rng(seed)
    N, ny, nx = mask.shape
    if slices is not None:
        allowed = np.zeros(N, dtype=bool)
        allowed[np.asarray(slices)] = True
        mask = mask & allowed[:, None, None]
    flat = np.flatnonzero(mask.reshape(-1))
    if flat.size == 0:
        raise ValueError("random_walks: empty mask")
    start = flat[rng.integers(0, flat.size, n_traj)]
    k = (start // (ny * nx)).astype(np.int64)
    iy = ((start // nx) % ny).astype(np.int64)
    ix = (start % nx).astype(np.int64)
    cells = np.empty((n_traj, n_wp, 2), dtype=np.int64)
    nb = np.array([(-1, -1), (-1, 0), (-1, 1), (0, -1), (0, 1), (1, -1), (1, 0), (1, 1)])
    for w in range(n_wp):
        cells[:, w, 0] = ix
        cells[:, w, 1] = iy
        cx = ix[:, None] + nb[None, :, 0]
        cy = iy[:, None] + nb[None, :, 1]
        inb = (cx >= 0) & (cx < nx) & (cy >= 0) & (cy < ny)
        ok = inb & mask[k[:, None], np.clip(cy, 0, ny - 1), np.clip(cx, 0, nx - 1)]
        r = rng.random((n_traj, 8)) * ok
        pick = np.argmax(r, axis=1)
        has = ok.any(axis=1)
        ix = np.where(has, cx[np.arange(n_traj), pick], ix)
        iy = np.where(has, cy[np.arange(n_traj), pick], iy)
    res = grid["res"]
    off = rng.uniform(0.1, 0.4, (n_traj, n_wp, 2)) * np.where(rng.random((n_traj, n_wp, 2)) < 0.5, -1, 1)
    x = grid["x0"] + res * (cells[..., 0] + 0.5 + off[..., 0])
    y = grid["y0"] + res * (cells[..., 1] + 0.5 + off[..., 1])
    kk = np.repeat(k[:, None], n_wp, 1)
    g = ground[kk, cells[..., 1], cells[..., 0]].astype(np.float64)
    g = np.where(np.isfinite(g), g, 0.0)
    z = g + d_ref + rng.normal(0.0, z_sigma, (n_traj, n_wp))
    wp = np.stack([x, y, z], -1).astype(np.float32)
    return np.ascontiguousarray(wp), np.ascontiguousarray(kk.astype(np.int32))


def submap_batch(seed: int = 3, n_items: int = 512, side_lo: int = 50, side_hi: int = 400,
                 pts_lo: int = 10_000, pts_hi: int = 1_000_000, res: float = 0.1,
                 slice_dz: float = 0.3):
    """Submaps of uneven size: one u ~ U(0,1) per item sets the side to
    round(side_lo * (side_hi/side_lo)^u) cells and the point count to
    round(pts_lo * (pts_hi/pts_lo)^u); floors ~ U{2..8}."""
    rng = np.random.default_rng(seed)
    items = []
    for i in range(n_items):
        u = rng.random()
        side = int(round(side_lo * (side_hi / side_lo) ** u))
        npts = int(round(pts_lo * (pts_hi / pts_lo) ** u))
        floors = int(rng.integers(2, 9))
        sc = multistorey_scene(seed, side * res, side * res, npts, n_floors=floors,
                               res=res, slice_dz=slice_dz, rng=rng)
        sc.name = f"submap{i}"
        items.append(sc)
    return items


def robot_profiles(seed: int = 4, n: int = 64):
    """Robot profiles: min interval U(0.4,0.8) m, max slope U(20,40) deg,
    max step U(0.1,0.3) m; the rest as the config-0 robot."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        r = dict(ROBOT_CONFIG0)
        r["min_interval"] = float(rng.uniform(0.4, 0.8))
        r["max_slope_deg"] = float(rng.uniform(20.0, 40.0))
        r["max_step"] = float(rng.uniform(0.1, 0.3))
        out.append(r)
    return out


# --------------------------------------------------------------------------
# inputs of the path search

def plan_layers(seed: int, L: int, ny: int, nx: int, c_barrier: float = 50.0, p_block: float = 0.2,
                p_same: float = 0.3, p_tie: float = 0.05):
    """Random layers for the path search: float32 c^T [L, ny, nx] uniform in
    [0, 20) with a ``p_block`` share of barrier cells, and e^G [L, ny, nx]
    where each layer repeats the ground of the layer below on a random
    ``p_same`` share of cells (where nodes merge and gateways can arise) and
    lies 0.5-3 m higher elsewhere; a ``p_tie`` share of cells copies the
    cost of the layer below (equal costs: no gateway)."""
    rng = np.random.default_rng(seed)
    cT = rng.uniform(0.0, 20.0, (L, ny, nx)).astype(np.float32)
    cT[rng.random((L, ny, nx)) < p_block] = np.float32(c_barrier)
    eG = np.zeros((L, ny, nx), np.float32)
    eG[0] = rng.uniform(0.0, 0.2, (ny, nx)).astype(np.float32)
    for l in range(1, L):
        same = rng.random((ny, nx)) < p_same
        eG[l] = np.where(same, eG[l - 1], eG[l - 1] + np.float32(rng.uniform(0.5, 3.0)))
    tie = rng.random((L, ny, nx)) < p_tie
    cT[1:][tie[1:]] = cT[:-1][tie[1:]]
    return cT, eG


def plan_serpentine(seed: int, ny: int, nx: int, pitch: int = 8, gap: int = 3, c_barrier: float = 50.0):
    """One layer with barrier walls across the map every ``pitch`` rows,
    each open for ``gap`` cells at alternating ends, so that a path from the
    top to the bottom winds through every corridor; costs uniform in [0, 5)."""
    rng = np.random.default_rng(seed)
    cT = rng.uniform(0.0, 5.0, (1, ny, nx)).astype(np.float32)
    for i, y in enumerate(range(pitch, ny, pitch)):
        cT[0, y, :] = np.float32(c_barrier)
        if i % 2 == 0:
            cT[0, y, nx - gap:] = cT[0, y - 1, nx - gap:]
        else:
            cT[0, y, :gap] = cT[0, y - 1, :gap]
    return cT, np.zeros((1, ny, nx), np.float32)


def plan_building(seed: int = 7, side: float = 100.0, n_floors: int = 6, per_cell: float = 4.0) -> Scene:
    """The path-search map: the six-storey building of the large map on a
    ``side`` x ``side`` footprint without beams (a beam across a staircase
    closes it), sampled densely enough (``per_cell`` points per 0.1 m cell
    and storey, plus 10 %) that floors and stairs are observed, so that paths
    exist through the slices from the ground floor to the top."""
    n_points = int(per_cell * (side / 0.1) ** 2 * n_floors * 1.1)
    sc = multistorey_scene(seed, side, side, n_points, n_floors=n_floors, beam_cover=0.0)
    sc.name = "plan-building"
    return sc


def traj_problems(seed: int, n: int, M: int, x_range, y_range, z_body: float, step: float = 0.6,
                  speed: float = 1.0, slices=(0,), turn: float = 0.5):
    """Seeded trajectory-optimisation problems: n trajectories of M pieces
    whose waypoints follow a random heading walk with the given step, inside
    the xy box, at body height z_body (+ N(0, 0.05)), starting and ending at
    rest.  Durations are step / speed times U(0.7, 1.3); each trajectory is
    assigned one of ``slices``.  Returns bound [n, 2, 3, 3] (start and goal:
    position, velocity, acceleration), slices [n, M] int32, knots
    [n, M-1, 3] and tau [n, M] (log-durations), all float64."""
    rng = np.random.default_rng(seed)
    pts = np.zeros((n, M + 1, 3))
    x0, x1 = x_range
    y0, y1 = y_range
    pts[:, 0, 0] = rng.uniform(x0, x1, n)
    pts[:, 0, 1] = rng.uniform(y0, y1, n)
    head = rng.uniform(0, 2 * math.pi, n)
    for m in range(1, M + 1):
        head = head + rng.normal(0, turn, n)
        nx_ = pts[:, m - 1, 0] + step * np.cos(head)
        ny_ = pts[:, m - 1, 1] + step * np.sin(head)
        out = (nx_ < x0) | (nx_ > x1) | (ny_ < y0) | (ny_ > y1)
        head = np.where(out, head + math.pi, head)
        pts[:, m, 0] = np.clip(np.where(out, pts[:, m - 1, 0] + step * np.cos(head), nx_), x0, x1)
        pts[:, m, 1] = np.clip(np.where(out, pts[:, m - 1, 1] + step * np.sin(head), ny_), y0, y1)
    pts[:, :, 2] = z_body + rng.normal(0, 0.05, (n, M + 1))
    bound = np.zeros((n, 2, 3, 3))
    bound[:, 0, 0] = pts[:, 0]
    bound[:, 1, 0] = pts[:, M]
    sl = np.asarray(slices, np.int32)[rng.integers(0, len(slices), n)]
    return dict(bound=bound, slices=np.repeat(sl[:, None], M, axis=1).astype(np.int32),
                knots=np.ascontiguousarray(pts[:, 1:M]),
                tau=np.log(step / speed * rng.uniform(0.7, 1.3, (n, M))))
