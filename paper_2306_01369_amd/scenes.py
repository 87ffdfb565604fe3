"""Seeded synthetic scenes: particle beds, containers and tool trajectories.

This module builds inputs only.  It places spheres on jittered lattices, draws
radii and tool twists from seeded NumPy generators (PCG64 via
``numpy.random.default_rng``) and writes kinematic body descriptions.  It holds
none of the simulation arithmetic (no hashing, contact tests, impulses or
integration), so both the GPU path and the CPU oracle can take their inputs
from it.

Body records are plain dicts::

    {"shape": "plane"|"box"|"capsule", "params": [4 floats],
     "R": 3x3 world<-body rotation, "t": 3-vector, "nu": 3, "omega": 3, "env": int}

Shapes follow the closed-form primitives of Sec. II-C (signed distance
functions): a plane is the body-frame half space z <= 0 with outward normal +z;
a box has half extents ``params[0:3]``; a capsule is the set within
``params[0]`` of the body-frame segment from (0,0,-params[1]) to (0,0,+params[1]).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

DENSITY = 2500.0          # kg/m^3, grain density used for m_i = rho*4/3*pi*r_i^3
GRAVITY = (0.0, 0.0, -9.81)


@dataclass
class Scene:
    """A complete simulation input.  Arrays are float32 as handed to both sides."""
    name: str
    x: np.ndarray                 # (n, 3) float32 positions [m]
    v: np.ndarray                 # (n, 3) float32 velocities [m/s]
    radius: np.ndarray            # (n,) float32 radii [m]
    bodies: list = field(default_factory=list)
    dt: float = 1e-3
    n_iters: int = 20
    mu: float = 0.5
    alpha: float = 0.2
    gravity: tuple = GRAVITY
    n_steps: int = 100
    env_offsets: np.ndarray | None = None   # (n_envs+1,) int64, None = one env
    # per-step twists (n_steps, n_bodies, 6) or None for constant twists
    twists: np.ndarray | None = None

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


# ----------------------------------------------------------------------------
# bodies
# ----------------------------------------------------------------------------

def _rot_z_to(nrm):
    """Rotation whose third column is the unit vector ``nrm`` (body +z -> nrm).

    Only used for axis-aligned container walls, so the result is exact in
    float32 (entries are 0 and +-1)."""
    nrm = np.asarray(nrm, dtype=np.float64)
    table = {
        (0, 0, 1): np.eye(3),
        (1, 0, 0): np.array([[0, 0, 1], [0, 1, 0], [-1, 0, 0]], float),
        (-1, 0, 0): np.array([[0, 0, -1], [0, 1, 0], [1, 0, 0]], float),
        (0, 1, 0): np.array([[1, 0, 0], [0, 0, 1], [0, -1, 0]], float),
        (0, -1, 0): np.array([[1, 0, 0], [0, 0, -1], [0, 1, 0]], float),
    }
    return table[tuple(int(round(c)) for c in nrm)]


def plane(point, normal, env=0):
    """Half-space container wall through ``point`` whose outward normal (pointing
    into the free region) is ``normal``."""
    return {"shape": "plane", "params": [0.0, 0.0, 0.0, 0.0],
            "R": _rot_z_to(normal), "t": np.asarray(point, float),
            "nu": np.zeros(3), "omega": np.zeros(3), "env": env}


def box_tool(center, half_extents, nu=(0, 0, 0), omega=(0, 0, 0), R=None, env=0):
    return {"shape": "box", "params": [*map(float, half_extents), 0.0],
            "R": np.eye(3) if R is None else np.asarray(R, float),
            "t": np.asarray(center, float), "nu": np.asarray(nu, float),
            "omega": np.asarray(omega, float), "env": env}


def capsule_tool(center, radius, half_length, nu=(0, 0, 0), omega=(0, 0, 0), R=None, env=0):
    return {"shape": "capsule", "params": [float(radius), float(half_length), 0.0, 0.0],
            "R": np.eye(3) if R is None else np.asarray(R, float),
            "t": np.asarray(center, float), "nu": np.asarray(nu, float),
            "omega": np.asarray(omega, float), "env": env}


def sdf_grid(fn, lo, hi, inv_spacing):
    """Samples of a distance field fn(points (m, 3) body frame) -> (m,) on the
    regular grid with knots at lo + k / inv_spacing covering [lo, hi]: the
    input format of grid bodies (values (nz, ny, nx), x fastest)."""
    lo = np.asarray(lo, np.float32).astype(np.float64)   # the origin as the grid stores it
    n = [int(np.ceil((hi[a] - lo[a]) * inv_spacing)) + 1 for a in range(3)]
    ax = [lo[a] + np.arange(n[a]) / inv_spacing for a in range(3)]
    zz, yy, xx = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    pts = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], 1)
    vals = np.asarray(fn(pts), np.float64).reshape(n[2], n[1], n[0])
    return {"values": vals.astype(np.float32), "origin": lo.astype(np.float32), "inv_spacing": float(inv_spacing)}


def ball_grid(radius, margin, inv_spacing):
    """Distance field of a ball of the given radius about the body origin."""
    m = radius + margin
    return sdf_grid(lambda p: np.linalg.norm(p, axis=1) - radius, (-m, -m, -m), (m, m, m), inv_spacing)


def bowl_grid(radius, thickness, margin, inv_spacing):
    """A scoop-like bowl: the lower half (z <= 0) of a spherical shell of
    inner radius ``radius`` and the given thickness, about the body origin,
    as the exact distance to that solid (shell distance, then the cut)."""
    R0, R1 = radius, radius + thickness
    m = R1 + margin

    def fn(p):
        r = np.linalg.norm(p, axis=1)
        shell = np.maximum(r - R1, R0 - r)               # full spherical shell
        # points above the cut plane: distance to the rim annulus in z = 0
        rho = np.linalg.norm(p[:, :2], axis=1)
        dr = np.maximum(np.maximum(R0 - rho, rho - R1), 0.0)
        above = np.sqrt(dr * dr + p[:, 2] ** 2)
        return np.where(p[:, 2] <= 0.0, shell, np.maximum(above, shell))

    return sdf_grid(fn, (-m, -m, -m), (m, m, m / 2), inv_spacing)


def affine_grid(normal, offset, lo, hi, inv_spacing):
    """The affine field n . p - offset (a plane's distance for a unit n)."""
    nrm = np.asarray(normal, np.float64)
    return sdf_grid(lambda p: p @ nrm - offset, lo, hi, inv_spacing)


def grid_tool(grid, center, nu=(0, 0, 0), omega=(0, 0, 0), R=None, env=0):
    return {"shape": "grid", "params": [0.0, 0.0, 0.0, 0.0], "grid": grid,
            "R": np.eye(3) if R is None else np.asarray(R, float),
            "t": np.asarray(center, float), "nu": np.asarray(nu, float),
            "omega": np.asarray(omega, float), "env": env}


# ----------------------------------------------------------------------------
# cameras (observations of the Gym-style environment, Sec. III-A)
# ----------------------------------------------------------------------------

def camera_pose(eye, target, up=(0.0, 0.0, 1.0)):
    """Row-major [R | t] (camera -> world) of a camera at ``eye`` whose +z axis
    points at ``target``; image x (columns) to the right, y (rows) downward."""
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    xa = np.cross(f, np.asarray(up, np.float64))
    xa /= np.linalg.norm(xa)
    ya = np.cross(f, xa)
    R = np.stack([xa, ya, f], axis=1)
    return np.concatenate([R, eye[:, None]], axis=1)


def sky_camera(x0, x1, y0, y1, height, width, rows, far=None, env=0):
    """Orthographic camera looking straight down on [x0, x1] x [y0, y1] from
    ``height``; far defaults to the height (the depth of the plane z = 0)."""
    pose = np.array([[1.0, 0.0, 0.0, 0.5 * (x0 + x1)],
                     [0.0, -1.0, 0.0, 0.5 * (y0 + y1)],
                     [0.0, 0.0, -1.0, height]])
    return {"env": env, "kind": "ortho", "width": int(width), "height": int(rows), "pose": pose,
            "params": (0.5 * (x1 - x0), 0.5 * (y1 - y0), height if far is None else far, 0.0)}


def perspective_camera(eye, target, fov_x_deg, width, rows, far, up=(0.0, 0.0, 1.0), env=0):
    """Perspective camera at ``eye`` looking at ``target`` with a horizontal
    field of view of ``fov_x_deg`` degrees and square pixels."""
    tx = float(np.tan(np.radians(fov_x_deg) / 2))
    return {"env": env, "kind": "perspective", "width": int(width), "height": int(rows),
            "pose": camera_pose(eye, target, up), "params": (tx, tx * rows / width, far, 0.0)}


def walled_box(x0, x1, y0, y1, env=0, ground_z=0.0):
    """Ground plane plus four side walls of an open-top container."""
    return [
        plane((0, 0, ground_z), (0, 0, 1), env),
        plane((x0, 0, 0), (1, 0, 0), env),
        plane((x1, 0, 0), (-1, 0, 0), env),
        plane((0, y0, 0), (0, 1, 0), env),
        plane((0, y1, 0), (0, -1, 0), env),
    ]


def random_rotation(rng):
    """Uniform random rotation from a unit quaternion (Shoemake's method)."""
    u1, u2, u3 = rng.random(3)
    a, b = math.sqrt(1 - u1), math.sqrt(u1)
    qx, qy = a * math.sin(2 * math.pi * u2), a * math.cos(2 * math.pi * u2)
    qz, qw = b * math.sin(2 * math.pi * u3), b * math.cos(2 * math.pi * u3)
    return np.array([
        [1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qz * qw), 2 * (qx * qz + qy * qw)],
        [2 * (qx * qy + qz * qw), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qx * qw)],
        [2 * (qx * qz - qy * qw), 2 * (qy * qz + qx * qw), 1 - 2 * (qx * qx + qy * qy)],
    ])


def uniform_ball(rng, radius):
    """Point uniform in the 3-ball of the given radius."""
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    return d * radius * rng.random() ** (1.0 / 3.0)


# ----------------------------------------------------------------------------
# particle beds
# ----------------------------------------------------------------------------

def jittered_lattice(counts, spacing, origin, jitter, rng):
    """Cubic lattice, index i = (a*counts[1] + b)*counts[2] + c at
    origin + spacing*(a, b, c) + U(-jitter, jitter)^3 (one (n, 3) draw)."""
    na, nb, nc = counts
    a, b, c = np.meshgrid(np.arange(na), np.arange(nb), np.arange(nc), indexing="ij")
    idx = np.stack([a.ravel(), b.ravel(), c.ravel()], axis=1).astype(np.float64)
    pos = np.asarray(origin, float) + spacing * idx
    pos += rng.uniform(-jitter, jitter, size=pos.shape)
    return pos


def packed_bed(n, r, x0, x1, y0, y1, rng, overlap=1e-3, jitter_frac=0.1):
    """A dense resting bed of ``n`` equal spheres inside [x0,x1]x[y0,y1].

    Simple-cubic layers filled bottom-up, row by row (index order is spatial
    order).  Neighbour spacing is s = 2r(1 - overlap) so every face neighbour
    touches (six contacts per interior grain, the coordination of a random
    close packing); each coordinate gets an independent U(+-jitter_frac *
    overlap * r) jitter, small enough that every face pair still overlaps and
    no diagonal pair does.  The bottom layer rests on z = 0 with the same
    overlap.  Returns float64 positions (n, 3)."""
    s = 2.0 * r * (1.0 - overlap)
    nx = int(math.floor(((x1 - x0) - 2 * r) / s)) + 1
    ny = int(math.floor(((y1 - y0) - 2 * r) / s)) + 1
    per_layer = nx * ny
    layers = -(-n // per_layer)
    ox = x0 + 0.5 * ((x1 - x0) - (nx - 1) * s)
    oy = y0 + 0.5 * ((y1 - y0) - (ny - 1) * s)
    oz = r * (1.0 - overlap)
    k = np.arange(n)
    layer, rem = np.divmod(k, per_layer)
    row, col = np.divmod(rem, nx)
    pos = np.stack([ox + s * col, oy + s * row, oz + s * layer], axis=1).astype(np.float64)
    pos += rng.uniform(-1.0, 1.0, size=pos.shape) * (jitter_frac * overlap * r)
    assert layers >= 1
    return pos


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------

def drop_scene(seed=0):
    """4,096 spheres, r = 5 mm, jittered 16^3 lattice (spacing 2.1r, jitter
    +-0.05r) falling onto the floor of a 0.2 m box; dt = 1 ms, 20 iterations,
    mu = 0.5, 100 steps."""
    r = 0.005
    rng = np.random.default_rng(seed)
    pos = jittered_lattice((16, 16, 16), 2.1 * r, (0.02125, 0.02125, 1.1 * r), 0.05 * r, rng)
    n = pos.shape[0]
    return Scene("drop-4096", _f32(pos), np.zeros((n, 3), np.float32),
                 np.full(n, r, np.float32), walled_box(0.0, 0.2, 0.0, 0.2),
                 dt=1e-3, n_iters=20, mu=0.5, alpha=0.2, n_steps=100)


def scoop_scene(seed=0, n=1 << 20, r=0.002):
    """1,048,576 spheres, r = 2 mm, resting bed in a 1 x 1 m walled box, with a
    0.05 x 0.1 x 0.2 m box tool whose bottom edge starts 1 cm above the bed at
    x = 0.3 m and moves at 0.2 m/s along (cos 30deg, 0, -sin 30deg)."""
    rng = np.random.default_rng(seed)
    pos = packed_bed(n, r, 0.0, 1.0, 0.0, 1.0, rng)
    s = 2.0 * r * (1.0 - 1e-3)
    per_layer = int(math.floor((1.0 - 2 * r) / s) + 1) ** 2
    full_layers = n // per_layer
    surface = r * (1 - 1e-3) + s * (full_layers - 1) + r
    half = (0.025, 0.05, 0.1)
    center = (0.3, 0.5, surface + 0.01 + half[2])
    speed = 0.2
    a = math.radians(30.0)
    tool = box_tool(center, half, nu=(speed * math.cos(a), 0.0, -speed * math.sin(a)))
    bodies = walled_box(0.0, 1.0, 0.0, 1.0) + [tool]
    return Scene(f"scoop-{n}", _f32(pos), np.zeros((n, 3), np.float32),
                 np.full(n, r, np.float32), bodies, dt=1e-3, n_iters=20, mu=0.5,
                 alpha=0.2, n_steps=200)


# The settled scoop bed is prepared by seeded settling: grains poured from a
# loose jittered lattice first compact without friction (a frictionless pour
# packs randomly and densely; with friction and no rotational degrees of
# freedom, columns of grains stacked almost vertically are stable and the pour
# stays loose), then settle with the workload's friction until no more than a
# fraction SETTLE_FAST_FRACTION of the grains (none below 100,000 grains, 10 of
# 2^20) moves faster than SETTLE_VMAX: in a wide bed a handful of grains
# squeezed between the floor, a wall and their neighbours creep at about
# 1 mm/s for thousands of steps while the rest are at rest.  Both phases use
# SETTLE_ITERS sweeps.  The plan is data; each simulator runs it in its own
# code.
SETTLE_ITERS = 100
SETTLE_COMPACT_STEPS = 300     # phase 1: mu = 0
SETTLE_VMAX = 1e-3             # phase 2: mu of the workload, until |v| < this ...
SETTLE_FAST_FRACTION = 1e-5    # ... for all but this fraction of the grains
SETTLE_CHECK_EVERY = 25        # steps between checks of the speeds in phase 2
SETTLE_MAX_STEPS = 3000        # phase 2 gives up after this many steps


def settle_fast_allowed(n):
    """Grains allowed above SETTLE_VMAX when settling n grains."""
    return int(math.floor(SETTLE_FAST_FRACTION * n))


def poured_lattice(n, r, x0, x1, y0, y1, rng, spacing=2.6, jitter=0.3):
    """The first n sites of a loose cubic lattice over [x0,x1] x [y0,y1],
    filled bottom-up (layer, then row, then column): spacing spacing*r, every
    coordinate jittered by U(+-jitter*r) (one (n, 3) draw), lowest centres at
    z = (1 + jitter) r.  spacing - 2 jitter >= 2 keeps every pair apart, so the
    pour starts without contacts.  Returns float64 positions (n, 3)."""
    s = spacing * r
    nx = int(math.floor((x1 - x0) / s))
    ny = int(math.floor((y1 - y0) / s))
    per_layer = nx * ny
    k = np.arange(n)
    layer, rem = np.divmod(k, per_layer)
    row, col = np.divmod(rem, nx)
    ox = x0 + 0.5 * ((x1 - x0) - (nx - 1) * s)
    oy = y0 + 0.5 * ((y1 - y0) - (ny - 1) * s)
    oz = (1.0 + jitter) * r
    pos = np.stack([ox + s * col, oy + s * row, oz + s * layer], axis=1).astype(np.float64)
    pos += rng.uniform(-jitter * r, jitter * r, size=pos.shape)
    return pos


def scoop_pour(seed=0, n=1 << 20, r=0.002, side=1.0):
    """The scoop bed before settling: n spheres (r = 2 mm) poured from a loose
    jittered lattice (spacing 2.6r, jitter +-0.3r; 192 x 192 sites per layer
    for the 1 x 1 m box) inside a walled side x side box, at rest.  Bodies are
    the walls only; the tool (scoop_tool) is placed on the settled surface.
    Settling follows the SETTLE_* plan; the workload then runs 20 sweeps with
    mu = 0.5."""
    rng = np.random.default_rng(seed)
    pos = poured_lattice(n, r, 0.0, side, 0.0, side, rng)
    return Scene(f"scoop-pour-{n}", _f32(pos), np.zeros((n, 3), np.float32),
                 np.full(n, r, np.float32), walled_box(0.0, side, 0.0, side),
                 dt=1e-3, n_iters=20, mu=0.5, alpha=0.2, n_steps=200)


def scoop_tool(surface, x=0.3, y=0.5, speed=0.2, angle_deg=30.0, half=(0.025, 0.05, 0.1), env=0):
    """The scoop bed's box tool (0.05 x 0.1 x 0.2 m): bottom face 1 cm above the
    bed surface at (x, y), moving at `speed` m/s along (cos a, 0, -sin a)."""
    a = math.radians(angle_deg)
    center = (x, y, surface + 0.01 + half[2])
    return box_tool(center, half, nu=(speed * math.cos(a), 0.0, -speed * math.sin(a)), env=env)


def column_scene(n=4096, r=0.005, seed=0, overlap=1e-3):
    """A resting column of equal spheres (the paper's 'particles at rest'
    benchmark shape) on a 8 x 8 footprint per layer, walled box around it."""
    rng = np.random.default_rng(seed)
    side = 8 * 2 * r * (1 - overlap) + 2 * r * overlap
    pos = packed_bed(n, r, 0.0, side, 0.0, side, rng, overlap=overlap)
    return Scene(f"column-{n}", _f32(pos), np.zeros((n, 3), np.float32),
                 np.full(n, r, np.float32), walled_box(0.0, side, 0.0, side),
                 n_steps=100)


def batched_scene(seed=0, n_envs=256, lo=8192, hi=65536, r=0.003, n_steps=100,
                  resample_every=20):
    """256 independent walled 0.3 x 0.3 m beds of U{8192..65536} spheres
    (r = 3 mm), each with a capsule tool (radius 2 cm, 15 cm between cap
    centres) in a random orientation starting 1 mm above its bed, driven by
    piecewise-constant random twists (|nu| <= 0.3 m/s, |omega| <= 1 rad/s,
    first segment moving down), resampled every 20 steps."""
    rng = np.random.default_rng(seed)
    counts = rng.integers(lo, hi + 1, size=n_envs)
    offsets = np.zeros(n_envs + 1, np.int64)
    offsets[1:] = np.cumsum(counts)
    xs, bodies = [], []
    n_seg = -(-n_steps // resample_every)
    tw = np.zeros((n_steps, 0, 6))
    twist_cols = []
    spacing_env = 0.5     # envs are laid out on a grid, 0.5 m apart (no overlap)
    grid = int(math.ceil(math.sqrt(n_envs)))
    for e in range(n_envs):
        erng = np.random.default_rng(1000 + seed + e)
        gx, gy = (e % grid) * spacing_env, (e // grid) * spacing_env
        pos = packed_bed(int(counts[e]), r, gx, gx + 0.3, gy, gy + 0.3, erng)
        xs.append(pos)
        top = float(pos[:, 2].max()) + r
        Rm = random_rotation(erng)
        # lowest point of the capsule above the bed by 1 mm
        axis = Rm[:, 2]
        low = 0.075 * abs(axis[2]) + 0.02
        center = (gx + 0.15, gy + 0.15, top + 0.001 + low)
        for wb in walled_box(gx, gx + 0.3, gy, gy + 0.3, env=e):
            bodies.append(wb)
            twist_cols.append(np.zeros((n_steps, 6)))
        cap = capsule_tool(center, 0.02, 0.075, R=Rm, env=e)
        seq = np.zeros((n_steps, 6))
        for sgi in range(n_seg):
            nu = uniform_ball(erng, 0.3)
            if sgi == 0 and nu[2] > 0:
                nu[2] = -nu[2]
            om = uniform_ball(erng, 1.0)
            seq[sgi * resample_every:(sgi + 1) * resample_every, :3] = nu
            seq[sgi * resample_every:(sgi + 1) * resample_every, 3:] = om
        cap["nu"], cap["omega"] = seq[0, :3].copy(), seq[0, 3:].copy()
        bodies.append(cap)
        twist_cols.append(seq)
    x = np.concatenate(xs, axis=0)
    n = x.shape[0]
    tw = np.stack(twist_cols, axis=1)   # (n_steps, n_bodies, 6)
    return Scene(f"batched-{n_envs}x", _f32(x), np.zeros((n, 3), np.float32),
                 np.full(n, r, np.float32), bodies, dt=1e-3, n_iters=20, mu=0.5,
                 alpha=0.2, n_steps=n_steps, env_offsets=offsets,
                 twists=tw.astype(np.float32))


def diff_scene(seed=0, n=32768, r=0.003):
    """32,768 spheres (r = 3 mm) resting in a 0.3 x 0.3 m walled footprint
    (13 full layers and part of a 14th); a capsule tool (radius 2 cm, 15 cm
    between cap centres, axis along y) whose lowest point starts 1 mm above
    the full layers at x = 0.1 m, moving at (0.2, 0, -0.1) m/s; 50 steps."""
    rng = np.random.default_rng(seed)
    pos = packed_bed(n, r, 0.0, 0.3, 0.0, 0.3, rng)
    top = surface_height(pos, r)
    Rm = np.array([[1, 0, 0], [0, 0, -1], [0, 1, 0]], float)   # axis along world y
    cap = capsule_tool((0.1, 0.15, top + 0.001 + 0.02), 0.02, 0.075, nu=(0.2, 0, -0.1), R=Rm)
    bodies = walled_box(0.0, 0.3, 0.0, 0.3) + [cap]
    return Scene(f"diff-{n}", _f32(pos), np.zeros((n, 3), np.float32),
                 np.full(n, r, np.float32), bodies, n_steps=50)


def surface_height(pos, r):
    """Top of the full layers of a bed: the 99th percentile of z plus r (a
    partly filled top layer holds fewer than 1% of the grains)."""
    return float(np.percentile(np.asarray(pos)[:, 2], 99.0)) + float(r)


def polydisperse_radii(n, rng, median=0.002, sigma=0.25, lo=0.001, hi=0.004):
    r = np.exp(math.log(median) + sigma * rng.normal(size=n))
    return np.clip(r, lo, hi)


def large_scene(seed=0, n=1 << 22, side=2.0, gap=1.02):
    """4,194,304 spheres with lognormal radii (median 2 mm, sigma 0.25, clipped
    to [1, 4] mm) filling a walled side x side m box, in random index order,
    with a box tool (0.05 x 0.3 x 0.2 m) and a capsule tool (radius 2 cm, 15 cm
    between cap centres) above the bed, moving down into it.

    The bed is built to settle within a few tens of steps: the radii are sorted
    and cut into horizontal layers, each a square lattice whose spacing is
    2.04 times the largest radius in it (jitter U(+-1.5%) of that radius across,
    U(+-0.5%) up);
    the layers are stacked in random order, each 2% of the radius sum above the
    one below, so the start has no contacts and compacts by grains sinking
    into the hollows of the layer beneath (falls of at most a few mm)."""
    rng = np.random.default_rng(seed)
    pos, rad, top = layered_polydisperse_bed(n, side, rng, gap=gap)
    box = box_tool((0.6, 1.0, top + 0.11), (0.025, 0.15, 0.1), nu=(0.2, 0.0, -0.3))
    cap = capsule_tool((1.4, 1.0, top + 0.03), 0.02, 0.075, nu=(-0.2, 0.0, -0.3), omega=(0.0, 1.0, 0.0),
                       R=np.array([[1.0, 0, 0], [0, 0, -1.0], [0, 1.0, 0]]))
    bodies = walled_box(0.0, side, 0.0, side) + [box, cap]
    return Scene(f"large-{n}", _f32(pos), np.zeros((n, 3), np.float32), _f32(rad), bodies, dt=1e-3,
                 n_iters=64, mu=0.5, alpha=0.2, n_steps=100)


def layered_polydisperse_bed(n, side, rng, gap=1.02):
    """The large bed's start (see large_scene): lognormal radii sorted and cut
    into square-lattice layers over a side x side footprint, stacked in random
    order `gap` times the sum of the layers' largest radii apart (1.02: 2%
    apart; below 1, vertically aligned grains of adjacent layers overlap),
    index order shuffled.  Returns (positions, radii, top of the highest
    layer)."""
    rad = np.sort(polydisperse_radii(n, rng))
    pos = np.zeros((n, 3))
    layers = []
    k = 0
    while k < n:
        # the layer's largest radius sets its spacing; it only grows as the
        # layer shrinks, so the loop ends
        rl = float(rad[k])
        while True:
            per_row = int(math.floor((side - 2.0 * rl) / (2.04 * rl))) + 1
            cnt = min(n - k, per_row * per_row)
            r_end = float(rad[k + cnt - 1])
            if r_end <= rl:
                break
            rl = r_end
        layers.append((k, cnt, per_row, 2.04 * rl, rl))
        k += cnt
    order = rng.permutation(len(layers))
    z = 0.0
    prev_r = 0.0
    for li in order:
        k0, cnt, per_row, sp, rl = layers[li]
        z += (prev_r + rl) * gap if prev_r else rl * 1.02
        idx = np.arange(cnt)
        row, col = np.divmod(idx, per_row)
        o = 0.5 * (side - (per_row - 1) * sp)
        pos[k0:k0 + cnt, 0] = o + sp * col
        pos[k0:k0 + cnt, 1] = o + sp * row
        pos[k0:k0 + cnt, 2] = z
        pos[k0:k0 + cnt, :2] += rng.uniform(-0.015 * rl, 0.015 * rl, size=(cnt, 2))
        pos[k0:k0 + cnt, 2] += rng.uniform(-0.005 * rl, 0.005 * rl, size=cnt)
        prev_r = rl
    perm = rng.permutation(n)
    pos, rad = pos[perm], rad[perm]
    return pos, rad, z + prev_r


def random_spheres(n, box, r, rng, r_jitter=0.0):
    """Uniform random centres in ``box`` = ((x0,x1),(y0,y1),(z0,z1)); radii
    r*(1+U(-r_jitter, r_jitter)).  Used for small brute-force tests."""
    lo = np.array([b[0] for b in box])
    hi = np.array([b[1] for b in box])
    x = lo + (hi - lo) * rng.random((n, 3))
    rad = r * (1.0 + r_jitter * rng.uniform(-1, 1, size=n))
    return _f32(x), _f32(rad)


def loose_lattice(n, r, origin, rng, spacing_factor=2.02, jitter_frac=0.06, shuffle=True):
    """n spheres on the first n sites of a cubic lattice (spacing
    spacing_factor * r, jitter U(+-jitter_frac * r) per coordinate), in random
    index order when shuffle is set: a physical (not over-packed) random input
    whose index order is not spatial."""
    side = int(math.ceil(n ** (1.0 / 3.0))) if n else 0
    pos = jittered_lattice((side, side, side), spacing_factor * r, origin, jitter_frac * r, rng)[:n]
    if shuffle and n:
        pos = pos[rng.permutation(n)]
    return _f32(pos), np.full(n, r, np.float32)


def scaled(scene: Scene, n: int, seed=0):
    """A smaller bed of the same structure as ``scene`` (same radius and
    packing) for tests that need the full-size recipe at oracle-friendly size."""
    r = float(scene.radius[0])
    rng = np.random.default_rng(seed)
    side = max(0.05, math.sqrt(n / 10.0) * 2 * r)
    pos = packed_bed(n, r, 0.0, side, 0.0, side, rng)
    return Scene(f"{scene.name}-scaled{n}", _f32(pos), np.zeros((n, 3), np.float32),
                 np.full(n, r, np.float32), walled_box(0.0, side, 0.0, side),
                 dt=scene.dt, n_iters=scene.n_iters, mu=scene.mu, alpha=scene.alpha,
                 n_steps=scene.n_steps)


def gear_grid(outer=0.03, depth=0.006, teeth=12, thickness=0.02, helix=20.0, bore=0.008, inv_spacing=512.0):
    """A helical gear sampled on a grid (body frame, axis z): a toothed disc of
    outer radius ``outer`` whose tooth profile turns by ``helix`` rad/m along
    the axis, with a central bore.  The field is a distance bound (radial gap
    to the profile, intersected with the slab and the bore), exact enough to
    stand in for a mesh's distance field."""
    m = 0.006

    def fn(p):
        rho = np.linalg.norm(p[:, :2], axis=1)
        th = np.arctan2(p[:, 1], p[:, 0])
        prof = outer - depth * (0.5 - 0.5 * np.cos(teeth * (th - helix * p[:, 2])))
        disc = np.maximum(rho - prof, np.abs(p[:, 2]) - 0.5 * thickness)
        return np.maximum(disc, bore - rho)

    lo = (-outer - m, -outer - m, -0.5 * thickness - m)
    hi = (outer + m, outer + m, 0.5 * thickness + m)
    return sdf_grid(fn, lo, hi, inv_spacing)


def tower_grid(radius, z0, z1, inv_spacing=256.0):
    """The wall of a vertical cylindrical tower of the given radius (solid
    outside the cylinder), sampled on a grid over the tower's height."""
    m = 0.01
    return sdf_grid(lambda p: radius - np.linalg.norm(p[:, :2], axis=1), (-radius - m, -radius - m, z0 - m),
                    (radius + m, radius + m, z1 + m), inv_spacing)


def gear_tower(n=16384, n_gears=10, seed=0, r=0.002, radius=0.1, height=0.5, omega_max=6.0):
    """The many-body benchmark of Sec. III-B (helical gears spinning in a tall
    cylindrical tower, particles recycled from the bottom to the top): n
    spheres on a loose lattice inside the tower (random index order), n_gears
    copies of one gear grid at random positions and axis orientations, each
    spinning about its own axis at a uniformly random rate in
    [-omega_max, omega_max] rad/s with its centre fixed.  Returns the scene
    and the cyclic boundary (z_lo, z_hi) to pass to the simulator."""
    rng = np.random.default_rng(seed)
    tower = tower_grid(radius, 0.0, height)
    gear = gear_grid()
    bodies = [grid_tool(tower, (0.0, 0.0, 0.0))]
    centres = []
    for _ in range(n_gears):
        for _try in range(200):
            c = np.array([rng.uniform(-0.05, 0.05), rng.uniform(-0.05, 0.05), rng.uniform(0.06, height - 0.06)])
            if all(np.linalg.norm(c - q) > 0.075 for q in centres):
                break
        centres.append(c)
        Rm = random_rotation(rng)
        w = rng.uniform(-omega_max, omega_max)
        bodies.append(grid_tool(gear, c, omega=w * Rm[:, 2], R=Rm))
    # particles: a cubic lattice inside the tower, outside every gear's box
    sp = 2.02 * r
    k = int(np.ceil(2 * radius / sp)) + 1
    g = np.arange(k) * sp - radius
    nz = int(np.ceil(height / sp))
    zz = 0.004 + np.arange(nz) * sp
    X, Y, Z = np.meshgrid(g, g, zz, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    pts = pts[np.linalg.norm(pts[:, :2], axis=1) < radius - 1.5 * r]
    keep = np.ones(len(pts), bool)
    for c in centres:
        keep &= np.linalg.norm(pts - c, axis=1) > 0.045
    pts = pts[keep]
    if len(pts) < n:
        raise ValueError(f"the tower holds only {len(pts)} lattice sites")
    pts = pts[np.sort(rng.choice(len(pts), n, replace=False))]
    pts += rng.uniform(-0.05 * r, 0.05 * r, size=pts.shape)
    pts = pts[rng.permutation(n)]
    sc = Scene(f"gears-{n}-{n_gears}", _f32(pts), np.zeros((n, 3), np.float32), np.full(n, r, np.float32),
               bodies, dt=1e-3, n_iters=20, mu=0.5, alpha=0.2, n_steps=100)
    return sc, (0.0, float(height))
