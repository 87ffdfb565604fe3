"""FP64 CPU oracle for the granular contact step -- TEST INFRASTRUCTURE ONLY.

Python view of ``liboracle.so`` (built from ``oracle.cpp`` by ``oracle.build``).
Only the test suite, the smoke check and the benchmark's CPU-baseline leg use
it; the product path never imports this package.

Every function cites the part of arXiv 2306.01369 it follows; the C++ source
states the readings taken where the paper is silent or garbled.
"""
from __future__ import annotations

import ctypes as C
import os
import math

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

SHAPES = {"plane": 0, "box": 1, "capsule": 2, "grid": 3}


class Body(C.Structure):
    _fields_ = [("shape", C.c_int32), ("env", C.c_int32), ("params", C.c_float * 4),
                ("R", C.c_double * 9), ("t", C.c_double * 3), ("nu", C.c_double * 3),
                ("omega", C.c_double * 3), ("gv", C.c_void_p), ("gn", C.c_int32 * 3), ("go", C.c_float * 3),
                ("gih", C.c_float), ("gpad", C.c_int32)]


class BodyTan(C.Structure):
    """Tangents of a body's pose and twist (forward-mode derivatives)."""
    _fields_ = [("R", C.c_double * 9), ("t", C.c_double * 3), ("nu", C.c_double * 3),
                ("omega", C.c_double * 3)]


class Camera(C.Structure):
    """A depth camera: pose = row-major [R | t] (camera -> world), looking
    along its +z axis; params = (p0, p1, far, 0)."""
    _fields_ = [("env", C.c_int32), ("kind", C.c_int32), ("width", C.c_int32), ("height", C.c_int32),
                ("pose", C.c_float * 12), ("params", C.c_float * 4)]


CAMERA_KINDS = {"ortho": 0, "perspective": 1}


class Params(C.Structure):
    _fields_ = [("dt", C.c_double), ("alpha", C.c_double), ("mu", C.c_double),
                ("relax", C.c_double), ("density", C.c_double), ("g", C.c_double * 3),
                ("n_iters", C.c_int32), ("mass_split", C.c_int32), ("inv_c", C.c_float),
                ("pad", C.c_int32), ("n_h", C.c_int64), ("cyc_lo", C.c_double), ("cyc_hi", C.c_double)]


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = C.CDLL(path)
        P = C.POINTER
        L.ggo_hash.restype = C.c_int64
        L.ggo_hash.argtypes = [C.c_int64] * 4
        L.ggo_cell_index.argtypes = [C.c_int64, C.c_void_p, C.c_float, C.c_int64, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_void_p]
        L.ggo_pair_touch.restype = C.c_int32
        L.ggo_pair_touch.argtypes = [C.c_void_p, C.c_void_p, C.c_float, C.c_float]
        L.ggo_sdf_f32.restype = C.c_float
        L.ggo_sdf_f32.argtypes = [P(Body), C.c_void_p]
        L.ggo_sdf_f64.restype = C.c_double
        L.ggo_sdf_f64.argtypes = [P(Body), C.c_void_p, C.c_void_p]
        L.ggo_pp_bruteforce.restype = C.c_int64
        L.ggo_pp_bruteforce.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                        C.c_void_p]
        L.ggo_pp_hashgrid.restype = C.c_int64
        L.ggo_pp_hashgrid.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_float,
                                      C.c_int64, C.c_int64, C.c_void_p, C.c_void_p]
        L.ggo_pb_contacts.restype = C.c_int64
        L.ggo_pb_contacts.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                      P(Body), C.c_int64, C.c_void_p]
        L.ggo_advance_bodies.argtypes = [C.c_int32, P(Body), C.c_double]
        L.ggo_step.restype = C.c_int64
        L.ggo_step.argtypes = [P(Params), C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_void_p, C.c_int32, P(Body), C.c_int32, C.c_int64,
                               C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int64]
        L.ggo_step_jvp.restype = C.c_int64
        L.ggo_step_jvp.argtypes = [P(Params), C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_int32, P(Body), P(BodyTan), C.c_int32,
                                   C.c_void_p, C.c_int64, C.c_int64, C.c_void_p]
        L.ggo_sizeof_body_tan.restype = C.c_int32
        L.ggo_num_threads.restype = C.c_int32
        L.ggo_sizeof_body.restype = C.c_int32
        L.ggo_sizeof_params.restype = C.c_int32
        L.ggo_render_depth.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_int32,
                                       P(Body), C.c_int32, P(Camera), C.c_void_p, C.c_int64, C.c_void_p]
        L.ggo_goal_reward.argtypes = [C.c_int64, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p]
        L.ggo_sizeof_camera.restype = C.c_int32
        assert L.ggo_sizeof_camera() == C.sizeof(Camera), "Camera layout mismatch"
        assert L.ggo_sizeof_body() == C.sizeof(Body), "Body layout mismatch"
        assert L.ggo_sizeof_params() == C.sizeof(Params), "Params layout mismatch"
        assert L.ggo_sizeof_body_tan() == C.sizeof(BodyTan), "BodyTan layout mismatch"
        _LIB = L
    return _LIB


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f32(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    if shape is not None:
        a = a.reshape(shape)
    return a


def default_cell(radius):
    """Cell size c = max(r_i + r_j) * (1 + 2^-10) and its binary32 reciprocal."""
    r = np.asarray(radius, dtype=np.float32)
    c = float(np.float32(2.0 * float(r.max()) * (1.0 + 2.0 ** -10))) if r.size else 1.0
    return c, float(np.float32(1.0) / np.float32(c))


def make_bodies(body_dicts):
    """ctypes bodies from scenes-style dicts.  A "grid" body carries
    b["grid"] = {"values": (nz, ny, nx), "origin", "inv_spacing"}; its values
    are kept alive on the returned array (attribute ``keep``)."""
    arr = (Body * max(1, len(body_dicts)))()
    keep = []
    for k, b in enumerate(body_dicts):
        B = arr[k]
        B.shape = SHAPES[b["shape"]]
        B.env = int(b.get("env", 0))
        if b["shape"] == "grid":
            g = b["grid"]
            vals = np.ascontiguousarray(g["values"], np.float32)
            keep.append(vals)
            B.gv = vals.ctypes.data
            B.gn[0], B.gn[1], B.gn[2] = vals.shape[2], vals.shape[1], vals.shape[0]
            for q in range(3):
                B.go[q] = float(g["origin"][q])
            B.gih = float(g["inv_spacing"])
            for q in range(4):
                B.params[q] = 0.0
        else:
            for q in range(4):
                B.params[q] = float(np.float32(b["params"][q]))
        R = np.asarray(b["R"], dtype=np.float64).reshape(9)
        for q in range(9):
            B.R[q] = float(R[q])
        for q in range(3):
            B.t[q] = float(b["t"][q])
            B.nu[q] = float(b["nu"][q])
            B.omega[q] = float(b["omega"][q])
    arr.keep = keep
    return arr


def bodies_to_f32_pose(arr, nb):
    """Round the FP64 poses to binary32 (the pose both sides see)."""
    for k in range(nb):
        for q in range(9):
            arr[k].R[q] = float(np.float32(arr[k].R[q]))
        for q in range(3):
            arr[k].t[q] = float(np.float32(arr[k].t[q]))
            arr[k].nu[q] = float(np.float32(arr[k].nu[q]))
            arr[k].omega[q] = float(np.float32(arr[k].omega[q]))
    return arr


# ------------------------------------------------- observations (Sec. III-A)

def make_cameras(cams):
    """ctypes cameras from dicts {"env", "kind" ("ortho" | "perspective"),
    "width", "height", "pose" (3 x 4), "params" (p0, p1, far[, 0])}."""
    arr = (Camera * max(1, len(cams)))()
    for k, c in enumerate(cams):
        A = arr[k]
        A.env = int(c.get("env", 0))
        A.kind = CAMERA_KINDS[c["kind"]]
        A.width, A.height = int(c["width"]), int(c["height"])
        pose = np.asarray(c["pose"], np.float32).reshape(12)
        for q in range(12):
            A.pose[q] = float(pose[q])
        prm = list(c["params"]) + [0.0] * (4 - len(c["params"]))
        for q in range(4):
            A.params[q] = float(np.float32(prm[q]))
    return arr


def _env_off(n, env_offsets):
    if env_offsets is None:
        return np.array([0, n], np.int64)
    return np.ascontiguousarray(env_offsets, np.int64)


def render_depth(x, radius, cams, bodies=(), env_offsets=None, pixels=None):
    """Depth images (Sec. III-A observations) of the binary32 positions x
    (n x 3) with radii `radius`: a list of (height, width) float32 arrays, or,
    when `pixels` (indices into the concatenated images) is given, the depths
    of those pixels only.  Plane bodies of each camera's environment are
    drawn; body poses are rounded to binary32 as the step sees them."""
    x = _f32(x, (-1, 3))
    r = _f32(radius)
    off = _env_off(len(x), env_offsets)
    A = make_cameras(cams)
    B = bodies_to_f32_pose(make_bodies(bodies), len(bodies))
    sizes = [int(c["width"]) * int(c["height"]) for c in cams]
    out = np.full(sum(sizes), np.nan, np.float32)
    pix = None if pixels is None else np.ascontiguousarray(pixels, np.int64)
    lib().ggo_render_depth(len(x), _ptr(x), _ptr(r), len(off) - 1, _ptr(off), len(bodies), B, len(cams), A,
                           _ptr(out), 0 if pix is None else len(pix), _ptr(pix))
    if pix is not None:
        return out[pix]
    imgs, at = [], 0
    for c, m in zip(cams, sizes):
        imgs.append(out[at:at + m].reshape(int(c["height"]), int(c["width"])))
        at += m
    return imgs


def goal_reward(x, boxes, env_offsets=None):
    """Goal-box reward per environment (Sec. III-A) and the particles inside:
    boxes = n_envs x (lo xyz, hi xyz)."""
    x = _f32(x, (-1, 3))
    off = _env_off(len(x), env_offsets)
    bx = _f32(boxes, (-1, 6))
    ne = len(off) - 1
    assert bx.shape[0] == ne
    rew = np.zeros(ne, np.float64)
    ins = np.zeros(ne, np.int64)
    lib().ggo_goal_reward(len(x), _ptr(x), ne, _ptr(off), _ptr(bx), _ptr(rew), _ptr(ins))
    return rew, ins


# ---------------------------------------------------------------- Eq. (6)

def spatial_hash(kappa, n_h):
    """Bucket of one cell: XOR of p_a*(kappa_a - q), floored mod n_h (Eq. (6))."""
    return int(lib().ggo_hash(int(kappa[0]), int(kappa[1]), int(kappa[2]), int(n_h)))


def cell_index(x, inv_c, n_h, bucket_offset=None, env_n_h=None):
    """(kappa (n,3) int64, h (n,) int64): kappa = rne(fl32(x * inv_c)) and h by Eq. (6)."""
    x = _f32(x, (-1, 3))
    n = x.shape[0]
    kappa = np.zeros((n, 3), np.int64)
    h = np.zeros(n, np.int64)
    bo = None if bucket_offset is None else np.ascontiguousarray(bucket_offset, np.int64)
    en = None if env_n_h is None else np.ascontiguousarray(env_n_h, np.int64)
    lib().ggo_cell_index(n, _ptr(x), C.c_float(inv_c), int(n_h), _ptr(bo), _ptr(en), _ptr(kappa), _ptr(h))
    return kappa, h


# ---------------------------------------------------------------- contacts

def pair_touch(xi, xj, ri, rj):
    a, b = _f32(xi), _f32(xj)
    return bool(lib().ggo_pair_touch(_ptr(a), _ptr(b), C.c_float(ri), C.c_float(rj)))


def pp_bruteforce(x, r, env=None):
    """O(n^2) contact set {(i, j): i < j, ||xi-xj||^2 <= (ri+rj)^2} (Sec. II-C)."""
    x, r = _f32(x, (-1, 3)), _f32(r)
    e = None if env is None else np.ascontiguousarray(env, np.int32)
    n = x.shape[0]
    cnt = lib().ggo_pp_bruteforce(n, _ptr(x), _ptr(r), _ptr(e), 0, None)
    out = np.zeros((max(cnt, 1), 2), np.int32)
    lib().ggo_pp_bruteforce(n, _ptr(x), _ptr(r), _ptr(e), cnt, _ptr(out))
    return out[:cnt]


def pp_hashgrid(x, r, inv_c, n_h, env=None):
    """Contact set through the linked hashmap of Alg. 2 and the 27-cell query
    (Sec. II-B).  Returns (pairs (C,2) sorted, candidates)."""
    x, r = _f32(x, (-1, 3)), _f32(r)
    e = None if env is None else np.ascontiguousarray(env, np.int32)
    n = x.shape[0]
    cand = np.zeros(1, np.int64)
    cnt = lib().ggo_pp_hashgrid(n, _ptr(x), _ptr(r), _ptr(e), C.c_float(inv_c), int(n_h), 0, None, _ptr(cand))
    out = np.zeros((max(cnt, 1), 2), np.int32)
    lib().ggo_pp_hashgrid(n, _ptr(x), _ptr(r), _ptr(e), C.c_float(inv_c), int(n_h), cnt, _ptr(out), _ptr(cand))
    return out[:cnt], int(cand[0])


def pb_contacts(x, r, body_dicts, env=None):
    """Particle-body contacts {(i, b): f32 SDF_b(x_i) - r_i <= 0} (Eq. (7))."""
    x, r = _f32(x, (-1, 3)), _f32(r)
    e = None if env is None else np.ascontiguousarray(env, np.int32)
    B = bodies_to_f32_pose(make_bodies(body_dicts), len(body_dicts))
    n = x.shape[0]
    cnt = lib().ggo_pb_contacts(n, _ptr(x), _ptr(r), _ptr(e), len(body_dicts), B, 0, None)
    out = np.zeros((max(cnt, 1), 2), np.int32)
    lib().ggo_pb_contacts(n, _ptr(x), _ptr(r), _ptr(e), len(body_dicts), B, cnt, _ptr(out))
    return out[:cnt]


def sdf32(body, x):
    B = bodies_to_f32_pose(make_bodies([body]), 1)
    return float(lib().ggo_sdf_f32(B, _ptr(_f32(x))))


def sdf64_body_frame(body, p):
    """FP64 SDF and unit gradient at body-frame point p (Sec. II-C)."""
    B = make_bodies([body])
    p = np.ascontiguousarray(p, np.float64)
    g = np.zeros(3)
    f = lib().ggo_sdf_f64(B, _ptr(p), _ptr(g))
    return float(f), g


# ---------------------------------------------------------------- the step

class Oracle:
    """FP64 simulation state stepped by the oracle (Alg. 1, Eqs. (1)-(7)).

    Positions/velocities are held in FP64; contact decisions use their
    binary32 rounding.  Body poses are FP64, advanced after each step."""

    def __init__(self, x, v, radius, bodies=(), *, dt=1e-3, alpha=0.2, mu=0.5, n_iters=20,
                 gravity=(0.0, 0.0, -9.81), relax=1.0, density=2500.0, mass_split=True,
                 cell_size=None, hash_size=None, env=None, cyclic_z=None):
        self.x = np.array(x, dtype=np.float64, copy=True).reshape(-1, 3)
        self.v = np.array(v, dtype=np.float64, copy=True).reshape(-1, 3)
        self.r = _f32(radius)
        self.n = self.x.shape[0]
        self.body_dicts = list(bodies)
        self.nb = len(self.body_dicts)
        self.B = bodies_to_f32_pose(make_bodies(self.body_dicts), self.nb)
        self.env = None if env is None else np.ascontiguousarray(env, np.int32)
        P = Params()
        P.dt, P.alpha, P.mu, P.relax, P.density = dt, alpha, mu, relax, density
        for a in range(3):
            P.g[a] = gravity[a]
        P.n_iters = n_iters
        P.mass_split = 1 if mass_split else 0
        if cell_size is None:
            cell_size, inv_c = default_cell(self.r)
        else:
            inv_c = float(np.float32(1.0) / np.float32(cell_size))
        P.inv_c = inv_c
        P.n_h = int(hash_size) if hash_size else max(1, 2 * self.n)
        if cyclic_z is not None:
            P.cyc_lo, P.cyc_hi = float(cyclic_z[0]), float(cyclic_z[1])
        self.P = P
        self.cell_size = cell_size
        self.stats = np.zeros(4, np.int64)

    def set_twists(self, tw, binary32=True):
        """tw: (n_bodies, 6) (nu, omega) for the next step, rounded to binary32
        (the values the GPU path receives) unless binary32 is False."""
        rnd = (lambda a: float(np.float32(a))) if binary32 else float
        for b in range(self.nb):
            for q in range(3):
                self.B[b].nu[q] = rnd(tw[b][q])
                self.B[b].omega[q] = rnd(tw[b][3 + q])

    def step(self, detail=False, n_hist=0, advance_bodies=True, fixed=None):
        """One step.  fixed = (pairs (C,2) int32, n_pp) uses that contact list
        instead of detecting (the contact set held fixed)."""
        n = self.n
        cap = 0
        fx, fpp, fpb = None, 0, 0
        if fixed is not None:
            fx = np.ascontiguousarray(fixed[0], np.int32)
            fpp = int(fixed[1])
            fpb = len(fx) - fpp
        if detail and fixed is not None:
            cap = len(fx)
        elif detail:
            # count first (dry detection) to size the outputs
            xf = self.x.astype(np.float32)
            pp, _ = pp_hashgrid(xf, self.r, self.P.inv_c, self.P.n_h, self.env)
            pbc = lib().ggo_pb_contacts(n, _ptr(_f32(xf)), _ptr(self.r), _ptr(self.env), self.nb, self.B, 0, None)
            cap = len(pp) + int(pbc)
        capm = max(cap, 1)
        pairs = np.zeros((capm, 2), np.int32) if detail else None
        imp = np.zeros((capm, 3)) if detail else None
        psi = np.zeros(capm) if detail else None
        nrm = np.zeros((capm, 3)) if detail else None
        dv = np.zeros((n, 3)) if detail else None
        hist = np.zeros((max(n_hist, 1), capm, 3)) if (detail and n_hist) else None
        Cn = lib().ggo_step(C.byref(self.P), n, _ptr(self.x), _ptr(self.v), _ptr(self.r), _ptr(self.env),
                            self.nb, self.B, 1 if advance_bodies else 0, cap, _ptr(pairs), _ptr(imp),
                            _ptr(psi), _ptr(nrm), _ptr(dv), int(n_hist), _ptr(hist), _ptr(self.stats),
                            _ptr(fx), fpp, fpb)
        if not detail:
            return None
        assert Cn == cap
        out = {"pairs": pairs[:cap], "impulses": imp[:cap], "psi": psi[:cap], "normals": nrm[:cap],
               "dv": dv, "n_pp": int(self.stats[1]), "n_pb": int(self.stats[2]),
               "candidates": int(self.stats[0])}
        if hist is not None:
            out["history"] = hist[:, :cap]
        return out

    def start_tangents(self, dx=None, dv=None):
        """Begin forward-mode differentiation: tangents of the current state
        (zero where None) and zero tangents of the body poses."""
        self.dx = np.zeros((self.n, 3)) if dx is None else np.array(dx, dtype=np.float64, copy=True).reshape(-1, 3)
        self.dv = np.zeros((self.n, 3)) if dv is None else np.array(dv, dtype=np.float64, copy=True).reshape(-1, 3)
        self.dB = (BodyTan * max(1, self.nb))()

    def set_twist_tangents(self, dtw):
        """dtw: (n_bodies, 6) tangents of (nu, omega) for the next step."""
        for b in range(self.nb):
            for q in range(3):
                self.dB[b].nu[q] = float(dtw[b][q])
                self.dB[b].omega[q] = float(dtw[b][3 + q])

    def step_jvp(self, advance_bodies=True, fixed=None):
        """One step carrying the tangents set by start_tangents (and
        set_twist_tangents): afterwards self.dx, self.dv hold the directional
        derivative of the state, with the decisions of the value run (the
        contact set, the normal clamp, the tangential scaling test)."""
        fx, fpp, fpb = None, 0, 0
        if fixed is not None:
            fx = np.ascontiguousarray(fixed[0], np.int32)
            fpp = int(fixed[1])
            fpb = len(fx) - fpp
        return int(lib().ggo_step_jvp(C.byref(self.P), self.n, _ptr(self.x), _ptr(self.v), _ptr(self.dx),
                                      _ptr(self.dv), _ptr(self.r), _ptr(self.env), self.nb, self.B, self.dB,
                                      1 if advance_bodies else 0, _ptr(fx), fpp, fpb, _ptr(self.stats)))

    def body_pose(self, b):
        R = np.array(self.B[b].R[:]).reshape(3, 3)
        t = np.array(self.B[b].t[:])
        return R, t


def num_threads():
    return int(lib().ggo_num_threads())


def scene_oracle(scene, **kw):
    """Oracle initialised from a scenes.Scene."""
    env = None
    if scene.env_offsets is not None:
        env = np.repeat(np.arange(len(scene.env_offsets) - 1, dtype=np.int32), np.diff(scene.env_offsets))
    args = dict(dt=scene.dt, alpha=scene.alpha, mu=scene.mu, n_iters=scene.n_iters,
                gravity=scene.gravity, env=env)
    args.update(kw)
    return Oracle(scene.x, scene.v, scene.radius, scene.bodies, **args)
